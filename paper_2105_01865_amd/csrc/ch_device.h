// ch_device.h -- device-side building blocks of libch: the per-cell
// explicit terms and the phases of the three directional passes of one
// RK3 substage of the Cahn-Hilliard update (arXiv 2105.01865, sec. 3 and
// sec. 3.1).
//
// Every phase is a plain function of (thread id, thread count, task) that
// touches only global memory and the work-group's LDS array, so a kernel is
// a sequence of phases separated by work-group barriers.  The functions are
// __host__ __device__: the HIP kernels call them per thread, and a host
// harness can run the same phases thread by thread, in order, to check the
// indexing on the CPU.
//
// Line solves.  Each directional factor of eq-fac, I + r (1,-4,6,-4,1), has
// constant coefficients, and its symbol factors as
//   1 + r (z - 2 + 1/z)^2 = c (1 + a1/z + a2/z^2) (1 + a1 z + a2 z^2),
// where x^2 + a1 x + a2 has its two (complex conjugate) roots inside the unit
// circle.  The solve is then a causal recurrence
//   w_i = b_i / c - a1 w_{i-1} - a2 w_{i-2}
// followed by an anti-causal one
//   y_i = w_i - a1 y_{i+1} - a2 y_{i+2},
// both stable, with responses that decay geometrically.  A chunk of a line
// needs only a warm-up of `tw` points before it (forward) and after it
// (backward) to reach the periodic solution -- or, through the even
// reflection of the data, the no-flux one -- to a tolerance the host picks
// from the decay rate.  This replaces a serial inversion per line by
// independent chunks that many threads march at once.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define CH_HD __host__ __device__ __forceinline__
#else
#define CH_HD inline
#endif

namespace chd {

enum { PASS_X = 0, PASS_Y = 1, PASS_Z = 2 };

// One box of the (possibly single-box) batch.  Plain data, copied to the
// device once per configuration.
struct BoxDesc {
    int32_t n[3];       // cells along x, y, z
    int32_t bc[3];      // 0 periodic, 1 no-flux
    int32_t nf[3];      // faces stored along x (u), y (v), z (w)
    int32_t x_rows;     // rows of one x-pass task
    int64_t c_off;      // first element of this box in C, E, q
    int64_t u_off, v_off, w_off;
    double inv_h, inv_h2, inv_pe, eps;
    double psi[4];      // psi'(C) = psi0 + psi1 C + psi2 C^2 + psi3 C^3
    // per RK3 substage k = 0, 1, 2
    double gdt[3];      // gamma_k dt
    double rdt[3];      // rho_k dt
    double bdt[3];      // alpha_k dt / Pe * kappa Cn^2 / h^4
    double a1[3], a2[3], ic[3];   // line-solve recurrences (ic = 1/c)
    int32_t tw[3];      // warm-up length of the recurrences
    int32_t seg[2];     // segment length of the y and z passes
    int32_t task0[3];   // first global task of this box in passes x, y, z
    int32_t ntask[3];   // tasks of this box in passes x, y, z
    int32_t mblk0;      // first mass block of this box
    int32_t nmblk;      // mass blocks of this box
};

// Launch-wide constants of one pass.
struct PassArgs {
    int32_t k;          // substage 0, 1, 2
    int32_t e_mode;     // x pass: 0 write E, 1 read old E and write E, 2 read old E
    int32_t lanes;      // y/z pass: x columns per task (32 or 64)
    int32_t rp;         // x pass: LDS row pitch (max rows + 1)
    int32_t tw_max;     // largest warm-up over boxes (LDS layout)
    int32_t nx_max;     // largest line length of this pass over boxes (LDS layout)
    int32_t kx;         // x pass: chunk length (0 = derive)
};

// Index of a cell that may lie outside [0, n): periodic wrap, or even
// reflection about the walls (C[-1-m] = C[m], C[n+m] = C[n-1-m]).
CH_HD int map_idx(int i, int n, int bc)
{
    if (i >= 0 && i < n) return i;
    if (n == 1) return 0;
    if (bc == 0) {
        int m = i % n;
        return m < 0 ? m + n : m;
    }
    int p = 2 * n;
    int m = i % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

// Fifth-order WENO (Jiang-Shu, point values as cell averages): value at the
// face between c and d with upwind side a.
template <typename T>
CH_HD T weno5(T a, T b, T c, T d, T e, T eps)
{
    const T sixth = T(1) / T(6);
    const T q0 = (T(2) * a - T(7) * b + T(11) * c) * sixth;
    const T q1 = (-b + T(5) * c + T(2) * d) * sixth;
    const T q2 = (T(2) * c + T(5) * d - e) * sixth;
    const T k13 = T(13) / T(12), qu = T(0.25);
    const T t0 = a - T(2) * b + c, u0 = a - T(4) * b + T(3) * c;
    const T t1 = b - T(2) * c + d, u1 = b - d;
    const T t2 = c - T(2) * d + e, u2 = T(3) * c - T(4) * d + e;
    const T s0 = k13 * t0 * t0 + qu * u0 * u0;
    const T s1 = k13 * t1 * t1 + qu * u1 * u1;
    const T s2 = k13 * t2 * t2 + qu * u2 * u2;
    const T e0 = eps + s0, e1 = eps + s1, e2 = eps + s2;
    const T w0 = T(0.1) / (e0 * e0);
    const T w1 = T(0.6) / (e1 * e1);
    const T w2 = T(0.3) / (e2 * e2);
    return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

template <typename T>
CH_HD T psi_prime(const double* p, T c)
{
    return ((T(p[3]) * c + T(p[2])) * c + T(p[1])) * c + T(p[0]);
}

// Fourth difference (1,-4,6,-4,1) in nested form: differences of adjacent
// values first, which keeps single precision accurate on smooth data.
template <typename T>
CH_HD T d4(T m2, T m1, T c0, T p1, T p2)
{
    const T a = m1 - m2, b = c0 - m1, c = p1 - c0, d = p2 - p1;
    return ((d - c) - (c - b)) - ((c - b) - (b - a));
}

// The explicit terms of cell (i, j, kz) of box bd.  Returns
//   E = -div(u C) + lap psi'(C) / Pe          (through *e_out)
//   B = sum_d (1,-4,6,-4,1)_d C              (return value, unscaled)
template <typename T>
CH_HD T cell_terms(const BoxDesc& bd, const T* __restrict__ C, const T* __restrict__ U,
                   const T* __restrict__ V, const T* __restrict__ W, int i, int j, int kz,
                   T* e_out)
{
    const int nx = bd.n[0], ny = bd.n[1], nz = bd.n[2];
    const int64_t plane = (int64_t)nx * ny;
    const T* Cb = C + bd.c_off;
    // C along each axis at offsets -3..3
    T cx[7], cy[7], cz[7];
    const int64_t rowz = (int64_t)kz * plane;
    const int64_t rowy = (int64_t)j * nx;
    for (int m = -3; m <= 3; ++m) {
        cx[m + 3] = Cb[rowz + rowy + map_idx(i + m, nx, bd.bc[0])];
        cy[m + 3] = Cb[rowz + (int64_t)map_idx(j + m, ny, bd.bc[1]) * nx + i];
        cz[m + 3] = Cb[(int64_t)map_idx(kz + m, nz, bd.bc[2]) * plane + rowy + i];
    }
    const T eps = T(bd.eps);
    // face velocities: low face = index of the cell, high face = next index
    // (wrapping to face 0 on a periodic axis)
    const int fx = bd.nf[0], fy = bd.nf[1];
    const int ih = (i + 1 == nx && bd.bc[0] == 0) ? 0 : i + 1;
    const int jh = (j + 1 == ny && bd.bc[1] == 0) ? 0 : j + 1;
    const int kh = (kz + 1 == nz && bd.bc[2] == 0) ? 0 : kz + 1;
    const T* Ub = U + bd.u_off;
    const T* Vb = V + bd.v_off;
    const T* Wb = W + bd.w_off;
    const int64_t ur = ((int64_t)kz * ny + j) * fx;
    const T ulo = Ub[ur + i], uhi = Ub[ur + ih];
    const int64_t vr = (int64_t)kz * fy * nx;
    const T vlo = Vb[vr + (int64_t)j * nx + i], vhi = Vb[vr + (int64_t)jh * nx + i];
    const T wlo = Wb[(int64_t)kz * plane + rowy + i], whi = Wb[(int64_t)kh * plane + rowy + i];

    // upwinded WENO face values: the left-biased stencil when the face
    // velocity is >= 0, the mirrored one otherwise
    T adv = T(0);
    {
        const T* c = cx;
        const bool pl = ulo >= T(0), ph = uhi >= T(0);
        const T flo = weno5<T>(pl ? c[0] : c[5], pl ? c[1] : c[4], pl ? c[2] : c[3],
                               pl ? c[3] : c[2], pl ? c[4] : c[1], eps);
        const T fhi = weno5<T>(ph ? c[1] : c[6], ph ? c[2] : c[5], ph ? c[3] : c[4],
                               ph ? c[4] : c[3], ph ? c[5] : c[2], eps);
        adv += uhi * fhi - ulo * flo;
    }
    {
        const T* c = cy;
        const bool pl = vlo >= T(0), ph = vhi >= T(0);
        const T flo = weno5<T>(pl ? c[0] : c[5], pl ? c[1] : c[4], pl ? c[2] : c[3],
                               pl ? c[3] : c[2], pl ? c[4] : c[1], eps);
        const T fhi = weno5<T>(ph ? c[1] : c[6], ph ? c[2] : c[5], ph ? c[3] : c[4],
                               ph ? c[4] : c[3], ph ? c[5] : c[2], eps);
        adv += vhi * fhi - vlo * flo;
    }
    {
        const T* c = cz;
        const bool pl = wlo >= T(0), ph = whi >= T(0);
        const T flo = weno5<T>(pl ? c[0] : c[5], pl ? c[1] : c[4], pl ? c[2] : c[3],
                               pl ? c[3] : c[2], pl ? c[4] : c[1], eps);
        const T fhi = weno5<T>(ph ? c[1] : c[6], ph ? c[2] : c[5], ph ? c[3] : c[4],
                               ph ? c[4] : c[3], ph ? c[5] : c[2], eps);
        adv += whi * fhi - wlo * flo;
    }
    // Laplacian of the bulk potential
    const T mu0 = psi_prime<T>(bd.psi, cx[3]);
    const T lap = (psi_prime<T>(bd.psi, cx[4]) - mu0) - (mu0 - psi_prime<T>(bd.psi, cx[2]))
                + (psi_prime<T>(bd.psi, cy[4]) - mu0) - (mu0 - psi_prime<T>(bd.psi, cy[2]))
                + (psi_prime<T>(bd.psi, cz[4]) - mu0) - (mu0 - psi_prime<T>(bd.psi, cz[2]));
    *e_out = -adv * T(bd.inv_h) + lap * T(bd.inv_h2) * T(bd.inv_pe);
    return d4<T>(cx[1], cx[2], cx[3], cx[4], cx[5]) + d4<T>(cy[1], cy[2], cy[3], cy[4], cy[5])
         + d4<T>(cz[1], cz[2], cz[3], cz[4], cz[5]);
}

// Box of a global task index (boxes sorted by task0 of the pass).
CH_HD int find_box(const BoxDesc* boxes, int nbox, int pass, int task)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].task0[pass] <= task) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Pass X: explicit terms, RHS and the x-line solve of eq-fac-1, for a task of
// `rows` complete x-lines (y0 .. y0+rows-1 at plane z).
// LDS: tb = (nx_max + 2 tw_max) x rp elements holding the RHS with halos,
// tw = (nx_max + tw_max) x rp elements holding the forward recurrence.
// Element of line position p (-tw <= p < nx + tw) and row r: tb[(p + tw) rp + r].
// ---------------------------------------------------------------------------
struct XTask {
    int z, y0, rows, nx, tw, kx;
};

CH_HD XTask x_task(const BoxDesc& bd, const PassArgs& pa, int task)
{
    XTask t;
    const int local = task - bd.task0[PASS_X];
    const int R = bd.x_rows;
    const int nyb = (bd.n[1] + R - 1) / R;
    t.z = local / nyb;
    t.y0 = (local % nyb) * R;
    t.rows = bd.n[1] - t.y0 < R ? bd.n[1] - t.y0 : R;
    t.nx = bd.n[0];
    t.tw = bd.tw[pa.k];
    t.kx = pa.kx;
    return t;
}

template <typename T>
CH_HD void x_phase_rhs(int tid, int nth, const BoxDesc& bd, const PassArgs& pa, const XTask& t,
                       const T* __restrict__ C, const T* __restrict__ U, const T* __restrict__ V,
                       const T* __restrict__ W, T* __restrict__ E, T* tb)
{
    const int nx = t.nx, k = pa.k, rp = pa.rp;
    const int64_t plane = (int64_t)bd.n[0] * bd.n[1];
    const T gdt = T(bd.gdt[k]), rdt = T(bd.rdt[k]), bdt = T(bd.bdt[k]);
    for (int item = tid; item < t.rows * nx; item += nth) {
        const int r = item / nx, i = item - r * nx;
        const int j = t.y0 + r;
        T e;
        const T b4 = cell_terms<T>(bd, C, U, V, W, i, j, t.z, &e);
        const int64_t at = bd.c_off + (int64_t)t.z * plane + (int64_t)j * nx + i;
        T rhs = gdt * e - bdt * b4;
        if (pa.e_mode != 0) rhs += rdt * E[at];
        if (pa.e_mode != 2) E[at] = e;
        tb[(i + t.tw) * rp + r] = rhs;
    }
}

template <typename T>
CH_HD void x_phase_halo(int tid, int nth, const BoxDesc& bd, const PassArgs& pa, const XTask& t,
                        T* tb)
{
    const int nx = t.nx, tw = t.tw, rp = pa.rp;
    const int span = 2 * tw;
    for (int item = tid; item < t.rows * span; item += nth) {
        const int r = item / span, m = item - r * span;
        const int p = m < tw ? m - tw : nx + (m - tw);
        const int s = map_idx(p, nx, bd.bc[0]);
        tb[(p + tw) * rp + r] = tb[(s + tw) * rp + r];
    }
}

// chunk length of the x solve: enough chunks to give every thread one
CH_HD int x_chunk(const XTask& t, int nth)
{
    if (t.kx > 0) return t.kx;
    const int per = nth / (t.rows > 0 ? t.rows : 1);
    const int len = t.nx + t.tw;
    int kx = (len + per - 1) / (per > 0 ? per : 1);
    return kx < 1 ? 1 : kx;
}

template <typename T, typename A>
CH_HD void x_phase_fwd(int tid, int nth, const BoxDesc& bd, const PassArgs& pa, const XTask& t,
                       const T* tb, A* twb)
{
    const int nx = t.nx, tw = t.tw, rp = pa.rp, k = pa.k;
    const int kx = x_chunk(t, nth);
    const int len = nx + tw;
    const int nch = (len + kx - 1) / kx;
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]), ic = A(bd.ic[k]);
    for (int item = tid; item < t.rows * nch; item += nth) {
        const int r = item % t.rows, c = item / t.rows;
        const int c0 = c * kx;
        const int c1 = c0 + kx < len ? c0 + kx : len;
        A w1 = A(0), w2 = A(0);
        for (int p = c0 - tw; p < c1; ++p) {
            const A w = A(tb[(p + tw) * rp + r]) * ic - a1 * w1 - a2 * w2;
            if (p >= c0) twb[p * rp + r] = w;
            w2 = w1;
            w1 = w;
        }
    }
}

template <typename T, typename A>
CH_HD void x_phase_bwd(int tid, int nth, const BoxDesc& bd, const PassArgs& pa, const XTask& t,
                       T* tb, const A* twb)
{
    const int nx = t.nx, tw = t.tw, rp = pa.rp, k = pa.k;
    const int kx = x_chunk(t, nth);
    const int nch = (nx + kx - 1) / kx;
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]);
    for (int item = tid; item < t.rows * nch; item += nth) {
        const int r = item % t.rows, c = item / t.rows;
        const int c0 = c * kx;
        const int e = c0 + kx < nx ? c0 + kx : nx;
        A y1 = A(0), y2 = A(0);
        for (int p = e + tw - 1; p >= c0; --p) {
            const A y = twb[p * rp + r] - a1 * y1 - a2 * y2;
            if (p < e) tb[(p + tw) * rp + r] = T(y);
            y2 = y1;
            y1 = y;
        }
    }
}

template <typename T>
CH_HD void x_phase_store(int tid, int nth, const BoxDesc& bd, const PassArgs& pa, const XTask& t,
                         const T* tb, T* __restrict__ Q)
{
    const int nx = t.nx, rp = pa.rp;
    const int64_t plane = (int64_t)bd.n[0] * bd.n[1];
    for (int item = tid; item < t.rows * nx; item += nth) {
        const int r = item / nx, i = item - r * nx;
        Q[bd.c_off + (int64_t)t.z * plane + (int64_t)(t.y0 + r) * nx + i] =
            tb[(i + t.tw) * rp + r];
    }
}

// ---------------------------------------------------------------------------
// Passes Y and Z: line solves of eq-fac-2 (q1 -> q2) and eq-fac-3
// (q2 -> dC, C += dC) for a task of `lanes` adjacent x columns and one
// segment [s0, s0 + len) of the line.  Lane l holds column x0 + l.  The
// forward recurrence reads q straight from global memory (coalesced across
// lanes) and keeps its values in LDS, wb[p * lanes + l] for 0 <= p < len + tw;
// the backward recurrence writes the result.
// ---------------------------------------------------------------------------
struct LTask {
    int plane;      // z (pass Y) or y (pass Z)
    int x0, s0, len, n, tw, bc;
    int64_t stride; // elements between consecutive line positions
    int64_t base;   // element of (x0, position 0) of this line family
};

CH_HD LTask l_task(const BoxDesc& bd, const PassArgs& pa, int pass, int task)
{
    LTask t;
    const int L = pa.lanes;
    const int nx = bd.n[0], ny = bd.n[1];
    const int axis = pass;                       // 1 = y, 2 = z
    const int n = bd.n[axis];
    const int S = bd.seg[axis - 1];
    const int nxb = (nx + L - 1) / L;
    const int nseg = (n + S - 1) / S;
    const int local = task - bd.task0[pass];
    t.plane = local / (nxb * nseg);
    const int rem = local - t.plane * (nxb * nseg);
    const int seg = rem / nxb;
    t.x0 = (rem - seg * nxb) * L;
    t.s0 = seg * S;
    t.len = n - t.s0 < S ? n - t.s0 : S;
    t.n = n;
    t.tw = bd.tw[pa.k];
    t.bc = bd.bc[axis];
    const int64_t plane = (int64_t)nx * ny;
    if (pass == PASS_Y) {
        t.stride = nx;
        t.base = bd.c_off + (int64_t)t.plane * plane + t.x0;
    } else {
        t.stride = plane;
        t.base = bd.c_off + (int64_t)t.plane * nx + t.x0;
    }
    return t;
}

template <typename T, typename A>
CH_HD void l_phase_fwd(int tid, int nth, const BoxDesc& bd, const PassArgs& pa, const LTask& t,
                       const T* __restrict__ Qin, A* wb)
{
    const int L = pa.lanes, k = pa.k;
    const int lane = tid % L, wv = tid / L, nw = nth / L;
    const int total = t.len + t.tw;
    const int kf = (total + nw - 1) / nw;
    const int c0 = wv * kf;
    const int c1 = c0 + kf < total ? c0 + kf : total;
    if (c0 >= c1) return;
    const bool live = t.x0 + lane < bd.n[0];
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]), ic = A(bd.ic[k]);
    A w1 = A(0), w2 = A(0);
    for (int p = c0 - t.tw; p < c1; ++p) {
        const int g = map_idx(t.s0 + p, t.n, t.bc);
        const A b = live ? A(Qin[t.base + (int64_t)g * t.stride + lane]) : A(0);
        const A w = b * ic - a1 * w1 - a2 * w2;
        if (p >= c0) wb[p * L + lane] = w;
        w2 = w1;
        w1 = w;
    }
}

// mode 0: Qout = y (pass Y); mode 1: Qout += y (pass Z, Qout = C)
template <typename T, typename A>
CH_HD void l_phase_bwd(int tid, int nth, const BoxDesc& bd, const PassArgs& pa, const LTask& t,
                       const A* wb, T* __restrict__ Qout, int mode)
{
    const int L = pa.lanes, k = pa.k;
    const int lane = tid % L, wv = tid / L, nw = nth / L;
    const int kb = (t.len + nw - 1) / nw;
    const int c0 = wv * kb;
    const int e = c0 + kb < t.len ? c0 + kb : t.len;
    if (c0 >= e) return;
    const bool live = t.x0 + lane < bd.n[0];
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]);
    A y1 = A(0), y2 = A(0);
    for (int p = e + t.tw - 1; p >= c0; --p) {
        const A y = wb[p * L + lane] - a1 * y1 - a2 * y2;
        if (p < e && live) {
            T* dst = Qout + t.base + (int64_t)(t.s0 + p) * t.stride + lane;
            if (mode == 0) *dst = T(y);
            else *dst = T(A(*dst) + y);
        }
        y2 = y1;
        y1 = y;
    }
}

// ---------------------------------------------------------------------------
// Mass: fixed-order partial sums of MASS_BLOCK elements per block, then a
// fixed-order sum of a box's partials.
// ---------------------------------------------------------------------------
enum { MASS_THREADS = 256, MASS_PER_THREAD = 16, MASS_BLOCK = MASS_THREADS * MASS_PER_THREAD };

template <typename T>
CH_HD double mass_thread_sum(int tid, const BoxDesc& bd, int blk, const T* C)
{
    const int64_t count = (int64_t)bd.n[0] * bd.n[1] * bd.n[2];
    const int64_t start = (int64_t)blk * MASS_BLOCK;
    double s = 0.0;
    for (int j = 0; j < MASS_PER_THREAD; ++j) {
        const int64_t e = start + (int64_t)j * MASS_THREADS + tid;
        if (e < count) s += double(C[bd.c_off + e]);
    }
    return s;
}

}  // namespace chd
