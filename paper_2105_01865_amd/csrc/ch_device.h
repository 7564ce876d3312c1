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
    int32_t zc;         // planes one x-pass task marches over
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
    int32_t lanes;      // y/z pass: x columns per task
    int32_t rmax;       // x pass: rows per task (LDS layout)
    int32_t tw_max;     // largest warm-up over boxes (LDS layout)
    int32_t nx_max;     // largest x extent over boxes (LDS layout)
    int32_t seg_max;    // y/z pass: longest segment over boxes (LDS layout)
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
// Execution of a work-group program.  A pass is written once as a sequence
// of phases; `ex.phase(f)` runs f(tid) for this thread and then waits at a
// work-group barrier on the GPU, and runs f for every thread in turn on the
// CPU.  Per-thread state that lives across phases is kept in `S* st` and
// addressed as st[ex.slot(tid)]: one local object on the GPU (registers),
// one per thread on the CPU.
// ---------------------------------------------------------------------------
#if defined(__HIPCC__)
struct GpuExec {
    int tid, nth;
    template <class F>
    __device__ __forceinline__ void phase(F&& f)
    {
        f(tid);
        __syncthreads();
    }
    __device__ __forceinline__ int slot(int) const { return 0; }
};
#endif

struct CpuExec {
    int nth;
    template <class F>
    void phase(F&& f)
    {
        for (int t = 0; t < nth; ++t) f(t);
    }
    int slot(int t) const { return t; }
};

// upwinded WENO value on a face from the six values c[0..5] of cells
// f-3 .. f+2 around the face between c[2] and c[3]
template <typename T>
CH_HD T face_weno(T vel, T c0, T c1, T c2, T c3, T c4, T c5, T eps)
{
    const bool p = vel >= T(0);
    return weno5<T>(p ? c0 : c5, p ? c1 : c4, p ? c2 : c3, p ? c3 : c2, p ? c4 : c1, eps);
}

// ---------------------------------------------------------------------------
// In-place chunked line solve of (I + r D4) y = b on an LDS tile.
// Element (p, l) of line l at position p (-tw <= p < n + tw) sits at
// tile[(p + tw) * pitch + l]; the halos hold the periodic or reflected
// continuation of b.  Thread tid works on line l = tid % nl, chunk
// c = tid / nl of length K.  Four phases, each followed by a barrier:
//   f1: forward warm-up over [c0 - tw, c0) (reads b)      -> state
//   f2: forward over the chunk, b -> w in place; the last chunk runs on to
//       n + tw so that every backward warm-up finds its w values
//   b1: backward warm-up over [e, e + tw) (reads w)       -> state
//   b2: backward over the chunk, w -> y in place
// ---------------------------------------------------------------------------
template <typename A>
struct LineState {
    A s1, s2;
};

struct Chunk {
    int l, c0, fend, bend;
    bool live;
};

// most chunks per line: every x-pass work-group has at least nx threads per
// line and every y/z work-group at least 8 threads per lane column
constexpr int X_CHAINS = 16;
constexpr int YZ_CHAINS = 8;

// Chunks of a line of n points: at most `cap` of them, none shorter than the
// warm-up.  The split depends only on the line (n, tw) and the pass, never on
// the launch, so a box gives bitwise the same result alone or in a batch.
CH_HD int line_chunk_len(int n, int tw, int cap)
{
    int nch = n / 16;
    if (nch > cap) nch = cap;
    if (nch < 1) nch = 1;
    int K = (n + nch - 1) / nch;
    if (K < tw) K = tw;
    return K < 1 ? 1 : K;
}

CH_HD Chunk line_chunk(int tid, int nl, int n, int tw, int cap)
{
    Chunk ch;
    const int K = line_chunk_len(n, tw, cap);
    ch.l = tid % nl;
    const int c = tid / nl;
    ch.c0 = c * K;
    ch.live = ch.c0 < n;
    const bool last = ch.c0 + K >= n;
    ch.fend = last ? n + tw : ch.c0 + K;
    ch.bend = ch.c0 + K < n ? ch.c0 + K : n;
    return ch;
}

// The recurrences walk the tile in batches of LB values: the batch's loads
// are independent of the chain and go out together.
constexpr int LB = 8;

template <typename A>
CH_HD void line_f1(const Chunk& ch, const A* tile, int pitch, int tw, A a1, A a2, A ic,
                   LineState<A>& st)
{
    A w1 = A(0), w2 = A(0);
    if (ch.live) {
        const A* base = tile + ch.l;
        for (int p0 = ch.c0 - tw; p0 < ch.c0; p0 += LB) {
            A v[LB];
#pragma unroll
            for (int j = 0; j < LB; ++j)
                v[j] = p0 + j < ch.c0 ? base[(p0 + j + tw) * pitch] : A(0);
#pragma unroll
            for (int j = 0; j < LB; ++j)
                if (p0 + j < ch.c0) {
                    const A w = v[j] * ic - a1 * w1 - a2 * w2;
                    w2 = w1;
                    w1 = w;
                }
        }
    }
    st.s1 = w1;
    st.s2 = w2;
}

template <typename A>
CH_HD void line_f2(const Chunk& ch, A* tile, int pitch, int tw, A a1, A a2, A ic,
                   const LineState<A>& st)
{
    if (!ch.live) return;
    A w1 = st.s1, w2 = st.s2;
    A* base = tile + ch.l;
    for (int p0 = ch.c0; p0 < ch.fend; p0 += LB) {
        A v[LB];
#pragma unroll
        for (int j = 0; j < LB; ++j)
            v[j] = p0 + j < ch.fend ? base[(p0 + j + tw) * pitch] : A(0);
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            const A w = v[j] * ic - a1 * w1 - a2 * w2;
            v[j] = w;
            w2 = w1;
            w1 = w;
        }
#pragma unroll
        for (int j = 0; j < LB; ++j)
            if (p0 + j < ch.fend) base[(p0 + j + tw) * pitch] = v[j];
    }
}

template <typename A>
CH_HD void line_b1(const Chunk& ch, const A* tile, int pitch, int tw, A a1, A a2,
                   LineState<A>& st)
{
    A y1 = A(0), y2 = A(0);
    if (ch.live) {
        const A* base = tile + ch.l;
        const int lo = ch.bend;
        for (int p0 = ch.bend + tw - 1; p0 >= lo; p0 -= LB) {
            A v[LB];
#pragma unroll
            for (int j = 0; j < LB; ++j)
                v[j] = p0 - j >= lo ? base[(p0 - j + tw) * pitch] : A(0);
#pragma unroll
            for (int j = 0; j < LB; ++j)
                if (p0 - j >= lo) {
                    const A y = v[j] - a1 * y1 - a2 * y2;
                    y2 = y1;
                    y1 = y;
                }
        }
    }
    st.s1 = y1;
    st.s2 = y2;
}

template <typename A>
CH_HD void line_b2(const Chunk& ch, A* tile, int pitch, int tw, A a1, A a2,
                   const LineState<A>& st)
{
    if (!ch.live) return;
    A y1 = st.s1, y2 = st.s2;
    A* base = tile + ch.l;
    for (int p0 = ch.bend - 1; p0 >= ch.c0; p0 -= LB) {
        A v[LB];
#pragma unroll
        for (int j = 0; j < LB; ++j)
            v[j] = p0 - j >= ch.c0 ? base[(p0 - j + tw) * pitch] : A(0);
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            const A y = v[j] - a1 * y1 - a2 * y2;
            v[j] = y;
            y2 = y1;
            y1 = y;
        }
#pragma unroll
        for (int j = 0; j < LB; ++j)
            if (p0 - j >= ch.c0) base[(p0 - j + tw) * pitch] = v[j];
    }
}

// ---------------------------------------------------------------------------
// Pass X: explicit terms, RHS and the x-line solve of eq-fac-1 for a task of
// `rows` complete x-lines (y0 .. y0+rows-1) marching over the planes
// z0 .. z0+nzc-1.  Thread tid owns the cells item = tid + nth m (m < MI) of
// the rows x nx plane tile for the whole march, and keeps for each the
// column of C at z-3 .. z+3 and the flux through its low z face in
// registers, so that each z face flux is computed once.  x and y face
// fluxes are computed once per face and exchanged through LDS.
//
// LDS (launch-wide pitches; all sizes from the largest box):
//   pb: (rmax + 6) x (nx_max + 6) T  C of the plane, rows y0-3 .. y0+rows+2,
//                                    columns -3 .. nx+2
//   fx: rmax x (nx_max + 1) T        flux through x face f of each row
//   fy: (rmax + 1) x nx_max T        flux through y face y0 + r
//   tb: (nx_max + 2 tw_max) x (rmax + 1) A   RHS -> solve tile
// ---------------------------------------------------------------------------
struct XLayout {
    size_t pb, fx, fy, tb, total;  // byte offsets and total size
    int pbp, fxp, fyp, tbp;        // pitches (elements)
};

CH_HD size_t al16(size_t b) { return (b + 15) & ~size_t(15); }

CH_HD XLayout x_layout(int nx_max, int rmax, int tw_max, int sT, int sA)
{
    XLayout L;
    L.pbp = nx_max + 6;
    L.fxp = nx_max + 1;
    L.fyp = nx_max;
    L.tbp = rmax + 1;
    L.pb = 0;
    L.fx = al16(L.pb + (size_t)(rmax + 6) * L.pbp * sT);
    L.fy = al16(L.fx + (size_t)rmax * L.fxp * sT);
    L.tb = al16(L.fy + (size_t)(rmax + 1) * L.fyp * sT);
    L.total = al16(L.tb + (size_t)(nx_max + 2 * tw_max) * L.tbp * sA);
    return L;
}

struct XZTask {
    int z0, nzc, y0, rows;
};

CH_HD XZTask xz_task(const BoxDesc& bd, int task)
{
    XZTask t;
    const int local = task - bd.task0[PASS_X];
    const int R = bd.x_rows;
    const int nyb = (bd.n[1] + R - 1) / R;
    const int zc = local / nyb;
    const int yb = local - zc * nyb;
    t.y0 = yb * R;
    t.rows = bd.n[1] - t.y0 < R ? bd.n[1] - t.y0 : R;
    t.z0 = zc * bd.zc;
    t.nzc = bd.n[2] - t.z0 < bd.zc ? bd.n[2] - t.z0 : bd.zc;
    return t;
}

template <typename T, typename A, int MI>
struct XState {
    T cz[MI][7];     // C at z-3 .. z+3 of each owned cell
    T fzl[MI];       // flux through the low z face of the current plane
    T pz[MI];        // z flux difference of the current plane
    T plap[MI];      // sum of second differences of psi'(C)
    T pb4[MI];       // sum of fourth differences of C
    int rx[MI];      // (row << 16) | x of each owned cell, -1 if none
    LineState<A> ls;
};

template <typename T, typename A, int MI, class X>
CH_HD void pass_x_program(X& ex, XState<T, A, MI>* st, const BoxDesc& bd, const PassArgs& pa,
                          int task, const T* __restrict__ C, const T* __restrict__ U,
                          const T* __restrict__ V, const T* __restrict__ W, T* __restrict__ E,
                          T* __restrict__ Q, unsigned char* smem)
{
    const XZTask t = xz_task(bd, task);
    const int nx = bd.n[0], ny = bd.n[1], nz = bd.n[2];
    const int fx = bd.nf[0], fy = bd.nf[1];
    const int k = pa.k, tw = bd.tw[k];
    const int nth = ex.nth;
    const XLayout L = x_layout(pa.nx_max, pa.rmax, pa.tw_max, (int)sizeof(T), (int)sizeof(A));
    T* pb = reinterpret_cast<T*>(smem + L.pb);
    T* fxb = reinterpret_cast<T*>(smem + L.fx);
    T* fyb = reinterpret_cast<T*>(smem + L.fy);
    A* tb = reinterpret_cast<A*>(smem + L.tb);
    const int64_t plane = (int64_t)nx * ny;
    const T* Cb = C + bd.c_off;
    const T* Ub = U + bd.u_off;
    const T* Vb = V + bd.v_off;
    const T* Wb = W + bd.w_off;
    T* Eb = E + bd.c_off;
    T* Qb = Q + bd.c_off;
    const T eps = T(bd.eps);
    const T gdt = T(bd.gdt[k]), rdt = T(bd.rdt[k]), bdt = T(bd.bdt[k]);
    const T inv_h = T(bd.inv_h), lap_s = T(bd.inv_h2 * bd.inv_pe);
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]), ic = A(bd.ic[k]);
    const int rows = t.rows;
    const int ncell = rows * nx;

    // owned cells
    ex.phase([&](int tid) {
        XState<T, A, MI>& s = st[ex.slot(tid)];
#pragma unroll
        for (int m = 0; m < MI; ++m) {
            const int item = tid + nth * m;
            s.rx[m] = item < ncell ? ((item / nx) << 16) | (item % nx) : -1;
        }
    });

    for (int zs = 0; zs < t.nzc; ++zs) {
        const int z = t.z0 + zs;
        // ---- load: C columns (queue), the plane tile with its halos
        ex.phase([&](int tid) {
            XState<T, A, MI>& s = st[ex.slot(tid)];
    #pragma unroll
        for (int m = 0; m < MI; ++m) {
                if (s.rx[m] < 0) continue;
                const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
                const int64_t col = (int64_t)(t.y0 + r) * nx + x;
                if (zs == 0) {
#pragma unroll
                    for (int q = 0; q < 7; ++q)
                        s.cz[m][q] = Cb[(int64_t)map_idx(z - 3 + q, nz, bd.bc[2]) * plane + col];
                } else {
#pragma unroll
                    for (int q = 0; q < 6; ++q) s.cz[m][q] = s.cz[m][q + 1];
                    s.cz[m][6] = Cb[(int64_t)map_idx(z + 3, nz, bd.bc[2]) * plane + col];
                }
                pb[(r + 3) * L.pbp + x + 3] = s.cz[m][3];
            }
            const int64_t zp = (int64_t)z * plane;
            // rows y0-3 .. y0-1 and y0+rows .. y0+rows+2
            for (int hr = 0; hr < 6; ++hr) {
                const int prow = hr < 3 ? hr : rows + hr;
                const int gy = map_idx(t.y0 - 3 + prow, ny, bd.bc[1]);
                for (int x = tid; x < nx; x += nth)
                    pb[prow * L.pbp + x + 3] = Cb[zp + (int64_t)gy * nx + x];
            }
            // columns -3..-1 and nx..nx+2 of every tile row
            for (int j = tid; j < 6 * (rows + 6); j += nth) {
                const int prow = j / 6, q = j - prow * 6;
                const int xc = q < 3 ? q - 3 : nx + q - 3;
                const int gy = map_idx(t.y0 - 3 + prow, ny, bd.bc[1]);
                pb[prow * L.pbp + xc + 3] = Cb[zp + (int64_t)gy * nx + map_idx(xc, nx, bd.bc[0])];
            }
        });
        // ---- faces, Laplacian of psi'(C), fourth differences
        ex.phase([&](int tid) {
            XState<T, A, MI>& s = st[ex.slot(tid)];
    #pragma unroll
        for (int m = 0; m < MI; ++m) {
                if (s.rx[m] < 0) continue;
                const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
                const int y = t.y0 + r;
                const T* row = pb + (r + 3) * L.pbp + x + 3;   // row[o] = C(x + o)
                const T* colm = pb + r * L.pbp + x + 3;        // colm[o * pbp] = C(y - 3 + o)
                // x: the low face of the cell, and face nx for the last cell
                const int64_t ur = ((int64_t)z * ny + y) * fx;
                {
                    const T ul = Ub[ur + x];
                    fxb[r * L.fxp + x] =
                        ul * face_weno<T>(ul, row[-3], row[-2], row[-1], row[0], row[1], row[2], eps);
                    if (x == nx - 1) {
                        const T uh = Ub[ur + (bd.bc[0] == 0 ? 0 : nx)];
                        fxb[r * L.fxp + nx] = uh * face_weno<T>(uh, row[-2], row[-1], row[0],
                                                                 row[1], row[2], row[3], eps);
                    }
                }
                // y: the low face, and the top face for the last row
                const int p = L.pbp;
                {
                    const T vl = Vb[((int64_t)z * fy + y) * nx + x];
                    fyb[r * L.fyp + x] = vl * face_weno<T>(vl, colm[0], colm[p], colm[2 * p],
                                                           colm[3 * p], colm[4 * p], colm[5 * p], eps);
                    if (r == rows - 1) {
                        const int yh = (y + 1 == ny && bd.bc[1] == 0) ? 0 : y + 1;
                        const T vh = Vb[((int64_t)z * fy + yh) * nx + x];
                        fyb[(r + 1) * L.fyp + x] =
                            vh * face_weno<T>(vh, colm[p], colm[2 * p], colm[3 * p], colm[4 * p],
                                              colm[5 * p], colm[6 * p], eps);
                    }
                }
                // z: the high face (the low one carries over from the plane below)
                const T* c = s.cz[m];
                {
                    const int64_t wc = (int64_t)y * nx + x;
                    if (zs == 0) {
                        const T wl = Wb[(int64_t)z * plane + wc];
                        s.fzl[m] = wl * face_weno<T>(wl, c[0], c[1], c[2], c[3], c[4], c[5], eps);
                    }
                    const int zh = (z + 1 == nz && bd.bc[2] == 0) ? 0 : z + 1;
                    const T wh = Wb[(int64_t)zh * plane + wc];
                    const T fzh = wh * face_weno<T>(wh, c[1], c[2], c[3], c[4], c[5], c[6], eps);
                    s.pz[m] = fzh - s.fzl[m];
                    s.fzl[m] = fzh;
                }
                const T mu0 = psi_prime<T>(bd.psi, c[3]);
                s.plap[m] = (psi_prime<T>(bd.psi, row[1]) - mu0) - (mu0 - psi_prime<T>(bd.psi, row[-1]))
                          + (psi_prime<T>(bd.psi, colm[4 * p]) - mu0)
                          - (mu0 - psi_prime<T>(bd.psi, colm[2 * p]))
                          + (psi_prime<T>(bd.psi, c[4]) - mu0) - (mu0 - psi_prime<T>(bd.psi, c[2]));
                s.pb4[m] = d4<T>(row[-2], row[-1], row[0], row[1], row[2])
                         + d4<T>(colm[p], colm[2 * p], colm[3 * p], colm[4 * p], colm[5 * p])
                         + d4<T>(c[1], c[2], c[3], c[4], c[5]);
            }
        });
        // ---- RHS into the solve tile
        ex.phase([&](int tid) {
            XState<T, A, MI>& s = st[ex.slot(tid)];
    #pragma unroll
        for (int m = 0; m < MI; ++m) {
                if (s.rx[m] < 0) continue;
                const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
                const T adv = (fxb[r * L.fxp + x + 1] - fxb[r * L.fxp + x])
                            + (fyb[(r + 1) * L.fyp + x] - fyb[r * L.fyp + x]) + s.pz[m];
                const T e = -adv * inv_h + s.plap[m] * lap_s;
                const int64_t at = (int64_t)z * plane + (int64_t)(t.y0 + r) * nx + x;
                T rhs = gdt * e - bdt * s.pb4[m];
                if (pa.e_mode != 0) rhs += rdt * Eb[at];
                if (pa.e_mode != 2) Eb[at] = e;
                tb[(x + tw) * L.tbp + r] = A(rhs);
            }
        });
        // ---- halo of the solve tile
        ex.phase([&](int tid) {
            const int span = 2 * tw;
            for (int j = tid; j < rows * span; j += nth) {
                const int r = j / span, q = j - r * span;
                const int pp = q < tw ? q - tw : nx + q - tw;
                tb[(pp + tw) * L.tbp + r] = tb[(map_idx(pp, nx, bd.bc[0]) + tw) * L.tbp + r];
            }
        });
        // ---- x solve
        ex.phase([&](int tid) {
            const Chunk ch = line_chunk(tid, rows, nx, tw, X_CHAINS);
            line_f1<A>(ch, tb, L.tbp, tw, a1, a2, ic, st[ex.slot(tid)].ls);
        });
        ex.phase([&](int tid) {
            const Chunk ch = line_chunk(tid, rows, nx, tw, X_CHAINS);
            line_f2<A>(ch, tb, L.tbp, tw, a1, a2, ic, st[ex.slot(tid)].ls);
        });
        ex.phase([&](int tid) {
            const Chunk ch = line_chunk(tid, rows, nx, tw, X_CHAINS);
            line_b1<A>(ch, tb, L.tbp, tw, a1, a2, st[ex.slot(tid)].ls);
        });
        ex.phase([&](int tid) {
            const Chunk ch = line_chunk(tid, rows, nx, tw, X_CHAINS);
            line_b2<A>(ch, tb, L.tbp, tw, a1, a2, st[ex.slot(tid)].ls);
        });
        // ---- store q
        ex.phase([&](int tid) {
            XState<T, A, MI>& s = st[ex.slot(tid)];
    #pragma unroll
        for (int m = 0; m < MI; ++m) {
                if (s.rx[m] < 0) continue;
                const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
                Qb[(int64_t)z * plane + (int64_t)(t.y0 + r) * nx + x] = T(tb[(x + tw) * L.tbp + r]);
            }
        });
    }
}

// ---------------------------------------------------------------------------
// Passes Y and Z: line solves of eq-fac-2 (q1 -> q2) and eq-fac-3
// (q2 -> dC, C += dC) for a task of `lanes` adjacent x columns and one
// segment [s0, s0 + len) of the line.  The segment and a warm-up halo of tw
// positions on each side are staged in LDS (coalesced rows of lanes
// elements), solved in place, and written back.
// LDS: (seg_max + 2 tw_max) x lanes A.
// ---------------------------------------------------------------------------
struct LTask {
    int plane;      // z (pass Y) or y (pass Z)
    int x0, s0, len, n, bc;
    int64_t stride; // elements between consecutive line positions
    int64_t base;   // element of (x0, position 0) of this line family
};

CH_HD LTask l_task(const BoxDesc& bd, const PassArgs& pa, int pass, int task)
{
    LTask t;
    const int Lw = pa.lanes;
    const int nx = bd.n[0], ny = bd.n[1];
    const int n = bd.n[pass];
    const int S = bd.seg[pass - 1];
    const int nxb = (nx + Lw - 1) / Lw;
    const int nseg = (n + S - 1) / S;
    const int local = task - bd.task0[pass];
    t.plane = local / (nxb * nseg);
    const int rem = local - t.plane * (nxb * nseg);
    const int seg = rem / nxb;
    t.x0 = (rem - seg * nxb) * Lw;
    t.s0 = seg * S;
    t.len = n - t.s0 < S ? n - t.s0 : S;
    t.n = n;
    t.bc = bd.bc[pass];
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

template <typename T, typename A, class X>
CH_HD void pass_line_program(X& ex, LineState<A>* st, const BoxDesc& bd, const PassArgs& pa,
                             int pass, int task, const T* __restrict__ Qin,
                             T* __restrict__ Qout, unsigned char* smem)
{
    const LTask t = l_task(bd, pa, pass, task);
    const int Lw = pa.lanes, nth = ex.nth, k = pa.k, tw = bd.tw[k];
    const int nlive = bd.n[0] - t.x0 < Lw ? bd.n[0] - t.x0 : Lw;
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]), ic = A(bd.ic[k]);
    A* tile = reinterpret_cast<A*>(smem);
    const int npos = t.len + 2 * tw;
    ex.phase([&](int tid) {
        const int l = tid % Lw;
        for (int q = tid / Lw; q < npos; q += nth / Lw) {
            const int g = map_idx(t.s0 + q - tw, t.n, t.bc);
            tile[q * Lw + l] = l < nlive ? A(Qin[t.base + (int64_t)g * t.stride + l]) : A(0);
        }
    });
    ex.phase([&](int tid) {
        const Chunk ch = line_chunk(tid, Lw, t.len, tw, YZ_CHAINS);
        line_f1<A>(ch, tile, Lw, tw, a1, a2, ic, st[ex.slot(tid)]);
    });
    ex.phase([&](int tid) {
        const Chunk ch = line_chunk(tid, Lw, t.len, tw, YZ_CHAINS);
        line_f2<A>(ch, tile, Lw, tw, a1, a2, ic, st[ex.slot(tid)]);
    });
    ex.phase([&](int tid) {
        const Chunk ch = line_chunk(tid, Lw, t.len, tw, YZ_CHAINS);
        line_b1<A>(ch, tile, Lw, tw, a1, a2, st[ex.slot(tid)]);
    });
    ex.phase([&](int tid) {
        const Chunk ch = line_chunk(tid, Lw, t.len, tw, YZ_CHAINS);
        line_b2<A>(ch, tile, Lw, tw, a1, a2, st[ex.slot(tid)]);
    });
    ex.phase([&](int tid) {
        const int l = tid % Lw;
        if (l >= nlive) return;
        for (int q = tid / Lw; q < t.len; q += nth / Lw) {
            T* dst = Qout + t.base + (int64_t)(t.s0 + q) * t.stride + l;
            const A y = tile[(q + tw) * Lw + l];
            if (pass == PASS_Z) *dst = T(A(*dst) + y);
            else *dst = T(y);
        }
    });
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
