// ch_kernels.hip -- HIP kernels of libch for gfx950 (CDNA4).
//
// One RK3 substage of the Cahn-Hilliard update is three launches
// (arXiv 2105.01865, eq-fac-1 .. eq-fac-3):
//   k_pass_x : explicit terms, RHS and the x-line solve; one work-group owns
//              complete x-lines, so the RHS goes straight into LDS and the
//              solve never leaves the chip
//   k_pass_y : y-line solve, x-columns across the lanes of a wave
//   k_pass_z : z-line solve and C += dC
// The path is stencil- and bandwidth-bound: no MFMA.  Work-group ids are
// remapped so that consecutive tasks (neighbouring lines that share stencil
// halos) land on the same XCD and its L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ch_device.h"
#include "ch_kernels.h"

namespace chk {

// Waves per SIMD the single-precision, one-cell-per-thread x kernel of the
// implicit scheme is compiled for (its register budget); the other variants
// keep the compiler's choice (forcing them spills).
#ifndef X_WAVES_F32_HINT
#define X_WAVES_F32_HINT 5
#endif

// Work-groups are dispatched round-robin over the 8 XCDs of the chip; give
// each XCD a contiguous range of tasks.
__device__ __forceinline__ int xcd_task(int wg, int nwg)
{
    const int nxcd = 8;
    const int per = nwg / nxcd, rem = nwg % nxcd;
    const int x = wg % nxcd, l = wg / nxcd;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + l;
}

// NT bounds the work-group size and so the registers per lane: 512 VGPRs per
// SIMD lane over the group's waves per SIMD (256 for 512 threads, 170 for
// 768, 128 for 1024).  E25 selects the explicit 25-point scheme (no solve,
// the new C is written to Q).
template <typename T, typename A, int MI, int NT, bool E25>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && MI == 1 && !E25 ? X_WAVES_F32_HINT : 1)))
k_pass_x(const chd::BoxDesc* __restrict__ boxes, int nbox, chd::PassArgs pa,
         const T* __restrict__ C, const T* __restrict__ U, const T* __restrict__ V,
         const T* __restrict__ W, T* __restrict__ E, T* __restrict__ Q)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int task = xcd_task(blockIdx.x, gridDim.x);
    const int b = chd::find_box(boxes, nbox, chd::PASS_X, task);
    chd::GpuExec ex{(int)threadIdx.x, (int)blockDim.x};
    chd::XState<T, A, MI> st;
    // double precision with registers to spare: uniform constants in lane registers
    constexpr bool VCONST = sizeof(T) == 8 && MI == 1 && NT <= 512 && !E25;
    chd::pass_x_program<T, A, MI, E25, chd::GpuExec, VCONST>(ex, &st, boxes[b], pa, task, C, U, V,
                                                             W, E, Q, smem);
}

// The row x-pass program (pass_x_row_program); NT bounds the group size, RM
// is the row mode (one row per task, several with per-thread row offsets, or
// several of whole waves).  Single precision with one row of a 512-cell line:
// at most 64 VGPRs (none spilled), so that four groups of 8 waves share a CU
// rather than three (the 512^3 x pass 941-955 -> 919-927 us; at 256 threads
// the same bound adds instructions and gains nothing).
template <typename T, typename A, int NT, int RM>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && RM == chd::XR_ONE && NT == 512 ? 8 : 1)))
k_pass_x_row(const chd::BoxDesc* __restrict__ boxes, int nbox, chd::PassArgs pa,
             const T* __restrict__ C, const T* __restrict__ U, const T* __restrict__ V,
             const T* __restrict__ W, T* __restrict__ E, T* __restrict__ Q)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int task = xcd_task(blockIdx.x, gridDim.x);
    const int b = chd::find_box(boxes, nbox, chd::PASS_X, task);
    chd::GpuExec ex{(int)threadIdx.x, (int)blockDim.x};
    chd::XRowState<T, A> st;
    chd::pass_x_row_program<T, A, RM, chd::GpuExec>(ex, &st, boxes[b], pa, task, C, U, V, W, E,
                                                    Q, smem);
}

// The segmented x-pass program (pass_x_seg_program): E read from Ein, the
// new one written to Eout.
template <typename T, typename A>
__global__ void __launch_bounds__(256)
k_pass_x_seg(const chd::BoxDesc* __restrict__ boxes, int nbox, chd::PassArgs pa,
             const T* __restrict__ C, const T* __restrict__ U, const T* __restrict__ V,
             const T* __restrict__ W, const T* __restrict__ Ein, T* __restrict__ Eout,
             T* __restrict__ Q)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int task = xcd_task(blockIdx.x, gridDim.x);
    const int b = chd::find_box(boxes, nbox, chd::PASS_X, task);
    chd::GpuExec ex{(int)threadIdx.x, (int)blockDim.x};
    chd::XSegState<T, A> st;
    chd::pass_x_seg_program<T, A, chd::GpuExec>(ex, &st, boxes[b], pa, task, C, U, V, W, Ein,
                                                Eout, Q, smem);
}

template <typename T, typename A, int PASS>
__global__ void __launch_bounds__(512)
k_pass_line(const chd::BoxDesc* __restrict__ boxes, int nbox, chd::PassArgs pa,
            const T* __restrict__ Qin, T* __restrict__ Qout)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int task = xcd_task(blockIdx.x, gridDim.x);
    const int b = chd::find_box(boxes, nbox, PASS, task);
    chd::GpuExec ex{(int)threadIdx.x, (int)blockDim.x};
    chd::LineState<A> st;
    chd::pass_line_program<T, A>(ex, &st, boxes[b], pa, PASS, task, Qin, Qout, smem);
}

// Mass, stage 1 body: block `blk` of box bd (MASS_BLOCK elements of C),
// summed in double in a fixed order, written to *partial.
template <typename T>
__device__ void mass_partial_body(const chd::BoxDesc& bd, int blk, const T* __restrict__ C,
                                  double* __restrict__ partial)
{
    __shared__ double sh[chd::MASS_THREADS];
    const int tid = threadIdx.x;
    sh[tid] = chd::mass_thread_sum<T>(tid, bd, blk, C);
    __syncthreads();
    for (int s = chd::MASS_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0) *partial = sh[0];
}

// Mass, stage 2 body: a box's nmblk partials summed in a fixed order and
// scaled by h^3.
__device__ void mass_final_body(const double* __restrict__ partial, int nmblk, double h3,
                                double* __restrict__ out)
{
    __shared__ double sh[chd::MASS_THREADS];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int i = tid; i < nmblk; i += chd::MASS_THREADS) s += partial[i];
    sh[tid] = s;
    __syncthreads();
    for (int st = chd::MASS_THREADS / 2; st > 0; st >>= 1) {
        if (tid < st) sh[tid] += sh[tid + st];
        __syncthreads();
    }
    if (tid == 0) *out = sh[0] * h3;
}

// Mass, stage 1: one fixed block of C per work-group (the box found from the
// block index).
template <typename T>
__global__ void __launch_bounds__(chd::MASS_THREADS)
k_mass_partial(const chd::BoxDesc* __restrict__ boxes, int nbox, const T* __restrict__ C,
               double* __restrict__ partial)
{
    const int blk = blockIdx.x;
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].mblk0 <= blk) lo = mid;
        else hi = mid - 1;
    }
    const chd::BoxDesc& bd = boxes[lo];
    mass_partial_body<T>(bd, blk - bd.mblk0, C, partial + blk);
}

// Mass, stage 2: one work-group per box.
__global__ void __launch_bounds__(chd::MASS_THREADS)
k_mass_final(const chd::BoxDesc* __restrict__ boxes, const double* __restrict__ partial,
             const double* __restrict__ h3, double* __restrict__ out)
{
    const chd::BoxDesc& bd = boxes[blockIdx.x];
    mass_final_body(partial + bd.mblk0, bd.nmblk, h3[blockIdx.x], out + blockIdx.x);
}

// The same two stages for one field described by value (no box table in
// device memory): the allocation-free mass.
template <typename T>
__global__ void __launch_bounds__(chd::MASS_THREADS)
k_mass_partial_one(chd::BoxDesc bd, const T* __restrict__ C, double* __restrict__ partial)
{
    mass_partial_body<T>(bd, blockIdx.x, C, partial + blockIdx.x);
}

__global__ void __launch_bounds__(chd::MASS_THREADS)
k_mass_final_one(int nmblk, const double* __restrict__ partial, double h3,
                 double* __restrict__ out)
{
    mass_final_body(partial, nmblk, h3, out);
}

// Velocity check: non-finite values anywhere, non-zero normal velocity on a
// no-flux wall.  Each work-group writes its two counts to flags[2 * wg].
template <typename T>
__global__ void __launch_bounds__(256)
k_check_velocity(const chd::BoxDesc* __restrict__ boxes, int nbox, const T* __restrict__ U,
                 const T* __restrict__ V, const T* __restrict__ W, int* __restrict__ flags)
{
    __shared__ int sh[2][256];
    int bad = 0, wall = 0;
    for (int b = 0; b < nbox; ++b) {
        const chd::BoxDesc& bd = boxes[b];
        const int nx = bd.n[0], ny = bd.n[1], nz = bd.n[2];
        const int64_t cnt[3] = {(int64_t)nz * ny * bd.nf[0], (int64_t)nz * bd.nf[1] * nx,
                                (int64_t)bd.nf[2] * ny * nx};
        const T* arr[3] = {U + bd.u_off, V + bd.v_off, W + bd.w_off};
        for (int d = 0; d < 3; ++d) {
            for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt[d];
                 e += (int64_t)gridDim.x * blockDim.x) {
                const T val = arr[d][e];
                if (!(val == val) || val - val != T(0)) ++bad;
                if (bd.bc[d] == 1) {
                    int64_t f;
                    if (d == 0) f = e % bd.nf[0];
                    else if (d == 1) f = (e / nx) % bd.nf[1];
                    else f = e / ((int64_t)ny * nx);
                    if ((f == 0 || f == bd.nf[d] - 1) && val != T(0)) ++wall;
                }
            }
        }
    }
    const int tid = threadIdx.x;
    sh[0][tid] = bad;
    sh[1][tid] = wall;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            sh[0][tid] += sh[0][tid + s];
            sh[1][tid] += sh[1][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        flags[2 * blockIdx.x] = sh[0][0];
        flags[2 * blockIdx.x + 1] = sh[1][0];
    }
}

// Coarse-to-fine velocity transfer, the separable tensor-product
// interpolation of sec. 3.4.  Work item = (band of JB target rows, target
// plane k), k fastest; each work-group takes a contiguous run of items
// (XCD-contiguous runs), so consecutive items are neighbouring target planes
// of one band, whose z stencils share most of their coarse planes: those
// rows come from L2 (at 512^3, 234 -> 201 us per FP32 component inside a
// step against the plane-major order):
//   A. the band's coarse rows, each combined over the 4 source planes of k's
//      z stencil, into LDS (coalesced along x; MA rows' loads in flight per
//      thread, through buffer resources on the 4 planes);
//   B. each target row of the band combines 4 of those rows (its y stencil)
//      into a second LDS row;
//   C. x stencil.  With the 6-point window property each thread owns 4
//      consecutive targets: it reads the 6 window points once and applies a
//      4 x 6 weight matrix built at start-up (4-wide stores); otherwise every
//      target reads its 4 taps.
// Band, z and y stencil entries are uniform per item and row, so they are
// read into scalar registers.  Every target element is written once, with
// non-temporal stores (nothing reads it back while it is in the caches, and
// streaming it out leaves them to the coarse rows, which are read again);
// the coarse data is read through the caches about (rows per band / band
// height) times per target plane.
template <typename T, int JB, int MA, bool PIPE>
__global__ void __launch_bounds__(256)
k_interp(InterpArgs a, const T* __restrict__ src, T* __restrict__ dst,
         const int* __restrict__ band, const int* __restrict__ izt, const T* __restrict__ wzt,
         const int* __restrict__ lyt, const T* __restrict__ wyt, const int* __restrict__ ixt,
         const double* __restrict__ wxt)
{
    typedef T T4 __attribute__((ext_vector_type(4)));
    constexpr int XQ = 4, NW = 6;
    extern __shared__ __align__(16) unsigned char smem[];
    const int sx = a.sx;
    T* zr = reinterpret_cast<T*>(smem);           // rmax x sx
    T* yr = zr + (size_t)a.rmax * sx;             // JB x sx
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nb = (a.tny + JB - 1) / JB;
    const int items = nb * a.tnz;
    const uint32_t pbytes = (uint32_t)(a.plane * sizeof(T));

    // x: thread -> targets xi0 .. xi0 + 3 of rows jj = rg0 (mod rgs)
    const int tc = (a.tnx + XQ - 1) / XQ;
    const bool win = a.xwin && tc <= nt;
    const int rgs = win ? nt / tc : 1;
    const int rg0 = win ? tid / tc : 0;
    const int xi0 = win ? XQ * (tid - rg0 * tc) : 0;
    const bool xact = win && rg0 < rgs;
    const bool vec = (a.tnx % XQ) == 0 && (reinterpret_cast<uintptr_t>(dst) % sizeof(T4)) == 0;
    int ws = 0;
    if (xact) ws = ixt[4 * xi0];
    int woff[NW];   // window points ws .. ws + NW - 1, cyclic in x
#pragma unroll
    for (int n = 0; n < NW; ++n) woff[n] = ws + n < sx ? ws + n : (ws + n) % sx;
    T M[XQ][NW];
#pragma unroll
    for (int q = 0; q < XQ; ++q)
#pragma unroll
        for (int n = 0; n < NW; ++n) M[q][n] = T(0);
    if (xact) {
#pragma unroll
        for (int q = 0; q < XQ; ++q)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bool ok = xi0 + q < a.tnx;
                int d = ok ? ixt[4 * (xi0 + q) + t] - ws : 0;
                if (d < 0) d += sx;
                const T w = ok ? T(wxt[4 * (xi0 + q) + t]) : T(0);
#pragma unroll
                for (int n = 0; n < NW; ++n) M[q][n] += d == n ? w : T(0);
            }
    }

    const int per = (items + a.nwg - 1) / a.nwg;
    const int it0 = xcd_task(blockIdx.x, a.nwg) * per;
    const int it1 = it0 + per < items ? it0 + per : items;
    // PIPE (one batch of loads covers an item: the coarse row fits the group
    // and no band is taller than the rows in flight): the next item's coarse
    // rows are loaded while this item's targets are stored, issued before
    // phase C and combined into LDS at the top of the next item.
    constexpr bool pipe = PIPE;
    T vp[PIPE ? MA : 1][4];
    auto issue = [&](int item) {   // the item's coarse rows at column tid
        if constexpr (!PIPE) return;
        const int b = item / a.tnz, k = item - b * a.tnz;
        const int base = band[2 * b], span = band[2 * b + 1];
        const chd::PlaneRef<T> p0(src + (int64_t)izt[4 * k] * a.plane, pbytes);
        const chd::PlaneRef<T> p1(src + (int64_t)izt[4 * k + 1] * a.plane, pbytes);
        const chd::PlaneRef<T> p2(src + (int64_t)izt[4 * k + 2] * a.plane, pbytes);
        const chd::PlaneRef<T> p3(src + (int64_t)izt[4 * k + 3] * a.plane, pbytes);
        const int cx = tid < sx ? tid : 0;
#pragma unroll
        for (int m = 0; m < (PIPE ? MA : 1); ++m) {
            int rr = base + m;
            if (rr >= a.sy) rr -= a.sy;
            const uint32_t boff = (uint32_t)((m < span ? rr * sx + cx : cx) * (int)sizeof(T));
            vp[m][0] = p0(boff);
            vp[m][1] = p1(boff);
            vp[m][2] = p2(boff);
            vp[m][3] = p3(boff);
        }
    };
    if (pipe && it0 < it1) issue(it0);
    for (int item = it0; item < it1; ++item) {
        const int b = item / a.tnz, k = item - b * a.tnz;
        const int j0 = b * JB;
        const int nj = a.tny - j0 < JB ? a.tny - j0 : JB;
        const int base = band[2 * b], span = band[2 * b + 1];
        __syncthreads();   // the previous item's readers are done with the LDS
        // A: coarse rows base .. base + span - 1 (cyclic), z stencil applied
        if constexpr (PIPE) {
            const T w0 = wzt[4 * k], w1 = wzt[4 * k + 1], w2 = wzt[4 * k + 2], w3 = wzt[4 * k + 3];
            if (tid < sx)
#pragma unroll
                for (int m = 0; m < (PIPE ? MA : 1); ++m)
                    if (m < span)
                        zr[m * sx + tid] =
                            ((w0 * vp[m][0] + w1 * vp[m][1]) + w2 * vp[m][2]) + w3 * vp[m][3];
        } else {
            const chd::PlaneRef<T> p0(src + (int64_t)izt[4 * k] * a.plane, pbytes);
            const chd::PlaneRef<T> p1(src + (int64_t)izt[4 * k + 1] * a.plane, pbytes);
            const chd::PlaneRef<T> p2(src + (int64_t)izt[4 * k + 2] * a.plane, pbytes);
            const chd::PlaneRef<T> p3(src + (int64_t)izt[4 * k + 3] * a.plane, pbytes);
            const T w0 = wzt[4 * k], w1 = wzt[4 * k + 1], w2 = wzt[4 * k + 2], w3 = wzt[4 * k + 3];
            for (int r0 = 0; r0 < span; r0 += MA)
                for (int cx = tid; cx < sx; cx += nt) {
                    T v[MA][4];
#pragma unroll
                    for (int m = 0; m < MA; ++m) {
                        int rr = base + r0 + m;
                        if (rr >= a.sy) rr -= a.sy;
                        const uint32_t boff =
                            (uint32_t)((r0 + m < span ? rr * sx + cx : cx) * (int)sizeof(T));
                        v[m][0] = p0(boff);
                        v[m][1] = p1(boff);
                        v[m][2] = p2(boff);
                        v[m][3] = p3(boff);
                    }
#pragma unroll
                    for (int m = 0; m < MA; ++m)
                        if (r0 + m < span)
                            zr[(r0 + m) * sx + cx] =
                                ((w0 * v[m][0] + w1 * v[m][1]) + w2 * v[m][2]) + w3 * v[m][3];
                }
        }
        __syncthreads();
        // B: the band's target rows, y stencil applied
        for (int cx = tid; cx < sx; cx += nt) {
#pragma unroll
            for (int jj = 0; jj < JB; ++jj) {
                if (jj < nj) {
                    const int* l = lyt + 4 * (j0 + jj);
                    const T* y = wyt + 4 * (j0 + jj);
                    yr[jj * sx + cx] = ((y[0] * zr[l[0] + cx] + y[1] * zr[l[1] + cx])
                                        + y[2] * zr[l[2] + cx]) + y[3] * zr[l[3] + cx];
                }
            }
        }
        __syncthreads();
        if (pipe && item + 1 < it1) issue(item + 1);
        // C: x stencil, every target point written once
        T* out = dst + ((int64_t)k * a.tny + j0) * a.tnx;
        if (win) {
            if (xact)
                for (int jj = rg0; jj < nj; jj += rgs) {
                    const T* row = yr + jj * sx;
                    T p[NW];
#pragma unroll
                    for (int n = 0; n < NW; ++n) p[n] = row[woff[n]];
                    T y[XQ];
#pragma unroll
                    for (int q = 0; q < XQ; ++q) {
                        T acc = M[q][0] * p[0];
#pragma unroll
                        for (int n = 1; n < NW; ++n) acc += M[q][n] * p[n];
                        y[q] = acc;
                    }
                    T* o = out + (int64_t)jj * a.tnx + xi0;
                    if (vec) {
                        __builtin_nontemporal_store(T4{y[0], y[1], y[2], y[3]},
                                                    reinterpret_cast<T4*>(o));
                    } else {
#pragma unroll
                        for (int q = 0; q < XQ; ++q)
                            if (xi0 + q < a.tnx) __builtin_nontemporal_store(y[q], o + q);
                    }
                }
        } else {
            for (int jj = 0; jj < nj; ++jj)
                for (int i = tid; i < a.tnx; i += nt) {
                    const T* row = yr + jj * sx;
                    T acc = T(0);
                    for (int t = 0; t < 4; ++t) acc += T(wxt[4 * i + t]) * row[ixt[4 * i + t]];
                    __builtin_nontemporal_store(acc, out + (int64_t)jj * a.tnx + i);
                }
        }
    }
}

// Solenoidal transfer, pieces other than the interpolation itself.
//
// Coarse normal gradient at the coarse cell centres, one row (k, j) per
// work-group: comp 0 differences u along x, 1 differences v along y, 2
// differences w along z (sz + 1 planes of w, cell heights 1 / dzinv[k]).
template <typename T>
__global__ void __launch_bounds__(256)
k_grad(const T* __restrict__ src, int comp, int sx, int sy, int sz,
       const double* __restrict__ dzinv, T* __restrict__ out)
{
    const int64_t plane = (int64_t)sx * sy;
    for (int64_t row = blockIdx.x; row < (int64_t)sy * sz; row += gridDim.x) {
        const int k = (int)(row / sy), j = (int)(row - (int64_t)k * sy);
        const T* p = src + row * sx;
        T* o = out + row * sx;
        if (comp == 0) {
            for (int i = threadIdx.x; i < sx; i += blockDim.x)
                o[i] = (p[i + 1 < sx ? i + 1 : 0] - p[i]) * T(sx);
        } else if (comp == 1) {
            const T* q = src + ((int64_t)k * sy + (j + 1 < sy ? j + 1 : 0)) * sx;
            for (int i = threadIdx.x; i < sx; i += blockDim.x) o[i] = (q[i] - p[i]) * T(sy);
        } else {
            const T s = T(dzinv[k]);
            for (int i = threadIdx.x; i < sx; i += blockDim.x) o[i] = (p[i + plane] - p[i]) * s;
        }
    }
}

// Largest closure magnitude of a work-group into part[blockIdx.x].
__device__ __forceinline__ void group_max(double v, double* __restrict__ part)
{
    __shared__ double red[4];
    for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
        part[blockIdx.x] = m;
    }
}

// Integration along x, one wavefront per row (in place): the row holds the
// interpolated gradient at the fine cell centres on entry and
//   u[i] = ref[row] + h sum_{i' < i} G[i']
// on exit.  Each lane takes CH consecutive points (32 bytes, two 16-byte
// vector accesses when the row allows), forms their prefix sums, and one
// wave-wide scan of the lane totals joins them.  The |h sum G| of the whole
// row is the closure left at the periodic seam.
template <typename T>
__global__ void __launch_bounds__(256)
k_scan_x(T* __restrict__ buf, const T* __restrict__ ref, int nx, int64_t nrows, T h,
         double* __restrict__ part)
{
    constexpr int CH = 32 / sizeof(T);
    typedef T TV __attribute__((ext_vector_type(CH / 2)));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool vec = nx % (64 * CH) == 0 && reinterpret_cast<uintptr_t>(buf) % 16 == 0;
    double mx = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * 4 + wv; row < nrows; row += (int64_t)gridDim.x * 4) {
        T* p = buf + row * nx;
        const T r = ref[row];
        T acc = T(0);
        for (int i0 = 0; i0 < nx; i0 += 64 * CH) {
            const int b0 = i0 + lane * CH;
            T g[CH];
            if (vec) {
                const TV lo = *reinterpret_cast<const TV*>(p + b0);
                const TV hi = *reinterpret_cast<const TV*>(p + b0 + CH / 2);
#pragma unroll
                for (int m = 0; m < CH / 2; ++m) {
                    g[m] = lo[m];
                    g[m + CH / 2] = hi[m];
                }
            } else {
#pragma unroll
                for (int m = 0; m < CH; ++m) g[m] = b0 + m < nx ? p[b0 + m] : T(0);
            }
            T loc[CH];
            T run = T(0);
#pragma unroll
            for (int m = 0; m < CH; ++m) {
                loc[m] = run;
                run += g[m];
            }
            T s = run;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const T t = __shfl_up(s, d);
                if (lane >= d) s += t;
            }
            const T ex = acc + (s - run);
            T o[CH];
#pragma unroll
            for (int m = 0; m < CH; ++m) o[m] = r + h * (ex + loc[m]);
            if (vec) {
                TV lo, hi;
#pragma unroll
                for (int m = 0; m < CH / 2; ++m) {
                    lo[m] = o[m];
                    hi[m] = o[m + CH / 2];
                }
                *reinterpret_cast<TV*>(p + b0) = lo;
                *reinterpret_cast<TV*>(p + b0 + CH / 2) = hi;
            } else {
#pragma unroll
                for (int m = 0; m < CH; ++m)
                    if (b0 + m < nx) p[b0 + m] = o[m];
            }
            acc += __shfl(s, 63);
        }
        mx = fmax(mx, (double)fabs(h * acc));
    }
    group_max(mx, part);
}

// Integration along y (in place), one thread per (k, i) column:
//   v[j] = ref[k][i] + h sum_{j' < j} G[j'].
template <typename T>
__global__ void __launch_bounds__(256)
k_scan_y(T* __restrict__ buf, const T* __restrict__ ref, int nx, int ny, int nz, T h,
         double* __restrict__ part)
{
    double mx = 0.0;
    const int64_t ncol = (int64_t)nz * nx;
    for (int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; col < ncol;
         col += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = col / nx, i = col - k * nx;
        T* p = buf + k * ny * nx + i;
        const T r = ref[col];
        T acc = T(0);
        int j = 0;
        for (; j + 8 <= ny; j += 8) {
            T g[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) g[q] = p[(int64_t)(j + q) * nx];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                p[(int64_t)(j + q) * nx] = r + h * acc;
                acc += g[q];
            }
        }
        for (; j < ny; ++j) {
            const T g = p[(int64_t)j * nx];
            p[(int64_t)j * nx] = r + h * acc;
            acc += g;
        }
        mx = fmax(mx, (double)fabs(h * acc));
    }
    group_max(mx, part);
}

// Integration along z (in place), one thread per (j, i) column: planes
// 0 .. nz-1 hold G on entry; w[k] = h sum_{k' < k} G[k'] (w = 0 on the
// bottom wall) and the top wall plane nz is set to 0.
template <typename T>
__global__ void __launch_bounds__(256)
k_scan_z(T* __restrict__ buf, int64_t plane, int nz, T h, double* __restrict__ part)
{
    double mx = 0.0;
    for (int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; col < plane;
         col += (int64_t)gridDim.x * blockDim.x) {
        T* p = buf + col;
        T acc = T(0);
        int k = 0;
        for (; k + 8 <= nz; k += 8) {
            T g[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) g[q] = p[(int64_t)(k + q) * plane];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                p[(int64_t)(k + q) * plane] = h * acc;
                acc += g[q];
            }
        }
        for (; k < nz; ++k) {
            const T g = p[(int64_t)k * plane];
            p[(int64_t)k * plane] = h * acc;
            acc += g;
        }
        p[(int64_t)nz * plane] = T(0);
        mx = fmax(mx, (double)fabs(h * acc));
    }
    group_max(mx, part);
}

// Drop labelling (the drop-size diagnostics of sec. 4): cells with
// C >= threshold, joined through faces (periodic axes wrap), by union-find
// on a label array.  A label points to a smaller linear index of the same
// drop or to itself (a root); unions link the larger root under the smaller
// with atomicMin, so every drop ends with its smallest index as its root.
// Loads of labels other threads may be changing go to the coherent level.
__device__ __forceinline__ int ccl_load(const int* lab, int a)
{
    return __hip_atomic_load(lab + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int ccl_find(const int* lab, int a)
{
    int b = ccl_load(lab, a);
    while (b != a) {   // labels only decrease along the chain: it ends
        a = b;
        b = ccl_load(lab, a);
    }
    return a;
}

__device__ void ccl_union(int* lab, int a, int b)
{
    // each retry lowers max(a, b) strictly, so the loop ends
    for (;;) {
        a = ccl_find(lab, a);
        b = ccl_find(lab, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(lab + b, a);
        if (old == b) return;
        b = old;   // b had been linked meanwhile: join a with b's parent
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_ccl_init(const T* __restrict__ C, int64_t n, T thr, int* __restrict__ lab)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        lab[i] = C[i] >= thr ? (int)i : -1;
}

// One (z, y) row per work-group and iteration, threads along x: every drop
// cell is joined with its -x, -y and -z neighbours (wrapping on periodic axes).
__global__ void __launch_bounds__(256)
k_ccl_union(int* lab, int nx, int ny, int nz, int px, int py, int pz)
{
    const int64_t plane = (int64_t)nx * ny;
    for (int64_t row = blockIdx.x; row < (int64_t)ny * nz; row += gridDim.x) {
        const int z = (int)(row / ny), y = (int)(row - (int64_t)z * ny);
        const int64_t r0 = row * nx;
        for (int x = threadIdx.x; x < nx; x += blockDim.x) {
            const int i = (int)(r0 + x);
            if (lab[i] < 0) continue;   // background stays background
            if (x > 0 || px) {
                const int j = x > 0 ? i - 1 : (int)(r0 + nx - 1);
                if (lab[j] >= 0) ccl_union(lab, i, j);
            }
            if (y > 0 || py) {
                const int j = y > 0 ? i - nx : (int)(i + (int64_t)(ny - 1) * nx);
                if (lab[j] >= 0) ccl_union(lab, i, j);
            }
            if (z > 0 || pz) {
                const int j = z > 0 ? (int)(i - plane) : (int)(i + (int64_t)(nz - 1) * plane);
                if (lab[j] >= 0) ccl_union(lab, i, j);
            }
        }
    }
}

__global__ void __launch_bounds__(256)
k_ccl_flatten(int* lab, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (lab[i] >= 0) lab[i] = ccl_find(lab, (int)i);
}

// Cells per drop: each wavefront reads windows of 64 consecutive labels
// (coalesced); the lanes that start a run of equal labels within a window
// (found with a ballot) add the run's length to cnt[root].
__global__ void __launch_bounds__(256)
k_ccl_count(const int* __restrict__ lab, int64_t n, int* __restrict__ cnt)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwave = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64;
         base < n; base += nwave * 64) {
        const int64_t i = base + lane;
        const int l = i < n ? lab[i] : -1;
        const int prev = __shfl_up(l, 1);
        const bool start = lane == 0 || l != prev;
        const unsigned long long runs = __ballot(start);
        if (start && l >= 0) {
            // next run start above this lane, or the window's end
            const unsigned long long above = lane == 63 ? 0ull : runs & (~0ull << (lane + 1));
            const int64_t end = above ? base + __ffsll((long long)above) - 1 : base + 64;
            atomicAdd(cnt + l, (int)((end < n ? end : n) - i));
        }
    }
}

// Roots and their cell counts into a list of at most cap entries (in no
// particular order); *count receives the number of drops.
__global__ void __launch_bounds__(256)
k_ccl_compact(const int* __restrict__ lab, const int* __restrict__ cnt, int64_t n, int cap,
              int* __restrict__ oroot, int* __restrict__ ocnt, int* __restrict__ count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (lab[i] == (int)i) {
            const int k = atomicAdd(count, 1);
            if (k < cap) {
                oroot[k] = (int)i;
                ocnt[k] = cnt[i];
            }
        }
}

// Split-density pressure step (sec. 3.2: eq-split, eq-newpoi, eq-u) on the
// staggered mesh: P and C at the cells, u / v / w on the low faces of the
// cells (w has nz + 1 planes between walls, zero on both).  The density is
// rho2 + (rho1 - rho2) clamp(C, 0, 1); a face takes the mean of its two
// cells, and 1/rho on a face is the refined hardware reciprocal (fast_rcp).
template <typename T>
__device__ __forceinline__ T press_rho(const PressArgs& a, T c)
{
    const T cc = c < T(0) ? T(0) : (c > T(1) ? T(1) : c);
    return T(a.rho2) + T(a.rho1 - a.rho2) * cc;
}

// Phat = 2 P - Pold, then Pold <- P (the next step's history).
template <typename T>
__global__ void __launch_bounds__(256)
k_press_prep(const T* __restrict__ P, T* __restrict__ Pold, T* __restrict__ phat, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T p = P[i];
        phat[i] = T(2) * p - Pold[i];
        Pold[i] = p;
    }
}

// The cell kernels of the pressure step take tiles of TX x-columns by TY
// rows and march each column up TZ planes, carrying the plane below in
// registers, so no plane is fetched twice for its z neighbours.  Planes are
// addressed through 32-bit byte offsets from a per-plane base (a plane is
// under 4 GiB).
struct PressTile {
    int tx, ty, tz;
};
constexpr PressTile RHS_TILE = {256, 2, 8}, UPD_TILE = {256, 1, 2};
constexpr PressTile RHS_TILE64 = {64, 4, 16}, UPD_TILE64 = {256, 1, 2};
template <typename T>
constexpr PressTile rhs_tile() { return sizeof(T) == 8 ? RHS_TILE64 : RHS_TILE; }
template <typename T>
constexpr PressTile upd_tile() { return sizeof(T) == 8 ? UPD_TILE64 : UPD_TILE; }

__host__ __device__ __forceinline__ int64_t press_tiles(PressTile p, int nx, int ny, int nz)
{
    return (int64_t)((nx + p.tx - 1) / p.tx) * ((ny + p.ty - 1) / p.ty) * ((nz + p.tz - 1) / p.tz);
}

// Column of thread t in task `task`: x, y and the march z0 .. z1 - 1; false
// for a thread past the mesh.
__device__ __forceinline__ bool press_column(PressTile p, int64_t task, int t, int nx, int ny,
                                             int nz, int* x, int* y, int* z0, int* z1)
{
    const int tx = (nx + p.tx - 1) / p.tx, ty = (ny + p.ty - 1) / p.ty;
    const int bx = (int)(task % tx);
    const int64_t rest = task / tx;
    const int by = (int)(rest % ty), bz = (int)(rest / ty);
    *x = bx * p.tx + t % p.tx;
    *y = by * p.ty + t / p.tx;
    *z0 = bz * p.tz;
    *z1 = *z0 + p.tz < nz ? *z0 + p.tz : nz;
    return *x < nx && *y < ny;
}

// Right-hand side of eq-newpoi at every cell:
// div[(1 - rho2/rho_f) grad Phat] + (rho2/dt) div u*.
template <typename T>
__global__ void __launch_bounds__(rhs_tile<T>().tx * rhs_tile<T>().ty)
k_press_rhs(PressArgs a, const T* __restrict__ C, const T* __restrict__ ph,
            const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
            T* __restrict__ rhs)
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t plane = (int64_t)nx * ny;
    constexpr uint32_t sT = sizeof(T);
    const uint32_t pbytes = (uint32_t)(plane * sT);
    const T ih = T(1.0 / a.h), r2 = T(a.rho2), sdiv = T(a.rho2 / a.dt);
    auto at = [&](const T* f, int z) { return chd::PlaneRef<T>(f + (int64_t)z * plane, pbytes); };
    const int64_t ntask = press_tiles(rhs_tile<T>(), nx, ny, nz);
    for (int64_t task = blockIdx.x; task < ntask; task += gridDim.x) {
        int x, y, z0, z1;
        if (!press_column(rhs_tile<T>(), task, (int)threadIdx.x, nx, ny, nz, &x, &y, &z0, &z1)) continue;
        const int xm = x > 0 ? x - 1 : nx - 1, xp = x + 1 < nx ? x + 1 : 0;
        const int ym = y > 0 ? y - 1 : ny - 1, yp = y + 1 < ny ? y + 1 : 0;
        const uint32_t oc = (uint32_t)(y * nx + x) * sT, oxm = (uint32_t)(y * nx + xm) * sT,
                       oxp = (uint32_t)(y * nx + xp) * sT, oym = (uint32_t)(ym * nx + x) * sT,
                       oyp = (uint32_t)(yp * nx + x) * sT;
        // rho and Phat of the column below the march (periodic wrap; not used
        // at the bottom wall) and at its first plane, and w on its low face
        T rlo = T(0), plo = T(0);
        if (z0 > 0 || !a.zwalls) {
            const int zb = z0 > 0 ? z0 - 1 : nz - 1;
            rlo = press_rho(a, at(C, zb)(oc));
            plo = at(ph, zb)(oc);
        }
        T rc = press_rho(a, at(C, z0)(oc)), pc = at(ph, z0)(oc);
        T wlo = at(w, z0)(oc);
        for (int z = z0; z < z1; ++z) {
            const int zp = z + 1 < nz ? z + 1 : 0;
            const bool up = !a.zwalls || z + 1 < nz;
            T rhi = T(0), phi = T(0);
            if (up) {
                rhi = press_rho(a, at(C, zp)(oc));
                phi = at(ph, zp)(oc);
            }
            const T whi = at(w, a.zwalls ? z + 1 : zp)(oc);
            const chd::PlaneRef<T> Cz = at(C, z), Pz = at(ph, z), Uz = at(u, z), Vz = at(v, z);
            // flux through the face between the cell and a neighbour (on the +
            // side when s = 1): (1 - rho2/rho_f) (Phat[hi] - Phat[lo]) / h
            auto flux = [&](T rn, T pn, int s) {
                const T rf = T(0.5) * (rc + rn);
                const T g = s > 0 ? pn - pc : pc - pn;
                return (T(1) - r2 * chd::fast_rcp(rf)) * g * ih;
            };
            T d = flux(press_rho(a, Cz(oxp)), Pz(oxp), 1) - flux(press_rho(a, Cz(oxm)), Pz(oxm), -1)
                + flux(press_rho(a, Cz(oyp)), Pz(oyp), 1) - flux(press_rho(a, Cz(oym)), Pz(oym), -1);
            if (up) d += flux(rhi, phi, 1);
            if (!a.zwalls || z > 0) d -= flux(rlo, plo, -1);
            const T du = Uz(oxp) - Uz(oc);
            const T dv = Vz(oyp) - Vz(oc);
            const T dw = whi - wlo;
            at(rhs, z).store(oc, d * ih + sdiv * (du + dv + dw) * ih);
            rlo = rc;
            plo = pc;
            rc = rhi;
            pc = phi;
            wlo = whi;
        }
    }
}

// Solve along z per (ky, kx) mode after the 2-D transforms in x and y
// (between walls): (1/h^2)(p[k+1] - 2 p[k] + p[k-1]) + lxy p[k] = f[k] with
// p[-1] = p[0], p[nz] = p[nz-1] (dP/dz = 0).  The rows are diagonally
// dominant for lxy < 0 and are eliminated from both ends at once: lane l
// (l < 32) of a wave takes mode g*32 + l from row 0 up to row M - 1 (M = nz/2),
// lane l + 32 the same mode from row nz - 1 down to M + 1; row M then
// couples the two eliminated halves,
//   (b_M - c_{M-1}/h^2 - e_{M+1}/h^2) p_M = f_M - (d_{M-1} + g_{M+1})/h^2,
// and each lane substitutes back over its half.  This halves the serial chain
// and doubles the threads of the plain Thomas sweep.  The mean mode (lxy = 0)
// is singular: its mean over z is removed from f, then p[0] = 0 and the rows
// 0 .. nz-2 give p[1 .. nz-1] by p[k+1] = 2 p[k] - p[k-1] + h^2 f[k]
// (p[-1] = p[0]), and the mean of p is removed.  Spectra are [nz][ny][nxh]
// complex (re, im interleaved); cp holds nz x nmodes reals of scratch, of
// which one per block of PK rows is used.  The result is scaled by `scale`
// (the inverse transform's 1 / (nx ny)).
template <typename T>
struct Cplx;
template <>
struct Cplx<float> {
    typedef float2 V;
};
template <>
struct Cplx<double> {
    typedef double2 V;
};

template <typename T>
__global__ void __launch_bounds__(256)
k_press_tri(T* __restrict__ spec, T* __restrict__ cp, int nx, int ny, int nz, double h,
            double scale)
{
    typedef typename Cplx<T>::V V;
    const int nxh = nx / 2 + 1;
    const int64_t nm = (int64_t)ny * nxh;
    const int64_t ngroups = (nm + 31) / 32;
    const double PI = 3.14159265358979323846;
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int M = nz / 2;
    const int len = half == 0 ? M : nz - 1 - M;   // rows eliminated by this lane
    const T ih2 = T(1.0 / (h * h));
    const T sc = T(scale);
    const int64_t st = nm;                          // complex elements between planes
    constexpr int PK = sizeof(T) == 4 ? 8 : 4;      // planes loaded ahead
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // the group loop is uniform over a wave: every lane reaches the exchange
    for (int64_t g = wave0; g < ngroups; g += nwaves) {
        const int64_t m = g * 32 + (lane & 31);
        const bool live = m < nm;
        const bool special = m == 0;
        const int64_t mm = live ? m : 0;
        const int j = (int)(mm / nxh), i = (int)(mm - (int64_t)j * nxh);
        const double sx = sin(PI * i / nx), sy = sin(PI * j / ny);
        const T lxy = T(-4.0 / (h * h) * (sx * sx + sy * sy));
        V* f = reinterpret_cast<V*>(spec) + mm;       // f[k] at f + k nm
        auto row = [&](int s) { return half == 0 ? s : nz - 1 - s; };
        auto diag = [&](int k) { return lxy - (k == 0 || k == nz - 1 ? ih2 : T(2) * ih2); };
        // elimination towards row M in blocks of PK rows: d into f, and into
        // cp at each block's first row the c entering the block (the block's
        // c are formed again from it on the way back)
        T c = T(0), dr = T(0), di = T(0);
        if (live && !special) {
            for (int s0 = 0; s0 < len; s0 += PK) {
                cp[row(s0) * nm + m] = c;
                V fv[PK];
#pragma unroll
                for (int q = 0; q < PK; ++q) fv[q] = f[row(s0 + q < len ? s0 + q : len - 1) * st];
#pragma unroll
                for (int q = 0; q < PK; ++q) {
                    const int sq = s0 + q;
                    if (sq >= len) break;
                    const int k = row(sq);
                    const T den = diag(k) - ih2 * c;
                    c = ih2 / den;
                    dr = (fv[q].x - ih2 * dr) / den;
                    di = (fv[q].y - ih2 * di) / den;
                    V o;
                    o.x = dr;
                    o.y = di;
                    f[k * st] = o;
                }
            }
        }
        // row M, read by the lower lane only, and the other half's last
        // coefficients (zero for an empty half), across the wave
        T fmr = T(0), fmi = T(0);
        if (live && !special && half == 0) {
            const V v = f[M * st];
            fmr = v.x;
            fmi = v.y;
        }
        const T oc = __shfl_xor(c, 32), odr = __shfl_xor(dr, 32), odi = __shfl_xor(di, 32);
        const T ofr = __shfl_xor(fmr, 32), ofi = __shfl_xor(fmi, 32);
        if (live && !special) {
            if (half == 1) {
                fmr = ofr;
                fmi = ofi;
            }
            const T den = diag(M) - ih2 * (c + oc);
            T xr = (fmr - ih2 * (dr + odr)) / den;
            T xi = (fmi - ih2 * (di + odi)) / den;
            if (half == 0) {
                V o;
                o.x = xr * sc;
                o.y = xi * sc;
                f[M * st] = o;
            }
            // back substitution from row M outwards, block by block: the
            // block's c again from its checkpoint (the same operations as on
            // the way up, so the same values), then its rows in reverse
            for (int s0 = len > 0 ? (len - 1) / PK * PK : -1; s0 >= 0; s0 -= PK) {
                V fv[PK];
                T cc[PK];
                T cin = cp[row(s0) * nm + m];
#pragma unroll
                for (int q = 0; q < PK; ++q) fv[q] = f[row(s0 + q < len ? s0 + q : len - 1) * st];
#pragma unroll
                for (int q = 0; q < PK; ++q) {
                    cc[q] = T(0);
                    if (s0 + q >= len) break;
                    const T den = diag(row(s0 + q)) - ih2 * cin;
                    cin = ih2 / den;
                    cc[q] = cin;
                }
#pragma unroll
                for (int q = PK - 1; q >= 0; --q) {
                    const int sq = s0 + q;
                    if (sq >= len) continue;
                    xr = fv[q].x - cc[q] * xr;
                    xi = fv[q].y - cc[q] * xi;
                    V o;
                    o.x = xr * sc;
                    o.y = xi * sc;
                    f[row(sq) * st] = o;
                }
            }
        }
        if (live && special && half == 0) {
            T* fs = spec;                  // mode 0: f[k] at fs + 2 k nm
            const int64_t s2 = 2 * nm;
            T mr = T(0), mi = T(0);
            for (int k = 0; k < nz; ++k) {
                mr += fs[k * s2];
                mi += fs[k * s2 + 1];
            }
            mr /= T(nz);
            mi /= T(nz);
            const T h2 = T(h * h);
            T pr = T(0), pi = T(0), qr = T(0), qi = T(0);   // p[k-1], p[k]
            T sr = T(0), si = T(0);
            for (int k = 0; k < nz; ++k) {
                const T fr = fs[k * s2] - mr, fi = fs[k * s2 + 1] - mi;
                fs[k * s2] = qr;         // p[k]
                fs[k * s2 + 1] = qi;
                sr += qr;
                si += qi;
                const T lr = k == 0 ? qr : pr, li = k == 0 ? qi : pi;
                const T nr = T(2) * qr - lr + h2 * fr, ni = T(2) * qi - li + h2 * fi;
                pr = qr;
                pi = qi;
                qr = nr;
                qi = ni;
            }
            sr /= T(nz);
            si /= T(nz);
            for (int k = 0; k < nz; ++k) {
                fs[k * s2] = (fs[k * s2] - sr) * sc;
                fs[k * s2 + 1] = (fs[k * s2 + 1] - si) * sc;
            }
        }
    }
}

// Periodic z: divide the 3-D spectrum [nz][ny][nxh] by the eigenvalue of the
// 7-point Laplacian, zero mode to 0, scaled by 1 / (nx ny nz).
template <typename T>
__global__ void __launch_bounds__(256)
k_press_div(T* __restrict__ spec, int nx, int ny, int nz, double h, double scale)
{
    const int nxh = nx / 2 + 1;
    const int64_t n = (int64_t)nz * ny * nxh;
    const double PI = 3.14159265358979323846;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % nxh);
        const int64_t r = e / nxh;
        const int j = (int)(r % ny), k = (int)(r / ny);
        const double sx = sin(PI * i / nx), sy = sin(PI * j / ny), sz = sin(PI * k / nz);
        const double lam = -4.0 / (h * h) * (sx * sx + sy * sy + sz * sz);
        const T f = (e == 0) ? T(0) : T(scale / lam);
        spec[2 * e] *= f;
        spec[2 * e + 1] *= f;
    }
}

// eq-u on the low faces of every cell (the wall faces of z stay as they are),
// z-marching tiles as for the right-hand side.
template <typename T>
__global__ void __launch_bounds__(upd_tile<T>().tx * upd_tile<T>().ty)
k_press_update(PressArgs a, const T* __restrict__ C, const T* __restrict__ P,
               const T* __restrict__ ph, T* __restrict__ u, T* __restrict__ v, T* __restrict__ w)
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t plane = (int64_t)nx * ny;
    constexpr uint32_t sT = sizeof(T);
    const uint32_t pbytes = (uint32_t)(plane * sT);
    const T ih = T(1.0 / a.h), ir2 = T(1.0 / a.rho2), dt = T(a.dt);
    auto at = [&](const T* f, int z) { return chd::PlaneRef<T>(f + (int64_t)z * plane, pbytes); };
    const int64_t ntask = press_tiles(upd_tile<T>(), nx, ny, nz);
    for (int64_t task = blockIdx.x; task < ntask; task += gridDim.x) {
        int x, y, z0, z1;
        if (!press_column(upd_tile<T>(), task, (int)threadIdx.x, nx, ny, nz, &x, &y, &z0, &z1)) continue;
        const int xm = x > 0 ? x - 1 : nx - 1, ym = y > 0 ? y - 1 : ny - 1;
        const uint32_t oc = (uint32_t)(y * nx + x) * sT, oxm = (uint32_t)(y * nx + xm) * sT,
                       oym = (uint32_t)(ym * nx + x) * sT;
        // rho, P and Phat of the column below the march (periodic wrap; not
        // used at the bottom wall)
        T rlo = T(0), qlo = T(0), hlo = T(0);
        if (z0 > 0 || !a.zwalls) {
            const int zb = z0 > 0 ? z0 - 1 : nz - 1;
            rlo = press_rho(a, at(C, zb)(oc));
            qlo = at(P, zb)(oc);
            hlo = at(ph, zb)(oc);
        }
        for (int z = z0; z < z1; ++z) {
            const chd::PlaneRef<T> Cz = at(C, z), Pz = at(P, z), Hz = at(ph, z);
            const T rc = press_rho(a, Cz(oc)), pc = Pz(oc), hc = Hz(oc);
            auto corr = [&](T rn, T qn, T hn) {   // face between a low neighbour and the cell
                const T rf = T(0.5) * (rc + rn);
                return dt * ((pc - qn) * ih * ir2 + (chd::fast_rcp(rf) - ir2) * (hc - hn) * ih);
            };
            const chd::PlaneRef<T> Uz = at(u, z), Vz = at(v, z), Wz = at(w, z);
            Uz.store(oc, Uz(oc) - corr(press_rho(a, Cz(oxm)), Pz(oxm), Hz(oxm)));
            Vz.store(oc, Vz(oc) - corr(press_rho(a, Cz(oym)), Pz(oym), Hz(oym)));
            if (!a.zwalls || z > 0) Wz.store(oc, Wz(oc) - corr(rlo, qlo, hlo));
            rlo = rc;
            qlo = pc;
            hlo = hc;
        }
    }
}

// ---------------------------------------------------------------------------
// host-side launchers (declared in ch_kernels.h)
// ---------------------------------------------------------------------------
template <typename T, typename A, int MI, int NT, bool E25>
static hipError_t launch_x(int nwg, int nth, size_t lds, hipStream_t st, const chd::BoxDesc* boxes,
                           int nbox, const chd::PassArgs& pa, const void* C, const void* U,
                           const void* V, const void* W, void* E, void* Q)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)&k_pass_x<T, A, MI, NT, E25>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_pass_x<T, A, MI, NT, E25>), dim3(nwg), dim3(nth), lds, st, boxes, nbox, pa,
                       (const T*)C, (const T*)U, (const T*)V, (const T*)W, (T*)E, (T*)Q);
    return hipGetLastError();
}

template <typename T, typename A, bool E25>
static hipError_t launch_x_mode(int mi, int nwg, int nth, size_t lds, hipStream_t st,
                                const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                                const void* C, const void* U, const void* V, const void* W,
                                void* E, void* Q)
{
    if (mi == 1 && nth <= 512)
        return launch_x<T, A, 1, 512, E25>(nwg, nth, lds, st, boxes, nbox, pa, C, U, V, W, E, Q);
    if (mi == 1)
        return launch_x<T, A, 1, 1024, E25>(nwg, nth, lds, st, boxes, nbox, pa, C, U, V, W, E, Q);
    if (nth <= 768)
        return launch_x<T, A, 2, 768, E25>(nwg, nth, lds, st, boxes, nbox, pa, C, U, V, W, E, Q);
    return launch_x<T, A, 2, 1024, E25>(nwg, nth, lds, st, boxes, nbox, pa, C, U, V, W, E, Q);
}

template <typename T, typename A, int NT, int RM>
static hipError_t launch_x_row(int nwg, int nth, size_t lds, hipStream_t st,
                               const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                               const void* C, const void* U, const void* V, const void* W,
                               void* E, void* Q)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)&k_pass_x_row<T, A, NT, RM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_pass_x_row<T, A, NT, RM>), dim3(nwg), dim3(nth), lds, st, boxes, nbox,
                       pa, (const T*)C, (const T*)U, (const T*)V, (const T*)W, (T*)E, (T*)Q);
    return hipGetLastError();
}

template <typename T, typename A, int RM>
static hipError_t launch_x_row_nt(int nwg, int nth, size_t lds, hipStream_t st,
                                  const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                                  const void* C, const void* U, const void* V, const void* W,
                                  void* E, void* Q)
{
    if (nth <= 256)
        return launch_x_row<T, A, 256, RM>(nwg, nth, lds, st, boxes, nbox, pa, C, U, V, W, E, Q);
    if (nth <= 512)
        return launch_x_row<T, A, 512, RM>(nwg, nth, lds, st, boxes, nbox, pa, C, U, V, W, E, Q);
    return launch_x_row<T, A, 1024, RM>(nwg, nth, lds, st, boxes, nbox, pa, C, U, V, W, E, Q);
}

template <typename T, typename A>
hipError_t launch_pass_x(int mi, int nwg, int nth, size_t lds, hipStream_t st,
                         const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                         const void* C, const void* U, const void* V, const void* W, void* E,
                         void* Q, bool e25, bool xrow, int xrm)
{
    if (xrow && !e25 && mi == 1) {
        if (xrm == chd::XR_WAVE)
            return launch_x_row_nt<T, A, chd::XR_WAVE>(nwg, nth, lds, st, boxes, nbox, pa, C, U,
                                                       V, W, E, Q);
        if (xrm == chd::XR_THREAD)
            return launch_x_row_nt<T, A, chd::XR_THREAD>(nwg, nth, lds, st, boxes, nbox, pa, C,
                                                         U, V, W, E, Q);
        return launch_x_row_nt<T, A, chd::XR_ONE>(nwg, nth, lds, st, boxes, nbox, pa, C, U, V,
                                                  W, E, Q);
    }
    if constexpr (std::is_same<T, A>::value) {
        if (e25)
            return launch_x_mode<T, A, true>(mi, nwg, nth, lds, st, boxes, nbox, pa, C, U, V, W,
                                             E, Q);
    } else {
        if (e25) return hipErrorInvalidValue;   // the explicit mode has no solve precision
    }
    return launch_x_mode<T, A, false>(mi, nwg, nth, lds, st, boxes, nbox, pa, C, U, V, W, E, Q);
}

template <typename T, typename A>
hipError_t launch_pass_x_seg(int nwg, int nth, size_t lds, hipStream_t st,
                             const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                             const void* C, const void* U, const void* V, const void* W,
                             const void* Ein, void* Eout, void* Q)
{
    if (nth > 256) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)&k_pass_x_seg<T, A>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_pass_x_seg<T, A>), dim3(nwg), dim3(nth), lds, st, boxes, nbox, pa,
                       (const T*)C, (const T*)U, (const T*)V, (const T*)W, (const T*)Ein, (T*)Eout,
                       (T*)Q);
    return hipGetLastError();
}

template <typename T, typename A>
hipError_t launch_pass_line(int pass, int nwg, int nthreads, size_t lds, hipStream_t st,
                            const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                            const void* Qin, void* Qout)
{
    const void* fn = pass == chd::PASS_Y ? (const void*)&k_pass_line<T, A, chd::PASS_Y>
                                         : (const void*)&k_pass_line<T, A, chd::PASS_Z>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    if (pass == chd::PASS_Y)
        hipLaunchKernelGGL((k_pass_line<T, A, chd::PASS_Y>), dim3(nwg), dim3(nthreads), lds, st,
                           boxes, nbox, pa, (const T*)Qin, (T*)Qout);
    else
        hipLaunchKernelGGL((k_pass_line<T, A, chd::PASS_Z>), dim3(nwg), dim3(nthreads), lds, st,
                           boxes, nbox, pa, (const T*)Qin, (T*)Qout);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mass(int nblk, int nbox, hipStream_t st, const chd::BoxDesc* boxes,
                       const void* C, double* partial, const double* h3, double* out)
{
    hipLaunchKernelGGL((k_mass_partial<T>), dim3(nblk), dim3(chd::MASS_THREADS), 0, st, boxes,
                       nbox, (const T*)C, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mass_final, dim3(nbox), dim3(chd::MASS_THREADS), 0, st, boxes, partial,
                       h3, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mass_one(hipStream_t st, const chd::BoxDesc& bd, const void* C,
                           double* partial, double h3, double* out)
{
    hipLaunchKernelGGL((k_mass_partial_one<T>), dim3(bd.nmblk), dim3(chd::MASS_THREADS), 0, st,
                       bd, (const T*)C, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mass_final_one, dim3(1), dim3(chd::MASS_THREADS), 0, st, bd.nmblk,
                       (const double*)partial, h3, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_check_velocity(hipStream_t st, const chd::BoxDesc* boxes, int nbox,
                                 const void* U, const void* V, const void* W, int* flags)
{
    hipLaunchKernelGGL((k_check_velocity<T>), dim3(CHECK_WGS), dim3(256), 0, st, boxes, nbox,
                       (const T*)U, (const T*)V, (const T*)W, flags);
    return hipGetLastError();
}

template <typename T, int JB, int MA, bool PIPE>
static hipError_t launch_interp_k(hipStream_t st, const InterpArgs& a)
{
    if (a.lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)&k_interp<T, JB, MA, PIPE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)a.lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_interp<T, JB, MA, PIPE>), dim3((unsigned)a.nwg), dim3(256), a.lds, st,
                       a, (const T*)a.src, (T*)a.dst, a.band, a.iz, (const T*)a.wz, a.ly,
                       (const T*)a.wy, a.ix, a.wx);
    return hipGetLastError();
}

template <typename T, int JB>
static hipError_t launch_interp_jb(hipStream_t st, const InterpArgs& a)
{
    constexpr int MA = sizeof(T) == 4 ? 20 : 12;  // rows of loads in flight
    // one batch of loads per item: coarse rows of at most 256 points, bands
    // of at most MA rows
    if (a.rmax <= MA && a.sx <= 256) return launch_interp_k<T, JB, MA, true>(st, a);
    return launch_interp_k<T, JB, MA, false>(st, a);
}

template <typename T>
hipError_t launch_interp(hipStream_t st, const InterpArgs& a)
{
    switch (a.jb) {
    case 32: return launch_interp_jb<T, 32>(st, a);
    case 16: return launch_interp_jb<T, 16>(st, a);
    case 8: return launch_interp_jb<T, 8>(st, a);
    case 4: return launch_interp_jb<T, 4>(st, a);
    case 2: return launch_interp_jb<T, 2>(st, a);
    case 1: return launch_interp_jb<T, 1>(st, a);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_grad(hipStream_t st, const void* src, int comp, int sx, int sy, int sz,
                       const double* dzinv, void* out)
{
    const int64_t rows = (int64_t)sy * sz;
    const int64_t nwg = rows < 262144 ? rows : 262144;
    hipLaunchKernelGGL((k_grad<T>), dim3((unsigned)nwg), dim3(256), 0, st, (const T*)src, comp,
                       sx, sy, sz, dzinv, (T*)out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scan(hipStream_t st, int dir, void* buf, const void* ref, int nx, int ny,
                       int nz, double h, double* part)
{
    const int nwg = scan_groups(dir, nx, ny, nz);
    if (dir == 0)
        hipLaunchKernelGGL((k_scan_x<T>), dim3(nwg), dim3(256), 0, st, (T*)buf, (const T*)ref,
                           nx, (int64_t)ny * nz, T(h), part);
    else if (dir == 1)
        hipLaunchKernelGGL((k_scan_y<T>), dim3(nwg), dim3(256), 0, st, (T*)buf, (const T*)ref,
                           nx, ny, nz, T(h), part);
    else
        hipLaunchKernelGGL((k_scan_z<T>), dim3(nwg), dim3(256), 0, st, (T*)buf,
                           (int64_t)nx * ny, nz, T(h), part);
    return hipGetLastError();
}

static unsigned grid_for(int64_t n)
{
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

template <typename T>
hipError_t launch_drops_label(hipStream_t st, const void* C, int nx, int ny, int nz,
                              const int bc[3], double thr, int* lab)
{
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL((k_ccl_init<T>), dim3(grid_for(n)), dim3(256), 0, st, (const T*)C, n,
                       T(thr), lab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t rows = (int64_t)ny * nz;
    hipLaunchKernelGGL(k_ccl_union, dim3((unsigned)(rows < 262144 ? rows : 262144)), dim3(256), 0,
                       st, lab, nx, ny, nz, bc[0] == 0, bc[1] == 0, bc[2] == 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ccl_flatten, dim3(grid_for(n)), dim3(256), 0, st, lab, n);
    return hipGetLastError();
}

hipError_t launch_drops_count(hipStream_t st, const int* lab, int64_t n, int* cnt, int cap,
                              int* oroot, int* ocnt, int* count)
{
    hipLaunchKernelGGL(k_ccl_count, dim3(grid_for(n)), dim3(256), 0, st, lab, n, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ccl_compact, dim3(grid_for(n)), dim3(256), 0, st, lab, cnt, n, cap,
                       oroot, ocnt, count);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_press_prep(hipStream_t st, const void* P, void* Pold, void* phat, int64_t n)
{
    hipLaunchKernelGGL((k_press_prep<T>), dim3(grid_for(n)), dim3(256), 0, st, (const T*)P,
                       (T*)Pold, (T*)phat, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_press_rhs(hipStream_t st, const PressArgs& a, const void* C, const void* phat,
                            const void* u, const void* v, const void* w, void* rhs)
{
    constexpr PressTile tl = rhs_tile<T>();
    const int64_t tiles = press_tiles(tl, a.nx, a.ny, a.nz);
    hipLaunchKernelGGL((k_press_rhs<T>), dim3((unsigned)(tiles < 1048576 ? tiles : 1048576)),
                       dim3(tl.tx * tl.ty), 0, st, a, (const T*)C, (const T*)phat, (const T*)u,
                       (const T*)v, (const T*)w, (T*)rhs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_press_solve(hipStream_t st, int zwalls, void* spec, void* cp, int nx, int ny,
                              int nz, double h)
{
    if (zwalls) {
        // one wave per 32 modes (two lanes per mode)
        const int64_t nm = (int64_t)ny * (nx / 2 + 1);
        hipLaunchKernelGGL((k_press_tri<T>), dim3(grid_for((nm + 31) / 32 * 64)), dim3(256), 0, st,
                           (T*)spec, (T*)cp, nx, ny, nz, h, 1.0 / ((double)nx * ny));
    } else {
        const int64_t n = (int64_t)nz * ny * (nx / 2 + 1);
        hipLaunchKernelGGL((k_press_div<T>), dim3(grid_for(n)), dim3(256), 0, st, (T*)spec, nx,
                           ny, nz, h, 1.0 / ((double)nx * ny * nz));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_press_update(hipStream_t st, const PressArgs& a, const void* C, const void* P,
                               const void* phat, void* u, void* v, void* w)
{
    constexpr PressTile tl = upd_tile<T>();
    const int64_t tiles = press_tiles(tl, a.nx, a.ny, a.nz);
    hipLaunchKernelGGL((k_press_update<T>), dim3((unsigned)(tiles < 1048576 ? tiles : 1048576)),
                       dim3(tl.tx * tl.ty), 0, st, a, (const T*)C, (const T*)P, (const T*)phat,
                       (T*)u, (T*)v, (T*)w);
    return hipGetLastError();
}

#define CH_INSTANTIATE(T, A)                                                                    \
    template hipError_t launch_pass_x<T, A>(int, int, int, size_t, hipStream_t,                 \
                                            const chd::BoxDesc*, int,                           \
                                            const chd::PassArgs&, const void*, const void*,     \
                                            const void*, const void*, void*, void*, bool,       \
                                            bool, int);                                         \
    template hipError_t launch_pass_x_seg<T, A>(int, int, size_t, hipStream_t,                  \
                                                const chd::BoxDesc*, int, const chd::PassArgs&, \
                                                const void*, const void*, const void*,          \
                                                const void*, const void*, void*, void*);        \
    template hipError_t launch_pass_line<T, A>(int, int, int, size_t, hipStream_t,              \
                                               const chd::BoxDesc*, int, const chd::PassArgs&,  \
                                               const void*, void*);

CH_INSTANTIATE(double, double)
CH_INSTANTIATE(float, float)
CH_INSTANTIATE(float, double)

template hipError_t launch_mass<double>(int, int, hipStream_t, const chd::BoxDesc*, const void*,
                                        double*, const double*, double*);
template hipError_t launch_mass<float>(int, int, hipStream_t, const chd::BoxDesc*, const void*,
                                       double*, const double*, double*);
template hipError_t launch_mass_one<double>(hipStream_t, const chd::BoxDesc&, const void*, double*,
                                            double, double*);
template hipError_t launch_mass_one<float>(hipStream_t, const chd::BoxDesc&, const void*, double*,
                                           double, double*);
template hipError_t launch_check_velocity<double>(hipStream_t, const chd::BoxDesc*, int,
                                                  const void*, const void*, const void*, int*);
template hipError_t launch_check_velocity<float>(hipStream_t, const chd::BoxDesc*, int,
                                                 const void*, const void*, const void*, int*);
template hipError_t launch_interp<double>(hipStream_t, const InterpArgs&);
template hipError_t launch_interp<float>(hipStream_t, const InterpArgs&);
template hipError_t launch_drops_label<double>(hipStream_t, const void*, int, int, int,
                                               const int*, double, int*);
template hipError_t launch_drops_label<float>(hipStream_t, const void*, int, int, int, const int*,
                                              double, int*);
template hipError_t launch_grad<double>(hipStream_t, const void*, int, int, int, int,
                                        const double*, void*);
template hipError_t launch_grad<float>(hipStream_t, const void*, int, int, int, int,
                                       const double*, void*);
template hipError_t launch_scan<double>(hipStream_t, int, void*, const void*, int, int, int,
                                        double, double*);
template hipError_t launch_scan<float>(hipStream_t, int, void*, const void*, int, int, int,
                                       double, double*);

template hipError_t launch_press_prep<double>(hipStream_t, const void*, void*, void*, int64_t);
template hipError_t launch_press_rhs<double>(hipStream_t, const PressArgs&, const void*, const void*,
                                          const void*, const void*, const void*, void*);
template hipError_t launch_press_solve<double>(hipStream_t, int, void*, void*, int, int, int, double);
template hipError_t launch_press_update<double>(hipStream_t, const PressArgs&, const void*,
                                             const void*, const void*, void*, void*, void*);
template hipError_t launch_press_prep<float>(hipStream_t, const void*, void*, void*, int64_t);
template hipError_t launch_press_rhs<float>(hipStream_t, const PressArgs&, const void*, const void*,
                                          const void*, const void*, const void*, void*);
template hipError_t launch_press_solve<float>(hipStream_t, int, void*, void*, int, int, int, double);
template hipError_t launch_press_update<float>(hipStream_t, const PressArgs&, const void*,
                                             const void*, const void*, void*, void*, void*);

}  // namespace chk
