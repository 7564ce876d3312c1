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
    chd::pass_x_program<T, A, MI, E25>(ex, &st, boxes[b], pa, task, C, U, V, W, E, Q, smem);
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

// Mass, stage 1: one fixed block of C per work-group, summed in double in a
// fixed order.
template <typename T>
__global__ void __launch_bounds__(chd::MASS_THREADS)
k_mass_partial(const chd::BoxDesc* __restrict__ boxes, int nbox, const T* __restrict__ C,
               double* __restrict__ partial)
{
    __shared__ double sh[chd::MASS_THREADS];
    const int blk = blockIdx.x;
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].mblk0 <= blk) lo = mid;
        else hi = mid - 1;
    }
    const chd::BoxDesc& bd = boxes[lo];
    const int tid = threadIdx.x;
    sh[tid] = chd::mass_thread_sum<T>(tid, bd, blk - bd.mblk0, C);
    __syncthreads();
    for (int s = chd::MASS_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0) partial[blk] = sh[0];
}

// Mass, stage 2: one work-group per box sums its partials in a fixed order
// and scales by h^3.
__global__ void __launch_bounds__(chd::MASS_THREADS)
k_mass_final(const chd::BoxDesc* __restrict__ boxes, const double* __restrict__ partial,
             const double* __restrict__ h3, double* __restrict__ out)
{
    __shared__ double sh[chd::MASS_THREADS];
    const chd::BoxDesc& bd = boxes[blockIdx.x];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int i = tid; i < bd.nmblk; i += chd::MASS_THREADS) s += partial[bd.mblk0 + i];
    sh[tid] = s;
    __syncthreads();
    for (int st = chd::MASS_THREADS / 2; st > 0; st >>= 1) {
        if (tid < st) sh[tid] += sh[tid + st];
        __syncthreads();
    }
    if (tid == 0) out[blockIdx.x] = sh[0] * h3[blockIdx.x];
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

// Coarse-to-fine velocity transfer, one target x-row per work-group and
// iteration: the 4 x 4 source rows of the row's z and y stencils are first
// combined into one coarse row in LDS (16 taps per coarse x point, coalesced
// reads), then every target point takes its 4-point x stencil from LDS.
// Exactly the separable tensor-product interpolation, summed z-y first.
template <typename T>
__global__ void __launch_bounds__(256)
k_interp(const T* __restrict__ src, int64_t sx, int64_t sy, int64_t tnx, int64_t tny,
         int64_t tnz, const int* __restrict__ ix, const double* __restrict__ wx,
         const int* __restrict__ iy, const double* __restrict__ wy,
         const int* __restrict__ iz, const double* __restrict__ wz, T* __restrict__ dst)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T* row = reinterpret_cast<T*>(smem);
    const int64_t nrows = tny * tnz;
    for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int64_t j = r % tny, k = r / tny;
        __syncthreads();   // the previous row's readers are done with `row`
        for (int64_t cx = threadIdx.x; cx < sx; cx += blockDim.x) {
            T acc = T(0);
            for (int c = 0; c < 4; ++c) {
                const T* plane = src + (int64_t)iz[4 * k + c] * sy * sx + cx;
                T accy = T(0);
                for (int b = 0; b < 4; ++b)
                    accy += T(wy[4 * j + b]) * plane[(int64_t)iy[4 * j + b] * sx];
                acc += T(wz[4 * k + c]) * accy;
            }
            row[cx] = acc;
        }
        __syncthreads();
        T* out = dst + r * tnx;
        for (int64_t i = threadIdx.x; i < tnx; i += blockDim.x) {
            T acc = T(0);
            for (int a = 0; a < 4; ++a) acc += T(wx[4 * i + a]) * row[ix[4 * i + a]];
            out[i] = acc;
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

template <typename T, typename A>
hipError_t launch_pass_x(int mi, int nwg, int nth, size_t lds, hipStream_t st,
                         const chd::BoxDesc* boxes, int nbox, const chd::PassArgs& pa,
                         const void* C, const void* U, const void* V, const void* W, void* E,
                         void* Q, bool e25)
{
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
hipError_t launch_check_velocity(hipStream_t st, const chd::BoxDesc* boxes, int nbox,
                                 const void* U, const void* V, const void* W, int* flags)
{
    hipLaunchKernelGGL((k_check_velocity<T>), dim3(CHECK_WGS), dim3(256), 0, st, boxes, nbox,
                       (const T*)U, (const T*)V, (const T*)W, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_interp(hipStream_t st, const void* src, int64_t sx, int64_t sy, int64_t tnx,
                         int64_t tny, int64_t tnz, const int* ix, const double* wx,
                         const int* iy, const double* wy, const int* iz, const double* wz,
                         void* dst)
{
    const int64_t rows = tny * tnz;
    const int64_t nwg = rows < 262144 ? rows : 262144;
    hipLaunchKernelGGL((k_interp<T>), dim3((unsigned)nwg), dim3(256), (size_t)sx * sizeof(T), st,
                       (const T*)src, sx, sy, tnx, tny, tnz, ix, wx, iy, wy, iz, wz, (T*)dst);
    return hipGetLastError();
}

#define CH_INSTANTIATE(T, A)                                                                    \
    template hipError_t launch_pass_x<T, A>(int, int, int, size_t, hipStream_t,                 \
                                            const chd::BoxDesc*, int,                           \
                                            const chd::PassArgs&, const void*, const void*,     \
                                            const void*, const void*, void*, void*, bool);      \
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
template hipError_t launch_check_velocity<double>(hipStream_t, const chd::BoxDesc*, int,
                                                  const void*, const void*, const void*, int*);
template hipError_t launch_check_velocity<float>(hipStream_t, const chd::BoxDesc*, int,
                                                 const void*, const void*, const void*, int*);
template hipError_t launch_interp<double>(hipStream_t, const void*, int64_t, int64_t, int64_t,
                                          int64_t, int64_t, const int*, const double*,
                                          const int*, const double*, const int*, const double*,
                                          void*);
template hipError_t launch_interp<float>(hipStream_t, const void*, int64_t, int64_t, int64_t,
                                         int64_t, int64_t, const int*, const double*,
                                         const int*, const double*, const int*, const double*,
                                         void*);

}  // namespace chk
