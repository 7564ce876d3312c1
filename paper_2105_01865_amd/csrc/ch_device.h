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

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

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
    int32_t xs;         // x segment of the segmented x program (0: whole lines)
    int32_t nxs;        // its segments per line
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
    int32_t zcmax;      // x pass: most planes per task (LDS layout)
};

// Index of a cell that may lie outside [0, n): periodic wrap, or even
// reflection about the walls (C[-1-m] = C[m], C[n+m] = C[n-1-m]).
CH_HD int map_idx(int i, int n, int bc)
{
    if (i >= 0 && i < n) return i;
    if (n == 1) return 0;
    if (i >= -n && i < 2 * n) {   // within one period: no division
        if (bc == 0) return i < 0 ? i + n : i - n;
        return i < 0 ? -1 - i : 2 * n - 1 - i;
    }
    // far out (warm-ups longer than the line): i lies in copy q of the line,
    // at offset r; under reflection every odd-numbered copy runs backwards
    const int q = i >= 0 ? i / n : -((n - 1 - i) / n);
    const int r = i - q * n;
    return (bc != 0 && (q & 1)) ? n - 1 - r : r;
}

// 1/x: on the GPU one hardware reciprocal (1 ulp) in single precision, and in
// double the hardware estimate refined by two Newton steps (r += r (1 - x r)),
// which leaves an error of a few ulp; a correctly rounded division on the host.
CH_HD double fast_rcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}
CH_HD float fast_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// One plane of a field seen from a wave-uniform base: elements are read and
// written at 32-bit byte offsets.  On the GPU it is a raw buffer resource
// (base, size in bytes; dword 3 = 32-bit data format), so the load unit
// forms the address from the scalar base and the lane offset with no
// per-lane 64-bit arithmetic, and an offset at or past `bytes` reads zero
// and drops a store.
#if !defined(__HIP_DEVICE_COMPILE__)
// host execution of the kernel code (tests): an access past a plane is a bug
inline void plane_overrun(uint32_t boff, uint32_t n)
{
    fprintf(stderr, "plane access at byte %u of a %u-byte plane\n", boff, n);
    abort();
}
#endif

#ifndef CH_BUFFER_LOADS
#define CH_BUFFER_LOADS 1
#endif

template <typename T>
struct PlaneRef {
#if defined(__HIP_DEVICE_COMPILE__) && CH_BUFFER_LOADS
    __amdgpu_buffer_rsrc_t rs;
    __device__ PlaneRef(const T* base, uint32_t bytes)
        : rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, (int)bytes,
                                               0x00020000))
    {
    }
    __device__ T operator()(uint32_t boff) const
    {
        if constexpr (sizeof(T) == 4) {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, boff, 0, 0));
        } else {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, boff, 0, 0));
        }
    }
    // element at lane offset voff plus the wave-uniform offset soff (which
    // takes the load's scalar offset field: no lane register for the sum)
    __device__ T operator()(uint32_t voff, uint32_t soff) const
    {
        if constexpr (sizeof(T) == 4) {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
        } else {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
        }
    }
    // the same load marked non-temporal: for data read once, so that it
    // does not push out of L2 what is read again (halo rows, the output a
    // following pass reads)
    __device__ T nt(uint32_t voff, uint32_t soff) const
    {
        if constexpr (sizeof(T) == 4) {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 2));
        } else {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 2));
        }
    }
    __device__ void store(uint32_t boff, T v) const { store(boff, 0u, v); }
    __device__ void store(uint32_t voff, uint32_t soff, T v) const
    {
        if constexpr (sizeof(T) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, voff, soff,
                                                  0);
        } else {
            typedef uint32_t u2 __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, voff, soff, 0);
        }
    }
#else
    const char* p;
    uint32_t n;
    CH_HD PlaneRef(const T* base, uint32_t bytes) : p(reinterpret_cast<const char*>(base)), n(bytes)
    {
    }
    CH_HD T operator()(uint32_t boff) const
    {
#if defined(__HIP_DEVICE_COMPILE__)
        return *reinterpret_cast<const T*>(p + boff);
#else
        if (boff + sizeof(T) > n) plane_overrun(boff, n);
        return *reinterpret_cast<const T*>(p + boff);
#endif
    }
    CH_HD T operator()(uint32_t voff, uint32_t soff) const { return (*this)(voff + soff); }
    CH_HD T nt(uint32_t voff, uint32_t soff) const { return (*this)(voff + soff); }
    CH_HD void store(uint32_t voff, uint32_t soff, T v) const { store(voff + soff, v); }
    CH_HD void store(uint32_t boff, T v) const
    {
#if defined(__HIP_DEVICE_COMPILE__)
        *reinterpret_cast<T*>(const_cast<char*>(p) + boff) = v;
#else
        if (boff + sizeof(T) > n) plane_overrun(boff, n);
        *reinterpret_cast<T*>(const_cast<char*>(p) + boff) = v;
#endif
    }
#endif
};

// Keep the instruction scheduler from moving code across this point, so
// that the work of two cells of one thread runs one after the other and
// shares its temporary registers.
CH_HD void sched_fence()
{
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_sched_barrier(0);
#endif
}

// Keep a wave-uniform value in a lane register from here on.
template <typename T>
CH_HD void in_vgpr(T& v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(v));
#else
    (void)v;
#endif
}

// Form v here: an empty asm statement takes it as an operand, so the
// compiler neither sinks its computation below this point nor recomputes it
// later (either would keep its inputs alive past here).
template <typename T>
CH_HD void pin(T& v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(v));
#else
    (void)v;
#endif
}

// A value the same in every lane, marked so (the compiler keeps it, and
// what is computed from it, in scalar registers).
CH_HD int uniform_i(int v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_readfirstlane(v);
#else
    return v;
#endif
}

// Wait until every global load the wave has issued has landed (vmcnt(0);
// expcnt and lgkmcnt untouched).  Used at the end of a loop's prologue: a load
// left pending there makes the compiler's conservative merge at the loop
// header wait, in every iteration, for the iteration's own prefetches.
CH_HD void wait_loads()
{
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_s_waitcnt(0x0F70);
#endif
}

// Fifth-order WENO (Jiang-Shu, point values as cell averages): value at the
// face between c and d with upwind side a.
//
// Arithmetic arranged for few instructions, exact in real arithmetic:
//  - everything is written in the first differences d1..d4 of the stencil:
//    per substencil k the second difference t_k and the combination u_k
//    (a - 4b + 3c, d - b, 3c - 4d + e), so that beta_k = 13/12 t_k^2 +
//    1/4 u_k^2 and the candidate value is q_k = c + t_k/12 + s_k u_k/4
//    (s = +1, +1, -1);
//  - the smoothness indicators and eps are scaled by 12/13 (the normalised
//    weights do not change): eps + beta is t^2 + (3/13) u^2 + (12/13) eps;
//  - the weights g_k / (eps + beta_k)^2 (g = 1/10, 6/10, 3/10) are formed
//    over the common denominator prod_k (eps + beta_k)^2, which leaves one
//    reciprocal; the factor 10 g_k is folded into the q_k - c coefficients,
//    which in the differences are (5 d2 - 2 d1)/6, d2 + 2 d3 and
//    2 d3 - d4/2.
// `epsw` is (12/13) eps.  weno5_inc returns the value minus c.
template <typename T>
CH_HD T weno5_inc(T d1, T d2, T d3, T d4, T epsw)
{
    const T k3 = T(3) / T(13);
    const T t0 = d2 - d1, t1 = d3 - d2, t2 = d4 - d3;
    const T u0 = T(3) * d2 - d1, u1 = d2 + d3, u2 = d4 - T(3) * d3;
    const T e0 = t0 * t0 + ((k3 * u0) * u0 + epsw);
    const T e1 = t1 * t1 + ((k3 * u1) * u1 + epsw);
    const T e2 = t2 * t2 + ((k3 * u2) * u2 + epsw);
    const T p0 = e0 * e0, p1 = e1 * e1, p2 = e2 * e2;
    const T p12 = p1 * p2, p02 = p0 * p2, p01 = p0 * p1;
    // 10 g_k (q_k - c)
    const T r0 = T(5) / T(6) * d2 - T(1) / T(3) * d1;
    const T r1 = d2 + T(2) * d3;
    const T r2 = T(2) * d3 - T(0.5) * d4;
    const T num = p12 * r0 + (p02 * r1 + p01 * r2);
    const T den = p12 + (T(6) * p02 + T(3) * p01);
    return num * fast_rcp(den);
}

template <typename T>
CH_HD T weno5(T a, T b, T c, T d, T e, T epsw)
{
    return c + weno5_inc<T>(b - a, c - b, d - c, e - d, epsw);
}

template <typename T>
struct Cubic {
    T c0, c1, c2, c3;
    CH_HD T operator()(T x) const { return ((c3 * x + c2) * x + c1) * x + c0; }
};

template <typename T>
CH_HD Cubic<T> cubic(const double* p)
{
    return Cubic<T>{T(p[0]), T(p[1]), T(p[2]), T(p[3])};
}

// compile-time integer tag
template <int V>
struct IC {
    static constexpr int value = V;
};

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
    // the first thread of tid's wave, as a wave-uniform value
    __device__ __forceinline__ int wave_base(int t) const
    {
        return __builtin_amdgcn_readfirstlane(t & ~63);
    }
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
    int wave_base(int t) const { return t & ~63; }
};

// upwinded WENO value on a face from the six values c[0..5] of cells
// f-3 .. f+2 around the face between c[2] and c[3]
template <typename T>
CH_HD T face_weno(T vel, T c0, T c1, T c2, T c3, T c4, T c5, T eps)
{
    const bool p = vel >= T(0);
    return weno5<T>(p ? c0 : c5, p ? c1 : c4, p ? c2 : c3, p ? c3 : c2, p ? c4 : c1, eps);
}

// The flux vel * value through the same face, from the five first
// differences D_j = c[j] - c[j-1] of the six cells and the two cells c2, c3
// next to the face.  Read from the downwind side the stencil's differences
// are the negated D in reverse order, and the increment is odd in the
// differences (exactly so in rounded arithmetic too), so
//   value = c2 + inc(D1, D2, D3, D4)  (vel >= 0),  c3 - inc(D5, D4, D3, D2),
// and vel * value = vel * centre + |vel| * inc.  One set of D serves both
// directions, neighbouring faces and the fourth differences.
template <typename T>
CH_HD T flux_weno_d(T vel, T D1, T D2, T D3, T D4, T D5, T c2, T c3, T eps)
{
    const bool p = vel >= T(0);
    const T inc = weno5_inc<T>(p ? D1 : D5, p ? D2 : D4, D3, p ? D4 : D2, eps);
    return vel * (p ? c2 : c3) + fabs(vel) * inc;
}

// Fourth difference (1,-4,6,-4,1) at the cell between D2 and D3 from the first
// differences D1 .. D4 of its five cells.
template <typename T>
CH_HD T d4_d(T D1, T D2, T D3, T D4)
{
    return (D4 - D1) + T(3) * (D2 - D3);
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
struct Chunk {
    int l, c0, fend, bend;
    bool live;
};

template <typename A>
struct LineState {
    A s1, s2;
    Chunk ch;   // the thread's (line, chunk), where a pass keeps it across phases
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

// Chunk of thread tid for chunks of length K (line_chunk_len).
CH_HD Chunk line_chunk_k(int tid, int nl, int n, int tw, int K)
{
    Chunk ch;
    ch.l = tid % nl;
    const int c = tid / nl;
    ch.c0 = c * K;
    ch.live = ch.c0 < n;
    const bool last = ch.c0 + K >= n;
    ch.fend = last ? n + tw : ch.c0 + K;
    ch.bend = ch.c0 + K < n ? ch.c0 + K : n;
    return ch;
}

CH_HD Chunk line_chunk(int tid, int nl, int n, int tw, int cap)
{
    return line_chunk_k(tid, nl, n, tw, line_chunk_len(n, tw, cap));
}

// Line pitch of an x solve tile whose lines hold `span` positions: odd, so
// that lanes walking different lines at the same position hit different
// LDS banks.
CH_HD int x_tile_pitch(int span) { return span | 1; }

// Halo positions -tw .. -1 and n .. n+tw-1 of the nl lines of an x solve tile
// (element (p, l) at tile[l * pitch + p + tw], a line contiguous) from the
// periodic or reflected continuation: lane q of each wave maps halo position
// q (and q + 64, ...) once, and the waves split the lines.
template <typename A>
CH_HD void x_tile_halos(int tid, int nth, A* tile, int pitch, int nl, int n, int tw, int bc)
{
    const int lane = tid & 63, wv = tid >> 6, nw = (nth + 63) >> 6;
    for (int q = lane; q < 2 * tw; q += 64) {
        const int pp = q < tw ? q - tw : n + q - tw;
        const int src = map_idx(pp, n, bc) + tw;
        for (int l = wv; l < nl; l += nw) tile[l * pitch + pp + tw] = tile[l * pitch + src];
    }
}

// The recurrences walk the tile in batches of LB values: the batch's loads
// are independent of the chain and go out together.
constexpr int LB = 8;

// Tile layouts of the line recurrences.  PS == 0: element (p, l) at
// tile[(p + tw) * pitch + l] (the lines across the fastest index: the y / z
// passes' column tiles).  PS > 0: element (p, l) at
// tile[l * pitch + (p + tw) * PS] (a line contiguous: the x solve tiles,
// whose position steps then fold into the LDS instructions' offsets).
template <int PS>
CH_HD int line_origin(int l, int tw, int pitch)
{
    return PS == 0 ? tw * pitch + l : l * pitch + tw * PS;
}
template <int PS>
CH_HD int line_step(int pitch)
{
    return PS == 0 ? pitch : PS;
}

template <typename A, int PS = 0>
CH_HD void line_f1(const Chunk& ch, const A* tile, int pitch, int tw, A a1, A a2, A ic,
                   LineState<A>& st)
{
    A w1 = A(0), w2 = A(0);
    if (ch.live) {
        const A* base = tile + line_origin<PS>(ch.l, tw, pitch);
        pitch = line_step<PS>(pitch);
        int p = ch.c0 - tw;
        for (; p + LB <= ch.c0; p += LB) {
            A v[LB];
#pragma unroll
            for (int j = 0; j < LB; ++j) v[j] = base[(p + j) * pitch];
#pragma unroll
            for (int j = 0; j < LB; ++j) {
                const A w = v[j] * ic - a1 * w1 - a2 * w2;
                w2 = w1;
                w1 = w;
            }
        }
        for (; p < ch.c0; ++p) {
            const A w = base[p * pitch] * ic - a1 * w1 - a2 * w2;
            w2 = w1;
            w1 = w;
        }
    }
    st.s1 = w1;
    st.s2 = w2;
}

template <typename A, int PS = 0>
CH_HD void line_f2(const Chunk& ch, A* tile, int pitch, int tw, A a1, A a2, A ic,
                   const LineState<A>& st)
{
    if (!ch.live) return;
    A w1 = st.s1, w2 = st.s2;
    A* base = tile + line_origin<PS>(ch.l, tw, pitch);
    pitch = line_step<PS>(pitch);
    int p = ch.c0;
    for (; p + LB <= ch.fend; p += LB) {
        A v[LB];
#pragma unroll
        for (int j = 0; j < LB; ++j) v[j] = base[(p + j) * pitch];
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            const A w = v[j] * ic - a1 * w1 - a2 * w2;
            v[j] = w;
            w2 = w1;
            w1 = w;
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) base[(p + j) * pitch] = v[j];
    }
    for (; p < ch.fend; ++p) {
        const A w = base[p * pitch] * ic - a1 * w1 - a2 * w2;
        base[p * pitch] = w;
        w2 = w1;
        w1 = w;
    }
}

template <typename A, int PS = 0>
CH_HD void line_b1(const Chunk& ch, const A* tile, int pitch, int tw, A a1, A a2,
                   LineState<A>& st)
{
    A y1 = A(0), y2 = A(0);
    if (ch.live) {
        const A* base = tile + line_origin<PS>(ch.l, tw, pitch);
        pitch = line_step<PS>(pitch);
        int p = ch.bend + tw - 1;
        for (; p - LB + 1 >= ch.bend; p -= LB) {
            A v[LB];
#pragma unroll
            for (int j = 0; j < LB; ++j) v[j] = base[(p - j) * pitch];
#pragma unroll
            for (int j = 0; j < LB; ++j) {
                const A y = v[j] - a1 * y1 - a2 * y2;
                y2 = y1;
                y1 = y;
            }
        }
        for (; p >= ch.bend; --p) {
            const A y = base[p * pitch] - a1 * y1 - a2 * y2;
            y2 = y1;
            y1 = y;
        }
    }
    st.s1 = y1;
    st.s2 = y2;
}

template <typename A, int PS = 0>
CH_HD void line_b2(const Chunk& ch, A* tile, int pitch, int tw, A a1, A a2,
                   const LineState<A>& st)
{
    if (!ch.live) return;
    A y1 = st.s1, y2 = st.s2;
    A* base = tile + line_origin<PS>(ch.l, tw, pitch);
    pitch = line_step<PS>(pitch);
    int p = ch.bend - 1;
    for (; p - LB + 1 >= ch.c0; p -= LB) {
        A v[LB];
#pragma unroll
        for (int j = 0; j < LB; ++j) v[j] = base[(p - j) * pitch];
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            const A y = v[j] - a1 * y1 - a2 * y2;
            v[j] = y;
            y2 = y1;
            y1 = y;
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) base[(p - j) * pitch] = v[j];
    }
    for (; p >= ch.c0; --p) {
        const A y = base[p * pitch] - a1 * y1 - a2 * y2;
        base[p * pitch] = y;
        y2 = y1;
        y1 = y;
    }
}

// ---------------------------------------------------------------------------
// Pass X: explicit terms, RHS and the x-line solve of eq-fac-1 for a task of
// `rows` complete x-lines (y0 .. y0+rows-1) over the planes z0 .. z0+nzc-1.
//
// March: thread tid owns the cells item = tid + nth m (m < MI) of the
// rows x nx plane tile and walks them up through the planes, keeping for
// each the column of C at z-3 .. z+3 and the flux through its low z face in
// registers, so each z face flux is computed once; x and y face fluxes are
// computed once per face and exchanged through LDS.  The RHS of every plane
// goes into one LDS tile of rows x nzc lines, which is then solved in place
// by all threads at once and written out.  Two barriers per plane: the RHS
// of plane z-1 is finished in the same phase that loads plane z.
//
// LDS (launch-wide pitches; all sizes from the largest box):
//   pb: (rmax + 6) x (nx_max + 6) T  C of the plane, rows y0-3 .. y0+rows+2,
//                                    columns -3 .. nx+2
//   fx: rmax x (nx_max + 1) T        flux through x face f of each row
//   fy: (rmax + 1) x nx_max T        flux through y face y0 + r
//   tb: rmax zcmax x pitch A         RHS -> solve tile: line zs * rows + r,
//                                    positions -tw .. nx+tw-1 contiguous
//                                    (pitch: nx_max + 2 tw_max, made odd)
// ---------------------------------------------------------------------------
struct XLayout {
    size_t pb, mb, fx, fy, tb, zm, zp, total;  // byte offsets and total size
    int pbp, mbp, fxp, fyp, tbp;               // pitches (elements)
};

CH_HD size_t al16(size_t b) { return (b + 15) & ~size_t(15); }

// e25: the explicit 25-point mode, which has no solve tile and keeps the
// owned row of the planes z-1 and z+1 (pitch mbp, one halo column a side).
CH_HD XLayout x_layout(int nx_max, int rmax, int zcmax, int tw_max, int sT, int sA,
                       bool e25 = false)
{
    XLayout L;
    L.pbp = nx_max + 6;
    L.mbp = nx_max + 2;
    L.fxp = nx_max + 1;
    L.fyp = nx_max;
    L.tbp = x_tile_pitch(nx_max + 2 * tw_max);
    L.pb = 0;
    L.mb = al16(L.pb + (size_t)(rmax + 6) * L.pbp * sT);
    L.fx = al16(L.mb + (size_t)(rmax + 2) * L.mbp * sT);
    L.fy = al16(L.fx + (size_t)rmax * L.fxp * sT);
    L.tb = al16(L.fy + (size_t)(rmax + 1) * L.fyp * sT);
    if (e25) {
        L.zm = L.tb;
        L.zp = al16(L.zm + (size_t)L.mbp * sT);
        L.total = al16(L.zp + (size_t)L.mbp * sT);
    } else {
        L.zm = L.zp = 0;
        L.total = al16(L.tb + (size_t)rmax * zcmax * L.tbp * sA);
    }
    return L;
}

struct XZTask {
    int z0, nzc, y0, rows;
    int x0, xlen;   // x segment (the whole line unless the box is segmented)
};

// Task order: x segments fastest, then rows, then chunks of planes.
CH_HD XZTask xz_task(const BoxDesc& bd, int task)
{
    XZTask t;
    int local = task - bd.task0[PASS_X];
    t.x0 = 0;
    t.xlen = bd.n[0];
    if (bd.xs > 0) {
        const int sg = local % bd.nxs;
        local /= bd.nxs;
        t.x0 = sg * bd.xs;
        t.xlen = bd.n[0] - t.x0 < bd.xs ? bd.n[0] - t.x0 : bd.xs;
    }
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

// Planes of x-pass inputs held in registers ahead of the plane being computed
// (1 or 2).  One plane keeps the state within 128 VGPRs in FP32.
#ifndef X_PREFETCH
#define X_PREFETCH 1
#endif

template <typename T, typename A, int MI>
struct XState {
    T cz[MI][7];     // C at z-3 .. z+3 of each owned cell
    T mq[MI][3];     // psi'(C) at z-1, z, z+1
    T fzl[MI];       // flux through the low z face of the current plane
    T pz[MI];        // z flux difference of the current plane
    T plap[MI];      // sum of second differences of psi'(C)
    T pb4[MI];       // sum of fourth differences of C
    T vel[MI][6];    // u, v, w on the low and high faces of the cell
    T eold[MI];      // E of the previous substage
    T eold_next[MI]; // E of the previous substage on this plane, until the
                     // RHS of the plane below has used eold
    // the next X_PREFETCH planes, loaded while this one is computed (set b
    // holds planes z0 + b, z0 + b + X_PREFETCH, ...)
    T ncz[X_PREFETCH][MI];       // C at z+3 of the plane
    T nvel[X_PREFETCH][MI][4];   // u low, u high, v low, v high
    T nwh[X_PREFETCH][MI];       // w on the high face
    T neold[X_PREFETCH][MI];     // old E
    T nhalo[X_PREFETCH][MI][6];  // C of the halo rows hr with hr mod rows equal to
                                 // the owned row, at the owned column
    int rx[MI];      // (row << 16) | x of each owned cell, -1 if none
    uint32_t col[MI];   // byte offset of the cell in a plane of C, E, v, w
    uint32_t colu[MI];  // byte offset of its low x face in a plane of u
    int cxp[MI];     // halo column (-3 .. nx+2) that copies the owned column in
                     // the C tile, or the column itself if none (nx >= 6)
    int cxm[MI];     // the same for the psi'(C) tile (-1 .. nx)
    int xmask[MI];   // all halo columns fed by the owned column (any nx)
    LineState<A> ls;
    // explicit 25-point mode: mixed second differences of the plane below
    // (xy and xz), and C of the rows y-1, y+1 at the planes z-2, z-1
    T pmix[MI];
    T hq[MI][2][2];
};

template <typename T, typename A, int MI, bool E25, class X, bool VCONST = false>
CH_HD void pass_x_program(X& ex, XState<T, A, MI>* st, const BoxDesc& bd, const PassArgs& pa,
                          int task, const T* __restrict__ C, const T* __restrict__ U,
                          const T* __restrict__ V, const T* __restrict__ W, T* __restrict__ E,
                          T* __restrict__ Q, unsigned char* smem)
{
    const XZTask t = xz_task(bd, task);
    const int nx = bd.n[0], ny = bd.n[1], nz = bd.n[2];
    const int fx = bd.nf[0], fy = bd.nf[1];
    const int bcx = bd.bc[0];
    const int k = pa.k, tw = bd.tw[k];
    const int nth = ex.nth;
    const XLayout L = x_layout(pa.nx_max, pa.rmax, pa.zcmax, pa.tw_max, (int)sizeof(T),
                               (int)sizeof(A), E25);
    constexpr uint32_t sT = sizeof(T);
    T* pb = reinterpret_cast<T*>(smem + L.pb);
    T* mb = reinterpret_cast<T*>(smem + L.mb);
    T* fxb = reinterpret_cast<T*>(smem + L.fx);
    T* fyb = reinterpret_cast<T*>(smem + L.fy);
    A* tb = reinterpret_cast<A*>(smem + L.tb);
    T* zmb = reinterpret_cast<T*>(smem + L.zm);   // explicit mode: owned row at z-1
    T* zpb = reinterpret_cast<T*>(smem + L.zp);   // and at z+1
    const int64_t plane = (int64_t)nx * ny;
    // bytes of one plane of C, E, q and w, of u, and of v
    const uint32_t pbytes = (uint32_t)(plane * sT);
    const uint32_t ubytes = (uint32_t)((int64_t)ny * fx * sT);
    const uint32_t vbytes = (uint32_t)((int64_t)fy * nx * sT);
    const T* Cb = C + bd.c_off;
    const T* Ub = U + bd.u_off;
    const T* Vb = V + bd.v_off;
    const T* Wb = W + bd.w_off;
    T* Eb = E + bd.c_off;
    T* Qb = Q + bd.c_off;
    T epsw = T(bd.eps * (12.0 / 13.0));
    T gdt = T(bd.gdt[k]), rdt = T(bd.rdt[k]), bdt = T(bd.bdt[k]);
    T inv_h = T(bd.inv_h), lap_s = T(bd.inv_h2 * bd.inv_pe);
    Cubic<T> mu = cubic<T>(bd.psi);
    if constexpr (VCONST) {
        // these constants live in lane registers, where the kernel has room,
        // instead of scalar registers, which run out in double precision
        in_vgpr(epsw);
        in_vgpr(gdt);
        in_vgpr(rdt);
        in_vgpr(bdt);
        in_vgpr(inv_h);
        in_vgpr(lap_s);
        in_vgpr(mu.c0);
        in_vgpr(mu.c1);
        in_vgpr(mu.c2);
        in_vgpr(mu.c3);
    }
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]), ic = A(bd.ic[k]);
    const int rows = t.rows;
    const int ncell = rows * nx;
    const int nlines = rows * t.nzc;
    // the six halo rows (y0-3 .. y0-1, y0+rows .. y0+rows+2), their tile rows,
    // and the owned row whose threads load them (hr mod rows)
    int hrow[6], hown[6];
    uint32_t hoffb[6];   // byte offsets of the halo rows in a plane
#pragma unroll
    for (int hr = 0; hr < 6; ++hr) {
        const int prow = hr < 3 ? hr : rows + hr;
        hrow[hr] = prow;
        hown[hr] = hr % rows;
        hoffb[hr] = (uint32_t)(map_idx(t.y0 - 3 + prow, ny, bd.bc[1]) * nx) * sT;
    }
    const bool one_copy = nx >= 6;   // every column feeds at most one halo column
    // byte offset, in a plane of v, of the row of the task's top y face (the
    // high face of the last row: periodic wrap, or the wall face ny)
    const int ytop = t.y0 + rows;
    const uint32_t vtopb = (uint32_t)((ytop == ny && bd.bc[1] == 0 ? 0 : ytop) * nx) * sT;

    // all global loads of plane z for the owned cells, into prefetch set b
    // (uniform plane bases, 32-bit offsets within a plane)
    auto fetch = [&](XState<T, A, MI>& s, auto bset, int z) {
        constexpr int b = decltype(bset)::value;
        const PlaneRef<T> Cq(Cb + (int64_t)map_idx(z + 3, nz, bd.bc[2]) * plane, pbytes);
        const PlaneRef<T> Uz(Ub + (int64_t)z * ny * fx, ubytes);
        const PlaneRef<T> Vz(Vb + (int64_t)z * fy * nx, vbytes);
        const PlaneRef<T> Wh(Wb + (int64_t)((z + 1 == nz && bd.bc[2] == 0) ? 0 : z + 1) * plane,
                             pbytes);
        const PlaneRef<T> Ez(Eb + (int64_t)z * plane, pbytes);
        const PlaneRef<T> Cz(Cb + (int64_t)z * plane, pbytes);
#pragma unroll
        for (int m = 0; m < MI; ++m) {
            if (s.rx[m] >= 0) {
                const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
                s.ncz[b][m] = Cq(s.col[m]);
                s.nvel[b][m][0] = Uz(s.colu[m]);
                s.nvel[b][m][1] = (x == nx - 1 && bcx != 0) ? Uz(s.colu[m] + sT) : T(0);
                s.nvel[b][m][2] = Vz(s.col[m]);
                s.nvel[b][m][3] = r == rows - 1 ? Vz((uint32_t)x * sT, vtopb) : T(0);
                s.nwh[b][m] = Wh(s.col[m]);
                s.neold[b][m] = pa.e_mode != 0 ? Ez(s.col[m]) : T(0);
                const uint32_t xb = (uint32_t)x * sT;
#pragma unroll
                for (int hr = 0; hr < 6; ++hr)
                    if (hown[hr] == r) s.nhalo[b][m][hr] = Cz(xb, hoffb[hr]);
            }
        }
    };
    // a value of an owned row at column x, and its copies in the halo columns:
    // the one column cx when nx >= 6, else every bit q of mask (column q - 3
    // for q < 3, nx + q - 3 otherwise)
    auto put = [&](T* tile, int pitch, int halo, int prow, int x, int cx, int mask, T v) {
        T* rp = tile + prow * pitch + halo;
        rp[x] = v;
        if (one_copy) {
            rp[cx] = v;
        } else if (mask) {
#pragma unroll
            for (int q = 3 - halo; q < 3 + halo; ++q)
                if ((mask >> q) & 1) rp[q < 3 ? q - 3 : nx + q - 3] = v;
        }
    };
    // RHS of plane zs of the owned cells into the solve tile; in the explicit
    // 25-point mode, C + dt (gamma N + rho N_old) into Q instead, with yz the
    // mixed yz difference and cc the C of each owned cell at plane zs
    auto rhs_plane = [&](XState<T, A, MI>& s, int zs, const T* yz, const T* cc) {
        const PlaneRef<T> Ez(Eb + (int64_t)(t.z0 + zs) * plane, pbytes);
        const PlaneRef<T> Qz(Qb + (int64_t)(t.z0 + zs) * plane, pbytes);
#pragma unroll
        for (int m = 0; m < MI; ++m) {
            if (s.rx[m] < 0) continue;
            const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
            const T fhi = x + 1 < nx ? fxb[r * L.fxp + x + 1]
                                     : fxb[r * L.fxp + (bcx == 0 ? 0 : nx)];
            const T adv = (fhi - fxb[r * L.fxp + x])
                        + (fyb[(r + 1) * L.fyp + x] - fyb[r * L.fyp + x]) + s.pz[m];
            const T e = -adv * inv_h + s.plap[m] * lap_s;
            if constexpr (E25) {
                // every term explicit: N = E - Cn^2/(h^4 Pe) (25-point lap^2 C),
                // kept in place of E for the next substage
                const T nk = e - bdt * (s.pb4[m] + T(2) * (s.pmix[m] + yz[m]));
                T rhs = gdt * nk;
                if (pa.e_mode != 0) rhs += rdt * s.eold[m];
                if (pa.e_mode != 2) Ez.store(s.col[m], nk);
                Qz.store(s.col[m], cc[m] + rhs);
            } else {
                T rhs = gdt * e - bdt * s.pb4[m];
                if (pa.e_mode != 0) rhs += rdt * s.eold[m];
                if (pa.e_mode != 2) Ez.store(s.col[m], e);
                tb[(zs * rows + r) * L.tbp + x + tw] = A(rhs);
            }
        }
    };

    // owned cells, the queue below the first plane, and the first plane's loads
    ex.phase([&](int tid) {
        XState<T, A, MI>& s = st[ex.slot(tid)];
        const T* Wz = Wb + (int64_t)t.z0 * plane;
#pragma unroll
        for (int m = 0; m < MI; ++m) {
            const int item = tid + nth * m;
            s.rx[m] = item < ncell ? ((item / nx) << 16) | (item % nx) : -1;
            int mask = 0;
            s.cxp[m] = 0;
            s.cxm[m] = 0;
            if (s.rx[m] >= 0) {
                const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
                const int y = t.y0 + r;
                s.col[m] = (uint32_t)(y * nx + x) * sT;
                s.colu[m] = (uint32_t)(y * fx + x) * sT;
                s.cxp[m] = x;
                s.cxm[m] = x;
                for (int q = 0; q < 6; ++q)
                    if (map_idx(q < 3 ? q - 3 : nx + q - 3, nx, bcx) == x) {
                        mask |= 1 << q;
                        s.cxp[m] = q < 3 ? q - 3 : nx + q - 3;
                        if (q == 2 || q == 3) s.cxm[m] = q == 2 ? -1 : nx;
                    }
#pragma unroll
                for (int q = 1; q < 7; ++q)
                    s.cz[m][q] = PlaneRef<T>(Cb + (int64_t)map_idx(t.z0 - 4 + q, nz, bd.bc[2]) * plane,
                                             pbytes)(s.col[m]);
                s.mq[m][1] = mu(s.cz[m][3]);   // psi'(C) at z0-2 .. z0 after the first shift
                s.mq[m][2] = mu(s.cz[m][4]);
                s.vel[m][4] = PlaneRef<T>(Wz, pbytes)(s.col[m]);
                if constexpr (E25) {
                    // rows y-1, y+1 at plane z0-1 (the first shift moves them down)
                    const PlaneRef<T> Cm(Cb + (int64_t)map_idx(t.z0 - 1, nz, bd.bc[2]) * plane,
                                         pbytes);
                    const uint32_t xb = (uint32_t)x * sT;
                    s.hq[m][0][0] = s.hq[m][1][0] = T(0);
                    s.hq[m][0][1] = Cm(xb, hoffb[2]);
                    s.hq[m][1][1] = Cm(xb, hoffb[3]);
                }
            }
            s.xmask[m] = mask;
        }
        wait_loads();
        fetch(s, IC<0>{}, t.z0);
        if (X_PREFETCH == 2 && t.nzc > 1) fetch(s, IC<X_PREFETCH - 1>{}, t.z0 + 1);
    });

    // one plane of the march; the prefetch set alternates, so the loop is
    // unrolled by two to keep the set index a constant
    auto plane_step = [&](auto bset, int zs) {
        constexpr int b = decltype(bset)::value;
        const int z = t.z0 + zs;
        // ---- take this plane's loads, start the loads X_PREFETCH planes up, RHS of
        //      the plane below
        ex.phase([&](int tid) {
            XState<T, A, MI>& s = st[ex.slot(tid)];
            // take this plane's loads out of the prefetch registers; the halo
            // rows go straight into the plane tiles
            T own[MI];
#pragma unroll
            for (int m = 0; m < MI; ++m) {
                if (s.rx[m] >= 0) {
#pragma unroll
                    for (int q = 0; q < 6; ++q) s.cz[m][q] = s.cz[m][q + 1];
                    s.cz[m][6] = s.ncz[b][m];
                    own[m] = s.cz[m][3];
                    s.vel[m][0] = s.nvel[b][m][0];
                    s.vel[m][1] = s.nvel[b][m][1];
                    s.vel[m][2] = s.nvel[b][m][2];
                    s.vel[m][3] = s.nvel[b][m][3];
                    if (zs > 0) s.vel[m][4] = s.vel[m][5];
                    s.vel[m][5] = s.nwh[b][m];
                    s.eold_next[m] = s.neold[b][m];
                    // halo rows (no halo columns: only owned rows are read
                    // across x), and psi'(C) of the two next to the tile
                    const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
#pragma unroll
                    for (int hr = 0; hr < 6; ++hr) {
                        if (hown[hr] != r) continue;
                        const T v = s.nhalo[b][m][hr];
                        if (E25 && (hr == 2 || hr == 3))   // the mixed xy term reads x +- 1
                            put(pb, L.pbp, 3, hrow[hr], x, s.cxp[m], s.xmask[m], v);
                        else
                            pb[hrow[hr] * L.pbp + 3 + x] = v;
                        if (hr == 2) mb[1 + x] = mu(v);
                        if (hr == 3) mb[(rows + 1) * L.mbp + 1 + x] = mu(v);
                    }
                }
            }
            // explicit mode: the mixed yz difference of the plane below, from the
            // rows y-1, y+1 at z-2, z-1 (queue) and z (this plane's halo)
            T yz[MI], cc[MI];
            if constexpr (E25) {
#pragma unroll
                for (int m = 0; m < MI; ++m) {
                    if (s.rx[m] < 0) continue;
                    const T* c = s.cz[m];
                    const T* hm = s.hq[m][0];
                    const T* hp = s.hq[m][1];
                    const T lo = (hm[0] - hm[1]) + (s.nhalo[b][m][2] - hm[1]);
                    const T mid = (c[1] - c[2]) + (c[3] - c[2]);
                    const T hi = (hp[0] - hp[1]) + (s.nhalo[b][m][3] - hp[1]);
                    yz[m] = (lo + hi) - T(2) * mid;
                    cc[m] = c[2];
                    s.hq[m][0][0] = hm[1];
                    s.hq[m][0][1] = s.nhalo[b][m][2];
                    s.hq[m][1][0] = hp[1];
                    s.hq[m][1][1] = s.nhalo[b][m][3];
                }
            }
            // start the loads X_PREFETCH planes up, before any store of this phase
            if (zs + X_PREFETCH < t.nzc) fetch(s, IC<b>{}, z + X_PREFETCH);
            // RHS of the plane below (stores E)
            if (zs > 0) rhs_plane(s, zs - 1, yz, cc);
#pragma unroll
            for (int m = 0; m < MI; ++m) {
                if (s.rx[m] < 0) continue;
                const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
                s.eold[m] = s.eold_next[m];
                s.mq[m][0] = s.mq[m][1];
                s.mq[m][1] = s.mq[m][2];
                s.mq[m][2] = mu(s.cz[m][4]);
                put(pb, L.pbp, 3, r + 3, x, s.cxp[m], s.xmask[m], own[m]);
                put(mb, L.mbp, 1, r + 1, x, s.cxm[m], s.xmask[m], s.mq[m][1]);
                if constexpr (E25) {
                    put(zmb, L.mbp, 1, 0, x, s.cxm[m], s.xmask[m], s.cz[m][2]);
                    put(zpb, L.mbp, 1, 0, x, s.cxm[m], s.xmask[m], s.cz[m][4]);
                }
            }
        });
        // ---- face fluxes, Laplacian of psi'(C), fourth differences
        ex.phase([&](int tid) {
            XState<T, A, MI>& s = st[ex.slot(tid)];
#pragma unroll
            for (int m = 0; m < MI; ++m) {
                if (s.rx[m] < 0) continue;
                const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
                const T* row = pb + (r + 3) * L.pbp + x + 3;   // row[o] = C(x + o)
                const T* colm = pb + r * L.pbp + x + 3;        // colm[o * pbp] = C(y - 3 + o)
                const T* mrow = mb + (r + 1) * L.mbp + x + 1;  // mrow[o] = psi'(C)(x + o)
                const int p = L.pbp, mp = L.mbp;
                const T* vl = s.vel[m];
                // Each direction's first differences (D_j = C_j - C_{j-1}) serve its
                // faces and its fourth difference; the directions are taken one
                // after the other so that only one set is live at a time.
                // x: C(x-2..x+2) minus the cell before; the low face of the cell,
                // and the wall face nx
                {
                    const T dX[5] = {row[-2] - row[-3], row[-1] - row[-2], row[0] - row[-1],
                                     row[1] - row[0], row[2] - row[1]};
                    fxb[r * L.fxp + x] = flux_weno_d<T>(vl[0], dX[0], dX[1], dX[2], dX[3], dX[4],
                                                        row[-1], row[0], epsw);
                    if (x == nx - 1 && bcx != 0)
                        fxb[r * L.fxp + nx] = vl[1] * face_weno<T>(vl[1], row[-2], row[-1], row[0],
                                                                     row[1], row[2], row[3], epsw);
                    s.pb4[m] = d4_d<T>(dX[1], dX[2], dX[3], dX[4]);
                }
                // y: rows y-2 .. y+2; the low face, and the top face for the last row
                {
                    T dY[5];
#pragma unroll
                    for (int j = 0; j < 5; ++j) dY[j] = colm[(j + 1) * p] - colm[j * p];
                    fyb[r * L.fyp + x] = flux_weno_d<T>(vl[2], dY[0], dY[1], dY[2], dY[3], dY[4],
                                                        colm[2 * p], colm[3 * p], epsw);
                    if (r == rows - 1)
                        fyb[(r + 1) * L.fyp + x] =
                            flux_weno_d<T>(vl[3], dY[1], dY[2], dY[3], dY[4], colm[6 * p] - colm[5 * p],
                                           colm[3 * p], colm[4 * p], epsw);
                    s.pb4[m] += d4_d<T>(dY[1], dY[2], dY[3], dY[4]);
                }
                // z: planes z-1 .. z+3; the high face (the low one carries over
                // from the plane below)
                const T* c = s.cz[m];
                {
                    T dZ[5];
#pragma unroll
                    for (int j = 0; j < 5; ++j) dZ[j] = c[j + 2] - c[j + 1];
                    if (zs == 0)   // the low face of the task's first plane, in the same
                                   // form as every face after it
                        s.fzl[m] = flux_weno_d<T>(vl[4], c[1] - c[0], c[2] - c[1], c[3] - c[2],
                                                  c[4] - c[3], c[5] - c[4], c[2], c[3], epsw);
                    const T fzh =
                        flux_weno_d<T>(vl[5], dZ[0], dZ[1], dZ[2], dZ[3], dZ[4], c[3], c[4], epsw);
                    s.pz[m] = fzh - s.fzl[m];
                    s.fzl[m] = fzh;
                    s.pb4[m] += d4_d<T>(dZ[0], dZ[1], dZ[2], dZ[3]);
                }
                const T mu0 = s.mq[m][1];
                s.plap[m] = ((mrow[1] + mrow[-1]) + (mrow[mp] + mrow[-mp]))
                          + (s.mq[m][2] + s.mq[m][0]) - T(6) * mu0;
                if constexpr (E25) {
                    // mixed second differences xy (rows y -+ 1 of this plane) and xz
                    // (the owned row at z -+ 1)
                    auto d2x = [](const T* q) { return (q[-1] - q[0]) + (q[1] - q[0]); };
                    const T dx0 = d2x(row);
                    const T xy = (d2x(row - p) + d2x(row + p)) - T(2) * dx0;
                    const T xz = (d2x(zmb + 1 + x) + d2x(zpb + 1 + x)) - T(2) * dx0;
                    s.pmix[m] = xy + xz;
                }
                if (m + 1 < MI) sched_fence();
            }
        });
    };
    for (int zs = 0; zs < t.nzc; zs += X_PREFETCH) {
        plane_step(IC<0>{}, zs);
        if (X_PREFETCH == 2 && zs + 1 < t.nzc) plane_step(IC<X_PREFETCH - 1>{}, zs + 1);
    }
    // ---- RHS of the last plane
    ex.phase([&](int tid) {
        XState<T, A, MI>& s = st[ex.slot(tid)];
        T yz[MI], cc[MI];
        if constexpr (E25) {
            // rows y -+ 1 at the plane above the chunk, loaded here once
            const int zl = t.z0 + t.nzc - 1;
            const PlaneRef<T> Cn1(Cb + (int64_t)map_idx(zl + 1, nz, bd.bc[2]) * plane, pbytes);
#pragma unroll
            for (int m = 0; m < MI; ++m) {
                if (s.rx[m] < 0) continue;
                const uint32_t xb = (uint32_t)(s.rx[m] & 0xffff) * sT;
                const T* c = s.cz[m];
                const T* hm = s.hq[m][0];
                const T* hp = s.hq[m][1];
                const T lo = (hm[0] - hm[1]) + (Cn1(xb, hoffb[2]) - hm[1]);
                const T mid = (c[2] - c[3]) + (c[4] - c[3]);
                const T hi = (hp[0] - hp[1]) + (Cn1(xb, hoffb[3]) - hp[1]);
                yz[m] = (lo + hi) - T(2) * mid;
                cc[m] = c[3];
            }
        }
        rhs_plane(s, t.nzc - 1, yz, cc);
    });
    if constexpr (E25) return;   // no solve: the new C is written
    // ---- halos of the solve tile; each thread's (line, chunk) of the solve
    ex.phase([&](int tid) {
        x_tile_halos<A>(tid, nth, tb, L.tbp, nlines, nx, tw, bcx);
        st[ex.slot(tid)].ls.ch = line_chunk(tid, nlines, nx, tw, X_CHAINS);
    });
    // ---- x solve of all lines at once
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_f1<A, 1>(ls.ch, tb, L.tbp, tw, a1, a2, ic, ls);
    });
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_f2<A, 1>(ls.ch, tb, L.tbp, tw, a1, a2, ic, ls);
    });
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_b1<A, 1>(ls.ch, tb, L.tbp, tw, a1, a2, ls);
    });
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_b2<A, 1>(ls.ch, tb, L.tbp, tw, a1, a2, ls);
    });
    // ---- store q, plane by plane, x fastest
    ex.phase([&](int tid) {
        XState<T, A, MI>& s = st[ex.slot(tid)];
        for (int zs = 0; zs < t.nzc; ++zs) {
            const PlaneRef<T> Qz(Qb + (int64_t)(t.z0 + zs) * plane, pbytes);
#pragma unroll
            for (int m = 0; m < MI; ++m) {
                if (s.rx[m] < 0) continue;
                const int r = s.rx[m] >> 16, x = s.rx[m] & 0xffff;
                Qz.store(s.col[m], T(tb[(zs * rows + r) * L.tbp + x + tw]));
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Pass X with one cell per thread and the y stencil in registers (the same
// arithmetic as pass_x_program, which the plan takes instead where this one
// does not apply: see plan_dt).
//
// A task is `rows` complete x-lines (rows = 1 whenever a line fills a
// work-group; narrow boxes of an ensemble take several) over nzc planes.
// Every thread owns one cell and marches it up through the planes.  The
// y-direction stencil of a cell is its own column, so the six halo rows of C
// go straight into the thread's registers, and the y differences, the y face
// fluxes and the y neighbours of psi'(C) are formed there.  LDS carries the
// owned rows (C and psi'(C) with their x halos), the x face fluxes, the y
// face fluxes that the rows of a task share, and the solve tile.  Each field
// of the box is one buffer resource with 32-bit byte offsets (every field of
// every box under 4 GiB): the plane goes into the scalar offset.  The row
// mode RM says where the row offsets live:
//   XR_ONE     one row per task: every row offset is uniform and goes there
//              too;
//   XR_THREAD  several rows per task, the row offsets per thread;
//   XR_WAVE    several rows per task, each of whole waves (nx a multiple of
//              64, or one row per task): the row is read from the wave's
//              first thread, so its offsets are uniform per wave.
// XR_THREAD and XR_WAVE map threads to cells alike and give the same bits.
// Threads past the task's cells read its last cell and store nothing.
//
// LDS of a box (launch size: the largest over boxes):
//   cr: rows x (nx + 6) T      C of the owned rows, columns -3 .. nx+2
//   mr: rows x (nx + 2) T      psi'(C) of the owned rows, columns -1 .. nx
//   fr: rows x (nx + 1) T      flux through x face f of each row
//   fy: rows x nx T            (several rows) flux through the low y face of
//                              each cell, which is the high face of the row below
//   tb: rows zc x pitch A      RHS -> solve tile: line zs rows + r, positions
//                              -tw .. nx+tw-1 contiguous (pitch nx + 2 tw_max,
//                              made odd)
// ---------------------------------------------------------------------------
enum : int { XR_ONE = 0, XR_THREAD = 1, XR_WAVE = 2 };

struct XRowLayout {
    size_t cr, mr, fr, fy, tb, total;   // byte offsets and total size
    int crp, mrp, frp, tbp;             // pitches (elements)
};

CH_HD XRowLayout x_row_layout(int nx, int rows, int zc, int tw_max, int sT, int sA)
{
    XRowLayout L;
    L.crp = nx + 6;
    L.mrp = nx + 2;
    L.frp = nx + 1;
    L.tbp = x_tile_pitch(nx + 2 * tw_max);
    L.cr = 0;
    L.mr = al16(L.cr + (size_t)rows * L.crp * sT);
    L.fr = al16(L.mr + (size_t)rows * L.mrp * sT);
    L.fy = al16(L.fr + (size_t)rows * L.frp * sT);
    L.tb = al16(L.fy + (rows > 1 ? (size_t)rows * nx * sT : 0));
    L.total = al16(L.tb + (size_t)rows * zc * L.tbp * sA);
    return L;
}

template <typename T, typename A>
struct XRowState {
    T c[7];                   // C at z-3 .. z+3 of the owned cell
    T mq[3];                  // psi'(C) at z-1, z, z+1
    T yh[6];                  // C of this plane at rows y-3, y-2, y-1, y+1, y+2, y+3
    T ul, vl, vh, wl, wh;     // u on the low x face, v on the low and high y faces,
                              // w on the low and high z faces
    T fzl;                    // flux through the low z face
    T eold;                   // E of the previous substage at the plane whose RHS is next
    T py, pz, plap, pb4;      // y and z flux differences, Laplacian of psi', sum of D4
                              // (several rows per task, below the last row: py is
                              // minus the low y face's flux until the RHS adds the
                              // high one, which the row above forms)
    T nc;                     // C at z+4 of the owned cell (the next plane's c[6])
    int cxp, cxm;             // halo columns of the C and psi' rows fed by the
                              // owned column (or the column itself)
    int r, x;                 // the owned cell (several rows per task)
    bool live;
    uint32_t ro, rou, rvt;    // byte offsets in a plane of its row of C (v, w, E, q),
                              // of u, and of v's high face
    uint32_t ho[6];           // and of its six halo rows
    LineState<A> ls;
};

template <typename T, typename A, int RM, class X, bool VCONST = false>
CH_HD void pass_x_row_program(X& ex, XRowState<T, A>* st, const BoxDesc& bd, const PassArgs& pa,
                              int task, const T* __restrict__ C, const T* __restrict__ U,
                              const T* __restrict__ V, const T* __restrict__ W,
                              T* __restrict__ E, T* __restrict__ Q, unsigned char* smem)
{
    constexpr bool MR = RM != XR_ONE;
    const XZTask t = xz_task(bd, task);
    const int nx = bd.n[0], ny = bd.n[1], nz = bd.n[2];
    const int fx = bd.nf[0], fy = bd.nf[1], fz = bd.nf[2];
    const int bcx = bd.bc[0];
    const int k = pa.k, tw = bd.tw[k];
    const int nth = ex.nth;
    const int rows = MR ? t.rows : 1;
    const XRowLayout L = x_row_layout(nx, MR ? bd.x_rows : 1, bd.zc, pa.tw_max, (int)sizeof(T),
                                      (int)sizeof(A));
    constexpr uint32_t sT = sizeof(T);
    T* crb = reinterpret_cast<T*>(smem + L.cr) + 3;   // row r: crb[r crp + x], -3 <= x < nx + 3
    T* mrb = reinterpret_cast<T*>(smem + L.mr) + 1;   // row r: mrb[r mrp + x], -1 <= x < nx + 1
    T* frb = reinterpret_cast<T*>(smem + L.fr);       // row r: frb[r frp + f], 0 <= f <= nx
    T* fyb = reinterpret_cast<T*>(smem + L.fy);       // row r: fyb[r nx + x] (MR)
    A* tb = reinterpret_cast<A*>(smem + L.tb);
    const int tbp = L.tbp;
    // bytes of a plane of C (E, q and w too), of u and of v
    const uint32_t pbytes = (uint32_t)((int64_t)nx * ny * sT);
    const uint32_t ubytes = (uint32_t)((int64_t)ny * fx * sT);
    const uint32_t vbytes = (uint32_t)((int64_t)fy * nx * sT);
    const PlaneRef<T> Cr(C + bd.c_off, (uint32_t)((int64_t)pbytes * nz));
    const PlaneRef<T> Ur(U + bd.u_off, (uint32_t)((int64_t)ubytes * nz));
    const PlaneRef<T> Vr(V + bd.v_off, (uint32_t)((int64_t)vbytes * nz));
    const PlaneRef<T> Wr(W + bd.w_off, (uint32_t)((int64_t)pbytes * fz));
    const PlaneRef<T> Er(E + bd.c_off, (uint32_t)((int64_t)pbytes * nz));
    const PlaneRef<T> Qr(Q + bd.c_off, (uint32_t)((int64_t)pbytes * nz));
    T epsw = T(bd.eps * (12.0 / 13.0));
    T gdt = T(bd.gdt[k]), rdt = T(bd.rdt[k]), bdt = T(bd.bdt[k]);
    T inv_h = T(bd.inv_h), lap_s = T(bd.inv_h2 * bd.inv_pe);
    Cubic<T> mu = cubic<T>(bd.psi);
    if constexpr (VCONST) {
        in_vgpr(epsw);
        in_vgpr(gdt);
        in_vgpr(rdt);
        in_vgpr(bdt);
        in_vgpr(inv_h);
        in_vgpr(lap_s);
        in_vgpr(mu.c0);
        in_vgpr(mu.c1);
        in_vgpr(mu.c2);
        in_vgpr(mu.c3);
    }
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]), ic = A(bd.ic[k]);
    const int z0 = t.z0, nzc = t.nzc;
    // byte offsets within a plane of row y: of C (and v, w), of u, of the
    // row of v's high face (periodic wrap, or the wall face ny), and of
    // halo row hr (y-3, y-2, y-1, y+1, y+2, y+3)
    auto row_off = [&](int y) { return (uint32_t)(y * nx) * sT; };
    auto row_offu = [&](int y) { return (uint32_t)(y * fx) * sT; };
    auto row_vtop = [&](int y) {
        return (uint32_t)((y + 1 == ny && bd.bc[1] == 0 ? 0 : y + 1) * nx) * sT;
    };
    auto halo_off = [&](int y, int hr) {
        return (uint32_t)(map_idx(y + (hr < 3 ? hr - 3 : hr - 2), ny, bd.bc[1]) * nx) * sT;
    };
    // one row per task: these are uniform
    const uint32_t yoff = row_off(t.y0), yoffu = row_offu(t.y0), vtop = row_vtop(t.y0);
    uint32_t hoff[6];
#pragma unroll
    for (int hr = 0; hr < 6; ++hr) hoff[hr] = halo_off(t.y0, hr);
    auto cplane = [&](int z) { return (uint32_t)map_idx(z, nz, bd.bc[2]) * pbytes; };
    // the owned cell of thread tid: row, column, and whether it is a cell
    auto cell = [&](const XRowState<T, A>& s, int tid, int* r, int* x) {
        if constexpr (MR) {
            *r = s.r;
            *x = s.x;
            return s.live;
        } else {
            (void)s;
            *r = 0;
            *x = tid < nx ? tid : nx - 1;
            return tid < nx;
        }
    };

    // The global loads of plane z go straight into the registers that hold
    // them while the plane is computed, each group issued after the last use
    // of the previous plane's values (behind a scheduling fence, so that the
    // two never live at once): u after the x face, v and the y halo rows
    // after the y faces, w after the z face, the old E after the RHS that
    // reads it.  Each has about one plane of work to arrive.  On the task's
    // last plane they load that plane again (just read, so from L2) rather
    // than branch: a load under a branch keeps the old value alive beside
    // the new one.  u, w and the old E are read by this cell alone, and go
    // through L2 non-temporally.
    auto load_u = [&](XRowState<T, A>& s, uint32_t xb, int z) {
        s.ul = Ur.nt(xb + (MR ? s.rou : yoffu), (uint32_t)z * ubytes);
    };
    auto load_vy = [&](XRowState<T, A>& s, uint32_t xb, int z) {
        const uint32_t zo = (uint32_t)z * pbytes;
        if constexpr (MR) {
            s.vl = Vr(xb + s.ro, (uint32_t)z * vbytes);
            s.vh = Vr(xb + s.rvt, (uint32_t)z * vbytes);
#pragma unroll
            for (int hr = 0; hr < 6; ++hr) s.yh[hr] = Cr(xb + s.ho[hr], zo);
        } else {
            s.vl = Vr(xb + yoff, (uint32_t)z * vbytes);
            s.vh = Vr(xb, (uint32_t)z * vbytes + vtop);
#pragma unroll
            for (int hr = 0; hr < 6; ++hr) s.yh[hr] = Cr(xb, zo + hoff[hr]);
        }
    };
    // w on the high face of plane z (periodic wrap, or the wall face nz)
    auto load_wh = [&](XRowState<T, A>& s, uint32_t xb, int z) {
        const uint32_t wo = (uint32_t)((z + 1 == nz && bd.bc[2] == 0) ? 0 : z + 1) * pbytes;
        s.wh = Wr.nt(xb + (MR ? s.ro : yoff), wo);
    };
    // RHS of plane zs of the owned cell into the solve tile (and E out); with
    // several rows per task the high y face of a row below the last is the
    // low face of the row above, formed there
    auto rhs_plane = [&](XRowState<T, A>& s, int r, int x, bool live, int zs) {
        const T* fr = frb + r * L.frp;
        const T fhi = x + 1 < nx ? fr[x + 1] : fr[bcx == 0 ? 0 : nx];
        if constexpr (MR)
            if (r + 1 < rows) s.py = fyb[(r + 1) * nx + x] + s.py;
        const T adv = ((fhi - fr[x]) + s.py) + s.pz;
        const T e = -adv * inv_h + s.plap * lap_s;
        T rhs = gdt * e - bdt * s.pb4;
        if (pa.e_mode != 0) rhs += rdt * s.eold;
        if (live) {
            if (pa.e_mode != 2)
                Er.store((uint32_t)x * sT + (MR ? s.ro : yoff), (uint32_t)(z0 + zs) * pbytes, e);
            tb[(zs * rows + r) * tbp + x + tw] = A(rhs);
        }
    };

    // the thread's cell and halo columns, the column below the first plane,
    // its loads
    ex.phase([&](int tid) {
        XRowState<T, A>& s = st[ex.slot(tid)];
        if constexpr (MR) {
            s.live = tid < rows * nx;
            const int item = s.live ? tid : rows * nx - 1;
            if constexpr (RM == XR_WAVE) {
                const int w0 = ex.wave_base(tid);
                s.r = (w0 < rows * nx ? w0 : rows * nx - 1) / nx;
            } else {
                s.r = item / nx;
            }
            s.x = item - s.r * nx;
            const int y = t.y0 + s.r;
            s.ro = row_off(y);
            s.rou = row_offu(y);
            s.rvt = row_vtop(y);
#pragma unroll
            for (int hr = 0; hr < 6; ++hr) s.ho[hr] = halo_off(y, hr);
        }
        int r, x;
        cell(s, tid, &r, &x);
        const uint32_t xb = (uint32_t)x * sT;
        const uint32_t ro = MR ? s.ro : yoff;
        s.cxp = x;
        s.cxm = x;
        for (int q = 0; q < 6; ++q) {
            const int hc = q < 3 ? q - 3 : nx + q - 3;
            if (map_idx(hc, nx, bcx) == x) {
                s.cxp = hc;
                if (q == 2 || q == 3) s.cxm = hc;
            }
        }
#pragma unroll
        for (int q = 1; q < 7; ++q) s.c[q] = Cr(xb + ro, cplane(z0 - 4 + q));
        s.mq[1] = mu(s.c[3]);   // psi'(C) at z0-2 .. z0 after the first shift
        s.mq[2] = mu(s.c[4]);
        wait_loads();
        s.nc = Cr(xb + ro, cplane(z0 + 3));
        load_u(s, xb, z0);
        load_vy(s, xb, z0);
        s.wl = Wr(xb + ro, (uint32_t)z0 * pbytes);
        load_wh(s, xb, z0);
    });

    for (int zs = 0; zs < nzc; ++zs) {
        const int z = z0 + zs;
        // ---- this plane's loads in, the next plane's loads out, the RHS of
        //      the plane below, the owned row into LDS
        ex.phase([&](int tid) {
            XRowState<T, A>& s = st[ex.slot(tid)];
            int r, x;
            const bool live = cell(s, tid, &r, &x);
            const uint32_t xb = (uint32_t)x * sT;
#pragma unroll
            for (int q = 0; q < 6; ++q) s.c[q] = s.c[q + 1];
            s.c[6] = s.nc;
            s.nc = Cr(xb + (MR ? s.ro : yoff), cplane(zs + 1 < nzc ? z + 4 : z + 3));
            if (zs > 0) rhs_plane(s, r, x, live, zs - 1);
            sched_fence();
            if (pa.e_mode != 0) s.eold = Er.nt(xb + (MR ? s.ro : yoff), (uint32_t)z * pbytes);
            s.mq[0] = s.mq[1];
            s.mq[1] = s.mq[2];
            s.mq[2] = mu(s.c[4]);
            if (live) {
                T* cr = crb + r * L.crp;
                T* mr = mrb + r * L.mrp;
                cr[x] = s.c[3];
                cr[s.cxp] = s.c[3];
                mr[x] = s.mq[1];
                mr[s.cxm] = s.mq[1];
            }
        });
        // ---- face fluxes, Laplacian of psi'(C), fourth differences
        ex.phase([&](int tid) {
            XRowState<T, A>& s = st[ex.slot(tid)];
            int r, x;
            const bool live = cell(s, tid, &r, &x);
            const T* row = crb + r * L.crp + x;   // row[o] = C(x + o)
            const T* mrow = mrb + r * L.mrp + x;  // mrow[o] = psi'(C)(x + o)
            T* fr = frb + r * L.frp;
            {
                const T dX[5] = {row[-2] - row[-3], row[-1] - row[-2], row[0] - row[-1],
                                 row[1] - row[0], row[2] - row[1]};
                const T f = flux_weno_d<T>(s.ul, dX[0], dX[1], dX[2], dX[3], dX[4], row[-1],
                                           row[0], epsw);
                if (live) fr[x] = f;
                s.pb4 = d4_d<T>(dX[1], dX[2], dX[3], dX[4]);
            }
            // the plane whose loads go out
            const int zn = uniform_i(zs + 1 < nzc ? z + 1 : z);
            sched_fence();
            load_u(s, (uint32_t)x * sT, zn);
            if (bcx != 0 && live && x == nx - 1) {
                // the wall face nx (its normal velocity is zero by the interface's rule)
                const T uw = Ur((uint32_t)(x + 1) * sT + (MR ? s.rou : yoffu),
                                (uint32_t)z * ubytes);
                fr[nx] = uw * face_weno<T>(uw, row[-2], row[-1], row[0], row[1], row[2], row[3],
                                           epsw);
            }
            // y: the owned column from the halo registers (with several rows per
            // task, the high face only in the task's last row: the others take
            // the low face of the row above from LDS when they form the RHS)
            {
                const T yc[7] = {s.yh[0], s.yh[1], s.yh[2], s.c[3], s.yh[3], s.yh[4], s.yh[5]};
                T dY[6];
#pragma unroll
                for (int j = 0; j < 6; ++j) dY[j] = yc[j + 1] - yc[j];
                const T fyl =
                    flux_weno_d<T>(s.vl, dY[0], dY[1], dY[2], dY[3], dY[4], yc[2], yc[3], epsw);
                if constexpr (MR) {
                    if (live) fyb[r * nx + x] = fyl;
                    if (r + 1 == rows)
                        s.py = flux_weno_d<T>(s.vh, dY[1], dY[2], dY[3], dY[4], dY[5], yc[3],
                                              yc[4], epsw) -
                               fyl;
                    else
                        s.py = -fyl;   // a + (-b) is a - b, bit for bit
                } else {
                    const T fyh = flux_weno_d<T>(s.vh, dY[1], dY[2], dY[3], dY[4], dY[5], yc[3],
                                                 yc[4], epsw);
                    s.py = fyh - fyl;
                }
                s.pb4 += d4_d<T>(dY[1], dY[2], dY[3], dY[4]);
            }
            // psi'(C) of the y neighbours (summed as in the Laplacian below);
            // what the y block formed is pinned before its inputs are reloaded
            T myy = mu(s.yh[3]) + mu(s.yh[2]);
            pin(myy);
            pin(s.py);
            sched_fence();
            load_vy(s, (uint32_t)x * sT, zn);
            // z: planes z-1 .. z+3; the high face (the low one carries over)
            {
                const T* c = s.c;
                T dZ[5];
#pragma unroll
                for (int j = 0; j < 5; ++j) dZ[j] = c[j + 2] - c[j + 1];
                if (zs == 0)   // the low face of the task's first plane, in the same form
                               // as every face after it
                    s.fzl = flux_weno_d<T>(s.wl, c[1] - c[0], c[2] - c[1], c[3] - c[2],
                                           c[4] - c[3], c[5] - c[4], c[2], c[3], epsw);
                const T fzh =
                    flux_weno_d<T>(s.wh, dZ[0], dZ[1], dZ[2], dZ[3], dZ[4], c[3], c[4], epsw);
                s.pz = fzh - s.fzl;
                s.fzl = fzh;
                s.pb4 += d4_d<T>(dZ[0], dZ[1], dZ[2], dZ[3]);
            }
            pin(s.pz);
            sched_fence();
            s.wl = s.wh;
            load_wh(s, (uint32_t)x * sT, zn);
            s.plap = ((mrow[1] + mrow[-1]) + myy) + (s.mq[2] + s.mq[0]) - T(6) * s.mq[1];
        });
    }
    // ---- RHS of the last plane
    ex.phase([&](int tid) {
        XRowState<T, A>& s = st[ex.slot(tid)];
        int r, x;
        const bool live = cell(s, tid, &r, &x);
        rhs_plane(s, r, x, live, nzc - 1);
    });
    const int nlines = rows * nzc;
    // ---- halos of the solve tile (periodic or reflected continuation); each
    //      thread's (line, chunk) of the x solve
    ex.phase([&](int tid) {
        x_tile_halos<A>(tid, nth, tb, tbp, nlines, nx, tw, bcx);
        st[ex.slot(tid)].ls.ch = line_chunk(tid, nlines, nx, tw, X_CHAINS);
    });
    // ---- x solve of the task's lines
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_f1<A, 1>(ls.ch, tb, tbp, tw, a1, a2, ic, ls);
    });
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_f2<A, 1>(ls.ch, tb, tbp, tw, a1, a2, ic, ls);
    });
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_b1<A, 1>(ls.ch, tb, tbp, tw, a1, a2, ls);
    });
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_b2<A, 1>(ls.ch, tb, tbp, tw, a1, a2, ls);
    });
    // ---- q out, plane by plane
    ex.phase([&](int tid) {
        const XRowState<T, A>& s = st[ex.slot(tid)];
        int r, x;
        if (!cell(s, tid, &r, &x)) return;
        const uint32_t o = (uint32_t)x * sT + (MR ? s.ro : yoff);
        for (int zs = 0; zs < nzc; ++zs)
            Qr.store(o, (uint32_t)(z0 + zs) * pbytes, T(tb[(zs * rows + r) * tbp + x + tw]));
    });
}

// ---------------------------------------------------------------------------
// Pass X over one row and one x segment per task, for periodic lines too long
// for one work-group (the arithmetic of pass_x_row_program, cell by cell).
//
// The segment [x0, x0 + S) is solved from the RHS of the segment extended by
// tw_max cells on each side (the recurrences' warm-ups), so a task computes
// the explicit terms of NE = S + 2 tw_max cells, and thread NE + 1 only the x
// face above the last one.  Extended position q (0 <= q <= NE) is the cell
// x0 - tw_max + q, wrapped.  The six C values beyond the extended range that
// its x stencils reach are loaded by threads 0..5.  E of the previous
// substage is read from Ein and the new one written to Eout, a different
// array: a task reads E at the cells of its neighbours' segments.  Only the
// segment's own cells are written (E and q).  Fields are addressed per plane
// (a buffer resource for each plane), so they may exceed 4 GiB.  Threads:
// x_seg_threads (positions 0 .. NE).
//
// LDS (launch-wide: S the longest segment):
//   cr: NE + 7 T    C at extended positions -3 .. NE + 3
//   mr: NE + 3 T    psi'(C) at -1 .. NE + 1
//   fr: NE + 1 T    flux through the low x face of position q, 0 .. NE
//   tb: zc x pitch A    RHS -> solve tile: line zs, positions -tw .. S+tw-1
//                       contiguous (pitch S + 2 tw_max, made odd)
// ---------------------------------------------------------------------------
struct XSegLayout {
    size_t cr, mr, fr, tb, total;   // byte offsets and total size
    int tbp;                        // pitch of the solve tile (elements)
};

CH_HD XSegLayout x_seg_layout(int S, int zc, int tw_max, int sT, int sA)
{
    const int ne = S + 2 * tw_max;
    XSegLayout L;
    L.tbp = x_tile_pitch(S + 2 * tw_max);
    L.cr = 0;
    L.mr = al16(L.cr + (size_t)(ne + 7) * sT);
    L.fr = al16(L.mr + (size_t)(ne + 3) * sT);
    L.tb = al16(L.fr + (size_t)(ne + 1) * sT);
    L.total = al16(L.tb + (size_t)zc * L.tbp * sA);
    return L;
}

// threads of a segment of S cells
CH_HD int x_seg_threads(int S, int tw_max) { return S + 2 * tw_max + 1; }

template <typename T, typename A>
struct XSegState {
    T c[7];                   // C at z-3 .. z+3 of the cell
    T mq[3];                  // psi'(C) at z-1, z, z+1
    T yh[6];                  // C of this plane at rows y-3, y-2, y-1, y+1, y+2, y+3
    T ul, vl, vh, wl, wh;     // face velocities (as in XRowState)
    T fzl;                    // flux through the low z face
    T eold;                   // E of the previous substage at the plane whose RHS is next
    T py, pz, plap, pb4;      // y and z flux differences, Laplacian of psi', sum of D4
    T xh;                     // threads 0..5: C beyond the extended range, this plane
    T nc;                     // C at z+4 of the cell (the next plane's c[6])
    uint32_t xb;              // byte offset of the cell in its row
    LineState<A> ls;
};

template <typename T, typename A, class X>
CH_HD void pass_x_seg_program(X& ex, XSegState<T, A>* st, const BoxDesc& bd, const PassArgs& pa,
                              int task, const T* __restrict__ C, const T* __restrict__ U,
                              const T* __restrict__ V, const T* __restrict__ W,
                              const T* __restrict__ Ein, T* __restrict__ Eout,
                              T* __restrict__ Q, unsigned char* smem)
{
    const XZTask t = xz_task(bd, task);   // one row, one segment
    const int nx = bd.n[0], ny = bd.n[1], nz = bd.n[2];
    const int fx = bd.nf[0], fy = bd.nf[1];
    const int k = pa.k, tw = bd.tw[k], twm = pa.tw_max;
    const int S = t.xlen, x0 = t.x0;
    const int NE = S + 2 * twm;
    const XSegLayout L = x_seg_layout(bd.xs, bd.zc, twm, (int)sizeof(T), (int)sizeof(A));
    constexpr uint32_t sT = sizeof(T);
    T* cr = reinterpret_cast<T*>(smem + L.cr) + 3;   // cr[q], -3 <= q <= NE + 3
    T* mr = reinterpret_cast<T*>(smem + L.mr) + 1;   // mr[q], -1 <= q <= NE + 1
    T* fr = reinterpret_cast<T*>(smem + L.fr);       // fr[q], 0 <= q <= NE
    A* tb = reinterpret_cast<A*>(smem + L.tb);
    const int tbp = L.tbp;
    const int64_t plane = (int64_t)nx * ny;
    const uint32_t pbytes = (uint32_t)(plane * sT);
    const uint32_t ubytes = (uint32_t)((int64_t)ny * fx * sT);
    const uint32_t vbytes = (uint32_t)((int64_t)fy * nx * sT);
    const T* Cb = C + bd.c_off;
    const T* Ub = U + bd.u_off;
    const T* Vb = V + bd.v_off;
    const T* Wb = W + bd.w_off;
    const T* Eib = Ein + bd.c_off;
    T* Eob = Eout + bd.c_off;
    T* Qb = Q + bd.c_off;
    auto Cp = [&](int z) { return PlaneRef<T>(Cb + (int64_t)z * plane, pbytes); };
    const T epsw = T(bd.eps * (12.0 / 13.0));
    const T gdt = T(bd.gdt[k]), rdt = T(bd.rdt[k]), bdt = T(bd.bdt[k]);
    const T inv_h = T(bd.inv_h), lap_s = T(bd.inv_h2 * bd.inv_pe);
    const Cubic<T> mu = cubic<T>(bd.psi);
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]), ic = A(bd.ic[k]);
    const int y = t.y0;
    const int z0 = t.z0, nzc = t.nzc;
    const uint32_t yoff = (uint32_t)(y * nx) * sT;
    const uint32_t yoffu = (uint32_t)(y * fx) * sT;
    const uint32_t vtop = (uint32_t)((y + 1 == ny && bd.bc[1] == 0 ? 0 : y + 1) * nx) * sT;
    uint32_t hoff[6];
#pragma unroll
    for (int hr = 0; hr < 6; ++hr)
        hoff[hr] = (uint32_t)(map_idx(y + (hr < 3 ? hr - 3 : hr - 2), ny, bd.bc[1]) * nx) * sT;
    // extended position of a thread (threads past NE + 1 repeat the last one)
    auto pos = [&](int tid) { return tid <= NE ? tid : NE; };
    auto cellb = [&](int q) { return (uint32_t)map_idx(x0 - twm + q, nx, 0) * sT; };
    // threads 0..5: the C beyond the extended range, at cr index hq
    auto hq = [&](int tid) { return tid < 3 ? tid - 3 : NE + 1 + (tid - 3); };

    // the loads of plane z, straight into the working registers (as in the
    // row program: each group after the last use of the previous plane's;
    // plain loads: on boxes this large the non-temporal hint measured
    // slower, 32.2 against 31.9 ms per 1536^3 x pass)
    auto load_u = [&](XSegState<T, A>& s, int z) {
        s.ul = PlaneRef<T>(Ub + (int64_t)z * ny * fx, ubytes)(s.xb, yoffu);
    };
    auto load_vy = [&](XSegState<T, A>& s, int z) {
        const PlaneRef<T> Vz(Vb + (int64_t)z * fy * nx, vbytes);
        s.vl = Vz(s.xb + yoff);
        s.vh = Vz(s.xb, vtop);
        const PlaneRef<T> Cz = Cp(z);
#pragma unroll
        for (int hr = 0; hr < 6; ++hr) s.yh[hr] = Cz(s.xb, hoff[hr]);
    };
    auto load_wh = [&](XSegState<T, A>& s, int z) {   // w on the high face of plane z
        s.wh = PlaneRef<T>(Wb + (int64_t)((z + 1 == nz && bd.bc[2] == 0) ? 0 : z + 1) * plane,
                           pbytes)(s.xb, yoff);
    };
    auto load_xh = [&](XSegState<T, A>& s, int tid, int z) {
        if (tid < 6) s.xh = Cp(z)(cellb(hq(tid)) + yoff);
    };
    // RHS of plane zs at extended position q into the solve tile (and E out
    // at the segment's own cells)
    auto rhs_plane = [&](XSegState<T, A>& s, int tid, int q, int zs) {
        const T adv = ((fr[q + 1] - fr[q]) + s.py) + s.pz;
        const T e = -adv * inv_h + s.plap * lap_s;
        T rhs = gdt * e - bdt * s.pb4;
        if (pa.e_mode != 0) rhs += rdt * s.eold;
        const int rel = q - twm;   // position in the segment
        if (tid == q && rel >= -tw && rel < S + tw) {
            if (pa.e_mode != 2 && rel >= 0 && rel < S)
                PlaneRef<T>(Eob + (int64_t)(z0 + zs) * plane, pbytes).store(s.xb + yoff, e);
            tb[zs * tbp + rel + tw] = A(rhs);
        }
    };

    ex.phase([&](int tid) {
        XSegState<T, A>& s = st[ex.slot(tid)];
        s.xb = cellb(pos(tid));
#pragma unroll
        for (int q = 1; q < 7; ++q) s.c[q] = Cp(map_idx(z0 - 4 + q, nz, bd.bc[2]))(s.xb + yoff);
        s.mq[1] = mu(s.c[3]);
        s.mq[2] = mu(s.c[4]);
        wait_loads();
        s.nc = Cp(map_idx(z0 + 3, nz, bd.bc[2]))(s.xb + yoff);
        load_u(s, z0);
        load_vy(s, z0);
        s.wl = PlaneRef<T>(Wb + (int64_t)z0 * plane, pbytes)(s.xb + yoff);
        load_wh(s, z0);
        load_xh(s, tid, z0);
    });

    for (int zs = 0; zs < nzc; ++zs) {
        const int z = z0 + zs;
        ex.phase([&](int tid) {
            XSegState<T, A>& s = st[ex.slot(tid)];
            const int q = pos(tid);
#pragma unroll
            for (int j = 0; j < 6; ++j) s.c[j] = s.c[j + 1];
            s.c[6] = s.nc;
            s.nc = Cp(map_idx(zs + 1 < nzc ? z + 4 : z + 3, nz, bd.bc[2]))(s.xb + yoff);
            if (zs > 0 && q < NE) rhs_plane(s, tid, q, zs - 1);
            sched_fence();
            if (pa.e_mode != 0)
                s.eold = PlaneRef<T>(Eib + (int64_t)z * plane, pbytes)(s.xb, yoff);
            s.mq[0] = s.mq[1];
            s.mq[1] = s.mq[2];
            s.mq[2] = mu(s.c[4]);
            if (tid == q) {
                cr[q] = s.c[3];
                mr[q] = s.mq[1];
            }
            if (tid < 6) {
                cr[hq(tid)] = s.xh;
                if (tid == 2) mr[-1] = mu(s.xh);
                if (tid == 3) mr[NE + 1] = mu(s.xh);
            }
            sched_fence();
            load_xh(s, tid, uniform_i(zs + 1 < nzc ? z + 1 : z));
        });
        ex.phase([&](int tid) {
            XSegState<T, A>& s = st[ex.slot(tid)];
            const int q = pos(tid);
            const T* row = cr + q;
            {
                const T dX[5] = {row[-2] - row[-3], row[-1] - row[-2], row[0] - row[-1],
                                 row[1] - row[0], row[2] - row[1]};
                const T f = flux_weno_d<T>(s.ul, dX[0], dX[1], dX[2], dX[3], dX[4], row[-1],
                                           row[0], epsw);
                if (tid == q) fr[q] = f;
                s.pb4 = d4_d<T>(dX[1], dX[2], dX[3], dX[4]);
            }
            // the plane whose loads go out (this one again on the task's last)
            const int zn = uniform_i(zs + 1 < nzc ? z + 1 : z);
            sched_fence();
            load_u(s, zn);
            {
                const T yc[7] = {s.yh[0], s.yh[1], s.yh[2], s.c[3], s.yh[3], s.yh[4], s.yh[5]};
                T dY[6];
#pragma unroll
                for (int j = 0; j < 6; ++j) dY[j] = yc[j + 1] - yc[j];
                const T fyl =
                    flux_weno_d<T>(s.vl, dY[0], dY[1], dY[2], dY[3], dY[4], yc[2], yc[3], epsw);
                const T fyh =
                    flux_weno_d<T>(s.vh, dY[1], dY[2], dY[3], dY[4], dY[5], yc[3], yc[4], epsw);
                s.py = fyh - fyl;
                s.pb4 += d4_d<T>(dY[1], dY[2], dY[3], dY[4]);
            }
            T myy = mu(s.yh[3]) + mu(s.yh[2]);
            pin(myy);
            pin(s.py);
            sched_fence();
            load_vy(s, zn);
            {
                const T* c = s.c;
                T dZ[5];
#pragma unroll
                for (int j = 0; j < 5; ++j) dZ[j] = c[j + 2] - c[j + 1];
                if (zs == 0)
                    s.fzl = flux_weno_d<T>(s.wl, c[1] - c[0], c[2] - c[1], c[3] - c[2],
                                           c[4] - c[3], c[5] - c[4], c[2], c[3], epsw);
                const T fzh =
                    flux_weno_d<T>(s.wh, dZ[0], dZ[1], dZ[2], dZ[3], dZ[4], c[3], c[4], epsw);
                s.pz = fzh - s.fzl;
                s.fzl = fzh;
                s.pb4 += d4_d<T>(dZ[0], dZ[1], dZ[2], dZ[3]);
            }
            pin(s.pz);
            sched_fence();
            s.wl = s.wh;
            load_wh(s, zn);
            s.plap = ((mr[q + 1] + mr[q - 1]) + myy) + (s.mq[2] + s.mq[0]) - T(6) * s.mq[1];
        });
    }
    ex.phase([&](int tid) {
        const int q = pos(tid);
        if (q < NE) rhs_plane(st[ex.slot(tid)], tid, q, nzc - 1);
    });
    // ---- solve the segment's lines from the computed warm-ups
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        ls.ch = line_chunk(tid, nzc, S, tw, X_CHAINS);
        line_f1<A, 1>(ls.ch, tb, tbp, tw, a1, a2, ic, ls);
    });
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_f2<A, 1>(ls.ch, tb, tbp, tw, a1, a2, ic, ls);
    });
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_b1<A, 1>(ls.ch, tb, tbp, tw, a1, a2, ls);
    });
    ex.phase([&](int tid) {
        LineState<A>& ls = st[ex.slot(tid)].ls;
        line_b2<A, 1>(ls.ch, tb, tbp, tw, a1, a2, ls);
    });
    // ---- q out at the segment's cells
    ex.phase([&](int tid) {
        const int rel = tid - twm;
        if (rel < 0 || rel >= S) return;
        const uint32_t o = st[ex.slot(tid)].xb + yoff;   // tid <= NE: its own cell
        for (int zs = 0; zs < nzc; ++zs)
            PlaneRef<T>(Qb + (int64_t)(z0 + zs) * plane, pbytes)
                .store(o, T(tb[zs * tbp + rel + tw]));
    });
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

// Lanes of a y/z task: x columns of 128 bytes of accumulators (the planner's
// `lanes`).
template <typename A>
constexpr int line_lanes()
{
    return 128 / (int)sizeof(A);
}

// The line passes' 16-byte fast path (below) can be compiled out, so that the
// host harness can hold it to the element-wise path.
#ifndef CH_LINE_VEC
#define CH_LINE_VEC 1
#endif

// Rows of a y/z tile are filled 8 at a time (see load16_to_lds), so the tile
// is allocated in whole blocks of 8 rows.
CH_HD int line_tile_rows(int npos) { return (npos + 7) & ~7; }

// 16 bytes of global memory straight into LDS, without registers: on the GPU
// the wave's 64 lanes write 64 consecutive 16-byte pieces from `wave_base`
// (lane L at wave_base + 16 L, which must be the same for the whole wave),
// so one instruction fills eight 128-byte tile rows.  The host runs the same
// per lane.  Waited for by wait_loads().
template <typename T>
CH_HD void load16_to_lds(const T* g, unsigned char* wave_base, int lane)
{
#if defined(__HIP_DEVICE_COMPILE__)
    (void)lane;
    // non-temporal: a line pass reads each element once, and leaves the
    // caches to its output, which the next pass reads
    __builtin_amdgcn_global_load_lds(
        g, (__attribute__((address_space(3))) void*)(wave_base), 16, 0, 2);
#else
    memcpy(wave_base + 16 * lane, g, 16);
#endif
}

// 16 bytes of T as one vector (the aligned loads and stores of the line
// passes' fast path)
template <typename T>
struct Vec16 {
    typedef T type __attribute__((vector_size(16)));
};

template <typename T, typename A, class X>
CH_HD void pass_line_program(X& ex, LineState<A>* st, const BoxDesc& bd, const PassArgs& pa,
                             int pass, int task, const T* __restrict__ Qin,
                             T* __restrict__ Qout, unsigned char* smem)
{
    constexpr int Lw = line_lanes<A>();
    const LTask t = l_task(bd, pa, pass, task);
    const int nth = ex.nth, k = pa.k, tw = bd.tw[k];
    const int nlive = bd.n[0] - t.x0 < Lw ? bd.n[0] - t.x0 : Lw;
    const A a1 = A(bd.a1[k]), a2 = A(bd.a2[k]), ic = A(bd.ic[k]);
    A* tile = reinterpret_cast<A*>(smem);
    const int npos = t.len + 2 * tw;
    // a thread walks rows q0, q0 + qstep, ... of the tile, LB rows per batch
    // with their loads in flight together; `dstep` is the distance in the
    // field between two rows of a batch
    const int qstep = nth / Lw;
    const int span = (LB - 1) * qstep;
    const int64_t dstep = (int64_t)qstep * t.stride;
    // Fast path: the field holds the solve's precision, the task's 32 (FP32)
    // or 16 (FP64) columns are all in the box, and rows start on 16 bytes:
    // rows go to LDS by 16-byte direct loads and come back as 16-byte vectors.
    constexpr int EPV = 16 / (int)sizeof(T);   // elements per 16 bytes
    const bool vec = CH_LINE_VEC && sizeof(T) == sizeof(A) && nlive == Lw && nth % 64 == 0 &&
                     ((t.base * (int64_t)sizeof(T)) & 15) == 0 &&
                     ((t.stride * (int64_t)sizeof(T)) & 15) == 0;
    // stage the segment with its halos; tile row q holds line position
    // s0 + q - tw.
    if (vec) {
        // wave w fills the blocks of 8 rows w, w + waves, ...; lane L takes
        // row L / 8 of the block and its 16-byte piece L % 8.  The padding
        // rows of the last block repeat the last position.
        ex.phase([&](int tid) {
            const int wave = tid / 64, lane = tid % 64, nwave = nth / 64;
            const T* colb = Qin + t.base + (lane % 8) * EPV;
            const int nblk = line_tile_rows(npos) / 8;
            for (int b = wave; b < nblk; b += nwave) {
                int q = b * 8 + lane / 8;
                if (q >= npos) q = npos - 1;
                const int pos = map_idx(t.s0 + q - tw, t.n, t.bc);
                load16_to_lds<T>(colb + (int64_t)pos * t.stride,
                                 reinterpret_cast<unsigned char*>(tile + b * 8 * Lw), lane);
            }
            wait_loads();
        });
    } else
    ex.phase([&](int tid) {
        const int l = tid % Lw;
        const bool on = l < nlive;
        const T* col = Qin + t.base + l;
        for (int q0 = tid / Lw; q0 < npos; q0 += qstep * LB) {
            const int i0 = t.s0 + q0 - tw;
            A* trow = tile + q0 * Lw + l;
            if (on && i0 >= 0 && i0 + span < t.n && q0 + span < npos) {
                const T* p = col + (int64_t)i0 * t.stride;
                A v[LB];
#pragma unroll
                for (int j = 0; j < LB; ++j) v[j] = A(p[j * dstep]);
#pragma unroll
                for (int j = 0; j < LB; ++j) trow[j * qstep * Lw] = v[j];
            } else {
                A v[LB];
#pragma unroll
                for (int j = 0; j < LB; ++j) {
                    const int q = q0 + j * qstep;
                    v[j] = A(0);
                    if (q < npos && on)
                        v[j] = A(col[(int64_t)map_idx(t.s0 + q - tw, t.n, t.bc) * t.stride]);
                }
#pragma unroll
                for (int j = 0; j < LB; ++j)
                    if (q0 + j * qstep < npos) trow[j * qstep * Lw] = v[j];
            }
        }
    });
    const int K = line_chunk_len(t.len, tw, YZ_CHAINS);
    ex.phase([&](int tid) {
        const Chunk ch = line_chunk_k(tid, Lw, t.len, tw, K);
        line_f1<A>(ch, tile, Lw, tw, a1, a2, ic, st[ex.slot(tid)]);
    });
    ex.phase([&](int tid) {
        const Chunk ch = line_chunk_k(tid, Lw, t.len, tw, K);
        line_f2<A>(ch, tile, Lw, tw, a1, a2, ic, st[ex.slot(tid)]);
    });
    ex.phase([&](int tid) {
        const Chunk ch = line_chunk_k(tid, Lw, t.len, tw, K);
        line_b1<A>(ch, tile, Lw, tw, a1, a2, st[ex.slot(tid)]);
    });
    ex.phase([&](int tid) {
        const Chunk ch = line_chunk_k(tid, Lw, t.len, tw, K);
        line_b2<A>(ch, tile, Lw, tw, a1, a2, st[ex.slot(tid)]);
    });
    // write the segment back (pass Z: C += dC); only the last batch of a
    // thread can reach past the segment
    if (vec) {
        // lane L of a wave takes row L / 8 of a block of 8 and its 16-byte
        // piece L % 8; four blocks per round, their loads of C in flight
        // together
        typedef typename Vec16<T>::type V;
        ex.phase([&](int tid) {
            const int wave = tid / 64, lane = tid % 64, nwave = nth / 64;
            const int r = lane / 8, e0 = (lane % 8) * EPV;
            const int nblk = line_tile_rows(t.len) / 8;
            T* colb = Qout + t.base + e0;
            for (int b0 = wave; b0 < nblk; b0 += 4 * nwave) {
                V c[4];
                if (pass == PASS_Z) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int q = (b0 + j * nwave) * 8 + r;
                        if (q < t.len)
                            c[j] = *reinterpret_cast<const V*>(colb + (int64_t)(t.s0 + q) * t.stride);
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int q = (b0 + j * nwave) * 8 + r;
                    if (q >= t.len) continue;
                    V d = *reinterpret_cast<const V*>(tile + (q + tw) * Lw + e0);
                    if (pass == PASS_Z) d = c[j] + d;
                    *reinterpret_cast<V*>(colb + (int64_t)(t.s0 + q) * t.stride) = d;
                }
            }
        });
        return;
    }
    ex.phase([&](int tid) {
        const int l = tid % Lw;
        if (l >= nlive) return;
        for (int q0 = tid / Lw; q0 < t.len; q0 += qstep * LB) {
            T* p = Qout + t.base + l + (int64_t)(t.s0 + q0) * t.stride;
            const A* trow = tile + (q0 + tw) * Lw + l;
            const bool full = q0 + span < t.len;
            if (pass == PASS_Z) {
                // C += dC: the LB reads of C go out together
                A c[LB];
#pragma unroll
                for (int j = 0; j < LB; ++j)
                    c[j] = full || q0 + j * qstep < t.len ? A(p[j * dstep]) : A(0);
#pragma unroll
                for (int j = 0; j < LB; ++j)
                    if (full || q0 + j * qstep < t.len)
                        p[j * dstep] = T(c[j] + trow[j * qstep * Lw]);
            } else {
#pragma unroll
                for (int j = 0; j < LB; ++j)
                    if (full || q0 + j * qstep < t.len) p[j * dstep] = T(trow[j * qstep * Lw]);
            }
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
