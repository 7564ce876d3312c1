// ch_lib.cpp -- host side of libch: the C ABI of include/ch.h.
//
// A state (single box) and a batch (many boxes) share one engine: the
// kernels always work on a table of boxes, and a state is a batch of one.
// Per RK3 substage the engine enqueues the three directional passes
// (x: explicit terms + RHS + x solve, y solve, z solve + update); with a
// non-null stream a whole step is captured once as a HIP graph and replayed.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ch.h"
#include "ch_device.h"
#include "ch_kernels.h"
#include "ch_plan.h"

namespace {

thread_local std::string g_err;

ch_status fail(ch_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(CH_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

// live handles, each with the kind of object it names: a handle of one kind
// passed where another is expected is rejected like a destroyed one
enum HandleKind { H_STATE = 1, H_BATCH = 2, H_INTERP = 3, H_POISSON = 4 };
constexpr HandleKind kind_of(const ch_state*) { return H_STATE; }
constexpr HandleKind kind_of(const ch_batch*) { return H_BATCH; }
constexpr HandleKind kind_of(const ch_interp*) { return H_INTERP; }
constexpr HandleKind kind_of(const ch_poisson*) { return H_POISSON; }

std::mutex g_mu;
std::unordered_map<const void*, HandleKind> g_live;

template <typename H>
void reg(const H* p)
{
    std::lock_guard<std::mutex> l(g_mu);
    g_live[p] = kind_of(p);
}
template <typename H>
bool live(const H* p)
{
    std::lock_guard<std::mutex> l(g_mu);
    if (!p) return false;
    const auto it = g_live.find(p);
    return it != g_live.end() && it->second == kind_of(p);
}
template <typename H>
void unreg(const H* p)
{
    std::lock_guard<std::mutex> l(g_mu);
    g_live.erase(p);
}

struct Engine {
    chp::Plan P;
    chd::BoxDesc* d_boxes = nullptr;
    chd::BoxDesc* d_xbox[3] = {nullptr, nullptr, nullptr};   // box tables of the x launches
    void* C = nullptr;
    void* E = nullptr;
    void* E2 = nullptr;   // the segmented x program's second E (allocated when used)
    void* qa = nullptr;
    void* qb = nullptr;
    double* d_partial = nullptr;
    double* d_h3 = nullptr;
    double* d_mass = nullptr;
    int* d_flags = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    // graph of one step
    hipGraphExec_t gexec = nullptr;
    // pointers and transfer handle (with its mode generation) of the captured step
    const void* gkey[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double prof_ms[4] = {0, 0, 0, 0};
    int64_t prof_n[4] = {0, 0, 0, 0};
    // fine velocity for the multiple-resolution step
    void* fu = nullptr;
    void* fv = nullptr;
    void* fw = nullptr;
    // drop labelling: labels and counts (one int per cell of the largest box
    // labelled so far), the root list (cap entries each) and its length
    int* d_lab = nullptr;
    int* d_cnt = nullptr;
    int64_t lab_n = 0;
    int* d_list = nullptr;
    int64_t list_cap = 0;
};

void free_engine(Engine& e)
{
    if (e.gexec) (void)hipGraphExecDestroy(e.gexec);
    for (auto& p : e.ev_pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (auto ev : e.ev_pool) (void)hipEventDestroy(ev);
    void* bufs[] = {e.C, e.E, e.E2, e.qa, e.qb, e.d_partial, e.d_h3, e.d_mass, e.d_flags,
                    e.d_boxes, e.d_xbox[0], e.d_xbox[1], e.d_xbox[2], e.fu, e.fv, e.fw,
                    e.d_lab, e.d_cnt,
                    e.d_list};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
}

ch_status init_engine(Engine& e, int nbox, const ch_grid* g, const double* Cn, const double* Pe,
                      const ch_psi* psi, const ch_bc* bc, const ch_opts* opt)
{
    chp::Plan& P = e.P;
    ch_status st = chp::plan_init(P, nbox, g, Cn, Pe, psi, bc, opt);
    if (st != CH_OK) return fail(st, "%s", P.err.c_str());
    HIP_TRY(hipGetDevice(&e.device));
    const size_t bytes = (size_t)P.tot[0] * chp::esize(P.prec);
    void** fields[4] = {&e.C, &e.E, &e.qa, &e.qb};
    for (void** f : fields) {
        if (hipMalloc(f, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *f = nullptr;
            return fail(CH_ENOMEM, "cannot allocate %zu bytes", bytes);
        }
        HIP_TRY(hipMemset(*f, 0, bytes));
    }
    HIP_TRY(hipMalloc(&e.d_partial, sizeof(double) * std::max(1, P.nmblk)));
    HIP_TRY(hipMalloc(&e.d_h3, sizeof(double) * nbox));
    HIP_TRY(hipMalloc(&e.d_mass, sizeof(double) * nbox));
    HIP_TRY(hipMalloc(&e.d_flags, sizeof(int) * 2 * chk::CHECK_WGS));
    HIP_TRY(hipMalloc(&e.d_boxes, sizeof(chd::BoxDesc) * nbox));
    if (nbox > 1)
        for (int g = 0; g < 3; ++g) HIP_TRY(hipMalloc(&e.d_xbox[g], sizeof(chd::BoxDesc) * nbox));
    std::vector<double> h3(nbox);
    for (int b = 0; b < nbox; ++b) h3[b] = P.g[b].h * P.g[b].h * P.g[b].h;
    HIP_TRY(hipMemcpy(e.d_h3, h3.data(), sizeof(double) * nbox, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(e.d_boxes, P.boxes.data(), sizeof(chd::BoxDesc) * nbox,
                      hipMemcpyHostToDevice));
    return CH_OK;
}

// New coefficients and launch configuration for dt; the table is read by
// work already in the stream, so wait before replacing it.
ch_status set_dt(Engine& e, double dt, bool e25 = false)
{
    e.P.e25 = e25;
    ch_status st = chp::plan_dt(e.P, dt);
    if (st != CH_OK) {
        e.P.dt = NAN;
        return fail(st, "%s", e.P.err.c_str());
    }
    HIP_TRY(hipStreamSynchronize(e.stream));
    if (e.P.xseg && !e.E2) {
        const size_t bytes = (size_t)e.P.tot[0] * chp::esize(e.P.prec);
        if (hipMalloc(&e.E2, bytes) != hipSuccess) {
            (void)hipGetLastError();
            e.E2 = nullptr;
            e.P.dt = NAN;
            return fail(CH_ENOMEM, "cannot allocate %zu bytes", bytes);
        }
    }
    HIP_TRY(hipMemcpy(e.d_boxes, e.P.boxes.data(), sizeof(chd::BoxDesc) * e.P.nbox,
                      hipMemcpyHostToDevice));
    if (e.P.nxl > 1)
        for (int g = 0; g < e.P.nxl; ++g)
            HIP_TRY(hipMemcpy(e.d_xbox[g], e.P.xbox[g].data(),
                              sizeof(chd::BoxDesc) * e.P.xbox[g].size(), hipMemcpyHostToDevice));
    if (e.gexec) {
        (void)hipGraphExecDestroy(e.gexec);
        e.gexec = nullptr;
    }
    return CH_OK;
}

hipEvent_t take_event(Engine& e)
{
    if (!e.ev_pool.empty()) {
        hipEvent_t ev = e.ev_pool.back();
        e.ev_pool.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    return ev;
}

template <typename T, typename A>
hipError_t enqueue_substage(Engine& e, int k, const void* u, const void* v, const void* w)
{
    
    for (int p = 0; p < 3; ++p) {
        hipEvent_t a = nullptr, b = nullptr;
        if (e.prof) {
            a = take_event(e);
            b = take_event(e);
            if (a) (void)hipEventRecord(a, e.stream);
        }
        hipError_t err;
        const chd::PassArgs pa = chp::pass_args(e.P, k, p);
        if (p == 0 && e.P.xseg)
            // substage 1 writes E, 2 reads it and writes E2, 3 reads E2
            err = chk::launch_pass_x_seg<T, A>(e.P.ntask[0], e.P.x_threads, e.P.lds[0],
                                               e.stream, e.d_boxes, e.P.nbox, pa, e.C, u, v, w,
                                               k == 2 ? e.E2 : e.E, k == 1 ? e.E2 : e.E, e.qa);
        else if (p == 0 && e.P.nxl > 1) {
            // one launch per row mode, each with its own work-group size
            err = hipSuccess;
            for (int g = 0; g < e.P.nxl && err == hipSuccess; ++g)
                err = chk::launch_pass_x<T, A>(e.P.mi, e.P.x_ntask[g], e.P.x_nth[g],
                                               e.P.x_lds[g], e.stream, e.d_xbox[g],
                                               (int)e.P.xbox[g].size(), pa, e.C, u, v, w, e.E,
                                               e.qa, false, true, e.P.x_rm[g]);
        } else if (p == 0)
            err = chk::launch_pass_x<T, A>(e.P.mi, e.P.ntask[0], e.P.x_threads, e.P.lds[0],
                                           e.stream, e.d_boxes, e.P.nbox, pa,
                                           e.C, u, v, w, e.E, e.qa, false, e.P.xrow,
                                           e.P.xrm);
        else if (p == 1)
            err = chk::launch_pass_line<T, A>(chd::PASS_Y, e.P.ntask[1], e.P.yz_threads,
                                              e.P.lds[1], e.stream, e.d_boxes, e.P.nbox, pa, e.qa,
                                              e.qb);
        else
            err = chk::launch_pass_line<T, A>(chd::PASS_Z, e.P.ntask[2], e.P.yz_threads,
                                              e.P.lds[2], e.stream, e.d_boxes, e.P.nbox, pa, e.qb,
                                              e.C);
        if (e.prof && a && b) {
            (void)hipEventRecord(b, e.stream);
            e.ev_pending.push_back({p, {a, b}});
        }
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// One substage of the explicit 25-point scheme: the x-pass program in its
// explicit mode writes C + RHS to qa, which then becomes C.
template <typename T>
hipError_t enqueue_substage_e25(Engine& e, int k, const void* u, const void* v, const void* w)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (e.prof) {
        a = take_event(e);
        b = take_event(e);
        if (a) (void)hipEventRecord(a, e.stream);
    }
    const chd::PassArgs pa = chp::pass_args(e.P, k, 0);
    hipError_t err = chk::launch_pass_x<T, T>(e.P.mi, e.P.ntask[0], e.P.x_threads, e.P.lds[0],
                                              e.stream, e.d_boxes, e.P.nbox, pa, e.C, u, v, w,
                                              e.E, e.qa, true, false, chd::XR_ONE);
    if (e.prof && a && b) {
        (void)hipEventRecord(b, e.stream);
        e.ev_pending.push_back({0, {a, b}});
    }
    if (err == hipSuccess) std::swap(e.C, e.qa);
    return err;
}

ch_status run_steps_e25(Engine& e, const void* u, const void* v, const void* w, double dt,
                        int nsteps)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CH_EINVAL, "dt must be > 0 and finite");
    if (nsteps < 0) return fail(CH_EINVAL, "nsteps must be >= 0");
    if (!u || !v || !w) return fail(CH_EINVAL, "null velocity");
    HIP_TRY(hipSetDevice(e.device));
    if (dt != e.P.dt || !e.P.e25) {
        ch_status st = set_dt(e, dt, true);
        if (st != CH_OK) return st;
    }
    // the buffers of C and qa trade places every substage: a captured step
    // of the implicit scheme would address the wrong one
    if (e.gexec && nsteps > 0) {
        (void)hipGraphExecDestroy(e.gexec);
        e.gexec = nullptr;
    }
    for (int s = 0; s < nsteps; ++s)
        for (int k = 0; k < 3; ++k) {
            hipError_t err = e.P.prec == CH_FP64 ? enqueue_substage_e25<double>(e, k, u, v, w)
                                                 : enqueue_substage_e25<float>(e, k, u, v, w);
            if (err != hipSuccess)
                return fail(CH_EHIP, "kernel launch failed: %s", hipGetErrorString(err));
        }
    return CH_OK;
}

struct InterpData;
hipError_t enqueue_interp(Engine& e, InterpData* ip, const void* uc, const void* vc,
                          const void* wc, void* u, void* v, void* w);

hipError_t enqueue_step(Engine& e, const void* u, const void* v, const void* w)
{
    for (int k = 0; k < 3; ++k) {
        hipError_t err;
        if (e.P.prec == CH_FP64) err = enqueue_substage<double, double>(e, k, u, v, w);
        else if (e.P.acc64) err = enqueue_substage<float, double>(e, k, u, v, w);
        else err = enqueue_substage<float, float>(e, k, u, v, w);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

ch_status resolve_profile(Engine& e)
{
    if (e.ev_pending.empty()) return CH_OK;
    HIP_TRY(hipStreamSynchronize(e.stream));
    for (auto& p : e.ev_pending) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        e.prof_ms[p.first] += ms;
        e.prof_n[p.first] += 1;
        e.ev_pool.push_back(p.second.first);
        e.ev_pool.push_back(p.second.second);
    }
    e.ev_pending.clear();
    return CH_OK;
}

// One coarse-to-fine (or fine-to-coarse) tensor-product transfer: the
// source is [.][sy][sx], the targets tn[0] x tn[1] x tn[2].
struct Transfer {
    int64_t sx = 0, sy = 0;
    int64_t tn[3] = {};
    // 1-D stencils per axis (x, y, z): 4 source indices and weights per target
    int* idx[3] = {};
    double* wt[3] = {};
    // y bands: height, widest band, LDS bytes, (first row, row count) per
    // band; y taps as band-local offsets x sx; y and z weights in the working
    // precision; whether the x taps of targets 4t .. 4t+3 lie in 6 points
    int jb = 0, rmax = 0, xwin = 0;
    size_t lds = 0;
    int* band = nullptr;
    int* ly = nullptr;
    void* wy = nullptr;
    void* wz = nullptr;
    bool ok = false;   // built (a source row too long for the LDS leaves it unbuilt)
};

// Transfers of one handle: the plain transfer of u, v, w; the fine cell
// centres from coarse cell centres (the gradients of the solenoidal
// transfer); its reference planes (u on x = 0, v on y = 0); C from the fine
// to the coarse cell centres.
enum { TR_U, TR_V, TR_W, TR_CENTRES, TR_UREF, TR_VREF, TR_C, TR_COUNT };

// One multiple-resolution transfer handle.
struct InterpData {
    int64_t nf[3];           // fine cells
    int64_t nc[3];           // coarse cells
    int prec = CH_FP64;
    hipStream_t stream = nullptr;
    Transfer tr[TR_COUNT];
    // solenoidal mode and its work buffers
    int solenoidal = 0;
    unsigned gen = 0;        // unique per handle and mode (graphs captured before are stale)
    void* grad = nullptr;    // one coarse cell-centred gradient [ncz][ncy][ncx]
    void* ref = nullptr;     // one reference plane (nz x max(nx, ny))
    double* dzinv = nullptr; // 1 / coarse cell heights
    double* part = nullptr;  // per-group closure maxima, 3 x chk::SCAN_WG
    std::vector<double> zf;  // coarse z faces
};

// work-groups of one transfer launch at most (each takes a contiguous run of
// work items)
constexpr int64_t INTERP_MAX_WG = 2048;

// source of InterpData::gen
std::atomic<unsigned> g_interp_gen{1};

void free_transfer(Transfer& t)
{
    for (int a = 0; a < 3; ++a) {
        if (t.idx[a]) (void)hipFree(t.idx[a]);
        if (t.wt[a]) (void)hipFree(t.wt[a]);
        t.idx[a] = nullptr;
        t.wt[a] = nullptr;
    }
    void* p[4] = {t.band, t.ly, t.wy, t.wz};
    for (void* q : p)
        if (q) (void)hipFree(q);
    t.band = t.ly = nullptr;
    t.wy = t.wz = nullptr;
    t.ok = false;
}

void free_solenoidal(InterpData& d)
{
    void* p[4] = {d.grad, d.ref, d.dzinv, d.part};
    for (void* q : p)
        if (q) (void)hipFree(q);
    d.grad = d.ref = nullptr;
    d.dzinv = d.part = nullptr;
}

// Device copy of a host table; false on failure.
bool upload(void** dptr, const void* data, size_t bytes)
{
    if (hipMalloc(dptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *dptr = nullptr;
        return false;
    }
    return hipMemcpy(*dptr, data, bytes, hipMemcpyHostToDevice) == hipSuccess;
}

// Device copy of stencil weights in the working precision; false on failure.
bool upload_weights(void** dptr, const std::vector<double>& w, int precision)
{
    if (precision == CH_FP64) return upload(dptr, w.data(), sizeof(double) * w.size());
    std::vector<float> f(w.begin(), w.end());
    return upload(dptr, f.data(), sizeof(float) * f.size());
}

// LDS per work-group the band height is chosen for: three groups per CU in
// single precision, two in double, which admits bands of 32 (16) rows at the
// 512^3-from-256^2 ratio; measured faster than more groups with half the
// band, since each item's fixed cost (three barriers, one load round) then
// covers fewer rows.  And the most one group may take.
constexpr size_t interp_lds_target(size_t esize) { return esize == 4 ? 54528 : 81920; }
constexpr size_t INTERP_LDS_MAX = 163840;

// Band table for one y stencil (4 taps per target row, rows cyclic in sy):
// band b starts at its first row's first tap and spans up to its farthest
// tap.  The band height is the largest of 32, 16, ..., 1 (no larger than the
// row count needs) whose LDS fits interp_lds_target, else 1; false when even
// that exceeds INTERP_LDS_MAX.
bool interp_bands(const std::vector<int>& iy, int64_t tny, int sx, int sy, size_t esize,
                  int* jb_out, int* rmax_out, size_t* lds_out, std::vector<int>* band)
{
    int jb0 = 32;
    while (jb0 > 1 && jb0 / 2 >= tny) jb0 /= 2;
    for (int jb = jb0; jb >= 1; jb /= 2) {
        const int64_t nb = (tny + jb - 1) / jb;
        std::vector<int> t(2 * nb);
        int rmax = 1;
        for (int64_t b = 0; b < nb; ++b) {
            const int base = iy[4 * b * jb];
            int span = 1;
            for (int64_t j = b * jb; j < std::min<int64_t>(tny, (b + 1) * jb); ++j)
                for (int q = 0; q < 4; ++q) span = std::max(span, (iy[4 * j + q] - base + sy) % sy + 1);
            t[2 * b] = base;
            t[2 * b + 1] = span;
            rmax = std::max(rmax, span);
        }
        const size_t lds = chk::interp_lds(rmax, jb, sx, esize);
        if (lds > interp_lds_target(esize) && jb > 1) continue;
        if (lds > INTERP_LDS_MAX) return false;
        *band = std::move(t);
        *jb_out = jb;
        *rmax_out = rmax;
        *lds_out = lds;
        return true;
    }
    return false;
}

// Whether the x taps of every 4 consecutive targets 4t .. 4t+3 lie within
// the 6 cyclically consecutive source points from target 4t's first tap.
bool interp_xwin(const std::vector<int>& ix, int64_t tnx, int sx)
{
    for (int64_t i0 = 0; i0 < tnx; i0 += 4) {
        const int ws = ix[4 * i0];
        for (int64_t i = i0; i < std::min<int64_t>(tnx, i0 + 4); ++i)
            for (int q = 0; q < 4; ++q)
                if ((ix[4 * i + q] - ws + sx) % sx >= 6) return false;
    }
    return true;
}

template <typename T>
hipError_t launch_transfer(const Transfer& t, hipStream_t st, const void* src, void* dst)
{
    if (!t.ok) return hipErrorInvalidValue;
    chk::InterpArgs ia;
    ia.src = src;
    ia.dst = dst;
    ia.sx = (int)t.sx;
    ia.sy = (int)t.sy;
    ia.plane = t.sx * t.sy;
    ia.tnx = (int)t.tn[0];
    ia.tny = (int)t.tn[1];
    ia.tnz = (int)t.tn[2];
    ia.jb = t.jb;
    ia.rmax = t.rmax;
    ia.xwin = t.xwin;
    ia.nwg = (int)std::min<int64_t>((t.tn[1] + t.jb - 1) / t.jb * t.tn[2], INTERP_MAX_WG);
    ia.lds = t.lds;
    ia.ix = t.idx[0];
    ia.wx = t.wt[0];
    ia.ly = t.ly;
    ia.wy = t.wy;
    ia.iz = t.idx[2];
    ia.wz = t.wz;
    ia.band = t.band;
    return chk::launch_interp<T>(st, ia);
}

// One component of the solenoidal transfer: its coarse normal gradient, that
// gradient at the fine cell centres (written into the component's fine
// array), then the integration from the reference plane in place.
template <typename T>
hipError_t solenoidal_component(InterpData* ip, hipStream_t st, int c, const void* src, void* dst)
{
    const int nx = (int)ip->nf[0], ny = (int)ip->nf[1], nz = (int)ip->nf[2];
    hipError_t err = chk::launch_grad<T>(st, src, c, (int)ip->nc[0], (int)ip->nc[1],
                                         (int)ip->nc[2], ip->dzinv, ip->grad);
    if (err == hipSuccess) err = launch_transfer<T>(ip->tr[TR_CENTRES], st, ip->grad, dst);
    if (err == hipSuccess && c < 2)
        err = launch_transfer<T>(ip->tr[c == 0 ? TR_UREF : TR_VREF], st, src, ip->ref);
    if (err == hipSuccess)
        err = chk::launch_scan<T>(st, c, dst, ip->ref, nx, ny, nz, 1.0 / ip->nf[c],
                                  ip->part + c * chk::SCAN_WG);
    return err;
}

template <typename T>
hipError_t interp_components(InterpData* ip, hipStream_t st, const void* uc, const void* vc,
                             const void* wc, void* u, void* v, void* w, Engine* prof_e)
{
    const void* src[3] = {uc, vc, wc};
    void* dst[3] = {u, v, w};
    for (int c = 0; c < 3; ++c) {
        hipEvent_t a = nullptr, b = nullptr;
        if (prof_e && prof_e->prof) {
            a = take_event(*prof_e);
            b = take_event(*prof_e);
            if (a) (void)hipEventRecord(a, st);
        }
        hipError_t err = ip->solenoidal
            ? solenoidal_component<T>(ip, st, c, src[c], dst[c])
            : launch_transfer<T>(ip->tr[c], st, src[c], dst[c]);
        if (prof_e && prof_e->prof && a && b) {
            (void)hipEventRecord(b, st);
            prof_e->ev_pending.push_back({3, {a, b}});
        }
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t enqueue_interp(Engine& e, InterpData* ip, const void* uc, const void* vc,
                          const void* wc, void* u, void* v, void* w)
{
    if (ip->prec == CH_FP64) return interp_components<double>(ip, e.stream, uc, vc, wc, u, v, w, &e);
    return interp_components<float>(ip, e.stream, uc, vc, wc, u, v, w, &e);
}

// Enqueue nsteps steps; with a non-null stream and graphs enabled, a step is
// captured once and replayed.
ch_status run_steps(Engine& e, const void* u, const void* v, const void* w, double dt,
                    int nsteps, InterpData* ip, const void* uc, const void* vc, const void* wc)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CH_EINVAL, "dt must be > 0 and finite");
    if (nsteps < 0) return fail(CH_EINVAL, "nsteps must be >= 0");
    if (!ip && (!u || !v || !w)) return fail(CH_EINVAL, "null velocity");
    if (ip && (!uc || !vc || !wc)) return fail(CH_EINVAL, "null coarse velocity");
    HIP_TRY(hipSetDevice(e.device));
    if (dt != e.P.dt || e.P.e25) {
        ch_status st = set_dt(e, dt);
        if (st != CH_OK) return st;
    }
    if (nsteps == 0) return CH_OK;
    const void* key[8] = {u, v, w, uc, vc, wc, ip,
                          ip ? reinterpret_cast<const void*>((uintptr_t)ip->gen) : nullptr};
    const bool use_graph = e.P.opt.use_graph && e.stream != nullptr && !e.prof;
    auto body = [&]() -> hipError_t {
        if (ip) {
            hipError_t err = enqueue_interp(e, ip, uc, vc, wc, e.fu, e.fv, e.fw);
            if (err != hipSuccess) return err;
            return enqueue_step(e, e.fu, e.fv, e.fw);
        }
        return enqueue_step(e, u, v, w);
    };
    if (use_graph) {
        bool same = e.gexec != nullptr;
        for (int m = 0; m < 8 && same; ++m) same = key[m] == e.gkey[m];
        if (!same) {
            if (e.gexec) {
                (void)hipGraphExecDestroy(e.gexec);
                e.gexec = nullptr;
            }
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(e.stream, hipStreamCaptureModeThreadLocal));
            hipError_t err = body();
            hipError_t err2 = hipStreamEndCapture(e.stream, &graph);
            if (err != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(CH_EHIP, "kernel launch during capture failed: %s",
                            hipGetErrorString(err));
            }
            if (err2 != hipSuccess)
                return fail(CH_EHIP, "graph capture failed: %s", hipGetErrorString(err2));
            hipError_t err3 = hipGraphInstantiate(&e.gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (err3 != hipSuccess) {
                e.gexec = nullptr;
                return fail(CH_EHIP, "graph instantiate failed: %s", hipGetErrorString(err3));
            }
            for (int m = 0; m < 8; ++m) e.gkey[m] = key[m];
        }
        for (int s = 0; s < nsteps; ++s) HIP_TRY(hipGraphLaunch(e.gexec, e.stream));
    } else {
        for (int s = 0; s < nsteps; ++s) {
            hipError_t err = body();
            if (err != hipSuccess)
                return fail(CH_EHIP, "kernel launch failed: %s", hipGetErrorString(err));
        }
    }
    return CH_OK;
}

// Drops of box `box`: labels, counts and the sorted (root, cells) list.
ch_status drops(Engine& e, int box, double thr, int64_t cap, int64_t* ndrops, int64_t* root,
                int64_t* cells)
{
    if (!ndrops || (cap > 0 && (!root || !cells))) return fail(CH_EINVAL, "null output");
    if (cap < 0) return fail(CH_EINVAL, "negative capacity");
    if (box < 0 || box >= e.P.nbox) return fail(CH_EINVAL, "box %d out of range", box);
    if (!std::isfinite(thr)) return fail(CH_EINVAL, "threshold must be finite");
    const chd::BoxDesc& d = e.P.boxes[box];
    const int64_t n = (int64_t)d.n[0] * d.n[1] * d.n[2];
    if (n >= 2147483647LL) return fail(CH_EUNSUPPORTED, "drop labelling needs fewer than 2^31 cells");
    HIP_TRY(hipSetDevice(e.device));
    if (n > e.lab_n) {
        if (e.d_lab) (void)hipFree(e.d_lab);
        if (e.d_cnt) (void)hipFree(e.d_cnt);
        e.d_lab = e.d_cnt = nullptr;
        e.lab_n = 0;
        if (hipMalloc(&e.d_lab, sizeof(int) * n) != hipSuccess ||
            hipMalloc(&e.d_cnt, sizeof(int) * n) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CH_ENOMEM, "cannot allocate the drop labels");
        }
        e.lab_n = n;
    }
    const size_t es = chp::esize(e.P.prec);
    const void* C = (const char*)e.C + d.c_off * es;
    const int bc[3] = {d.bc[0], d.bc[1], d.bc[2]};
    hipError_t err = e.P.prec == CH_FP64
        ? chk::launch_drops_label<double>(e.stream, C, d.n[0], d.n[1], d.n[2], bc, thr, e.d_lab)
        : chk::launch_drops_label<float>(e.stream, C, d.n[0], d.n[1], d.n[2], bc, thr, e.d_lab);
    if (err != hipSuccess) return fail(CH_EHIP, "drop labelling failed: %s", hipGetErrorString(err));
    HIP_TRY(hipMemsetAsync(e.d_cnt, 0, sizeof(int) * n, e.stream));
    // the root list: sized from a first pass if the cached one is too short
    int64_t want = std::max<int64_t>(e.list_cap, 1024);
    for (int pass = 0; pass < 2; ++pass) {
        if (want > e.list_cap) {
            if (e.d_list) (void)hipFree(e.d_list);
            e.d_list = nullptr;
            e.list_cap = 0;
            if (hipMalloc(&e.d_list, sizeof(int) * (2 * want + 1)) != hipSuccess) {
                (void)hipGetLastError();
                return fail(CH_ENOMEM, "cannot allocate the drop list");
            }
            e.list_cap = want;
        }
        int* count = e.d_list + 2 * e.list_cap;
        HIP_TRY(hipMemsetAsync(count, 0, sizeof(int), e.stream));
        if (pass == 1) HIP_TRY(hipMemsetAsync(e.d_cnt, 0, sizeof(int) * n, e.stream));
        err = chk::launch_drops_count(e.stream, e.d_lab, n, e.d_cnt, (int)e.list_cap, e.d_list,
                                      e.d_list + e.list_cap, count);
        if (err != hipSuccess)
            return fail(CH_EHIP, "drop counting failed: %s", hipGetErrorString(err));
        int found = 0;
        HIP_TRY(hipMemcpyAsync(&found, count, sizeof(int), hipMemcpyDeviceToHost, e.stream));
        HIP_TRY(hipStreamSynchronize(e.stream));
        if (found <= e.list_cap) {
            std::vector<int> r(found), c(found);
            if (found > 0) {
                HIP_TRY(hipMemcpy(r.data(), e.d_list, sizeof(int) * found, hipMemcpyDeviceToHost));
                HIP_TRY(hipMemcpy(c.data(), e.d_list + e.list_cap, sizeof(int) * found,
                                  hipMemcpyDeviceToHost));
            }
            std::vector<int> order(found);
            for (int q = 0; q < found; ++q) order[q] = q;
            std::sort(order.begin(), order.end(), [&](int a, int b) { return r[a] < r[b]; });
            for (int64_t q = 0; q < std::min<int64_t>(cap, found); ++q) {
                root[q] = r[order[q]];
                cells[q] = c[order[q]];
            }
            *ndrops = found;
            return CH_OK;
        }
        want = found;
    }
    return fail(CH_EHIP, "drop list did not settle");
}

// Launch-plan autotuning: every candidate (x rows per task, planes per task)
// that the plan admits for dt is timed over `steps` steps (after one untimed
// step) with the given velocity, from the same C each time; then, with the
// fastest of those, the y / z segment lengths 128 and 64.  The fastest plan
// stays as the engine's options.  C is restored; E and q are scratch.
ch_status autotune(Engine& e, const void* u, const void* v, const void* w, double dt, int steps,
                   ch_tune* out)
{
    if (!u || !v || !w || !out) return fail(CH_EINVAL, "null argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CH_EINVAL, "dt must be > 0");
    steps = std::max(1, std::min(steps, 1000));
    HIP_TRY(hipSetDevice(e.device));
    HIP_TRY(hipStreamSynchronize(e.stream));
    const size_t bytes = (size_t)e.P.tot[0] * chp::esize(e.P.prec);
    void* save = nullptr;
    if (hipMalloc(&save, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CH_ENOMEM, "cannot allocate the copy of C for autotuning");
    }
    HIP_TRY(hipMemcpy(save, e.C, bytes, hipMemcpyDeviceToDevice));
    const bool prof = e.prof;
    e.prof = false;
    const int keep_rows = e.P.opt.x_rows, keep_zc = e.P.opt.z_chunk;
    // the automatic plan first (its timing also warms the device up) and
    // again last, where its time is taken
    std::vector<std::pair<int, int>> cand = {{0, 0}};
    for (int r : {1, 2, 4})
        for (int z : {0, 4, 6, 8, 10, 12, 14, 16, 20, 24}) cand.push_back({r, z});
    cand.push_back({0, 0});
    hipEvent_t t0 = nullptr, t1 = nullptr;
    ch_status st = CH_OK;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
        st = fail(CH_EHIP, "cannot create events");
    int best_r = keep_rows, best_z = keep_zc, tried = 0;
    double best_ms = INFINITY, auto_ms = NAN;
    for (size_t c = 0; c < cand.size() && st == CH_OK; ++c) {
        e.P.opt.x_rows = cand[c].first;
        e.P.opt.z_chunk = cand[c].second;
        if (set_dt(e, dt) != CH_OK) continue;   // not admitted for this dt
        hipError_t err = hipMemcpyAsync(e.C, save, bytes, hipMemcpyDeviceToDevice, e.stream);
        if (err == hipSuccess) err = enqueue_step(e, u, v, w);
        if (err == hipSuccess) err = hipEventRecord(t0, e.stream);
        for (int k = 0; k < steps && err == hipSuccess; ++k) err = enqueue_step(e, u, v, w);
        if (err == hipSuccess) err = hipEventRecord(t1, e.stream);
        if (err == hipSuccess) err = hipEventSynchronize(t1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, t0, t1);
        if (err != hipSuccess) {
            st = fail(CH_EHIP, "autotuning step failed: %s", hipGetErrorString(err));
            break;
        }
        if (c > 0) ++tried;
        const double per = ms / steps;
        if (c + 1 == cand.size()) auto_ms = per;
        if (c > 0 && per < best_ms) {
            best_ms = per;
            best_r = cand[c].first;
            best_z = cand[c].second;
        }
    }
    // then the segment length of the y and z passes, with the chosen x plan
    const int keep_seg = e.P.opt.seg_len;
    int best_seg = keep_seg;
    for (int seg : {128, 64}) {
        if (st != CH_OK) break;
        e.P.opt.x_rows = best_r;
        e.P.opt.z_chunk = best_z;
        e.P.opt.seg_len = seg;
        if (set_dt(e, dt) != CH_OK) continue;
        hipError_t err = hipMemcpyAsync(e.C, save, bytes, hipMemcpyDeviceToDevice, e.stream);
        if (err == hipSuccess) err = enqueue_step(e, u, v, w);
        if (err == hipSuccess) err = hipEventRecord(t0, e.stream);
        for (int k = 0; k < steps && err == hipSuccess; ++k) err = enqueue_step(e, u, v, w);
        if (err == hipSuccess) err = hipEventRecord(t1, e.stream);
        if (err == hipSuccess) err = hipEventSynchronize(t1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, t0, t1);
        if (err != hipSuccess) {
            st = fail(CH_EHIP, "autotuning step failed: %s", hipGetErrorString(err));
            break;
        }
        ++tried;
        if (ms / steps < best_ms) {
            best_ms = ms / steps;
            best_seg = seg;
        }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    e.prof = prof;
    e.P.opt.seg_len = st == CH_OK ? best_seg : keep_seg;
    e.P.opt.x_rows = st == CH_OK ? best_r : keep_rows;
    e.P.opt.z_chunk = st == CH_OK ? best_z : keep_zc;
    ch_status st2 = set_dt(e, dt);
    hipError_t err = hipMemcpy(e.C, save, bytes, hipMemcpyDeviceToDevice);
    (void)hipFree(save);
    if (st != CH_OK) return st;
    if (st2 != CH_OK) return st2;
    if (err != hipSuccess) return fail(CH_EHIP, "cannot restore C: %s", hipGetErrorString(err));
    out->x_rows = e.P.x_rows;
    out->z_chunk = e.P.zc;
    out->seg_len = e.P.seg_cap;
    out->ms_per_step = best_ms;
    out->auto_ms_per_step = auto_ms;
    out->candidates = tried;
    return CH_OK;
}

ch_status mass(Engine& e, double* out)
{
    if (!out) return fail(CH_EINVAL, "null output");
    HIP_TRY(hipSetDevice(e.device));
    hipError_t err = e.P.prec == CH_FP64
        ? chk::launch_mass<double>(e.P.nmblk, e.P.nbox, e.stream, e.d_boxes, e.C, e.d_partial,
                                   e.d_h3, e.d_mass)
        : chk::launch_mass<float>(e.P.nmblk, e.P.nbox, e.stream, e.d_boxes, e.C, e.d_partial,
                                  e.d_h3, e.d_mass);
    if (err != hipSuccess) return fail(CH_EHIP, "mass kernel failed: %s", hipGetErrorString(err));
    HIP_TRY(hipMemcpyAsync(out, e.d_mass, sizeof(double) * e.P.nbox, hipMemcpyDeviceToHost,
                           e.stream));
    HIP_TRY(hipStreamSynchronize(e.stream));
    return CH_OK;
}

ch_status copy_field(Engine& e, void* dst, const void* src, int on_device, bool in)
{
    if (!dst || !src) return fail(CH_EINVAL, "null field pointer");
    HIP_TRY(hipSetDevice(e.device));
    const size_t bytes = (size_t)e.P.tot[0] * chp::esize(e.P.prec);
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice
                                   : (in ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost);
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, kind, e.stream));
    if (!in || !on_device) HIP_TRY(hipStreamSynchronize(e.stream));
    return CH_OK;
}

ch_status check_velocity(Engine& e, const void* u, const void* v, const void* w)
{
    if (!u || !v || !w) return fail(CH_EINVAL, "null velocity");
    HIP_TRY(hipSetDevice(e.device));
    hipError_t err = e.P.prec == CH_FP64
        ? chk::launch_check_velocity<double>(e.stream, e.d_boxes, e.P.nbox, u, v, w, e.d_flags)
        : chk::launch_check_velocity<float>(e.stream, e.d_boxes, e.P.nbox, u, v, w, e.d_flags);
    if (err != hipSuccess) return fail(CH_EHIP, "check kernel failed: %s", hipGetErrorString(err));
    std::vector<int> flags(2 * chk::CHECK_WGS);
    HIP_TRY(hipMemcpyAsync(flags.data(), e.d_flags, sizeof(int) * flags.size(),
                           hipMemcpyDeviceToHost, e.stream));
    HIP_TRY(hipStreamSynchronize(e.stream));
    long long bad = 0, wall = 0;
    for (int i = 0; i < chk::CHECK_WGS; ++i) {
        bad += flags[2 * i];
        wall += flags[2 * i + 1];
    }
    if (bad) return fail(CH_ENONFINITE, "%lld non-finite velocity values", bad);
    if (wall) return fail(CH_EINVAL, "%lld non-zero normal velocities on no-flux walls", wall);
    return CH_OK;
}

ch_status profile_read(Engine& e, int kernel, double* ms, int64_t* n)
{
    if (kernel < 0 || kernel > 3) return fail(CH_EINVAL, "unknown kernel class %d", kernel);
    ch_status st = resolve_profile(e);
    if (st != CH_OK) return st;
    if (ms) *ms = e.prof_ms[kernel];
    if (n) *n = e.prof_n[kernel];
    return CH_OK;
}

ch_status profile_enable(Engine& e, int on)
{
    ch_status st = resolve_profile(e);
    if (st != CH_OK) return st;
    e.prof = on != 0;
    for (int k = 0; k < 4; ++k) {
        e.prof_ms[k] = 0.0;
        e.prof_n[k] = 0;
    }
    return CH_OK;
}

// Build one transfer: source axes src[3] (x, y, z) of a [.][sy][sx] array,
// target coordinates tgt[3].  A y-row extent that does not fit the LDS
// leaves it unbuilt (ok = false) with CH_OK; other failures return an error.
ch_status build_transfer(Transfer& t, const chp::SrcAxis* const src[3],
                         const std::vector<double>* const tgt[3], int64_t sx, int64_t sy,
                         int precision)
{
    t.sx = sx;
    t.sy = sy;
    std::vector<int> idx[3];
    std::vector<double> wt[3];
    for (int a = 0; a < 3; ++a) {
        const std::vector<double>& q = *tgt[a];
        if (!chp::hermite_stencils(*src[a], q, &idx[a], &wt[a]))
            return fail(CH_EINVAL, "transfer target outside the source axis");
        t.tn[a] = (int64_t)q.size();
    }
    std::vector<int> band;
    if (!interp_bands(idx[1], t.tn[1], (int)sx, (int)sy, precision == CH_FP64 ? 8 : 4, &t.jb,
                      &t.rmax, &t.lds, &band))
        return CH_OK;
    std::vector<int> ly(idx[1].size());
    for (size_t q = 0; q < ly.size(); ++q) {
        const int base = band[2 * ((q / 4) / t.jb)];
        ly[q] = (int)(((idx[1][q] - base + sy) % sy) * sx);
    }
    t.xwin = interp_xwin(idx[0], t.tn[0], (int)sx) ? 1 : 0;
    bool good = true;
    for (int a = 0; a < 3 && good; a += 2)
        good = upload((void**)&t.idx[a], idx[a].data(), sizeof(int) * idx[a].size()) &&
               upload((void**)&t.wt[a], wt[a].data(), sizeof(double) * wt[a].size());
    good = good && upload((void**)&t.band, band.data(), sizeof(int) * band.size()) &&
           upload((void**)&t.ly, ly.data(), sizeof(int) * ly.size()) &&
           upload_weights(&t.wy, wt[1], precision) && upload_weights(&t.wz, wt[2], precision);
    if (!good) {
        free_transfer(t);
        return fail(CH_ENOMEM, "cannot upload interpolation tables");
    }
    t.ok = true;
    return CH_OK;
}

}  // namespace

struct ch_state {
    Engine e;
};
struct ch_batch {
    Engine e;
};
struct ch_interp {
    InterpData d;
};
// Split-density pressure step: mesh, transforms and work arrays.
struct ch_poisson {
    int nx = 0, ny = 0, nz = 0, zwalls = 0, prec = CH_FP64;
    double h = 0.0;
    hipStream_t stream = nullptr;
    hipfftHandle fwd = 0, inv = 0;
    bool have_fwd = false, have_inv = false;
    void* phat = nullptr;   // 2 P^l - P^{l-1}
    void* rhs = nullptr;    // eq-newpoi right-hand side
    void* spec = nullptr;   // its transform, nz x ny x (nx/2 + 1) complex
    void* cp = nullptr;     // Thomas scratch, nz x ny x (nx/2 + 1) reals
};

// ---- allocation-free mass ---------------------------------------------------
// Partial sums of ch_mass_field_noalloc: one array per GPU, for the life of
// the process.  Host code never uses this name as an address (on the host it
// is only a stand-in); the device address comes from hipGetSymbolAddress,
// once per device, and is kept in g_scratch_ptr.
constexpr int NOALLOC_PARTIALS = 1 << 20;
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];

static std::mutex g_scratch_mu;
static std::unordered_map<int, double*> g_scratch_ptr;

// Device address of `scratch` on the current device (looked up on the
// first call there).
static ch_status scratch_ptr(double** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> l(g_scratch_mu);
    const auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return CH_OK;
    }
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(CH_EHIP, "no device address for the mass scratch array");
    g_scratch_ptr[dev] = (double*)p;
    *out = (double*)p;
    return CH_OK;
}

extern "C" {

void ch_default_opts(ch_opts* o)
{
    if (o) chp::default_opts(o);
}

const char* ch_last_error(void) { return g_err.c_str(); }

ch_status ch_create(const ch_grid* g, double Cn, double Pe, const ch_psi* psi, const ch_bc* bc,
                    const ch_opts* opt, ch_state** out)
{
    if (!out) return fail(CH_EINVAL, "null output handle");
    *out = nullptr;
    ch_state* s = new (std::nothrow) ch_state();
    if (!s) return fail(CH_ENOMEM, "host allocation failed");
    ch_status st = init_engine(s->e, 1, g, &Cn, &Pe, psi, bc, opt);
    if (st == CH_OK && s->e.P.opt.dt_hint > 0.0) st = set_dt(s->e, s->e.P.opt.dt_hint);
    if (st != CH_OK) {
        free_engine(s->e);
        delete s;
        return st;
    }
    reg(s);
    *out = s;
    return CH_OK;
}

#define CHECK_STATE(s) \
    if (!live(s)) return fail(CH_EHANDLE, "invalid or destroyed handle")

ch_status ch_set_stream(ch_state* s, void* stream)
{
    CHECK_STATE(s);
    if (s->e.gexec) {
        (void)hipGraphExecDestroy(s->e.gexec);
        s->e.gexec = nullptr;
    }
    s->e.stream = (hipStream_t)stream;
    return CH_OK;
}

ch_status ch_set_field(ch_state* s, const void* C, int on_device)
{
    CHECK_STATE(s);
    return copy_field(s->e, s->e.C, C, on_device, true);
}

ch_status ch_get_field(ch_state* s, void* C, int on_device)
{
    CHECK_STATE(s);
    return copy_field(s->e, C, s->e.C, on_device, false);
}

ch_status ch_step(ch_state* s, const void* u, const void* v, const void* w, double dt,
                  int nsteps)
{
    CHECK_STATE(s);
    return run_steps(s->e, u, v, w, dt, nsteps, nullptr, nullptr, nullptr, nullptr);
}

ch_status ch_step_explicit25(ch_state* s, const void* u, const void* v, const void* w,
                             double dt, int nsteps)
{
    CHECK_STATE(s);
    return run_steps_e25(s->e, u, v, w, dt, nsteps);
}

ch_status ch_mass(ch_state* s, double* out)
{
    CHECK_STATE(s);
    return mass(s->e, out);
}

ch_status ch_mass_field_noalloc(const void* C, int64_t nx, int64_t ny, int64_t nz, double h,
                                int precision, void* stream, double* out_dev)
{
    if (!C || !out_dev) return fail(CH_EINVAL, "null pointer");
    if (nx < 1 || ny < 1 || nz < 1) return fail(CH_EINVAL, "extents must be >= 1");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(CH_EINVAL, "h must be > 0 and finite");
    if (precision != CH_FP64 && precision != CH_FP32) return fail(CH_EINVAL, "unknown precision");
    // cells within NOALLOC_PARTIALS blocks, and each extent within the box
    // table's 32-bit fields
    if (nx > INT32_MAX || ny > INT32_MAX || nz > INT32_MAX ||
        (double)nx * (double)ny * (double)nz > (double)NOALLOC_PARTIALS * chd::MASS_BLOCK)
        return fail(CH_EINVAL, "field larger than %lld cells (the scratch array's limit)",
                    (long long)NOALLOC_PARTIALS * chd::MASS_BLOCK);
    const int64_t cells = nx * ny * nz;
    chd::BoxDesc bd{};
    bd.n[0] = (int)nx;
    bd.n[1] = (int)ny;
    bd.n[2] = (int)nz;
    bd.c_off = 0;
    bd.mblk0 = 0;
    bd.nmblk = (int)((cells + chd::MASS_BLOCK - 1) / chd::MASS_BLOCK);
    double* partial = nullptr;
    ch_status st = scratch_ptr(&partial);
    if (st != CH_OK) return st;
    const hipStream_t hs = (hipStream_t)stream;
    const double h3 = h * h * h;
    const hipError_t err = precision == CH_FP64
        ? chk::launch_mass_one<double>(hs, bd, C, partial, h3, out_dev)
        : chk::launch_mass_one<float>(hs, bd, C, partial, h3, out_dev);
    if (err != hipSuccess) return fail(CH_EHIP, "mass kernels failed: %s", hipGetErrorString(err));
    return CH_OK;
}

ch_status ch_check_velocity(ch_state* s, const void* u, const void* v, const void* w)
{
    CHECK_STATE(s);
    return check_velocity(s->e, u, v, w);
}

void ch_destroy(ch_state* s)
{
    if (!s || !live(s)) return;
    unreg(s);
    if (s->e.stream) (void)hipStreamSynchronize(s->e.stream);
    else (void)hipDeviceSynchronize();
    free_engine(s->e);
    delete s;
}

ch_status ch_profile_enable(ch_state* s, int on)
{
    CHECK_STATE(s);
    return profile_enable(s->e, on);
}

ch_status ch_profile_read(ch_state* s, int kernel, double* total_ms, int64_t* launches)
{
    CHECK_STATE(s);
    return profile_read(s->e, kernel, total_ms, launches);
}

ch_status ch_get_config(const ch_state* s, int cfg[8])
{
    CHECK_STATE(s);
    if (!cfg) return fail(CH_EINVAL, "null output");
    const chp::Plan& P = s->e.P;
    cfg[0] = P.x_rows;
    cfg[1] = P.seg_cap;
    cfg[2] = P.yz_threads;
    for (int k = 0; k < 3; ++k) cfg[3 + k] = P.boxes[0].tw[k];
    cfg[6] = P.acc64 ? 1 : 0;
    cfg[7] = P.zc;
    return CH_OK;
}

static ch_status x_program(const chp::Plan& P, int* kind)
{
    if (!kind) return fail(CH_EINVAL, "null output");
    if (std::isnan(P.dt)) return fail(CH_EINVAL, "no plan yet: step once or pass dt_hint");
    *kind = P.xseg ? 3 : P.nxl > 1 ? 4 : P.xrow ? (P.xrow_multi ? 2 : 1) : 0;
    return CH_OK;
}

ch_status ch_get_x_program(const ch_state* s, int* kind)
{
    CHECK_STATE(s);
    return x_program(s->e.P, kind);
}

// ---- batch -----------------------------------------------------------------
ch_status ch_batch_create(int nbox, const ch_grid* g, const double* Cn, const double* Pe,
                          const ch_psi* psi, const ch_bc* bc, const ch_opts* opt,
                          ch_batch** out)
{
    if (!out) return fail(CH_EINVAL, "null output handle");
    *out = nullptr;
    ch_batch* b = new (std::nothrow) ch_batch();
    if (!b) return fail(CH_ENOMEM, "host allocation failed");
    ch_status st = init_engine(b->e, nbox, g, Cn, Pe, psi, bc, opt);
    if (st == CH_OK && b->e.P.opt.dt_hint > 0.0) st = set_dt(b->e, b->e.P.opt.dt_hint);
    if (st != CH_OK) {
        free_engine(b->e);
        delete b;
        return st;
    }
    reg(b);
    *out = b;
    return CH_OK;
}

ch_status ch_batch_field_offsets(const ch_batch* b, int64_t* c_off, int64_t* u_off,
                                 int64_t* v_off, int64_t* w_off, int64_t totals[4])
{
    CHECK_STATE(b);
    for (int i = 0; i < b->e.P.nbox; ++i) {
        const chd::BoxDesc& d = b->e.P.boxes[i];
        if (c_off) c_off[i] = d.c_off;
        if (u_off) u_off[i] = d.u_off;
        if (v_off) v_off[i] = d.v_off;
        if (w_off) w_off[i] = d.w_off;
    }
    if (totals)
        for (int m = 0; m < 4; ++m) totals[m] = b->e.P.tot[m];
    return CH_OK;
}

ch_status ch_batch_set_stream(ch_batch* b, void* stream)
{
    CHECK_STATE(b);
    if (b->e.gexec) {
        (void)hipGraphExecDestroy(b->e.gexec);
        b->e.gexec = nullptr;
    }
    b->e.stream = (hipStream_t)stream;
    return CH_OK;
}

ch_status ch_batch_set_field(ch_batch* b, const void* C, int on_device)
{
    CHECK_STATE(b);
    return copy_field(b->e, b->e.C, C, on_device, true);
}

ch_status ch_batch_get_field(ch_batch* b, void* C, int on_device)
{
    CHECK_STATE(b);
    return copy_field(b->e, C, b->e.C, on_device, false);
}

ch_status ch_batch_step(ch_batch* b, const void* u, const void* v, const void* w, double dt,
                        int nsteps)
{
    CHECK_STATE(b);
    return run_steps(b->e, u, v, w, dt, nsteps, nullptr, nullptr, nullptr, nullptr);
}

ch_status ch_batch_mass(ch_batch* b, double* out)
{
    CHECK_STATE(b);
    return mass(b->e, out);
}

void ch_batch_destroy(ch_batch* b)
{
    if (!b || !live(b)) return;
    unreg(b);
    if (b->e.stream) (void)hipStreamSynchronize(b->e.stream);
    else (void)hipDeviceSynchronize();
    free_engine(b->e);
    delete b;
}

ch_status ch_batch_profile_enable(ch_batch* b, int on)
{
    CHECK_STATE(b);
    return profile_enable(b->e, on);
}

ch_status ch_batch_profile_read(ch_batch* b, int kernel, double* total_ms, int64_t* launches)
{
    CHECK_STATE(b);
    return profile_read(b->e, kernel, total_ms, launches);
}

ch_status ch_batch_get_x_program(const ch_batch* b, int* kind)
{
    CHECK_STATE(b);
    return x_program(b->e.P, kind);
}

// ---- multiple resolution -----------------------------------------------------
ch_status ch_interp_create(const ch_grid* fine, int64_t ncx, int64_t ncy, int64_t ncz,
                           const double* zf, int precision, ch_interp** out)
{
    if (!out || !fine || !zf) return fail(CH_EINVAL, "null argument");
    *out = nullptr;
    if (precision != CH_FP64 && precision != CH_FP32)
        return fail(CH_EINVAL, "unknown precision %d", precision);
    if (ncx < 4 || ncy < 4 || ncz < 4 || fine->nx < 1 || fine->ny < 1 || fine->nz < 1)
        return fail(CH_EINVAL, "meshes too small");
    if ((double)ncx * ncy * (ncz + 1) >= 2147483647.0)
        return fail(CH_EINVAL, "coarse mesh too large");
    // the kernels count (row, plane) work items and reference-plane points in
    // 32 bits (element addresses are 64-bit)
    if ((double)fine->ny * (fine->nz + 1) >= 2147483647.0 ||
        (double)fine->nx * (fine->nz + 1) >= 2147483647.0)
        return fail(CH_EINVAL, "fine mesh too large");
    if (ncx > (precision == CH_FP64 ? 4096 : 8192))
        return fail(CH_EUNSUPPORTED, "coarse x extent above %d (five rows in LDS)",
                    precision == CH_FP64 ? 4096 : 8192);
    if (zf[0] != 0.0 || zf[ncz] != 1.0) return fail(CH_EINVAL, "zf must run from 0 to 1");
    for (int64_t k = 0; k < ncz; ++k)
        if (!(zf[k + 1] > zf[k])) return fail(CH_EINVAL, "zf must increase");
    ch_interp* ip = new (std::nothrow) ch_interp();
    if (!ip) return fail(CH_ENOMEM, "host allocation failed");
    InterpData& d = ip->d;
    const int64_t nx = fine->nx, ny = fine->ny, nz = fine->nz;
    d.nf[0] = nx;
    d.nf[1] = ny;
    d.nf[2] = nz;
    d.nc[0] = ncx;
    d.nc[1] = ncy;
    d.nc[2] = ncz;
    d.prec = precision;
    d.gen = g_interp_gen.fetch_add(1);
    d.zf.assign(zf, zf + ncz + 1);
    auto pts = [](int64_t n, double off) {
        std::vector<double> t(n);
        for (int64_t i = 0; i < n; ++i) t[i] = (i + off) / n;
        return t;
    };
    using chp::SrcAxis;
    const SrcAxis cxf{pts(ncx, 0.0), chp::AXIS_PERIODIC}, cxc{pts(ncx, 0.5), chp::AXIS_PERIODIC},
        cyf{pts(ncy, 0.0), chp::AXIS_PERIODIC}, cyc{pts(ncy, 0.5), chp::AXIS_PERIODIC};
    SrcAxis czc{{}, chp::AXIS_MIRROR}, czf{{}, chp::AXIS_ANTI};
    for (int64_t k = 0; k < ncz; ++k) czc.s.push_back(0.5 * (zf[k] + zf[k + 1]));
    for (int64_t k = 0; k <= ncz; ++k) czf.s.push_back(zf[k]);
    const std::vector<double> fxf = pts(nx, 0.0), fxc = pts(nx, 0.5), fyf = pts(ny, 0.0),
                              fyc = pts(ny, 0.5), fzc = pts(nz, 0.5), zero(1, 0.0);
    std::vector<double> fzf(nz + 1);   // z faces including both walls
    for (int64_t k = 0; k <= nz; ++k) fzf[k] = (double)k / nz;
    const SrcAxis sfx{fxc, chp::AXIS_PERIODIC}, sfy{fyc, chp::AXIS_PERIODIC},
        sfz{fzc, chp::AXIS_MIRROR};
    std::vector<double> ccx(cxc.s), ccy(cyc.s), ccz(czc.s);
    // u: x faces, y and z centres; v: x centres, y faces, z centres; w: x
    // and y centres, z faces; then the solenoidal transfer's pieces and the
    // projection of C
    const SrcAxis* srcs[TR_COUNT][3] = {{&cxf, &cyc, &czc}, {&cxc, &cyf, &czc}, {&cxc, &cyc, &czf},
                                    {&cxc, &cyc, &czc}, {&cxf, &cyc, &czc}, {&cxc, &cyf, &czc},
                                    {&sfx, &sfy, &sfz}};
    const std::vector<double>* tgts[TR_COUNT][3] = {
        {&fxf, &fyc, &fzc}, {&fxc, &fyf, &fzc}, {&fxc, &fyc, &fzf}, {&fxc, &fyc, &fzc},
        {&zero, &fyc, &fzc}, {&fxc, &zero, &fzc}, {&ccx, &ccy, &ccz}};
    ch_status st = CH_OK;
    for (int c = 0; c < TR_COUNT && st == CH_OK; ++c) {
        const bool fine_src = c == TR_C;
        st = build_transfer(d.tr[c], srcs[c], tgts[c], fine_src ? nx : ncx, fine_src ? ny : ncy,
                            precision);
        if (st == CH_OK && !d.tr[c].ok && c != TR_C)
            st = fail(CH_EUNSUPPORTED, "coarse x extent too long for the transfer's LDS rows");
    }
    if (st != CH_OK) {
        for (int c = 0; c < TR_COUNT; ++c) free_transfer(d.tr[c]);
        delete ip;
        return st;
    }
    reg(ip);
    *out = ip;
    return CH_OK;
}

ch_status ch_interp_set_solenoidal(ch_interp* ip, int on)
{
    CHECK_STATE(ip);
    InterpData& d = ip->d;
    if ((on != 0) == (d.solenoidal != 0)) return CH_OK;
    if (d.stream) HIP_TRY(hipStreamSynchronize(d.stream));
    else HIP_TRY(hipDeviceSynchronize());
    d.gen = g_interp_gen.fetch_add(1);
    if (!on) {
        free_solenoidal(d);
        d.solenoidal = 0;
        return CH_OK;
    }
    const size_t es = d.prec == CH_FP64 ? 8 : 4;
    const size_t ncell = (size_t)d.nc[0] * d.nc[1] * d.nc[2];
    const size_t nref = (size_t)d.nf[2] * std::max(d.nf[0], d.nf[1]);
    std::vector<double> dzinv(d.nc[2]);
    for (int64_t k = 0; k < d.nc[2]; ++k) dzinv[k] = 1.0 / (d.zf[k + 1] - d.zf[k]);
    const std::vector<double> zeros(3 * chk::SCAN_WG, 0.0);
    const bool good = hipMalloc(&d.grad, ncell * es) == hipSuccess &&
                      hipMalloc(&d.ref, nref * es) == hipSuccess &&
                      upload((void**)&d.dzinv, dzinv.data(), sizeof(double) * dzinv.size()) &&
                      upload((void**)&d.part, zeros.data(), sizeof(double) * zeros.size());
    if (!good) {
        (void)hipGetLastError();
        free_solenoidal(d);
        return fail(CH_ENOMEM, "cannot allocate the solenoidal transfer's buffers");
    }
    d.solenoidal = 1;
    return CH_OK;
}

ch_status ch_interp_closure(ch_interp* ip, double out[3])
{
    CHECK_STATE(ip);
    if (!out) return fail(CH_EINVAL, "null output");
    InterpData& d = ip->d;
    out[0] = out[1] = out[2] = 0.0;
    if (!d.solenoidal) return CH_OK;
    if (d.stream) HIP_TRY(hipStreamSynchronize(d.stream));
    else HIP_TRY(hipDeviceSynchronize());
    std::vector<double> part(3 * chk::SCAN_WG);
    HIP_TRY(hipMemcpy(part.data(), d.part, sizeof(double) * part.size(), hipMemcpyDeviceToHost));
    for (int c = 0; c < 3; ++c) {
        const int g = chk::scan_groups(c, (int)d.nf[0], (int)d.nf[1], (int)d.nf[2]);
        for (int q = 0; q < g; ++q) out[c] = std::max(out[c], part[c * chk::SCAN_WG + q]);
    }
    return CH_OK;
}

ch_status ch_interp_project_c(ch_interp* ip, const void* Cf, void* Cc)
{
    CHECK_STATE(ip);
    if (!Cf || !Cc) return fail(CH_EINVAL, "null pointer");
    InterpData& d = ip->d;
    if (!d.tr[TR_C].ok)
        return fail(CH_EUNSUPPORTED, "fine x extent too long for the projection's LDS rows");
    hipError_t err = d.prec == CH_FP64 ? launch_transfer<double>(d.tr[TR_C], d.stream, Cf, Cc)
                                       : launch_transfer<float>(d.tr[TR_C], d.stream, Cf, Cc);
    if (err != hipSuccess) return fail(CH_EHIP, "projection failed: %s", hipGetErrorString(err));
    return CH_OK;
}

ch_status ch_interp_set_stream(ch_interp* ip, void* stream)
{
    CHECK_STATE(ip);
    ip->d.stream = (hipStream_t)stream;
    return CH_OK;
}

ch_status ch_interp_apply(ch_interp* ip, const void* uc, const void* vc, const void* wc,
                          void* u, void* v, void* w)
{
    CHECK_STATE(ip);
    if (!uc || !vc || !wc || !u || !v || !w) return fail(CH_EINVAL, "null pointer");
    hipError_t err = ip->d.prec == CH_FP64
        ? interp_components<double>(&ip->d, ip->d.stream, uc, vc, wc, u, v, w, nullptr)
        : interp_components<float>(&ip->d, ip->d.stream, uc, vc, wc, u, v, w, nullptr);
    if (err != hipSuccess) return fail(CH_EHIP, "interpolation failed: %s", hipGetErrorString(err));
    return CH_OK;
}

void ch_interp_destroy(ch_interp* ip)
{
    if (!ip || !live(ip)) return;
    unreg(ip);
    if (ip->d.stream) (void)hipStreamSynchronize(ip->d.stream);
    else (void)hipDeviceSynchronize();
    for (int c = 0; c < TR_COUNT; ++c) free_transfer(ip->d.tr[c]);
    free_solenoidal(ip->d);
    delete ip;
}

ch_status ch_autotune(ch_state* s, const void* u, const void* v, const void* w, double dt,
                      int steps, ch_tune* out)
{
    CHECK_STATE(s);
    return autotune(s->e, u, v, w, dt, steps, out);
}

ch_status ch_batch_autotune(ch_batch* b, const void* u, const void* v, const void* w, double dt,
                            int steps, ch_tune* out)
{
    CHECK_STATE(b);
    return autotune(b->e, u, v, w, dt, steps, out);
}

ch_status ch_drops(ch_state* s, double threshold, int64_t cap, int64_t* ndrops, int64_t* root,
                   int64_t* cells)
{
    CHECK_STATE(s);
    return drops(s->e, 0, threshold, cap, ndrops, root, cells);
}

ch_status ch_batch_drops(ch_batch* b, int box, double threshold, int64_t cap, int64_t* ndrops,
                         int64_t* root, int64_t* cells)
{
    CHECK_STATE(b);
    return drops(b->e, box, threshold, cap, ndrops, root, cells);
}

static void poisson_free(ch_poisson* p)
{
    if (p->have_fwd) (void)hipfftDestroy(p->fwd);
    if (p->have_inv) (void)hipfftDestroy(p->inv);
    void* bufs[4] = {p->phat, p->rhs, p->spec, p->cp};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

ch_status ch_poisson_create(const ch_grid* g, int z_walls, int precision, ch_poisson** out)
{
    if (!g || !out) return fail(CH_EINVAL, "null argument");
    *out = nullptr;
    if (precision != CH_FP64 && precision != CH_FP32)
        return fail(CH_EINVAL, "unknown precision %d", precision);
    if (g->nx < 2 || g->ny < 2 || g->nz < 2 || !(g->h > 0.0))
        return fail(CH_EINVAL, "the pressure mesh needs at least 2 cells per axis and h > 0");
    if ((double)g->nx * g->ny * (g->nz + 1) >= 2147483647.0)
        return fail(CH_EUNSUPPORTED, "pressure mesh of 2^31 cells or more");
    if ((double)g->nx * g->ny * (precision == CH_FP64 ? 8.0 : 4.0) >= 4294967296.0)
        return fail(CH_EUNSUPPORTED, "pressure mesh plane of 4 GiB or more");
    ch_poisson* p = new (std::nothrow) ch_poisson();
    if (!p) return fail(CH_ENOMEM, "host allocation failed");
    p->nx = (int)g->nx;
    p->ny = (int)g->ny;
    p->nz = (int)g->nz;
    p->h = g->h;
    p->zwalls = z_walls ? 1 : 0;
    p->prec = precision;
    const size_t es = precision == CH_FP64 ? 8 : 4;
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const size_t nm = (size_t)p->ny * (p->nx / 2 + 1);
    const hipfftType tf = precision == CH_FP64 ? HIPFFT_D2Z : HIPFFT_R2C;
    const hipfftType ti = precision == CH_FP64 ? HIPFFT_Z2D : HIPFFT_C2R;
    hipfftResult r1, r2;
    if (p->zwalls) {
        int dims[2] = {p->ny, p->nx};
        r1 = hipfftPlanMany(&p->fwd, 2, dims, nullptr, 1, 0, nullptr, 1, 0, tf, p->nz);
        p->have_fwd = r1 == HIPFFT_SUCCESS;
        r2 = hipfftPlanMany(&p->inv, 2, dims, nullptr, 1, 0, nullptr, 1, 0, ti, p->nz);
        p->have_inv = r2 == HIPFFT_SUCCESS;
    } else {
        r1 = hipfftPlan3d(&p->fwd, p->nz, p->ny, p->nx, tf);
        p->have_fwd = r1 == HIPFFT_SUCCESS;
        r2 = hipfftPlan3d(&p->inv, p->nz, p->ny, p->nx, ti);
        p->have_inv = r2 == HIPFFT_SUCCESS;
    }
    if (!p->have_fwd || !p->have_inv) {
        poisson_free(p);
        return fail(CH_EHIP, "hipFFT plan creation failed (%d, %d)", (int)r1, (int)r2);
    }
    if (hipMalloc(&p->phat, n * es) != hipSuccess || hipMalloc(&p->rhs, n * es) != hipSuccess ||
        hipMalloc(&p->spec, 2 * nm * p->nz * es) != hipSuccess ||
        (p->zwalls && hipMalloc(&p->cp, nm * p->nz * es) != hipSuccess)) {
        (void)hipGetLastError();
        poisson_free(p);
        return fail(CH_ENOMEM, "cannot allocate the pressure work arrays");
    }
    reg(p);
    *out = p;
    return CH_OK;
}

ch_status ch_poisson_set_stream(ch_poisson* p, void* stream)
{
    CHECK_STATE(p);
    p->stream = (hipStream_t)stream;
    return CH_OK;
}

static hipError_t poisson_enqueue(ch_poisson* p, const void* rhs, void* P)
{
    if (hipfftSetStream(p->fwd, p->stream) != HIPFFT_SUCCESS ||
        hipfftSetStream(p->inv, p->stream) != HIPFFT_SUCCESS)
        return hipErrorLaunchFailure;
    hipfftResult r;
    if (p->prec == CH_FP64)
        r = hipfftExecD2Z(p->fwd, (hipfftDoubleReal*)const_cast<void*>(rhs),
                          (hipfftDoubleComplex*)p->spec);
    else
        r = hipfftExecR2C(p->fwd, (hipfftReal*)const_cast<void*>(rhs), (hipfftComplex*)p->spec);
    if (r != HIPFFT_SUCCESS) return hipErrorLaunchFailure;
    hipError_t err = p->prec == CH_FP64
        ? chk::launch_press_solve<double>(p->stream, p->zwalls, p->spec, p->cp, p->nx, p->ny,
                                          p->nz, p->h)
        : chk::launch_press_solve<float>(p->stream, p->zwalls, p->spec, p->cp, p->nx, p->ny,
                                         p->nz, p->h);
    if (err != hipSuccess) return err;
    if (p->prec == CH_FP64)
        r = hipfftExecZ2D(p->inv, (hipfftDoubleComplex*)p->spec, (hipfftDoubleReal*)P);
    else
        r = hipfftExecC2R(p->inv, (hipfftComplex*)p->spec, (hipfftReal*)P);
    return r == HIPFFT_SUCCESS ? hipSuccess : hipErrorLaunchFailure;
}

ch_status ch_poisson_solve(ch_poisson* p, const void* rhs, void* P)
{
    CHECK_STATE(p);
    if (!rhs || !P) return fail(CH_EINVAL, "null pointer");
    hipError_t err = poisson_enqueue(p, rhs, P);
    if (err != hipSuccess) return fail(CH_EHIP, "Poisson solve failed: %s", hipGetErrorString(err));
    return CH_OK;
}

ch_status ch_pressure_step(ch_poisson* p, const void* C, double rho1, double rho2, double dt,
                           void* u, void* v, void* w, void* P, void* Pold)
{
    CHECK_STATE(p);
    if (!C || !u || !v || !w || !P || !Pold) return fail(CH_EINVAL, "null pointer");
    if (!(rho2 > 0.0) || !(rho1 >= rho2) || !(dt > 0.0) || !std::isfinite(rho1))
        return fail(CH_EINVAL, "need 0 < rho2 <= rho1 (finite) and dt > 0");
    const chk::PressArgs a{p->nx, p->ny, p->nz, p->zwalls, p->h, rho1, rho2, dt};
    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    hipError_t err;
    if (p->prec == CH_FP64) {
        err = chk::launch_press_prep<double>(p->stream, P, Pold, p->phat, n);
        if (err == hipSuccess)
            err = chk::launch_press_rhs<double>(p->stream, a, C, p->phat, u, v, w, p->rhs);
    } else {
        err = chk::launch_press_prep<float>(p->stream, P, Pold, p->phat, n);
        if (err == hipSuccess)
            err = chk::launch_press_rhs<float>(p->stream, a, C, p->phat, u, v, w, p->rhs);
    }
    if (err == hipSuccess) err = poisson_enqueue(p, p->rhs, P);
    if (err == hipSuccess)
        err = p->prec == CH_FP64
            ? chk::launch_press_update<double>(p->stream, a, C, P, p->phat, u, v, w)
            : chk::launch_press_update<float>(p->stream, a, C, P, p->phat, u, v, w);
    if (err != hipSuccess) return fail(CH_EHIP, "pressure step failed: %s", hipGetErrorString(err));
    return CH_OK;
}

void ch_poisson_destroy(ch_poisson* p)
{
    if (!p || !live(p)) return;
    unreg(p);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    poisson_free(p);
}

ch_status ch_step_multires(ch_state* s, ch_interp* ip, const void* uc, const void* vc,
                           const void* wc, double dt, int nsteps)
{
    CHECK_STATE(s);
    if (!live(ip)) return fail(CH_EHANDLE, "invalid or destroyed interpolation handle");
    Engine& e = s->e;
    const chd::BoxDesc& d = e.P.boxes[0];
    if (ip->d.nf[0] != d.n[0] || ip->d.nf[1] != d.n[1] || ip->d.nf[2] != d.n[2])
        return fail(CH_EINVAL, "interpolation target mesh differs from the state's");
    if (d.bc[0] != CH_PERIODIC || d.bc[1] != CH_PERIODIC || d.bc[2] != CH_NOFLUX)
        return fail(CH_EUNSUPPORTED, "the multiple-resolution step needs periodic x, y and "
                                     "no-flux z");
    if (ip->d.prec != e.P.prec) return fail(CH_EINVAL, "precision mismatch");
    if (!e.fu) {
        const size_t es = chp::esize(e.P.prec);
        const size_t nu = (size_t)d.nf[0] * d.n[1] * d.n[2];
        const size_t nv = (size_t)d.n[0] * d.nf[1] * d.n[2];
        const size_t nw = (size_t)d.n[0] * d.n[1] * d.nf[2];
        if (hipMalloc(&e.fu, nu * es) != hipSuccess || hipMalloc(&e.fv, nv * es) != hipSuccess ||
            hipMalloc(&e.fw, nw * es) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CH_ENOMEM, "cannot allocate the fine velocity");
        }
    }
    return run_steps(e, nullptr, nullptr, nullptr, dt, nsteps, &ip->d, uc, vc, wc);
}

}  // extern "C"
