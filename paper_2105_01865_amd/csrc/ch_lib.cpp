// ch_lib.cpp -- host side of libch: the C ABI of include/ch.h.
//
// A state (single box) and a batch (many boxes) share one engine: the
// kernels always work on a table of boxes, and a state is a batch of one.
// Per RK3 substage the engine enqueues the three directional passes
// (x: explicit terms + RHS + x solve, y solve, z solve + update); with a
// non-null stream a whole step is captured once as a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
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

// live handles
std::mutex g_mu;
std::unordered_set<const void*> g_live;

void reg(const void* p)
{
    std::lock_guard<std::mutex> l(g_mu);
    g_live.insert(p);
}
bool live(const void* p)
{
    std::lock_guard<std::mutex> l(g_mu);
    return p && g_live.count(p);
}
void unreg(const void* p)
{
    std::lock_guard<std::mutex> l(g_mu);
    g_live.erase(p);
}

struct Engine {
    chp::Plan P;
    chd::BoxDesc* d_boxes = nullptr;
    void* C = nullptr;
    void* E = nullptr;
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
    const void* gkey[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
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
};

void free_engine(Engine& e)
{
    if (e.gexec) (void)hipGraphExecDestroy(e.gexec);
    for (auto& p : e.ev_pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (auto ev : e.ev_pool) (void)hipEventDestroy(ev);
    void* bufs[] = {e.C, e.E, e.qa, e.qb, e.d_partial, e.d_h3, e.d_mass, e.d_flags, e.d_boxes,
                    e.fu, e.fv, e.fw};
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
    HIP_TRY(hipMemcpy(e.d_boxes, e.P.boxes.data(), sizeof(chd::BoxDesc) * e.P.nbox,
                      hipMemcpyHostToDevice));
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
        if (p == 0)
            err = chk::launch_pass_x<T, A>(e.P.mi, e.P.ntask[0], e.P.x_threads, e.P.lds[0],
                                           e.stream, e.d_boxes, e.P.nbox, pa,
                                           e.C, u, v, w, e.E, e.qa, false);
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
                                              e.E, e.qa, true);
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

// One multiple-resolution transfer descriptor.
struct InterpData {
    int64_t nf[3];           // fine cells
    int64_t nc[3];           // coarse cells
    int prec = CH_FP64;
    hipStream_t stream = nullptr;
    // 1-D stencils per component (u, v, w) and axis (x, y, z)
    int* idx[3][3] = {};
    double* wt[3][3] = {};
    int64_t tn[3][3] = {};   // targets per component and axis
};

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
        const int64_t sx = ip->nc[0], sy = ip->nc[1];
        hipError_t err = chk::launch_interp<T>(st, src[c], sx, sy, ip->tn[c][0], ip->tn[c][1],
                                               ip->tn[c][2], ip->idx[c][0], ip->wt[c][0],
                                               ip->idx[c][1], ip->wt[c][1], ip->idx[c][2],
                                               ip->wt[c][2], dst[c]);
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
    const void* key[6] = {u, v, w, uc, vc, wc};
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
        for (int m = 0; m < 6 && same; ++m) same = key[m] == e.gkey[m];
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
            for (int m = 0; m < 6; ++m) e.gkey[m] = key[m];
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

// ---- multiple resolution: 1-D cubic Hermite stencils -----------------------
// Source points s[0..n) on an axis: periodic (period 1), or between walls at
// 0 and 1, continued evenly (cell-centred values) or oddly (face values that
// include both walls, s[0] = 0, s[n-1] = 1).
enum { SRC_PERIODIC = 0, SRC_EVEN = 1, SRC_ODD = 2 };

struct Src {
    std::vector<double> s;
    int kind;
    // coordinate, stored index and sign of extended point m
    double at(long m, long* idx, double* sgn) const
    {
        const long n = (long)s.size();
        *sgn = 1.0;
        if (kind == SRC_PERIODIC) {
            long q = m >= 0 ? m / n : -((-m + n - 1) / n);
            long r = m - q * n;
            *idx = r;
            return s[r] + (double)q;
        }
        if (kind == SRC_EVEN) {
            if (m < 0) { *idx = -1 - m; return -s[-1 - m]; }
            if (m >= n) { *idx = 2 * n - 1 - m; return 2.0 - s[2 * n - 1 - m]; }
            *idx = m;
            return s[m];
        }
        if (m < 0) { *idx = -m; *sgn = -1.0; return -s[-m]; }
        if (m >= n) { *idx = 2 * n - 2 - m; *sgn = -1.0; return 2.0 - s[2 * n - 2 - m]; }
        *idx = m;
        return s[m];
    }
};

void hermite(const Src& src, double t, int idx[4], double w[4])
{
    long id;
    double sg;
    long m = -2;
    while (src.at(m + 1, &id, &sg) <= t) ++m;   // s_m <= t < s_{m+1}
    double x[4], sgn[4];
    long ii[4];
    for (int p = 0; p < 4; ++p) x[p] = src.at(m - 1 + p, &ii[p], &sgn[p]);
    const double D = x[2] - x[1], u = (t - x[1]) / D;
    const double u2 = u * u, u3 = u2 * u;
    const double b00 = 2 * u3 - 3 * u2 + 1, b10 = u3 - 2 * u2 + u;
    const double b01 = -2 * u3 + 3 * u2, b11 = u3 - u2;
    const double g1 = D / (x[2] - x[0]), g2 = D / (x[3] - x[1]);
    const double ww[4] = {-b10 * g1, b00 - b11 * g2, b01 + b10 * g1, b11 * g2};
    for (int p = 0; p < 4; ++p) {
        idx[p] = (int)ii[p];
        w[p] = ww[p] * sgn[p];
    }
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
    if (ncx > 8192) return fail(CH_EUNSUPPORTED, "coarse x extent above 8192 (one row in LDS)");
    if (zf[0] != 0.0 || zf[ncz] != 1.0) return fail(CH_EINVAL, "zf must run from 0 to 1");
    for (int64_t k = 0; k < ncz; ++k)
        if (!(zf[k + 1] > zf[k])) return fail(CH_EINVAL, "zf must increase");
    ch_interp* ip = new (std::nothrow) ch_interp();
    if (!ip) return fail(CH_ENOMEM, "host allocation failed");
    InterpData& d = ip->d;
    d.nf[0] = fine->nx;
    d.nf[1] = fine->ny;
    d.nf[2] = fine->nz;
    d.nc[0] = ncx;
    d.nc[1] = ncy;
    d.nc[2] = ncz;
    d.prec = precision;
    Src cxf{{}, SRC_PERIODIC}, cxc{{}, SRC_PERIODIC}, cyf{{}, SRC_PERIODIC},
        cyc{{}, SRC_PERIODIC}, czc{{}, SRC_EVEN}, czf{{}, SRC_ODD};
    for (int64_t i = 0; i < ncx; ++i) {
        cxf.s.push_back((double)i / ncx);
        cxc.s.push_back((i + 0.5) / ncx);
    }
    for (int64_t j = 0; j < ncy; ++j) {
        cyf.s.push_back((double)j / ncy);
        cyc.s.push_back((j + 0.5) / ncy);
    }
    for (int64_t k = 0; k < ncz; ++k) czc.s.push_back(0.5 * (zf[k] + zf[k + 1]));
    for (int64_t k = 0; k <= ncz; ++k) czf.s.push_back(zf[k]);
    const int64_t nx = fine->nx, ny = fine->ny, nz = fine->nz;
    auto faces = [](int64_t n) {
        std::vector<double> t(n);
        for (int64_t i = 0; i < n; ++i) t[i] = (double)i / n;
        return t;
    };
    auto centres = [](int64_t n) {
        std::vector<double> t(n);
        for (int64_t i = 0; i < n; ++i) t[i] = (i + 0.5) / n;
        return t;
    };
    std::vector<double> zfaces(nz + 1);
    for (int64_t k = 0; k <= nz; ++k) zfaces[k] = (double)k / nz;
    // component u: x faces, y centres, z centres; v: x centres, y faces, z
    // centres; w: x centres, y centres, z faces
    const Src* srcs[3][3] = {{&cxf, &cyc, &czc}, {&cxc, &cyf, &czc}, {&cxc, &cyc, &czf}};
    const std::vector<double> tgts[3][3] = {{faces(nx), centres(ny), centres(nz)},
                                            {centres(nx), faces(ny), centres(nz)},
                                            {centres(nx), centres(ny), zfaces}};
    ch_status st = CH_OK;
    for (int c = 0; c < 3 && st == CH_OK; ++c)
        for (int a = 0; a < 3 && st == CH_OK; ++a) {
            const std::vector<double>& t = tgts[c][a];
            std::vector<int> idx(4 * t.size());
            std::vector<double> wt(4 * t.size());
            for (size_t q = 0; q < t.size(); ++q) hermite(*srcs[c][a], t[q], &idx[4 * q], &wt[4 * q]);
            d.tn[c][a] = (int64_t)t.size();
            if (hipMalloc(&d.idx[c][a], sizeof(int) * idx.size()) != hipSuccess ||
                hipMalloc(&d.wt[c][a], sizeof(double) * wt.size()) != hipSuccess) {
                st = fail(CH_ENOMEM, "cannot allocate interpolation tables");
                break;
            }
            if (hipMemcpy(d.idx[c][a], idx.data(), sizeof(int) * idx.size(),
                          hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(d.wt[c][a], wt.data(), sizeof(double) * wt.size(),
                          hipMemcpyHostToDevice) != hipSuccess)
                st = fail(CH_EHIP, "cannot upload interpolation tables");
        }
    if (st != CH_OK) {
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) {
                if (d.idx[c][a]) (void)hipFree(d.idx[c][a]);
                if (d.wt[c][a]) (void)hipFree(d.wt[c][a]);
            }
        delete ip;
        return st;
    }
    reg(ip);
    *out = ip;
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
    for (int c = 0; c < 3; ++c)
        for (int a = 0; a < 3; ++a) {
            if (ip->d.idx[c][a]) (void)hipFree(ip->d.idx[c][a]);
            if (ip->d.wt[c][a]) (void)hipFree(ip->d.wt[c][a]);
        }
    delete ip;
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
