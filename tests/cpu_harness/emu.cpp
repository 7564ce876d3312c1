// emu.cpp -- CPU harness for the device code of libch (test infrastructure).
//
// Runs the exact phase functions of the HIP kernels (ch_device.h) with the
// exact launch plan of the library (ch_plan.h) on the CPU: every work-group
// of every pass, every thread of a phase in turn, a barrier between phases.
// Built with AddressSanitizer and UBSan, with LDS buffers of exactly the
// planned size, it checks the kernels' indexing without a GPU.
//
// usage: emu PARAMS IN_DIR OUT_DIR
//   PARAMS: "nbox prec kappa eps solve x_rows seg_len waves z_chunk dt nsteps mode
//           x_general"
//           then per box "nx ny nz h Cn Pe bcx bcy bcz"; mode 0 is the
//           factorised implicit scheme, 1 the explicit 25-point scheme
//   IN_DIR/{C,u,v,w}.bin: packed float64 arrays (the library's layout)
//   OUT_DIR/C.bin: packed float64 result; OUT_DIR/mass.txt: per-box mass;
//   OUT_DIR/plan.txt: x_rows seg_cap chains tw_max acc64 ntask0..2 lds0..2 z_chunk xrow
//           nxl xrm0 xrm1 xrm2 nth0 nth1 nth2
//           (xrow: 0 general x program, 1 row program, 2 row program with
//           several rows in some task, 3 segmented program, 4 row program in
//           one launch per row mode; nxl: the row program's launches; xrm0 ..
//           xrm2: the row mode of each (of the single launch in xrm0): 0 one
//           row, 1 several rows with per-thread offsets, 2 several rows of
//           whole waves; nth0 .. nth2: the threads per work-group of each)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ch.h"
#include "../../paper_2105_01865_amd/csrc/ch_device.h"
#include "../../paper_2105_01865_amd/csrc/ch_plan.h"

static std::vector<double> read_bin(const std::string& path, size_t n)
{
    std::vector<double> v(n);
    FILE* f = fopen(path.c_str(), "rb");
    if (!f || fread(v.data(), sizeof(double), n, f) != n) {
        fprintf(stderr, "cannot read %s (%zu values)\n", path.c_str(), n);
        exit(2);
    }
    fclose(f);
    return v;
}

template <typename T>
static T* dev_copy(const std::vector<double>& v)
{
    // exact-size heap copy: AddressSanitizer flags any access past the end
    T* p = (T*)malloc(sizeof(T) * (v.size() ? v.size() : 1));
    for (size_t i = 0; i < v.size(); ++i) p[i] = T(v[i]);
    return p;
}

template <typename T, typename A, int MI, bool E25 = false>
static void run_x(chp::Plan& P, int k, T* C, T* E, T* qa, const T* u, const T* v, const T* w)
{
    const chd::BoxDesc* boxes = P.boxes.data();
    const chd::PassArgs pa = chp::pass_args(P, k, 0);
    chd::CpuExec ex{P.x_threads};
    std::vector<chd::XState<T, A, MI>> st(ex.nth);
    for (int task = 0; task < P.ntask[0]; ++task) {
        unsigned char* lds = (unsigned char*)malloc(P.lds[0]);
        memset(lds, 0xff, P.lds[0]);
        const int b = chd::find_box(boxes, P.nbox, chd::PASS_X, task);
        chd::pass_x_program<T, A, MI, E25>(ex, st.data(), boxes[b], pa, task, C, u, v, w, E, qa,
                                           lds);
        free(lds);
    }
}

// one task of the row x-pass program in row mode rm
template <typename T, typename A>
static void xrow_task(int rm, chd::CpuExec& ex, chd::XRowState<T, A>* st, const chd::BoxDesc& bd,
                      const chd::PassArgs& pa, int task, const T* C, const T* u, const T* v,
                      const T* w, T* E, T* qa, unsigned char* lds)
{
    if (rm == chd::XR_WAVE)
        chd::pass_x_row_program<T, A, chd::XR_WAVE>(ex, st, bd, pa, task, C, u, v, w, E, qa, lds);
    else if (rm == chd::XR_THREAD)
        chd::pass_x_row_program<T, A, chd::XR_THREAD>(ex, st, bd, pa, task, C, u, v, w, E, qa,
                                                      lds);
    else
        chd::pass_x_row_program<T, A, chd::XR_ONE>(ex, st, bd, pa, task, C, u, v, w, E, qa, lds);
}

// the row x-pass program
template <typename T, typename A>
static void run_xrow(chp::Plan& P, int k, T* C, T* E, T* qa, const T* u, const T* v, const T* w)
{
    const chd::BoxDesc* boxes = P.boxes.data();
    const chd::PassArgs pa = chp::pass_args(P, k, 0);
    chd::CpuExec ex{P.x_threads};
    std::vector<chd::XRowState<T, A>> st(ex.nth);
    if (P.nxl > 1) {
        // one launch per row mode, each with its own work-group size
        for (int g = 0; g < P.nxl; ++g) {
            const chd::BoxDesc* gb = P.xbox[g].data();
            const int nb = (int)P.xbox[g].size();
            chd::CpuExec exg{P.x_nth[g]};
            std::vector<chd::XRowState<T, A>> stg(exg.nth);
            for (int task = 0; task < P.x_ntask[g]; ++task) {
                unsigned char* lds = (unsigned char*)malloc(P.x_lds[g]);
                memset(lds, 0xff, P.x_lds[g]);
                const int b = chd::find_box(gb, nb, chd::PASS_X, task);
                xrow_task<T, A>(P.x_rm[g], exg, stg.data(), gb[b], pa, task, C, u, v, w, E, qa,
                                lds);
                free(lds);
            }
        }
        return;
    }
    for (int task = 0; task < P.ntask[0]; ++task) {
        unsigned char* lds = (unsigned char*)malloc(P.lds[0]);
        memset(lds, 0xff, P.lds[0]);
        const int b = chd::find_box(boxes, P.nbox, chd::PASS_X, task);
        xrow_task<T, A>(P.xrm, ex, st.data(), boxes[b], pa, task, C, u, v, w, E, qa, lds);
        free(lds);
    }
}

// the segmented x-pass program: E read from Ein, written to Eout
template <typename T, typename A>
static void run_xseg(chp::Plan& P, int k, T* C, const T* Ein, T* Eout, T* qa, const T* u,
                     const T* v, const T* w)
{
    const chd::BoxDesc* boxes = P.boxes.data();
    const chd::PassArgs pa = chp::pass_args(P, k, 0);
    chd::CpuExec ex{P.x_threads};
    std::vector<chd::XSegState<T, A>> st(ex.nth);
    for (int task = 0; task < P.ntask[0]; ++task) {
        unsigned char* lds = (unsigned char*)malloc(P.lds[0]);
        memset(lds, 0xff, P.lds[0]);
        const int b = chd::find_box(boxes, P.nbox, chd::PASS_X, task);
        chd::pass_x_seg_program<T, A>(ex, st.data(), boxes[b], pa, task, C, u, v, w, Ein, Eout,
                                      qa, lds);
        free(lds);
    }
}

template <typename T, typename A>
static void run(chp::Plan& P, T* C, T* E, T* qa, T* qb, const T* u, const T* v, const T* w,
                int nsteps, T* E2)
{
    const chd::BoxDesc* boxes = P.boxes.data();
    for (int s = 0; s < nsteps; ++s)
        for (int k = 0; k < 3; ++k) {
            // pass x
            if (P.xseg) run_xseg<T, A>(P, k, C, k == 2 ? E2 : E, k == 1 ? E2 : E, qa, u, v, w);
            else if (P.xrow) run_xrow<T, A>(P, k, C, E, qa, u, v, w);
            else if (P.mi == 1) run_x<T, A, 1>(P, k, C, E, qa, u, v, w);
            else run_x<T, A, 2>(P, k, C, E, qa, u, v, w);
            // passes y, z
            for (int pass = 1; pass <= 2; ++pass) {
                const chd::PassArgs pa = chp::pass_args(P, k, pass);
                const T* in = pass == 1 ? qa : qb;
                T* out = pass == 1 ? qb : C;
                chd::CpuExec ex{P.yz_threads};
                std::vector<chd::LineState<A>> st(ex.nth);
                for (int task = 0; task < P.ntask[pass]; ++task) {
                    unsigned char* lds = (unsigned char*)malloc(P.lds[pass]);
                    memset(lds, 0xff, P.lds[pass]);
                    const int b = chd::find_box(boxes, P.nbox, pass, task);
                    chd::pass_line_program<T, A>(ex, st.data(), boxes[b], pa, pass, task, in, out,
                                                 lds);
                    free(lds);
                }
            }
        }
}

template <typename T>
static std::vector<double> masses(const chp::Plan& P, const T* C)
{
    std::vector<double> out(P.nbox);
    for (int b = 0; b < P.nbox; ++b) {
        const chd::BoxDesc& bd = P.boxes[b];
        std::vector<double> partial(bd.nmblk);
        for (int blk = 0; blk < bd.nmblk; ++blk) {
            double sh[chd::MASS_THREADS];
            for (int tid = 0; tid < chd::MASS_THREADS; ++tid)
                sh[tid] = chd::mass_thread_sum<T>(tid, bd, blk, C);
            for (int s = chd::MASS_THREADS / 2; s > 0; s >>= 1)
                for (int tid = 0; tid < s; ++tid) sh[tid] += sh[tid + s];
            partial[blk] = sh[0];
        }
        double sh[chd::MASS_THREADS];
        for (int tid = 0; tid < chd::MASS_THREADS; ++tid) {
            double s = 0.0;
            for (int i = tid; i < bd.nmblk; i += chd::MASS_THREADS) s += partial[i];
            sh[tid] = s;
        }
        for (int s = chd::MASS_THREADS / 2; s > 0; s >>= 1)
            for (int tid = 0; tid < s; ++tid) sh[tid] += sh[tid + s];
        const double h = P.g[b].h;
        out[b] = sh[0] * (h * h * h);
    }
    return out;
}

// the explicit 25-point scheme: one x-pass program per substage, C + RHS
// into qa, which becomes C
template <typename T>
static void run_e25(chp::Plan& P, T*& C, T* E, T*& qa, const T* u, const T* v, const T* w,
                    int nsteps)
{
    for (int s = 0; s < nsteps; ++s)
        for (int k = 0; k < 3; ++k) {
            if (P.mi == 1) run_x<T, T, 1, true>(P, k, C, E, qa, u, v, w);
            else run_x<T, T, 2, true>(P, k, C, E, qa, u, v, w);
            std::swap(C, qa);
        }
}

template <typename T>
static int go(chp::Plan& P, const std::string& in, const std::string& out, int nsteps)
{
    std::vector<double> C0 = read_bin(in + "/C.bin", P.tot[0]);
    T* C = dev_copy<T>(C0);
    std::vector<double> zero(P.tot[0], 0.0);
    T* E = dev_copy<T>(zero);
    T* E2 = dev_copy<T>(zero);
    T* qa = dev_copy<T>(zero);
    T* qb = dev_copy<T>(zero);
    T* u = dev_copy<T>(read_bin(in + "/u.bin", P.tot[1]));
    T* v = dev_copy<T>(read_bin(in + "/v.bin", P.tot[2]));
    T* w = dev_copy<T>(read_bin(in + "/w.bin", P.tot[3]));
    if (P.e25) run_e25<T>(P, C, E, qa, u, v, w, nsteps);
    else if (P.prec == CH_FP64) run<T, T>(P, C, E, qa, qb, u, v, w, nsteps, E2);
    else if (P.acc64) run<T, double>(P, C, E, qa, qb, u, v, w, nsteps, E2);
    else run<T, float>(P, C, E, qa, qb, u, v, w, nsteps, E2);
    std::vector<double> res(P.tot[0]);
    for (int64_t i = 0; i < P.tot[0]; ++i) res[i] = double(C[i]);
    FILE* f = fopen((out + "/C.bin").c_str(), "wb");
    fwrite(res.data(), sizeof(double), res.size(), f);
    fclose(f);
    std::vector<double> m = masses<T>(P, C);
    f = fopen((out + "/mass.txt").c_str(), "w");
    for (double x : m) fprintf(f, "%.17g\n", x);
    fclose(f);
    f = fopen((out + "/plan.txt").c_str(), "w");
    fprintf(f, "%d %d %d %d %d %d %d %d %zu %zu %zu %d %d %d %d %d %d %d %d %d\n", P.x_rows,
            P.seg_cap,
            P.yz_threads, P.tw_max, P.acc64 ? 1 : 0, P.ntask[0], P.ntask[1], P.ntask[2], P.lds[0],
            P.lds[1], P.lds[2], P.zc,
            P.xseg ? 3 : P.nxl > 1 ? 4 : P.xrow ? (P.xrow_multi ? 2 : 1) : 0, P.nxl,
            P.nxl > 1 ? P.x_rm[0] : P.xrm, P.nxl > 1 ? P.x_rm[1] : -1,
            P.nxl > 2 ? P.x_rm[2] : -1, P.nxl > 1 ? P.x_nth[0] : P.x_threads,
            P.nxl > 1 ? P.x_nth[1] : -1, P.nxl > 2 ? P.x_nth[2] : -1);
    fclose(f);
    free(C); free(E); free(E2); free(qa); free(qb); free(u); free(v); free(w);
    return 0;
}

int main(int argc, char** argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: emu PARAMS IN_DIR OUT_DIR\n");
        return 2;
    }
    FILE* f = fopen(argv[1], "r");
    if (!f) return 2;
    int nbox, prec, solve, x_rows, seg, waves, zchunk, nsteps, mode, xgen;
    double kappa, eps, dt;
    if (fscanf(f, "%d %d %lf %lf %d %d %d %d %d %lf %d %d %d", &nbox, &prec, &kappa, &eps, &solve,
               &x_rows, &seg, &waves, &zchunk, &dt, &nsteps, &mode, &xgen) != 13)
        return 2;
    std::vector<ch_grid> g(nbox);
    std::vector<double> Cn(nbox), Pe(nbox);
    std::vector<ch_bc> bc(nbox);
    for (int b = 0; b < nbox; ++b) {
        long long nx, ny, nz;
        if (fscanf(f, "%lld %lld %lld %lf %lf %lf %d %d %d", &nx, &ny, &nz, &g[b].h, &Cn[b],
                   &Pe[b], &bc[b].x, &bc[b].y, &bc[b].z) != 9)
            return 2;
        g[b].nx = nx;
        g[b].ny = ny;
        g[b].nz = nz;
    }
    fclose(f);
    ch_opts o;
    chp::default_opts(&o);
    o.precision = prec;
    o.kappa = kappa;
    o.weno_eps = eps;
    o.solve_fp64 = solve;
    o.x_rows = x_rows;
    o.seg_len = seg;
    o.waves_yz = waves;
    o.z_chunk = zchunk;
    o.x_general = xgen;
    chp::Plan P;
    P.e25 = mode == 1;
    if (chp::plan_init(P, nbox, g.data(), Cn.data(), Pe.data(), nullptr, bc.data(), &o) != CH_OK ||
        chp::plan_dt(P, dt) != CH_OK) {
        fprintf(stderr, "plan failed: %s\n", P.err.c_str());
        return 3;
    }
    if (prec == CH_FP64) return go<double>(P, argv[2], argv[3], nsteps);
    return go<float>(P, argv[2], argv[3], nsteps);
}
