// ch_plan.h -- host-side planning of libch, free of any HIP call: the box
// table (layout of the packed fields, per-box constants), the coefficients
// of one time step dt (RK3 weights, the factorised line-solve recurrences
// and their warm-up lengths) and the launch configuration (tasks and LDS
// per pass).  The library and the CPU harness of the tests share it.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "../../include/ch.h"
#include "ch_device.h"

namespace chp {

// Low-storage RK3 constants (gamma_k, rho_k); alpha_k = gamma_k + rho_k.
constexpr double RK_G[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
constexpr double RK_R[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

constexpr size_t LDS_BUDGET = 64 * 1024;   // default per work-group
constexpr size_t LDS_HARD = 160 * 1024;    // gfx950 LDS per CU
// Waves per SIMD that the x kernel's registers allow (512 VGPRs per lane
// over 96 in single precision (the kernel is built for 5 waves), 140 in
// double, for one cell per thread).
// The x tile's LDS budget is the CU's LDS shared by the work-groups that
// many waves make room for.
constexpr int X_WAVES_F32 = 5;
constexpr int X_WAVES_F64 = 3;
// the same for the row program (78 VGPRs in single precision, 123 in double)
constexpr int XROW_WAVES_F32 = 6;
constexpr int XROW_WAVES_F64 = 4;
// work-group size the segmented x program aims at (segment + warm-ups + 1)
constexpr int SEG_THREADS = 256;
constexpr int X_MAX_THREADS = 1024;        // largest x-pass work-group

// cells of an x-pass plane tile per thread: one, two for very long x lines
inline int x_items(int nx) { return nx > X_MAX_THREADS ? 2 : 1; }

// Factor 1 + r (z - 2 + 1/z)^2 = c (1 + a1/z + a2/z^2)(1 + a1 z + a2 z^2)
// and choose the warm-up length: the smallest T for which the response of
// the forward-then-backward recurrences beyond T points stays below tol
// relative to the data.
inline bool recurrence(double r, double tol, double* a1, double* a2, double* ic, int* tw)
{
    if (!(r > 0.0)) {
        *a1 = 0.0;
        *a2 = 0.0;
        *ic = 1.0;
        *tw = 0;
        return true;
    }
    const std::complex<double> beta(2.0, 1.0 / std::sqrt(r));
    const std::complex<double> disc = std::sqrt(beta * beta - 4.0);
    std::complex<double> z = 0.5 * (beta + disc);
    if (std::abs(z) >= 1.0) z = 0.5 * (beta - disc);
    if (!(std::abs(z) < 1.0)) return false;
    *a1 = -2.0 * z.real();
    *a2 = std::norm(z);
    const double c = r / *a2;
    *ic = 1.0 / c;
    // impulse response h of 1 / (1 + a1 S^-1 + a2 S^-2)
    const int NMAX = 1 << 14;
    std::vector<double> h(NMAX);
    h[0] = 1.0;
    h[1] = -*a1;
    double sum = std::fabs(h[0]) + std::fabs(h[1]);
    for (int n = 2; n < NMAX; ++n) {
        h[n] = -*a1 * h[n - 1] - *a2 * h[n - 2];
        sum += std::fabs(h[n]);
    }
    // error <= 2 tail(T) sum / c: the forward truncation carried through the
    // backward filter, plus the backward truncation
    double tail = 0.0;
    int T = NMAX;
    for (int n = NMAX - 1; n >= 0; --n) {
        tail += std::fabs(h[n]);
        if (2.0 * tail * sum / c > tol) {
            T = n + 1;
            break;
        }
    }
    if (T >= 4096) return false;
    *tw = T;
    return true;
}

struct Plan {
    int nbox = 0;
    int prec = CH_FP64;
    ch_opts opt{};
    std::vector<ch_grid> g;
    std::vector<double> Cn, Pe;
    std::vector<ch_psi> psi;
    std::vector<ch_bc> bc;
    std::vector<chd::BoxDesc> boxes;
    int64_t tot[4] = {0, 0, 0, 0};   // packed lengths of C (and E, q), u, v, w
    int nmblk = 0;                   // mass blocks
    // for the current dt
    double dt = NAN;
    bool acc64 = true;
    bool e25 = false;   // explicit 25-point scheme: no line solves, one row per x task
    bool xrow = false;        // the x pass runs the one-cell-per-thread row program
    bool xrow_multi = false;  // ... with several rows in some task
    int xrm = 0;              // its row mode (chd::XR_ONE, XR_THREAD or XR_WAVE)
    bool xseg = false;        // the x pass runs the segmented program (long lines)
    // The x pass of a batch whose boxes take different row modes in the row
    // program runs as one launch per mode (nxl of them, at most 3: one row
    // per task, several with per-thread row offsets, several of whole
    // waves), each over a box table of its own whose x tasks are numbered
    // from 0 and with a work-group size of its own (the y and z passes keep
    // the whole table).
    int nxl = 1;
    std::vector<chd::BoxDesc> xbox[3];
    int x_ntask[3] = {0, 0, 0};
    size_t x_lds[3] = {0, 0, 0};
    int x_rm[3] = {0, 0, 0};    // row mode of each launch
    int x_nth[3] = {0, 0, 0};   // its threads per work-group
    std::vector<int> box_th, box_rm;   // each box's work-group size and row mode
    int tw_max = 0;
    int x_rows = 0, x_threads = 256, zc = 1, mi = 1, lanes = 32, yz_threads = 256, seg_cap = 0;
    int ntask[3] = {0, 0, 0};
    size_t lds[3] = {0, 0, 0};
    int nx_max = 0, seg_max[2] = {0, 0};
    std::string err;

    ch_status fail(ch_status st, const std::string& m)
    {
        err = m;
        return st;
    }
};

inline size_t esize(int prec) { return prec == CH_FP64 ? 8 : 4; }

inline void default_opts(ch_opts* o)
{
    *o = ch_opts{};
    o->precision = CH_FP64;
    o->kappa = 4.0;
    o->weno_eps = 1e-6;
    o->solve_fp64 = CH_SOLVE_AUTO;
    o->use_graph = 1;
}

inline ch_status plan_init(Plan& P, int nbox, const ch_grid* g, const double* Cn,
                           const double* Pe, const ch_psi* psi, const ch_bc* bc,
                           const ch_opts* opt)
{
    if (nbox < 1 || !g || !Cn || !Pe) return P.fail(CH_EINVAL, "null argument");
    ch_opts o;
    default_opts(&o);
    if (opt) o = *opt;
    if (o.precision != CH_FP64 && o.precision != CH_FP32)
        return P.fail(CH_EINVAL, "unknown precision");
    if (!(o.kappa >= 0.0) || !std::isfinite(o.kappa))
        return P.fail(CH_EINVAL, "kappa must be >= 0 and finite");
    if (!(o.weno_eps > 0.0) || !std::isfinite(o.weno_eps))
        return P.fail(CH_EINVAL, "weno_eps must be > 0 and finite");
    if (o.solve_fp64 < CH_SOLVE_AUTO || o.solve_fp64 > CH_SOLVE_NATIVE)
        return P.fail(CH_EINVAL, "unknown solve_fp64 mode");
    if (!(o.dt_hint >= 0.0) || !std::isfinite(o.dt_hint))
        return P.fail(CH_EINVAL, "dt_hint must be >= 0 and finite");
    if (o.x_general != 0 && o.x_general != 1) return P.fail(CH_EINVAL, "x_general must be 0 or 1");
    if (o.x_rows < 0 || o.x_rows > 64 || o.seg_len < 0 || o.waves_yz < 0 || o.waves_yz > 8 ||
        o.z_chunk < 0)
        return P.fail(CH_EINVAL, "launch options out of range");
    if (o.precision == CH_FP64 && o.solve_fp64 == CH_SOLVE_NATIVE) o.solve_fp64 = CH_SOLVE_FP64;
    P.nbox = nbox;
    P.prec = o.precision;
    P.opt = o;
    P.g.assign(g, g + nbox);
    P.Cn.assign(Cn, Cn + nbox);
    P.Pe.assign(Pe, Pe + nbox);
    const ch_psi dw = {{0.0, 0.5, -1.5, 1.0}};
    const ch_bc per = {CH_PERIODIC, CH_PERIODIC, CH_PERIODIC};
    P.psi.assign(nbox, dw);
    P.bc.assign(nbox, per);
    if (psi) P.psi.assign(psi, psi + nbox);
    if (bc) P.bc.assign(bc, bc + nbox);
    for (int b = 0; b < nbox; ++b) {
        const int64_t n[3] = {P.g[b].nx, P.g[b].ny, P.g[b].nz};
        const int bb[3] = {P.bc[b].x, P.bc[b].y, P.bc[b].z};
        for (int d = 0; d < 3; ++d) {
            if (!(n[d] == 1 || n[d] >= 8))
                return P.fail(CH_EINVAL, "box " + std::to_string(b) + ": axis " +
                                             std::to_string(d) + " has " + std::to_string(n[d]) +
                                             " cells; need 1 or at least 8");
            if (n[d] > (1 << 20)) return P.fail(CH_EINVAL, "axis too long");
            if (bb[d] != CH_PERIODIC && bb[d] != CH_NOFLUX)
                return P.fail(CH_EINVAL, "unknown boundary condition");
        }
        // byte offsets within one plane of a field (faces included) are
        // 32-bit in the kernels
        if ((double)(n[0] + 1) * (double)(n[1] + 1) * 8.0 >= 4294967296.0)
            return P.fail(CH_EINVAL, "a plane of the mesh is too large");
        if (!(P.g[b].h > 0.0) || !std::isfinite(P.g[b].h))
            return P.fail(CH_EINVAL, "h must be > 0 and finite");
        if (!(P.Cn[b] > 0.0) || !std::isfinite(P.Cn[b]))
            return P.fail(CH_EINVAL, "Cn must be > 0 and finite");
        if (!(P.Pe[b] > 0.0) || !std::isfinite(P.Pe[b]))
            return P.fail(CH_EINVAL, "Pe must be > 0 and finite");
        for (int m = 0; m < 4; ++m)
            if (!std::isfinite(P.psi[b].c[m])) return P.fail(CH_EINVAL, "psi must be finite");
    }
    P.boxes.assign(nbox, chd::BoxDesc{});
    int64_t off[4] = {0, 0, 0, 0};
    int64_t mblk = 0;
    for (int b = 0; b < nbox; ++b) {
        chd::BoxDesc& d = P.boxes[b];
        const ch_grid& gg = P.g[b];
        d.n[0] = (int)gg.nx;
        d.n[1] = (int)gg.ny;
        d.n[2] = (int)gg.nz;
        d.bc[0] = P.bc[b].x;
        d.bc[1] = P.bc[b].y;
        d.bc[2] = P.bc[b].z;
        for (int a = 0; a < 3; ++a) d.nf[a] = d.n[a] + (d.bc[a] == CH_NOFLUX ? 1 : 0);
        const int64_t cells = gg.nx * gg.ny * gg.nz;
        d.c_off = off[0];
        d.u_off = off[1];
        d.v_off = off[2];
        d.w_off = off[3];
        off[0] += cells;
        off[1] += (int64_t)d.nf[0] * gg.ny * gg.nz;
        off[2] += (int64_t)gg.nx * d.nf[1] * gg.nz;
        off[3] += (int64_t)gg.nx * gg.ny * d.nf[2];
        d.inv_h = 1.0 / gg.h;
        d.inv_h2 = 1.0 / (gg.h * gg.h);
        d.inv_pe = 1.0 / P.Pe[b];
        d.eps = o.weno_eps;
        for (int m = 0; m < 4; ++m) d.psi[m] = P.psi[b].c[m];
        d.mblk0 = (int)mblk;
        const int64_t nb = (cells + chd::MASS_BLOCK - 1) / chd::MASS_BLOCK;
        d.nmblk = (int)nb;
        mblk += nb;
        if (mblk > 2000000000LL) return P.fail(CH_EUNSUPPORTED, "batch too large");
    }
    for (int m = 0; m < 4; ++m) P.tot[m] = off[m];
    P.nmblk = (int)mblk;
    return CH_OK;
}

// Coefficients, warm-ups and launch configuration for the time step dt.
inline ch_status plan_dt(Plan& P, double dt)
{
    const double tol = P.prec == CH_FP64 ? std::ldexp(1.0, -58) : std::ldexp(1.0, -28);
    double rmax = 0.0;
    P.tw_max = 0;
    for (int b = 0; b < P.nbox; ++b) {
        chd::BoxDesc& d = P.boxes[b];
        const double h = P.g[b].h, Cn = P.Cn[b], Pe = P.Pe[b], kap = P.opt.kappa;
        // the per-direction fourth differences carry kappa; the explicit
        // 25-point operator is Cn^2/h^4 times the full discrete lap^2, and it
        // enters the explicit operator N with weight 1/Pe
        const double bih = (P.e25 ? 1.0 : kap) * Cn * Cn / (h * h * h * h);
        for (int k = 0; k < 3; ++k) {
            const double al = RK_G[k] + RK_R[k];
            d.gdt[k] = RK_G[k] * dt;
            d.rdt[k] = RK_R[k] * dt;
            d.bdt[k] = al * dt / Pe * bih;
            if (P.e25) {
                d.bdt[k] = bih / Pe;   // the biharmonic is an explicit term (gamma/rho)
                d.a1[k] = d.a2[k] = 0.0;
                d.ic[k] = 1.0;
                d.tw[k] = 0;
                continue;
            }
            const double r = 0.5 * al * dt / Pe * bih;
            rmax = std::max(rmax, r);
            int tw = 0;
            if (!recurrence(r, tol, &d.a1[k], &d.a2[k], &d.ic[k], &tw))
                return P.fail(CH_EUNSUPPORTED, "time step too large for the line solver");
            d.tw[k] = tw;
            P.tw_max = std::max(P.tw_max, tw);
        }
    }
    P.acc64 = P.prec == CH_FP64 || P.opt.solve_fp64 == CH_SOLVE_FP64 ||
              (P.opt.solve_fp64 == CH_SOLVE_AUTO && rmax > 0.25);
    const size_t sT = esize(P.prec), sA = P.acc64 ? 8 : 4;
    int nxm = 0, nym = 0, lmax = 0;
    int64_t cells = 0;
    for (int b = 0; b < P.nbox; ++b) {
        nxm = std::max(nxm, P.boxes[b].n[0]);
        nym = std::max(nym, P.boxes[b].n[1]);
        lmax = std::max({lmax, P.boxes[b].n[1], P.boxes[b].n[2]});
        cells += (int64_t)P.boxes[b].n[0] * P.boxes[b].n[1] * P.boxes[b].n[2];
    }
    P.nx_max = nxm;
    P.mi = x_items(nxm);
    const int xcap = X_MAX_THREADS * P.mi;
    if (nxm > xcap) return P.fail(CH_EUNSUPPORTED, "x extent too large");
    // ---- x pass: rows per task and planes per task
    // chunks per x line (fixed by the line: see line_chunk_len)
    auto nch_x = [](int n) { return std::max(1, std::min(n / 16, chd::X_CHAINS)); };
    // Lines longer than a work-group, periodic in x: the segmented program,
    // one row and one segment of at most SEG_THREADS - 2 tw_max - 1 cells per
    // task, segments of a line balanced.
    bool seg_ok = !P.e25 && P.opt.x_general == 0 && nxm > X_MAX_THREADS;
    for (int b = 0; b < P.nbox && seg_ok; ++b) seg_ok = P.boxes[b].bc[0] == CH_PERIODIC;
    P.xseg = false;
    if (seg_ok) {
        const int smax = SEG_THREADS - 2 * P.tw_max - 1;
        if (smax >= 64) {
            int S = 0;
            for (int b = 0; b < P.nbox; ++b) {
                chd::BoxDesc& d = P.boxes[b];
                d.nxs = (d.n[0] + smax - 1) / smax;
                d.xs = (d.n[0] + d.nxs - 1) / d.nxs;
                S = std::max(S, d.xs);
            }
            P.xseg = true;
            P.mi = 1;
            P.xrow = P.xrow_multi = false;
            P.x_rows = 1;
            P.x_threads = (chd::x_seg_threads(S, P.tw_max) + 63) / 64 * 64;
            int zlim = 64;
            for (int b = 0; b < P.nbox; ++b) {
                const int lim = P.x_threads / nch_x(P.boxes[b].xs);
                if (P.boxes[b].n[2] > lim) zlim = std::min(zlim, lim);
            }
            const int xwaves = sT == 4 ? XROW_WAVES_F32 : XROW_WAVES_F64;
            const int groups = std::max(1, xwaves / std::max(1, (P.x_threads / 64 + 3) / 4));
            const size_t xbudget = LDS_HARD / (size_t)groups;
            auto slds = [&](int zc) {
                return chd::x_seg_layout(S, zc, P.tw_max, (int)sT, (int)sA).total;
            };
            int zc = P.opt.z_chunk;
            if (zc == 0) {
                int64_t tasks = 0;
                for (int b = 0; b < P.nbox; ++b)
                    tasks += (int64_t)P.boxes[b].n[1] * P.boxes[b].n[2] * P.boxes[b].nxs;
                zc = (int)std::max<int64_t>(1, std::min<int64_t>(16, tasks / 2048));
                zc = std::min(zc, zlim);
                while (zc > 1 && slds(zc) > xbudget) --zc;
            }
            if (zc > zlim) return P.fail(CH_EINVAL, "z_chunk too large for this x segment");
            if (slds(zc) > LDS_HARD) return P.fail(CH_EUNSUPPORTED, "x tile too large for LDS");
            P.zc = zc;
        }
    }
    if (!P.xseg)
        for (int b = 0; b < P.nbox; ++b) P.boxes[b].xs = P.boxes[b].nxs = 0;
    if (!P.xseg) {
    // the one-row x program: every box's columns feed at most one halo
    // column each (nx >= 6), and every field of every box is under 4 GiB
    // (32-bit byte offsets from one buffer resource per field)
    bool row_ok = !P.e25 && P.opt.x_general == 0 && P.mi == 1;
    for (int b = 0; b < P.nbox && row_ok; ++b) {
        const chd::BoxDesc& d = P.boxes[b];
        const double n0 = d.n[0], n1 = d.n[1], n2 = d.n[2], s = (double)sT;
        row_ok = d.n[0] >= 6 && n0 * n1 * n2 * s < 4294967296.0 &&
                 (double)d.nf[0] * n1 * n2 * s < 4294967296.0 &&
                 n0 * d.nf[1] * n2 * s < 4294967296.0 && n0 * n1 * d.nf[2] * s < 4294967296.0;
    }
    auto threads_for = [&](int R) { return ((R * nxm + P.mi - 1) / P.mi + 63) / 64 * 64; };
    // rows per task of box b in the row program with `threads` threads: as
    // many as fill the group, so narrow boxes of an ensemble keep it busy
    // (an explicit z_chunk caps them so that every line of a task keeps its
    // chunks' threads)
    auto rows_row = [&](int b, int threads) {
        int r = std::min(P.boxes[b].n[1], threads / P.boxes[b].n[0]);
        if (P.opt.z_chunk > 0)
            r = std::min(r, threads / (std::min(P.opt.z_chunk, P.boxes[b].n[2]) *
                                       nch_x(P.boxes[b].n[0])));
        return std::max(1, r);
    };
    auto xlds = [&](int R, int zc) {
        if (row_ok) {
            size_t m = 0;
            const int th = threads_for(R);
            for (int b = 0; b < P.nbox; ++b)
                m = std::max(m, chd::x_row_layout(P.boxes[b].n[0], rows_row(b, th),
                                                  std::min(zc, P.boxes[b].n[2]), P.tw_max,
                                                  (int)sT, (int)sA).total);
            return m;
        }
        return chd::x_layout(nxm, R, zc, P.tw_max, (int)sT, (int)sA, P.e25).total;
    };
    const int xwaves = row_ok ? (sT == 4 ? XROW_WAVES_F32 : XROW_WAVES_F64)
                              : (sT == 4 ? X_WAVES_F32 : X_WAVES_F64);
    auto xbudget_th = [&](int threads) {
        const int per_simd = (threads / 64 + 3) / 4;   // waves of one group per SIMD
        const int groups = std::max(1, xwaves / std::max(1, per_simd));
        // measured on gfx950: five groups of the single-precision kernel
        // share a CU only with about 2 KB of LDS headroom each
        return LDS_HARD / (size_t)groups - (groups >= 5 ? 2048 : 0);
    };
    auto xbudget_for = [&](int R) { return xbudget_th(threads_for(R)); };
    int R = P.e25 ? 1 : P.opt.x_rows;   // the explicit mode reads rows y -+ 1 as halo
    if (R == 0) {
        // about 256 threads per work-group: one row of a long line, several
        // of short ones (each extra row also shares its y faces)
        R = std::max(1, std::min({256 / std::max(1, nxm), std::max(1, nym), 16}));
        while (R > 1 && (R * nxm > xcap || xlds(R, 1) > xbudget_for(R))) --R;
    }
    if (R * nxm > xcap) return P.fail(CH_EINVAL, "x_rows too large for the x extent");
    P.x_rows = R;
    P.x_threads = threads_for(R);
    if (P.x_threads > X_MAX_THREADS) return P.fail(CH_EINVAL, "x_rows too large for the x extent");
    P.xrow = row_ok;
    P.xrow_multi = false;
    // Rows per task of each box and the threads of its work-group.  One size
    // for all by default; for the automatic plan of a batch, each box takes
    // 192 or 256 threads, whichever leaves fewer of them idle (more rows on
    // a tie), and boxes of one row mode share a launch of the largest size
    // among them (a 128-cell line: two rows of 256 instead of one of 192).
    std::vector<int> brows(P.nbox), bth(P.nbox, P.x_threads), bmode(P.nbox, chd::XR_ONE);
    auto mode_of = [&](int b, int r) {
        return r == 1 ? chd::XR_ONE : P.boxes[b].n[0] % 64 == 0 ? chd::XR_WAVE : chd::XR_THREAD;
    };
    for (int b = 0; b < P.nbox; ++b) {
        brows[b] = row_ok ? rows_row(b, P.x_threads) : std::min(R, P.boxes[b].n[1]);
        bmode[b] = row_ok ? mode_of(b, brows[b]) : chd::XR_ONE;
    }
    if (row_ok && P.opt.x_rows == 0 && P.nbox > 1) {
        int gth[3] = {0, 0, 0};
        for (int b = 0; b < P.nbox; ++b) {
            const int nx = P.boxes[b].n[0];
            int T = (nx + 63) / 64 * 64;
            if (nx <= 256) {
                double best = -1.0;
                for (int c : {192, 256}) {
                    if (nx > c) continue;
                    const double use = (double)(rows_row(b, c) * nx) / c;
                    if (use >= best - 1e-12) {
                        best = use;
                        T = c;
                    }
                }
            }
            bth[b] = T;
            bmode[b] = mode_of(b, rows_row(b, T));
            gth[bmode[b]] = std::max(gth[bmode[b]], bmode[b] == chd::XR_ONE ? (nx + 63) / 64 * 64 : T);
        }
        P.x_threads = 0;
        for (int b = 0; b < P.nbox; ++b) {
            bth[b] = gth[bmode[b]];
            // a box of several rows keeps several with its launch's size
            brows[b] = bmode[b] == chd::XR_ONE ? 1 : rows_row(b, bth[b]);
            P.x_threads = std::max(P.x_threads, bth[b]);
        }
    }
    auto rows_of = [&](int b) { return brows[b]; };
    for (int b = 0; b < P.nbox && row_ok; ++b) P.xrow_multi = P.xrow_multi || rows_of(b) > 1;
    // LDS of box b's task at zc planes, and whether every box's fits the
    // groups per CU that its work-group size allows
    auto blds = [&](int b, int zc) {
        return row_ok ? chd::x_row_layout(P.boxes[b].n[0], rows_of(b),
                                          std::min(zc, P.boxes[b].n[2]), P.tw_max, (int)sT,
                                          (int)sA).total
                      : chd::x_layout(nxm, R, zc, P.tw_max, (int)sT, (int)sA, P.e25).total;
    };
    auto lds_fits = [&](int zc, bool hard) {
        for (int b = 0; b < P.nbox; ++b)
            if (blds(b, zc) > (hard ? LDS_HARD : xbudget_th(bth[b]))) return false;
        return true;
    };
    // planes per task: every line of a task needs its chunks' threads
    int zlim = 64;
    // (a box takes min(z_chunk, nz) planes, so one whose nz fits sets no limit)
    for (int b = 0; b < P.nbox && !P.e25; ++b) {
        const int lim = bth[b] / (rows_of(b) * nch_x(P.boxes[b].n[0]));
        if (P.boxes[b].n[2] > lim) zlim = std::min(zlim, lim);
    }
    int zc = P.opt.z_chunk;
    if (zc == 0) {
        // enough tasks to fill the chip a few times over, marching as far as
        // that allows (each task reloads 6 planes to start its march)
        const int64_t rows_total = cells / std::max(1, nxm);
        zc = (int)std::max<int64_t>(1, std::min<int64_t>(16, rows_total / R / 2048));
        zc = std::min(zc, zlim);
        while (zc > 1 && !lds_fits(zc, false)) --zc;
    }
    if (zc > zlim) return P.fail(CH_EINVAL, "z_chunk too large for this x extent");
    if (!lds_fits(zc, true)) return P.fail(CH_EUNSUPPORTED, "x tile too large for LDS");
    P.zc = zc;
    P.lds[0] = 0;
    for (int b = 0; b < P.nbox; ++b) {
        P.boxes[b].x_rows = rows_of(b);
        P.lds[0] = std::max(P.lds[0], blds(b, zc));
    }
    P.box_th = bth;
    P.box_rm = bmode;
    }   // !P.xseg
    // ---- y/z passes: lanes of 128 bytes, whole lines when they fit
    P.lanes = (int)(128 / sA);
    // at least YZ_CHAINS threads per lane column (see line_chunk)
    P.yz_threads = std::max(chd::YZ_CHAINS * P.lanes, 64 * (P.opt.waves_yz > 0 ? P.opt.waves_yz : 4));
    int seg = P.opt.seg_len > 0 ? P.opt.seg_len
                                : (int)(LDS_BUDGET / (P.lanes * sA)) - 2 * P.tw_max;
    if (seg < 16) seg = (int)(LDS_HARD / (P.lanes * sA)) - 2 * P.tw_max;
    if (seg < 1) return P.fail(CH_EUNSUPPORTED, "line-solve warm-up too long");
    if (P.opt.seg_len == 0 && seg < lmax) {
        const int nseg = (lmax + seg - 1) / seg;
        seg = (lmax + nseg - 1) / nseg;
    }
    seg = std::min(seg, lmax);
    P.seg_cap = seg;
    int64_t t0[3] = {0, 0, 0};
    P.seg_max[0] = P.seg_max[1] = 0;
    for (int b = 0; b < P.nbox; ++b) {
        chd::BoxDesc& d = P.boxes[b];
        const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
        if (P.xseg) d.x_rows = 1;
        d.zc = std::min(P.zc, nz);
        d.seg[0] = std::min(seg, ny);
        d.seg[1] = std::min(seg, nz);
        P.seg_max[0] = std::max(P.seg_max[0], d.seg[0]);
        P.seg_max[1] = std::max(P.seg_max[1], d.seg[1]);
        const int64_t nxb = (nx + P.lanes - 1) / P.lanes;
        const int64_t tt[3] = {(int64_t)((nz + d.zc - 1) / d.zc) * ((ny + d.x_rows - 1) / d.x_rows) *
                                   (P.xseg ? d.nxs : 1),
                               (int64_t)nz * nxb * ((ny + d.seg[0] - 1) / d.seg[0]),
                               (int64_t)ny * nxb * ((nz + d.seg[1] - 1) / d.seg[1])};
        for (int p = 0; p < 3; ++p) {
            if (t0[p] + tt[p] > 2000000000LL)
                return P.fail(CH_EUNSUPPORTED, "too many work-groups");
            d.task0[p] = (int)t0[p];
            d.ntask[p] = (int)tt[p];
            t0[p] += tt[p];
        }
    }
    for (int p = 0; p < 3; ++p) P.ntask[p] = (int)t0[p];
    // the row program's x launches: one per row mode among the boxes, each
    // with the largest work-group size of its boxes
    P.nxl = 1;
    P.xrm = chd::XR_ONE;
    if (P.xrow) {
        int present[3] = {0, 0, 0};
        for (int b = 0; b < P.nbox; ++b) present[P.box_rm[b]] = 1;
        P.xrm = present[chd::XR_THREAD] ? chd::XR_THREAD
              : present[chd::XR_WAVE] ? chd::XR_WAVE : chd::XR_ONE;
        const int modes = present[0] + present[1] + present[2];
        if (modes > 1 || P.nbox > 1) {
            int g = 0, gi[3] = {-1, -1, -1};
            for (int m = 0; m < 3; ++m)
                if (present[m]) gi[m] = g++;
            for (int k = 0; k < 3; ++k) {
                P.xbox[k].clear();
                P.x_ntask[k] = 0;
                P.x_lds[k] = 0;
                P.x_nth[k] = 0;
                P.x_rm[k] = chd::XR_ONE;
            }
            for (int m = 0; m < 3; ++m)
                if (gi[m] >= 0) P.x_rm[gi[m]] = m;
            for (int b = 0; b < P.nbox; ++b) {
                const int k = gi[P.box_rm[b]];
                chd::BoxDesc d = P.boxes[b];
                d.task0[0] = P.x_ntask[k];
                P.x_ntask[k] += d.ntask[0];
                P.x_lds[k] = std::max(P.x_lds[k], chd::x_row_layout(d.n[0], d.x_rows, d.zc,
                                                                    P.tw_max, (int)sT,
                                                                    (int)sA).total);
                P.x_nth[k] = std::max(P.x_nth[k], P.box_th[b]);
                P.xbox[k].push_back(d);
            }
            // one launch: the whole table (its tasks already numbered from 0)
            if (g > 1) P.nxl = g;
            else {
                P.xrm = P.x_rm[0];
                P.x_threads = P.x_nth[0];
            }
        }
    }
    if (P.xseg) {
        int S = 0;
        for (int b = 0; b < P.nbox; ++b) S = std::max(S, P.boxes[b].xs);
        P.lds[0] = chd::x_seg_layout(S, P.zc, P.tw_max, (int)sT, (int)sA).total;
    }
    P.lds[1] = (size_t)chd::line_tile_rows(P.seg_max[0] + 2 * P.tw_max) * P.lanes * sA;
    P.lds[2] = (size_t)chd::line_tile_rows(P.seg_max[1] + 2 * P.tw_max) * P.lanes * sA;
    for (int p = 1; p < 3; ++p)
        if (P.lds[p] > LDS_HARD) return P.fail(CH_EUNSUPPORTED, "line segment too long for LDS");
    P.dt = dt;
    return CH_OK;
}

inline chd::PassArgs pass_args(const Plan& P, int k, int pass)
{
    chd::PassArgs pa{};
    pa.k = k;
    pa.e_mode = k;       // substage 1 writes E, 2 reads and writes, 3 reads
    pa.lanes = P.lanes;
    pa.rmax = P.x_rows;
    pa.tw_max = P.tw_max;
    pa.nx_max = P.nx_max;
    pa.seg_max = pass == 2 ? P.seg_max[1] : P.seg_max[0];
    pa.zcmax = P.zc;
    return pa;
}

// ---- multiple resolution: 1-D transfer stencils (sec. 3.4) ---------------
// The transfer from one mesh to another is a tensor product of 1-D cubic
// Hermite interpolants with four source points per direction.  The slope at
// a source point is the chord slope through its two neighbours.  These
// helpers build, for every target coordinate, the four stored source
// indices and weights, once per transfer.
//
// A source axis lists its stored points s[0..n) in increasing order and
// says how the sequence continues beyond its ends:
//   AXIS_PERIODIC  period 1: the point n + j sits at s[j] + 1;
//   AXIS_MIRROR    cell-centred values between walls at 0 and 1, continued
//                  evenly: the image of s[j] across a wall carries +s[j]'s
//                  value;
//   AXIS_ANTI      face values that include both walls (s[0] = 0,
//                  s[n-1] = 1), continued oddly: the image of s[j] across a
//                  wall carries minus its value, and the walls themselves are
//                  not repeated.
enum { AXIS_PERIODIC = 0, AXIS_MIRROR = 1, AXIS_ANTI = 2 };

struct SrcAxis {
    std::vector<double> s;
    int kind = AXIS_PERIODIC;
};

// The source axis with `pad` images added on each side, written out as
// arrays: position, the stored point that carries the value, and the sign
// of that value.  Entry e is the point e - pad of the continued sequence.
struct PaddedAxis {
    int pad = 0;
    std::vector<double> x;
    std::vector<int> from;
    std::vector<double> sign;
};

inline PaddedAxis pad_axis(const SrcAxis& a, int pad)
{
    const int n = (int)a.s.size();
    PaddedAxis out;
    // images in order of increasing position: the left ones first
    std::vector<double> lx, rx, ls, rs;
    std::vector<int> lf, rf;
    // a reflected axis has as many images per side as stored points (less
    // the wall itself when it is stored)
    const int lim = a.kind == AXIS_PERIODIC ? pad : std::min(pad, a.kind == AXIS_MIRROR ? n : n - 1);
    out.pad = lim;
    for (int g = lim; g >= 1; --g) {
        // the g-th image left of s[0], and the g-th right of s[n-1]
        int jl, jr;
        double pl, pr, sg = 1.0;
        if (a.kind == AXIS_PERIODIC) {
            // whole periods away, for axes shorter than the padding too
            const int q = (g + n - 1) / n;
            jl = q * n - g;
            jr = g - 1 - (q - 1) * n;
            pl = a.s[jl] - q;
            pr = a.s[jr] + q;
        } else if (a.kind == AXIS_MIRROR) {
            jl = g - 1;                 // mirror of s[g-1] about 0
            jr = n - g;                 // mirror of s[n-g] about 1
            pl = -a.s[jl];
            pr = 2.0 - a.s[jr];
        } else {
            jl = g;                     // the wall point s[0] is its own image
            jr = n - 1 - g;
            pl = -a.s[jl];
            pr = 2.0 - a.s[jr];
            sg = -1.0;
        }
        lx.push_back(pl);
        lf.push_back(jl);
        ls.push_back(sg);
        rx.insert(rx.begin(), pr);
        rf.insert(rf.begin(), jr);
        rs.insert(rs.begin(), sg);
    }
    out.x = lx;
    out.from = lf;
    out.sign = ls;
    for (int j = 0; j < n; ++j) {
        out.x.push_back(a.s[j]);
        out.from.push_back(j);
        out.sign.push_back(1.0);
    }
    out.x.insert(out.x.end(), rx.begin(), rx.end());
    out.from.insert(out.from.end(), rf.begin(), rf.end());
    out.sign.insert(out.sign.end(), rs.begin(), rs.end());
    return out;
}

// Slope of the chord through (xa, fa) and (xb, fb).
inline double chord_slope(double xa, double fa, double xb, double fb)
{
    return (fb - fa) / (xb - xa);
}

// The cubic on [x1, x2] with values f1, f2 and slopes d1, d2 at its ends,
// evaluated at t in power form about x1 (Horner).
inline double hermite_cubic(double x1, double x2, double f1, double f2, double d1, double d2,
                            double t)
{
    const double L = x2 - x1, tau = (t - x1) / L;
    const double c1 = L * d1;
    const double c2 = 3.0 * (f2 - f1) - 2.0 * L * d1 - L * d2;
    const double c3 = 2.0 * (f1 - f2) + L * d1 + L * d2;
    return f1 + tau * (c1 + tau * (c2 + tau * c3));
}

// Stored indices and weights of the four source points that interpolate the
// axis at t (the reflection sign folded into the weight).  t must lie
// within the padded axis, between its second and its second-to-last point.
inline bool hermite_stencil(const PaddedAxis& P, double t, int idx[4], double w[4])
{
    // the interval [x[e], x[e+1]) holding t
    const auto it = std::upper_bound(P.x.begin(), P.x.end(), t);
    const long e = (long)(it - P.x.begin()) - 1;
    if (e < 1 || e + 2 >= (long)P.x.size()) return false;
    const double* x = &P.x[e - 1];
    // each weight is the interpolant of the data that is 1 at one of the
    // four points and 0 at the others
    for (int p = 0; p < 4; ++p) {
        double f[4] = {0.0, 0.0, 0.0, 0.0};
        f[p] = 1.0;
        const double d1 = chord_slope(x[0], f[0], x[2], f[2]);
        const double d2 = chord_slope(x[1], f[1], x[3], f[3]);
        w[p] = hermite_cubic(x[1], x[2], f[1], f[2], d1, d2, t) * P.sign[e - 1 + p];
        idx[p] = P.from[e - 1 + p];
    }
    return true;
}

// Stencils of every target coordinate: idx[4 q + p], w[4 q + p].
inline bool hermite_stencils(const SrcAxis& a, const std::vector<double>& tgt,
                             std::vector<int>* idx, std::vector<double>* w)
{
    if (a.s.size() < 2) return false;
    const PaddedAxis P = pad_axis(a, 3);
    idx->assign(4 * tgt.size(), 0);
    w->assign(4 * tgt.size(), 0.0);
    for (size_t q = 0; q < tgt.size(); ++q)
        if (!hermite_stencil(P, tgt[q], &(*idx)[4 * q], &(*w)[4 * q])) return false;
    return true;
}

}  // namespace chp
