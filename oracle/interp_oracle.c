/*
 * interp_oracle.c -- plain FP64 CPU oracle for the multiple-resolution
 * velocity transfer of sec. 3.4 (multi-resolution meshes for C and u):
 * the staggered velocity of a coarse mesh, uniform and periodic in x and y
 * and stretched between two walls in z, is interpolated to the faces of the
 * fine uniform mesh on which C lives, with a tensor-product cubic Hermite
 * interpolant using four source points per direction (64 in 3-D).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; it shares no code with the GPU
 * library.
 *
 * Readings where the paper is silent (listed in the design notes):
 *   - The Hermite slopes are the chord slopes through the two neighbours,
 *       m_i = (f_{i+1} - f_{i-1}) / (s_{i+1} - s_{i-1}),
 *     so the four points are s_{i-1} .. s_{i+2} around the target interval
 *     [s_i, s_{i+1}] (on a uniform axis this is the Catmull-Rom spline).
 *   - Beyond a wall the source is continued by reflection: tangential
 *     components (cell-centred in z) evenly, the wall-normal component
 *     (on z faces, zero on the walls) oddly.
 *   - oracle_interp_velocity is the plain form: u, v and w interpolated
 *     directly.  oracle_solenoidal_velocity is the paper's variant that
 *     keeps the fine field divergence-free (its readings are listed there).
 *   - oracle_project_c is the back-coupling of C: fine cell centres to
 *     coarse cell centres by the same interpolant (C continues evenly
 *     beyond the walls).
 *
 * Geometry (unit box):
 *   coarse: ncx x ncy cells of width 1/ncx, 1/ncy; ncz cells between the
 *           face positions zf[0] = 0 < zf[1] < ... < zf[ncz] = 1.
 *   fine:   nfx x nfy x nfz cells of width 1/nfx, 1/nfy, 1/nfz.
 *   u: x faces (periodic, n_x of them), y and z centres
 *   v: y faces (periodic), x and z centres
 *   w: z faces including both walls (n_z + 1), x and y centres
 * Arrays are x-fastest, [z][y][x].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

enum { AX_PERIODIC = 0, AX_WALL_EVEN = 1, AX_WALL_ODD = 2 };

typedef struct {
    int64_t n;          /* number of stored source points */
    const double* s;    /* their coordinates, increasing */
    double L;           /* period or wall-to-wall length (walls at 0 and L) */
    int kind;
} axis_t;

/* Extended source sequence: coordinate of point m and the stored index and
 * sign that give its value. */
static double ext_coord(const axis_t* a, int64_t m, int64_t* idx, double* sign)
{
    int64_t n = a->n;
    *sign = 1.0;
    if (a->kind == AX_PERIODIC) {
        int64_t q = m / n, r = m % n;
        if (r < 0) { r += n; q -= 1; }
        *idx = r;
        return a->s[r] + (double)q * a->L;
    }
    if (a->kind == AX_WALL_EVEN) {
        if (m < 0) { *idx = -1 - m; return -a->s[-1 - m]; }
        if (m >= n) { *idx = 2 * n - 1 - m; return 2.0 * a->L - a->s[2 * n - 1 - m]; }
        *idx = m;
        return a->s[m];
    }
    /* odd reflection about the walls, which are the points 0 and n-1 */
    if (m < 0) { *idx = -m; *sign = -1.0; return -a->s[-m]; }
    if (m >= n) { *idx = 2 * n - 2 - m; *sign = -1.0; return 2.0 * a->L - a->s[2 * n - 2 - m]; }
    *idx = m;
    return a->s[m];
}

/* Four source indices and weights (sign of the reflection folded in) that
 * interpolate the source at coordinate t. */
void oracle_hermite_stencil(int64_t n, const double* s, double L, int kind, double t,
                            int64_t idx[4], double wt[4])
{
    axis_t a = {n, s, L, kind};
    int64_t i0, dummy;
    double sg;
    /* largest m with s_m <= t */
    int64_t m = -2;
    while (ext_coord(&a, m + 1, &dummy, &sg) <= t) ++m;
    i0 = m;
    double x[4], sgn[4];
    int64_t id[4];
    for (int p = 0; p < 4; ++p) x[p] = ext_coord(&a, i0 - 1 + p, &id[p], &sgn[p]);
    /* x[1] <= t < x[2] */
    double D = x[2] - x[1];
    double tau = (t - x[1]) / D;
    double h00 = 2 * tau * tau * tau - 3 * tau * tau + 1;
    double h10 = tau * tau * tau - 2 * tau * tau + tau;
    double h01 = -2 * tau * tau * tau + 3 * tau * tau;
    double h11 = tau * tau * tau - tau * tau;
    /* f(t) = h00 f1 + h10 D m1 + h01 f2 + h11 D m2,
       m1 = (f2 - f0)/(x2 - x0),  m2 = (f3 - f1)/(x3 - x1) */
    double g1 = D / (x[2] - x[0]);
    double g2 = D / (x[3] - x[1]);
    double w[4];
    w[0] = -h10 * g1;
    w[1] = h00 - h11 * g2;
    w[2] = h01 + h10 * g1;
    w[3] = h11 * g2;
    for (int p = 0; p < 4; ++p) {
        idx[p] = id[p];
        wt[p] = w[p] * sgn[p];
    }
}

/* Interpolate one component: source axes ax[3] (x, y, z), source array src
 * of shape [ax[2].n][ax[1].n][ax[0].n]; targets t_x[nx], t_y[ny], t_z[nz];
 * output dst [nz][ny][nx]. */
static void interp_component(const axis_t ax[3], const double* src,
                             int64_t nx, const double* tx, int64_t ny, const double* ty,
                             int64_t nz, const double* tz, double* dst)
{
    /* the 1-D stencils of every target coordinate, computed once */
    int64_t* ix = malloc(sizeof(int64_t) * 4 * nx);
    int64_t* iy = malloc(sizeof(int64_t) * 4 * ny);
    int64_t* iz = malloc(sizeof(int64_t) * 4 * nz);
    double* wx = malloc(sizeof(double) * 4 * nx);
    double* wy = malloc(sizeof(double) * 4 * ny);
    double* wz = malloc(sizeof(double) * 4 * nz);
    for (int64_t i = 0; i < nx; ++i)
        oracle_hermite_stencil(ax[0].n, ax[0].s, ax[0].L, ax[0].kind, tx[i], ix + 4 * i, wx + 4 * i);
    for (int64_t j = 0; j < ny; ++j)
        oracle_hermite_stencil(ax[1].n, ax[1].s, ax[1].L, ax[1].kind, ty[j], iy + 4 * j, wy + 4 * j);
    for (int64_t k = 0; k < nz; ++k)
        oracle_hermite_stencil(ax[2].n, ax[2].s, ax[2].L, ax[2].kind, tz[k], iz + 4 * k, wz + 4 * k);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double acc = 0.0;
                for (int c = 0; c < 4; ++c)
                    for (int b = 0; b < 4; ++b)
                        for (int a = 0; a < 4; ++a)
                            acc += wz[4 * k + c] * wy[4 * j + b] * wx[4 * i + a]
                                 * src[(iz[4 * k + c] * ax[1].n + iy[4 * j + b]) * ax[0].n
                                       + ix[4 * i + a]];
                dst[(k * ny + j) * nx + i] = acc;
            }
    free(ix); free(iy); free(iz); free(wx); free(wy); free(wz);
}

/* Coarse staggered velocity -> fine staggered velocity (sec. 3.4). */
int oracle_interp_velocity(const int64_t nc[3], const double* zf, const double* uc,
                           const double* vc, const double* wc, const int64_t nf[3],
                           double* uf, double* vf, double* wf)
{
    int64_t ncx = nc[0], ncy = nc[1], ncz = nc[2];
    int64_t nfx = nf[0], nfy = nf[1], nfz = nf[2];
    double* cxf = malloc(sizeof(double) * ncx);   /* coarse x faces  */
    double* cxc = malloc(sizeof(double) * ncx);   /* coarse x centres */
    double* cyf = malloc(sizeof(double) * ncy);
    double* cyc = malloc(sizeof(double) * ncy);
    double* czc = malloc(sizeof(double) * ncz);   /* coarse z centres */
    double* fxf = malloc(sizeof(double) * nfx);
    double* fxc = malloc(sizeof(double) * nfx);
    double* fyf = malloc(sizeof(double) * nfy);
    double* fyc = malloc(sizeof(double) * nfy);
    double* fzf = malloc(sizeof(double) * (nfz + 1));
    double* fzc = malloc(sizeof(double) * nfz);
    if (!cxf || !cxc || !cyf || !cyc || !czc || !fxf || !fxc || !fyf || !fyc || !fzf || !fzc)
        return -1;
    for (int64_t i = 0; i < ncx; ++i) { cxf[i] = (double)i / ncx; cxc[i] = (i + 0.5) / ncx; }
    for (int64_t j = 0; j < ncy; ++j) { cyf[j] = (double)j / ncy; cyc[j] = (j + 0.5) / ncy; }
    for (int64_t k = 0; k < ncz; ++k) czc[k] = 0.5 * (zf[k] + zf[k + 1]);
    for (int64_t i = 0; i < nfx; ++i) { fxf[i] = (double)i / nfx; fxc[i] = (i + 0.5) / nfx; }
    for (int64_t j = 0; j < nfy; ++j) { fyf[j] = (double)j / nfy; fyc[j] = (j + 0.5) / nfy; }
    for (int64_t k = 0; k <= nfz; ++k) fzf[k] = (double)k / nfz;
    for (int64_t k = 0; k < nfz; ++k) fzc[k] = (k + 0.5) / nfz;

    axis_t au[3] = {{ncx, cxf, 1.0, AX_PERIODIC}, {ncy, cyc, 1.0, AX_PERIODIC},
                    {ncz, czc, 1.0, AX_WALL_EVEN}};
    axis_t av[3] = {{ncx, cxc, 1.0, AX_PERIODIC}, {ncy, cyf, 1.0, AX_PERIODIC},
                    {ncz, czc, 1.0, AX_WALL_EVEN}};
    axis_t aw[3] = {{ncx, cxc, 1.0, AX_PERIODIC}, {ncy, cyc, 1.0, AX_PERIODIC},
                    {ncz + 1, zf, 1.0, AX_WALL_ODD}};
    interp_component(au, uc, nfx, fxf, nfy, fyc, nfz, fzc, uf);
    interp_component(av, vc, nfx, fxc, nfy, fyf, nfz, fzc, vf);
    interp_component(aw, wc, nfx, fxc, nfy, fyc, nfz + 1, fzf, wf);
    free(cxf); free(cxc); free(cyf); free(cyc); free(czc);
    free(fxf); free(fxc); free(fyf); free(fyc); free(fzf); free(fzc);
    return 0;
}

/* Coordinates of the coarse and fine meshes (see the header comment). */
typedef struct {
    int64_t ncx, ncy, ncz, nfx, nfy, nfz;
    double *cxf, *cxc, *cyf, *cyc, *czc, *fxf, *fxc, *fyf, *fyc, *fzf, *fzc;
    const double* zf;
} meshes_t;

static void meshes_free(meshes_t* m)
{
    free(m->cxf); free(m->cxc); free(m->cyf); free(m->cyc); free(m->czc);
    free(m->fxf); free(m->fxc); free(m->fyf); free(m->fyc); free(m->fzf); free(m->fzc);
}

static int meshes_init(meshes_t* m, const int64_t nc[3], const double* zf, const int64_t nf[3])
{
    m->ncx = nc[0]; m->ncy = nc[1]; m->ncz = nc[2];
    m->nfx = nf[0]; m->nfy = nf[1]; m->nfz = nf[2];
    m->zf = zf;
    m->cxf = malloc(sizeof(double) * m->ncx); m->cxc = malloc(sizeof(double) * m->ncx);
    m->cyf = malloc(sizeof(double) * m->ncy); m->cyc = malloc(sizeof(double) * m->ncy);
    m->czc = malloc(sizeof(double) * m->ncz);
    m->fxf = malloc(sizeof(double) * m->nfx); m->fxc = malloc(sizeof(double) * m->nfx);
    m->fyf = malloc(sizeof(double) * m->nfy); m->fyc = malloc(sizeof(double) * m->nfy);
    m->fzf = malloc(sizeof(double) * (m->nfz + 1)); m->fzc = malloc(sizeof(double) * m->nfz);
    if (!m->cxf || !m->cxc || !m->cyf || !m->cyc || !m->czc || !m->fxf || !m->fxc || !m->fyf ||
        !m->fyc || !m->fzf || !m->fzc) {
        meshes_free(m);
        return -1;
    }
    for (int64_t i = 0; i < m->ncx; ++i) { m->cxf[i] = (double)i / m->ncx; m->cxc[i] = (i + 0.5) / m->ncx; }
    for (int64_t j = 0; j < m->ncy; ++j) { m->cyf[j] = (double)j / m->ncy; m->cyc[j] = (j + 0.5) / m->ncy; }
    for (int64_t k = 0; k < m->ncz; ++k) m->czc[k] = 0.5 * (zf[k] + zf[k + 1]);
    for (int64_t i = 0; i < m->nfx; ++i) { m->fxf[i] = (double)i / m->nfx; m->fxc[i] = (i + 0.5) / m->nfx; }
    for (int64_t j = 0; j < m->nfy; ++j) { m->fyf[j] = (double)j / m->nfy; m->fyc[j] = (j + 0.5) / m->nfy; }
    for (int64_t k = 0; k <= m->nfz; ++k) m->fzf[k] = (double)k / m->nfz;
    for (int64_t k = 0; k < m->nfz; ++k) m->fzc[k] = (k + 0.5) / m->nfz;
    return 0;
}

/* Solenoidal coarse-to-fine transfer (sec. 3.4): instead of the velocity,
 * its normal gradients are interpolated, and each fine component is then
 * integrated along its own direction from a reference plane.  Readings where
 * the paper is brief:
 *   - The normal gradients are the coarse cell-centred differences
 *       gx = (u[i+1] - u[i]) ncx,  gy = (v[j+1] - v[j]) ncy,
 *       gz = (w[k+1] - w[k]) / (zf[k+1] - zf[k]),
 *     and all three go to the fine cell centres through one and the same
 *     interpolant (cell-centred source in every direction, even continuation
 *     beyond the walls), so the interpolated gradients add up to the
 *     interpolated coarse divergence.
 *   - The reference planes are the low domain boundaries: u on the fine
 *     x face 0 and v on the fine y face 0, interpolated from the coarse
 *     velocity like the plain transfer does; w on the bottom wall is zero.
 *   - Integration runs upward from the reference plane,
 *       u[i] = u[0] + hx sum_{i' < i} Gx[i'],  i = 1 .. nfx - 1,
 *     and likewise for v along y and w along z (w[k], k = 1 .. nfz - 1);
 *     the top wall keeps w = 0.  The fine divergence is then the
 *     interpolated coarse divergence in every cell but the last one of each
 *     line, where the line's closure sum hx sum_{all i'} Gx[i'] (zero for a
 *     periodic line whose coarse cells all carry the same total weight) is
 *     left over.  resid[0..2] receive the largest |closure sum| over the
 *     x, y and z lines (velocity units).
 */
int oracle_solenoidal_velocity(const int64_t nc[3], const double* zf, const double* uc,
                               const double* vc, const double* wc, const int64_t nf[3],
                               double* uf, double* vf, double* wf, double resid[3])
{
    meshes_t m;
    if (meshes_init(&m, nc, zf, nf)) return -1;
    const int64_t ncx = m.ncx, ncy = m.ncy, ncz = m.ncz, nfx = m.nfx, nfy = m.nfy, nfz = m.nfz;
    const int64_t ncell = ncx * ncy * ncz, nfine = nfx * nfy * nfz;
    double* g = malloc(sizeof(double) * ncell);
    double* G = malloc(sizeof(double) * nfine);
    double* ref = malloc(sizeof(double) * (nfx > nfy ? nfx : nfy) * nfz);
    double* zero1 = malloc(sizeof(double));
    if (!g || !G || !ref || !zero1) {
        free(g); free(G); free(ref); free(zero1); meshes_free(&m);
        return -1;
    }
    zero1[0] = 0.0;
    axis_t ac[3] = {{ncx, m.cxc, 1.0, AX_PERIODIC}, {ncy, m.cyc, 1.0, AX_PERIODIC},
                    {ncz, m.czc, 1.0, AX_WALL_EVEN}};
    const double hx = 1.0 / nfx, hy = 1.0 / nfy, hz = 1.0 / nfz;
    for (int d = 0; d < 3; ++d) resid[d] = 0.0;

    /* u: gradient along x, reference plane x = 0, integrate along x */
    for (int64_t k = 0; k < ncz; ++k)
        for (int64_t j = 0; j < ncy; ++j)
            for (int64_t i = 0; i < ncx; ++i) {
                const int64_t r = (k * ncy + j) * ncx;
                g[r + i] = (uc[r + (i + 1) % ncx] - uc[r + i]) * ncx;
            }
    interp_component(ac, g, nfx, m.fxc, nfy, m.fyc, nfz, m.fzc, G);
    {
        axis_t au[3] = {{ncx, m.cxf, 1.0, AX_PERIODIC}, {ncy, m.cyc, 1.0, AX_PERIODIC},
                        {ncz, m.czc, 1.0, AX_WALL_EVEN}};
        interp_component(au, uc, 1, zero1, nfy, m.fyc, nfz, m.fzc, ref);   /* [nfz][nfy] */
    }
    for (int64_t k = 0; k < nfz; ++k)
        for (int64_t j = 0; j < nfy; ++j) {
            const int64_t r = (k * nfy + j) * nfx;
            double acc = 0.0;
            for (int64_t i = 0; i < nfx; ++i) {
                uf[r + i] = ref[k * nfy + j] + hx * acc;
                acc += G[r + i];
            }
            if (fabs(hx * acc) > resid[0]) resid[0] = fabs(hx * acc);
        }

    /* v: gradient along y, reference plane y = 0, integrate along y */
    for (int64_t k = 0; k < ncz; ++k)
        for (int64_t j = 0; j < ncy; ++j)
            for (int64_t i = 0; i < ncx; ++i)
                g[(k * ncy + j) * ncx + i] =
                    (vc[(k * ncy + (j + 1) % ncy) * ncx + i] - vc[(k * ncy + j) * ncx + i]) * ncy;
    interp_component(ac, g, nfx, m.fxc, nfy, m.fyc, nfz, m.fzc, G);
    {
        axis_t av[3] = {{ncx, m.cxc, 1.0, AX_PERIODIC}, {ncy, m.cyf, 1.0, AX_PERIODIC},
                        {ncz, m.czc, 1.0, AX_WALL_EVEN}};
        interp_component(av, vc, nfx, m.fxc, 1, zero1, nfz, m.fzc, ref);   /* [nfz][nfx] */
    }
    for (int64_t k = 0; k < nfz; ++k)
        for (int64_t i = 0; i < nfx; ++i) {
            double acc = 0.0;
            for (int64_t j = 0; j < nfy; ++j) {
                const int64_t e = (k * nfy + j) * nfx + i;
                vf[e] = ref[k * nfx + i] + hy * acc;
                acc += G[e];
            }
            if (fabs(hy * acc) > resid[1]) resid[1] = fabs(hy * acc);
        }

    /* w: gradient along z, zero on the bottom wall, integrate along z; the
       top wall stays zero */
    for (int64_t k = 0; k < ncz; ++k)
        for (int64_t j = 0; j < ncy; ++j)
            for (int64_t i = 0; i < ncx; ++i)
                g[(k * ncy + j) * ncx + i] =
                    (wc[((k + 1) * ncy + j) * ncx + i] - wc[(k * ncy + j) * ncx + i])
                    / (zf[k + 1] - zf[k]);
    interp_component(ac, g, nfx, m.fxc, nfy, m.fyc, nfz, m.fzc, G);
    for (int64_t j = 0; j < nfy; ++j)
        for (int64_t i = 0; i < nfx; ++i) {
            double acc = 0.0;
            for (int64_t k = 0; k < nfz; ++k) {
                const int64_t e = (k * nfy + j) * nfx + i;
                wf[e] = hz * acc;
                acc += G[e];
            }
            wf[(nfz * nfy + j) * nfx + i] = 0.0;
            if (fabs(hz * acc) > resid[2]) resid[2] = fabs(hz * acc);
        }
    free(g); free(G); free(ref); free(zero1);
    meshes_free(&m);
    return 0;
}

/* Back-coupling of C (sec. 3.4): the fine cell-centred field interpolated to
 * the coarse cell centres (x, y periodic; beyond the walls C continues
 * evenly).  Cf [nfz][nfy][nfx] -> Cc [ncz][ncy][ncx]. */
int oracle_project_c(const int64_t nf[3], const double* Cf, const int64_t nc[3],
                     const double* zf, double* Cc)
{
    meshes_t m;
    if (meshes_init(&m, nc, zf, nf)) return -1;
    axis_t af[3] = {{m.nfx, m.fxc, 1.0, AX_PERIODIC}, {m.nfy, m.fyc, 1.0, AX_PERIODIC},
                    {m.nfz, m.fzc, 1.0, AX_WALL_EVEN}};
    interp_component(af, Cf, m.ncx, m.cxc, m.ncy, m.cyc, m.ncz, m.czc, Cc);
    meshes_free(&m);
    return 0;
}
