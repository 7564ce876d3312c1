/*
 * ch_oracle.c -- plain FP64 CPU oracle for the Cahn-Hilliard update of
 * Liu, Ng, Chong, Lohse & Verzicco, "An efficient phase-field method for
 * turbulent multiphase flows" (arXiv 2105.01865).
 *
 * TEST INFRASTRUCTURE.  This file is the slow, obviously correct reference
 * that the GPU library is checked against.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header, table or helper with the GPU library: every function below
 * is written directly from the paper's equations, in the paper's order, in
 * double precision, with plain loops (OpenMP only splits the outermost loop
 * over independent cells or lines).
 *
 * What it computes (sec. 2.1 and sec. 3 of the paper):
 *
 *   dC/dt + div(u C) = (1/Pe) [ -Cn^2 lap^2 C + lap psi'(C) ]       (eq-ch)
 *
 *   - psi'(C) is a cubic  p0 + p1 C + p2 C^2 + p3 C^3; the paper's double
 *     well psi = C^2 (C-1)^2 / 4 gives (0, 0.5, -1.5, 1)          (sec. 1, eq-ch)
 *   - C at cell centres of a uniform mesh of spacing h, u at the cell faces
 *     (staggered mesh, sec. 3)
 *   - advection: fifth-order WENO face values, upwinded by the face velocity,
 *     conservative flux form (sec. 3)
 *   - lap psi'(C): central second-order 7-point Laplacian (sec. 3)
 *   - the biharmonic term with the new scheme: per direction d,
 *       A_d C = kappa Cn^2 / h^4 (C_{-2} - 4 C_{-1} + 6 C - 4 C_{+1} + C_{+2})
 *     with kappa = 4 in 3-D as printed in eq-a3d (kappa = 2 reproduces the
 *     2-D eq-a2d)
 *   - time: low-storage RK3 with Crank-Nicolson on the biharmonic term, in
 *     delta form (eq-re) with the approximate factorisation (eq-fac) into
 *     three directional pentadiagonal solves (eq-fac-1 .. eq-fac-3).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - RK3 constants gamma = (8/15, 5/12, 3/4), rho = (0, -17/60, -5/12),
 *     alpha = gamma + rho; within substage k the CN part uses alpha_k dt.
 *   - WENO5 is the Jiang-Shu point-value construction with eps = 1e-6 and
 *     power 2; a face takes the left-biased stencil when its velocity is
 *     >= 0 and the mirrored one otherwise.
 *   - Boundary rows: periodic (cyclic) or no-flux (even reflection of C over
 *     the wall, zero normal velocity on the wall faces).
 *   - No mass correction is applied (its reference is not available).
 *
 * Layout: every field is x-fastest, index (k*ny + j)*nx + i.  The face
 * velocity along axis d has n_d faces when d is periodic (face n_d is face 0)
 * and n_d + 1 faces when d is no-flux; face i is the low face of cell i.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PERIODIC 0
#define ORC_NOFLUX 1

/* ------------------------------------------------------------------------ */
/* Boundary handling: map an index that may lie outside [0, n) onto the     */
/* stored cell that holds its value.                                        */
/* Periodic: wrap.  No-flux: even reflection about the wall faces, so that  */
/* C[-1-m] = C[m] and C[n+m] = C[n-1-m] (a reflection of period 2n).        */
/* ------------------------------------------------------------------------ */
static int64_t ghost(int64_t i, int64_t n, int bc)
{
    if (bc == ORC_PERIODIC) {
        int64_t m = i % n;
        return m < 0 ? m + n : m;
    }
    int64_t p = 2 * n;
    int64_t m = i % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

typedef struct {
    int64_t n[3];   /* nx, ny, nz */
    int bc[3];
} grid_t;

static int64_t cell(const grid_t* g, int64_t i, int64_t j, int64_t k)
{
    return (k * g->n[1] + j) * g->n[0] + i;
}

/* C at cell (i,j,k) shifted by m cells along axis d, with ghosts. */
static double c_at(const grid_t* g, const double* C, int64_t i, int64_t j, int64_t k,
                   int d, int64_t m)
{
    int64_t p[3] = {i, j, k};
    p[d] = ghost(p[d] + m, g->n[d], g->bc[d]);
    return C[cell(g, p[0], p[1], p[2])];
}

/* Number of faces stored along axis d. */
static int64_t nfaces(const grid_t* g, int d)
{
    return g->bc[d] == ORC_PERIODIC ? g->n[d] : g->n[d] + 1;
}

/* Velocity on face f (0 <= f <= n_d) along axis d of the row through
 * (i,j,k); the other two indices select the row. */
static double face_vel(const grid_t* g, const double* u, int d, int64_t f,
                       int64_t i, int64_t j, int64_t k)
{
    int64_t nf = nfaces(g, d);
    if (g->bc[d] == ORC_PERIODIC) f = ghost(f, g->n[d], ORC_PERIODIC);
    int64_t p[3] = {i, j, k};
    p[d] = f;
    int64_t dims[3] = {g->n[0], g->n[1], g->n[2]};
    dims[d] = nf;
    return u[(p[2] * dims[1] + p[1]) * dims[0] + p[0]];
}

/* ------------------------------------------------------------------------ */
/* psi'(C) as a cubic (eq-ch-d / eq-ch).                                    */
/* ------------------------------------------------------------------------ */
double oracle_psi_prime(double C, const double psi[4])
{
    return psi[0] + psi[1] * C + psi[2] * C * C + psi[3] * C * C * C;
}

/* ------------------------------------------------------------------------ */
/* Fifth-order WENO reconstruction (Jiang-Shu, point values) of the value    */
/* at the face between c and d from the five values a..e, upwind side a.    */
/* ------------------------------------------------------------------------ */
double oracle_weno5(double a, double b, double c, double d, double e, double eps)
{
    /* three third-order candidate reconstructions */
    double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
    double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
    /* smoothness indicators */
    double s0 = 13.0 / 12.0 * (a - 2.0 * b + c) * (a - 2.0 * b + c)
              + 0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
    double s1 = 13.0 / 12.0 * (b - 2.0 * c + d) * (b - 2.0 * c + d)
              + 0.25 * (b - d) * (b - d);
    double s2 = 13.0 / 12.0 * (c - 2.0 * d + e) * (c - 2.0 * d + e)
              + 0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);
    /* nonlinear weights from the optimal linear weights 1/10, 6/10, 3/10 */
    double w0 = 0.1 / ((eps + s0) * (eps + s0));
    double w1 = 0.6 / ((eps + s1) * (eps + s1));
    double w2 = 0.3 / ((eps + s2) * (eps + s2));
    return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

/* Upwinded WENO value of C on face f (between cells f-1 and f) along d. */
static double face_value(const grid_t* g, const double* C, int d, int64_t f,
                         int64_t i, int64_t j, int64_t k, double U, double eps)
{
    /* (i,j,k) with index d replaced by the cell f: offsets are relative to f */
    int64_t p[3] = {i, j, k};
    p[d] = 0;
    double v[6]; /* C at cells f-3 .. f+2 */
    for (int m = -3; m <= 2; ++m) {
        int64_t q[3] = {p[0], p[1], p[2]};
        q[d] = ghost(f + m, g->n[d], g->bc[d]);
        v[m + 3] = C[cell(g, q[0], q[1], q[2])];
    }
    if (U >= 0.0) return oracle_weno5(v[0], v[1], v[2], v[3], v[4], eps);
    return oracle_weno5(v[5], v[4], v[3], v[2], v[1], eps);
}

/* ------------------------------------------------------------------------ */
/* div(u C) with face fluxes F = U * C_face (conservative form).            */
/* ------------------------------------------------------------------------ */
void oracle_advection(const int64_t n[3], const int bc[3], double h, double eps,
                      const double* C, const double* u, const double* v,
                      const double* w, double* adv)
{
    grid_t g = {{n[0], n[1], n[2]}, {bc[0], bc[1], bc[2]}};
    const double* vel[3] = {u, v, w};
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n[2]; ++k)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                int64_t idx[3] = {i, j, k};
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    int64_t lo = idx[d], hi = idx[d] + 1;
                    double Ulo = face_vel(&g, vel[d], d, lo, i, j, k);
                    double Uhi = face_vel(&g, vel[d], d, hi, i, j, k);
                    double Flo = Ulo * face_value(&g, C, d, lo, i, j, k, Ulo, eps);
                    double Fhi = Uhi * face_value(&g, C, d, hi, i, j, k, Uhi, eps);
                    s += (Fhi - Flo) / h;
                }
                adv[cell(&g, i, j, k)] = s;
            }
}

/* ------------------------------------------------------------------------ */
/* lap psi'(C), central 7-point Laplacian of the bulk potential.            */
/* ------------------------------------------------------------------------ */
void oracle_lap_mu(const int64_t n[3], const int bc[3], double h, const double psi[4],
                   const double* C, double* out)
{
    grid_t g = {{n[0], n[1], n[2]}, {bc[0], bc[1], bc[2]}};
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n[2]; ++k)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                double mu0 = oracle_psi_prime(C[cell(&g, i, j, k)], psi);
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double mm = oracle_psi_prime(c_at(&g, C, i, j, k, d, -1), psi);
                    double mp = oracle_psi_prime(c_at(&g, C, i, j, k, d, +1), psi);
                    s += (mp - 2.0 * mu0 + mm) / (h * h);
                }
                out[cell(&g, i, j, k)] = s;
            }
}

/* ------------------------------------------------------------------------ */
/* New biharmonic scheme (eq-divbi, eq-a3d): B = sum_d A_d C,               */
/* A_d = kappa Cn^2/h^4 (1, -4, 6, -4, 1) along d.                          */
/* ------------------------------------------------------------------------ */
void oracle_biharm(const int64_t n[3], const int bc[3], double h, double Cn, double kappa,
                   const double* C, double* B)
{
    grid_t g = {{n[0], n[1], n[2]}, {bc[0], bc[1], bc[2]}};
    const double row[5] = {1.0, -4.0, 6.0, -4.0, 1.0};
    double scale = kappa * Cn * Cn / (h * h * h * h);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n[2]; ++k)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    for (int m = -2; m <= 2; ++m)
                        s += row[m + 2] * c_at(&g, C, i, j, k, d, m);
                B[cell(&g, i, j, k)] = scale * s;
            }
}

/* ------------------------------------------------------------------------ */
/* Standard second-order 25-point biharmonic with mixed derivatives         */
/* (eq-disbi, extended to 3-D): Cn^2 (dxx + dyy + dzz)^2 C, i.e.            */
/* Cn^2/h^4 [ sum_d D4_d + 2 sum_{d<e} D2_d D2_e ] C.                       */
/* ------------------------------------------------------------------------ */
void oracle_biharm25(const int64_t n[3], const int bc[3], double h, double Cn,
                     const double* C, double* B)
{
    grid_t g = {{n[0], n[1], n[2]}, {bc[0], bc[1], bc[2]}};
    const double row4[5] = {1.0, -4.0, 6.0, -4.0, 1.0};
    const double row2[3] = {1.0, -2.0, 1.0};
    double scale = Cn * Cn / (h * h * h * h);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n[2]; ++k)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    for (int m = -2; m <= 2; ++m)
                        s += row4[m + 2] * c_at(&g, C, i, j, k, d, m);
                for (int d = 0; d < 3; ++d)
                    for (int e = d + 1; e < 3; ++e)
                        for (int a = -1; a <= 1; ++a)
                            for (int b = -1; b <= 1; ++b) {
                                int64_t p[3] = {i, j, k};
                                p[d] = ghost(p[d] + a, g.n[d], g.bc[d]);
                                p[e] = ghost(p[e] + b, g.n[e], g.bc[e]);
                                s += 2.0 * row2[a + 1] * row2[b + 1]
                                   * C[cell(&g, p[0], p[1], p[2])];
                            }
                B[cell(&g, i, j, k)] = scale * s;
            }
}

/* ------------------------------------------------------------------------ */
/* Explicit CH operator without the biharmonic term:                        */
/*   E = -div(u C) + (1/Pe) lap psi'(C)                                     */
/* ------------------------------------------------------------------------ */
void oracle_explicit(const int64_t n[3], const int bc[3], double h, double Pe,
                     const double psi[4], double eps, const double* C,
                     const double* u, const double* v, const double* w, double* E)
{
    int64_t N = n[0] * n[1] * n[2];
    double* adv = (double*)malloc(sizeof(double) * N);
    double* lap = (double*)malloc(sizeof(double) * N);
    oracle_advection(n, bc, h, eps, C, u, v, w, adv);
    oracle_lap_mu(n, bc, h, psi, C, lap);
    for (int64_t p = 0; p < N; ++p) E[p] = -adv[p] + lap[p] / Pe;
    free(adv);
    free(lap);
}

/* ------------------------------------------------------------------------ */
/* Line solver for (I + r D4) y = b on one line of n points (eq-fac-1..3).  */
/*                                                                          */
/* The matrix rows come straight from the stencil (1,-4,6,-4,1) with the    */
/* ghost map above, so the boundary rows follow from the boundary condition  */
/* (the paper leaves them to it, after eq-a2d).  Entries within two of the  */
/* diagonal form a banded matrix T, factorised by Gaussian elimination      */
/* without pivoting (the matrix is symmetric positive definite); the        */
/* periodic wrap puts the remaining entries in the corners, handled with     */
/* the Sherman-Morrison-Woodbury formula  M = T + U V^T.                    */
/* ------------------------------------------------------------------------ */
#define MAXCORNER 8

typedef struct {
    int64_t n;
    double* band;     /* n x 5: T[i][i+d], d = -2..2, after factorisation: L and U */
    int ncorner;      /* number of rows with entries outside the band */
    int64_t crow[MAXCORNER];
    double* V;        /* ncorner x n: corner entries of each such row */
    double* Z;        /* ncorner x n: T^{-1} e_{crow} */
    double S[MAXCORNER * MAXCORNER]; /* I + V^T Z, LU-factorised in place */
} line_solver_t;

static void band_factor(double* A, int64_t n)
{
    /* A[i*5 + (d+2)] = T[i][i+d]; elimination keeps the band. */
    for (int64_t i = 0; i < n; ++i) {
        double piv = A[i * 5 + 2];
        for (int64_t r = i + 1; r <= i + 2 && r < n; ++r) {
            int dc = (int)(i - r); /* column i relative to row r: -1 or -2 */
            double l = A[r * 5 + dc + 2] / piv;
            A[r * 5 + dc + 2] = l; /* store the multiplier in place of the zeroed entry */
            for (int64_t c = i + 1; c <= i + 2 && c < n; ++c)
                A[r * 5 + (int)(c - r) + 2] -= l * A[i * 5 + (int)(c - i) + 2];
        }
    }
}

static void band_solve(const double* A, int64_t n, double* x)
{
    /* forward: L has unit diagonal and multipliers at d = -1, -2 */
    for (int64_t i = 0; i < n; ++i) {
        double s = x[i];
        if (i >= 1) s -= A[i * 5 + 1] * x[i - 1];
        if (i >= 2) s -= A[i * 5 + 0] * x[i - 2];
        x[i] = s;
    }
    /* backward: U has the diagonal and d = +1, +2 */
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = x[i];
        if (i + 1 < n) s -= A[i * 5 + 3] * x[i + 1];
        if (i + 2 < n) s -= A[i * 5 + 4] * x[i + 2];
        x[i] = s / A[i * 5 + 2];
    }
}

static void small_lu(double* S, int k)
{
    for (int i = 0; i < k; ++i)
        for (int r = i + 1; r < k; ++r) {
            double l = S[r * k + i] / S[i * k + i];
            S[r * k + i] = l;
            for (int c = i + 1; c < k; ++c) S[r * k + c] -= l * S[i * k + c];
        }
}

static void small_solve(const double* S, int k, double* x)
{
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < i; ++c) x[i] -= S[i * k + c] * x[c];
    for (int i = k - 1; i >= 0; --i) {
        for (int c = i + 1; c < k; ++c) x[i] -= S[i * k + c] * x[c];
        x[i] /= S[i * k + i];
    }
}

static int solver_init(line_solver_t* s, int64_t n, double r, int bc)
{
    const double row[5] = {1.0, -4.0, 6.0, -4.0, 1.0};
    memset(s, 0, sizeof(*s));
    s->n = n;
    s->band = (double*)calloc((size_t)n * 5, sizeof(double));
    s->V = (double*)calloc((size_t)n * MAXCORNER, sizeof(double));
    s->Z = (double*)calloc((size_t)n * MAXCORNER, sizeof(double));
    if (!s->band || !s->V || !s->Z) return -1;
    for (int64_t i = 0; i < n; ++i) {
        s->band[i * 5 + 2] += 1.0;
        for (int m = -2; m <= 2; ++m) {
            int64_t col = ghost(i + m, n, bc);
            double val = r * row[m + 2];
            int64_t d = col - i;
            if (d >= -2 && d <= 2) {
                s->band[i * 5 + (int)d + 2] += val;
            } else {
                int c;
                for (c = 0; c < s->ncorner; ++c)
                    if (s->crow[c] == i) break;
                if (c == s->ncorner) {
                    if (s->ncorner == MAXCORNER) return -1;
                    s->crow[s->ncorner++] = i;
                }
                s->V[(size_t)c * n + col] += val;
            }
        }
    }
    band_factor(s->band, n);
    int k = s->ncorner;
    for (int c = 0; c < k; ++c) {
        double* z = s->Z + (size_t)c * n;
        z[s->crow[c]] = 1.0;
        band_solve(s->band, n, z);
    }
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            double acc = (a == b) ? 1.0 : 0.0;
            for (int64_t p = 0; p < n; ++p) acc += s->V[(size_t)a * n + p] * s->Z[(size_t)b * n + p];
            s->S[a * k + b] = acc;
        }
    small_lu(s->S, k);
    return 0;
}

static void solver_apply(const line_solver_t* s, double* x)
{
    int64_t n = s->n;
    int k = s->ncorner;
    band_solve(s->band, n, x);
    if (k == 0) return;
    double t[MAXCORNER];
    for (int a = 0; a < k; ++a) {
        double acc = 0.0;
        for (int64_t p = 0; p < n; ++p) acc += s->V[(size_t)a * n + p] * x[p];
        t[a] = acc;
    }
    small_solve(s->S, k, t);
    for (int a = 0; a < k; ++a)
        for (int64_t p = 0; p < n; ++p) x[p] -= s->Z[(size_t)a * n + p] * t[a];
}

static void solver_free(line_solver_t* s)
{
    free(s->band);
    free(s->V);
    free(s->Z);
}

/* One line: y = (I + r D4)^{-1} b.  Returns 0 on success. */
int oracle_line_solve(int64_t n, double r, int bc, const double* b, double* y)
{
    line_solver_t s;
    if (solver_init(&s, n, r, bc)) { solver_free(&s); return -1; }
    memcpy(y, b, sizeof(double) * n);
    solver_apply(&s, y);
    solver_free(&s);
    return 0;
}

/* Solve (I + r D4_d) along every line of axis d of the field f, in place. */
static int solve_axis(const grid_t* g, int d, double r, double* f)
{
    line_solver_t s;
    int64_t n = g->n[d];
    if (solver_init(&s, n, r, g->bc[d])) { solver_free(&s); return -1; }
    int64_t o1 = (d == 0) ? 1 : 0, o2 = (d == 2) ? 1 : 2; /* the two other axes */
    int64_t n1 = g->n[o1], n2 = g->n[o2];
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < n2; ++b) {
        double* line = (double*)malloc(sizeof(double) * n);
        for (int64_t a = 0; a < n1; ++a) {
            int64_t p[3];
            p[o1] = a;
            p[o2] = b;
            for (int64_t m = 0; m < n; ++m) {
                p[d] = m;
                line[m] = f[cell(g, p[0], p[1], p[2])];
            }
            solver_apply(&s, line);
            for (int64_t m = 0; m < n; ++m) {
                p[d] = m;
                f[cell(g, p[0], p[1], p[2])] = line[m];
            }
        }
        free(line);
    }
    solver_free(&s);
    return 0;
}

/* Low-storage RK3 constants (the reading of the cited scheme). */
static const double RK_GAMMA[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
static const double RK_RHO[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

/* ------------------------------------------------------------------------ */
/* nsteps full RK3 steps of the CH equation, C updated in place.            */
/*                                                                          */
/* Substage k (eq-re with beta = -1/Pe and the CN weight alpha_k dt):       */
/*   E^k   = -div(u C) + (1/Pe) lap psi'(C)                                 */
/*   rhs   = dt (gamma_k E^k + rho_k E^{k-1}) - alpha_k dt/Pe sum_d A_d C    */
/*   (1 + alpha_k dt/(2 Pe) A_x) q1 = rhs                   (eq-fac-1)       */
/*   (1 + alpha_k dt/(2 Pe) A_y) q2 = q1                    (eq-fac-2)       */
/*   (1 + alpha_k dt/(2 Pe) A_z) dC = q2                    (eq-fac-3)       */
/*   C    += dC                                                             */
/* Returns 0 on success.                                                    */
/* ------------------------------------------------------------------------ */
int oracle_step(const int64_t n[3], const int bc[3], double h, double Cn, double Pe,
                const double psi[4], double kappa, double eps, double* C,
                const double* u, const double* v, const double* w, double dt,
                int nsteps)
{
    grid_t g = {{n[0], n[1], n[2]}, {bc[0], bc[1], bc[2]}};
    int64_t N = n[0] * n[1] * n[2];
    double* E = (double*)calloc((size_t)N, sizeof(double));
    double* Eold = (double*)calloc((size_t)N, sizeof(double));
    double* B = (double*)malloc(sizeof(double) * N);
    double* q = (double*)malloc(sizeof(double) * N);
    int rc = 0;
    if (!E || !Eold || !B || !q) rc = -1;
    for (int st = 0; st < nsteps && rc == 0; ++st) {
        for (int k = 0; k < 3 && rc == 0; ++k) {
            double alpha = RK_GAMMA[k] + RK_RHO[k];
            oracle_explicit(n, bc, h, Pe, psi, eps, C, u, v, w, E);
            oracle_biharm(n, bc, h, Cn, kappa, C, B);
            for (int64_t p = 0; p < N; ++p)
                q[p] = dt * (RK_GAMMA[k] * E[p] + RK_RHO[k] * Eold[p])
                     - alpha * dt * B[p] / Pe;
            double r = alpha * dt * kappa * Cn * Cn / (2.0 * Pe * h * h * h * h);
            for (int d = 0; d < 3 && rc == 0; ++d) rc = solve_axis(&g, d, r, q);
            for (int64_t p = 0; p < N; ++p) C[p] += q[p];
            double* t = Eold;
            Eold = E;
            E = t;
        }
    }
    free(E);
    free(Eold);
    free(B);
    free(q);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Explicit-biharmonic variant (the paper's baseline of eq-disbi): no      */
/* Crank-Nicolson and no line solves.  The paper advances every term with   */
/* the low-storage RK3 and treats explicitly all terms it does not put on   */
/* CN (sec. 2), so here the 25-point biharmonic joins the explicit terms:   */
/*   N^k = -div(u C) + lap psi'(C)/Pe - B25(C)/Pe                           */
/*   C  += dt (gamma_k N^k + rho_k N^{k-1})                                 */
/* ------------------------------------------------------------------------ */
int oracle_step_explicit25(const int64_t n[3], const int bc[3], double h, double Cn,
                           double Pe, const double psi[4], double eps, double* C,
                           const double* u, const double* v, const double* w,
                           double dt, int nsteps)
{
    int64_t N = n[0] * n[1] * n[2];
    double* E = (double*)malloc(sizeof(double) * N);
    double* Nk = (double*)calloc((size_t)N, sizeof(double));
    double* Nold = (double*)calloc((size_t)N, sizeof(double));
    double* B = (double*)malloc(sizeof(double) * N);
    if (!E || !Nk || !Nold || !B) { free(E); free(Nk); free(Nold); free(B); return -1; }
    for (int st = 0; st < nsteps; ++st)
        for (int k = 0; k < 3; ++k) {
            /* every term explicit: N = -div(u C) + lap psi'(C)/Pe - B(C)/Pe */
            oracle_explicit(n, bc, h, Pe, psi, eps, C, u, v, w, E);
            oracle_biharm25(n, bc, h, Cn, C, B);
            for (int64_t p = 0; p < N; ++p) {
                Nk[p] = E[p] - B[p] / Pe;
                C[p] += dt * (RK_GAMMA[k] * Nk[p] + RK_RHO[k] * Nold[p]);
            }
            double* t = Nold;
            Nold = Nk;
            Nk = t;
        }
    free(E);
    free(Nk);
    free(Nold);
    free(B);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Mass h^3 sum C (the quantity behind the mass-loss measure of sec. 4.3.1), */
/* summed pairwise in a fixed order.                                        */
/* ------------------------------------------------------------------------ */
static double pairwise_sum(const double* x, int64_t n)
{
    if (n <= 16) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += x[i];
        return s;
    }
    int64_t half = n / 2;
    return pairwise_sum(x, half) + pairwise_sum(x + half, n - half);
}

double oracle_mass(int64_t count, double h, const double* C)
{
    return h * h * h * pairwise_sum(C, count);
}

/* Threads the oracle's parallel loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the threads of the parallel loops (n <= 0: one per processor). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}
