/*
 * CPU FP64 oracle, part 2: the iterative method, written plainly.
 *
 * TEST INFRASTRUCTURE ONLY. The product library never links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do. It shares no code, header or table with the HIP path.
 *
 * What it computes (arXiv:1306.3159):
 *   - kernels phi_3 / phi_4, J and S (Sec. III.A, eqs. tensor_product,
 *     JS_invariance), the periodic 7-point Laplacian (Sec. III.A);
 *   - a geometric multigrid V-cycle for alpha I - D L (Sec. III.E,
 *     eq. Helmholtz). The paper takes its multigrid from a library and does
 *     not specify it; this reading is V(2,2) red-black Gauss-Seidel (red =
 *     (i+j+k) even; pre-smoothing red then black, post-smoothing black then
 *     red), full-weighting restriction R = P^T/8, cell-centred trilinear
 *     prolongation P, the rediscretised coarse operator alpha I - D L_{2h},
 *     and a dense (pseudo-)inverse on the coarsest grid;
 *   - MG-preconditioned CG for the reactive system B c = f
 *     (eqs. unsteady_system, steady_state, Pinv_Poisson). For alpha = 0 the
 *     preconditioner is P MG(P r) + e (e^T r)/(e^T B e), P = I - e e^T/n;
 *   - the absorbing saddle point (eq. saddle_point, zeta = 1, xi = 1/dV_f):
 *     Schur-complement GMRES(30) with modified Gram-Schmidt on
 *     G = J A^+ S (eqs. c_exact, r_schur), with the periodic null-space
 *     handling of Appendix A (mean sink strength fixed by the source, the
 *     fluctuating part on mean-zero vectors, cbar recovered from J c = 0);
 *   - backward-Euler steps (eq. c_np1).
 *
 * Grids are natural layout [z][y][x], x fastest, cell k centred at (k+1/2)h.
 * Positions q are [N][3] (x, y, z) in physical units.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny, nz;
    double h, D;
    int w;
    int N;
    const double* q;
    const double* kappa;
} ora_problem;

typedef struct {
    int iters;          /* outer iterations (CG or GMRES) */
    int inner_iters;    /* total inner CG iterations (absorbing) */
    int vcycles;        /* total V-cycles applied */
    double rel_resid;   /* final relative residual as measured by the solver */
} ora_stats;

/* ------------------------------------------------------------------ */
/* Kernels (Peskin 2002 four-point; Roma-Peskin-Berger three-point).   */
/* ------------------------------------------------------------------ */

static double ora_phi4(double r) {
    double a = fabs(r);
    if (a <= 1.0) {
        double s = 1.0 + 4.0 * a - 4.0 * a * a;
        return (3.0 - 2.0 * a + sqrt(s > 0.0 ? s : 0.0)) / 8.0;
    }
    if (a < 2.0) {
        double s = -7.0 + 12.0 * a - 4.0 * a * a;
        return (5.0 - 2.0 * a - sqrt(s > 0.0 ? s : 0.0)) / 8.0;
    }
    return 0.0;
}

static double ora_phi3(double r) {
    double a = fabs(r);
    if (a <= 0.5) {
        double s = 1.0 - 3.0 * a * a;
        return (1.0 + sqrt(s > 0.0 ? s : 0.0)) / 3.0;
    }
    if (a < 1.5) {
        double s = 1.0 - 3.0 * (1.0 - a) * (1.0 - a);
        return (5.0 - 3.0 * a - sqrt(s > 0.0 ? s : 0.0)) / 6.0;
    }
    return 0.0;
}

double ora_kernel(int w, double r) { return w == 3 ? ora_phi3(r) : ora_phi4(r); }

static int wrapi(int i, int n) { int m = i % n; return m < 0 ? m + n : m; }

/* Cells of one axis touched by a blob at coordinate qa: for each of the
 * w candidate cells k around qa/h - 1/2, the weight phi((qa - (k+1/2)h)/h)
 * with k taken as the integer (unwrapped) index; the grid index is k mod n. */
static void axis_support(double qa, int n, double h, int w, int* idx, double* wt) {
    double s = qa / h - 0.5;
    int k0 = (int)floor(s) - (w == 4 ? 1 : 0);
    if (w == 3) k0 = (int)floor(s + 0.5) - 1;
    for (int j = 0; j < w; ++j) {
        int k = k0 + j;
        wt[j] = ora_kernel(w, s - (double)k);
        idx[j] = wrapi(k, n);
    }
}

void ora_interp(const ora_problem* P, const double* c, double* out) {
    for (int i = 0; i < P->N; ++i) {
        int ix[4], iy[4], iz[4];
        double wx[4], wy[4], wz[4];
        axis_support(P->q[3 * i + 0], P->nx, P->h, P->w, ix, wx);
        axis_support(P->q[3 * i + 1], P->ny, P->h, P->w, iy, wy);
        axis_support(P->q[3 * i + 2], P->nz, P->h, P->w, iz, wz);
        double acc = 0.0;
        for (int c3 = 0; c3 < P->w; ++c3)
            for (int b = 0; b < P->w; ++b)
                for (int a = 0; a < P->w; ++a)
                    acc += wz[c3] * wy[b] * wx[a] *
                           c[((size_t)iz[c3] * P->ny + iy[b]) * P->nx + ix[a]];
        out[i] = acc;
    }
}

/* out += S lam  (S = h^-3 J^T) */
void ora_spread_add(const ora_problem* P, const double* lam, double* out) {
    double inv = 1.0 / (P->h * P->h * P->h);
    for (int i = 0; i < P->N; ++i) {
        int ix[4], iy[4], iz[4];
        double wx[4], wy[4], wz[4];
        axis_support(P->q[3 * i + 0], P->nx, P->h, P->w, ix, wx);
        axis_support(P->q[3 * i + 1], P->ny, P->h, P->w, iy, wy);
        axis_support(P->q[3 * i + 2], P->nz, P->h, P->w, iz, wz);
        for (int c3 = 0; c3 < P->w; ++c3)
            for (int b = 0; b < P->w; ++b)
                for (int a = 0; a < P->w; ++a)
                    out[((size_t)iz[c3] * P->ny + iy[b]) * P->nx + ix[a]] +=
                        inv * wz[c3] * wy[b] * wx[a] * lam[i];
    }
}

void ora_spread(const ora_problem* P, const double* lam, double* out) {
    memset(out, 0, sizeof(double) * (size_t)P->nx * P->ny * P->nz);
    ora_spread_add(P, lam, out);
}

/* ------------------------------------------------------------------ */
/* Grid operators.                                                    */
/* ------------------------------------------------------------------ */

#define IDX(x, y, z) (((size_t)(z) * ny + (y)) * nx + (x))

/* y = alpha x - D L x */
void ora_apply_A(int nx, int ny, int nz, double h, double D, double alpha,
                 const double* x, double* y) {
    double s = D / (h * h);
#pragma omp parallel for
    for (int z = 0; z < nz; ++z)
        for (int yy = 0; yy < ny; ++yy)
            for (int xx = 0; xx < nx; ++xx) {
                double c = x[IDX(xx, yy, z)];
                double nb = x[IDX(wrapi(xx - 1, nx), yy, z)] + x[IDX(wrapi(xx + 1, nx), yy, z)] +
                            x[IDX(xx, wrapi(yy - 1, ny), z)] + x[IDX(xx, wrapi(yy + 1, ny), z)] +
                            x[IDX(xx, yy, wrapi(z - 1, nz))] + x[IDX(xx, yy, wrapi(z + 1, nz))];
                y[IDX(xx, yy, z)] = alpha * c - s * (nb - 6.0 * c);
            }
}

/* y = B x = alpha x - D L x + S kappa J x */
void ora_apply_B(const ora_problem* P, double alpha, const double* x, double* y) {
    ora_apply_A(P->nx, P->ny, P->nz, P->h, P->D, alpha, x, y);
    if (P->N > 0 && P->kappa) {
        double* jx = (double*)malloc(sizeof(double) * P->N);
        ora_interp(P, x, jx);
        for (int i = 0; i < P->N; ++i) jx[i] *= P->kappa[i];
        ora_spread_add(P, jx, y);
        free(jx);
    }
}

/* One Gauss-Seidel half-sweep over cells of one colour ((x+y+z) % 2 == color). */
void ora_gs_color(int nx, int ny, int nz, double h, double D, double alpha,
                  double* u, const double* f, int color) {
    double s = D / (h * h);
    double diag = alpha + 6.0 * s;
#pragma omp parallel for
    for (int z = 0; z < nz; ++z)
        for (int yy = 0; yy < ny; ++yy)
            for (int xx = 0; xx < nx; ++xx) {
                if (((xx + yy + z) & 1) != color) continue;
                double nb = u[IDX(wrapi(xx - 1, nx), yy, z)] + u[IDX(wrapi(xx + 1, nx), yy, z)] +
                            u[IDX(xx, wrapi(yy - 1, ny), z)] + u[IDX(xx, wrapi(yy + 1, ny), z)] +
                            u[IDX(xx, yy, wrapi(z - 1, nz))] + u[IDX(xx, yy, wrapi(z + 1, nz))];
                u[IDX(xx, yy, z)] = (f[IDX(xx, yy, z)] + s * nb) / diag;
            }
}

/* r = f - (alpha I - D L) u */
void ora_residual(int nx, int ny, int nz, double h, double D, double alpha,
                  const double* u, const double* f, double* r) {
    size_t n = (size_t)nx * ny * nz;
    ora_apply_A(nx, ny, nz, h, D, alpha, u, r);
    for (size_t i = 0; i < n; ++i) r[i] = f[i] - r[i];
}

/* Full weighting: coarse cell I gets sum over fine cells 2I-1..2I+2 per axis
 * with 1-D weights (1,3,3,1)/8, i.e. R = P^T / 8 for the trilinear P below.
 * (nx, ny, nz) are the fine sizes. */
void ora_restrict(int nx, int ny, int nz, const double* r, double* rc) {
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    static const double w1[4] = {1.0 / 8, 3.0 / 8, 3.0 / 8, 1.0 / 8};
#pragma omp parallel for
    for (int Z = 0; Z < cz; ++Z)
        for (int Y = 0; Y < cy; ++Y)
            for (int X = 0; X < cx; ++X) {
                double acc = 0.0;
                for (int c = 0; c < 4; ++c)
                    for (int b = 0; b < 4; ++b)
                        for (int a = 0; a < 4; ++a)
                            acc += w1[c] * w1[b] * w1[a] *
                                   r[IDX(wrapi(2 * X - 1 + a, nx), wrapi(2 * Y - 1 + b, ny),
                                         wrapi(2 * Z - 1 + c, nz))];
                rc[((size_t)Z * cy + Y) * cx + X] = acc;
            }
}

/* Cell-centred trilinear prolongation, added: fine cell x = 2I + s takes
 * 3/4 of coarse I and 1/4 of coarse I-1 (s = 0) or I+1 (s = 1), per axis. */
void ora_prolong_add(int nx, int ny, int nz, const double* ec, double* u) {
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
#pragma omp parallel for
    for (int z = 0; z < nz; ++z)
        for (int yy = 0; yy < ny; ++yy)
            for (int xx = 0; xx < nx; ++xx) {
                int I[2], J[2], K[2];
                double wi[2] = {0.75, 0.25}, wj[2] = {0.75, 0.25}, wk[2] = {0.75, 0.25};
                I[0] = xx / 2; I[1] = wrapi((xx & 1) ? xx / 2 + 1 : xx / 2 - 1, cx);
                J[0] = yy / 2; J[1] = wrapi((yy & 1) ? yy / 2 + 1 : yy / 2 - 1, cy);
                K[0] = z / 2;  K[1] = wrapi((z & 1) ? z / 2 + 1 : z / 2 - 1, cz);
                double acc = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            acc += wk[c] * wj[b] * wi[a] * ec[((size_t)K[c] * cy + J[b]) * cx + I[a]];
                u[IDX(xx, yy, z)] += acc;
            }
}
#undef IDX

/* ------------------------------------------------------------------ */
/* Multigrid hierarchy.                                               */
/* ------------------------------------------------------------------ */

#define ORA_MAX_LEVELS 16

typedef struct {
    int nlev;
    int nx[ORA_MAX_LEVELS], ny[ORA_MAX_LEVELS], nz[ORA_MAX_LEVELS];
    double h[ORA_MAX_LEVELS];
    double D, alpha;
    double* u[ORA_MAX_LEVELS];
    double* f[ORA_MAX_LEVELS];
    double* r[ORA_MAX_LEVELS];
    double* cinv;   /* dense (pseudo-)inverse of the coarsest operator */
    int ncoarse;
    int nu1, nu2;
} ora_mg;

/* Coarsen while every dimension is even and larger than 4. */
int ora_mg_levels(int nx, int ny, int nz, int* out_dims) {
    int l = 0;
    for (;;) {
        if (out_dims) { out_dims[3 * l] = nx; out_dims[3 * l + 1] = ny; out_dims[3 * l + 2] = nz; }
        ++l;
        if ((nx & 1) || (ny & 1) || (nz & 1) || nx <= 4 || ny <= 4 || nz <= 4) break;
        if (l >= ORA_MAX_LEVELS) break;
        nx /= 2; ny /= 2; nz /= 2;
    }
    return l;
}

/* Gauss-Jordan inverse with partial pivoting of an m x m matrix (in place into inv). */
static int gauss_jordan(int m, double* a, double* inv) {
    for (int i = 0; i < m * m; ++i) inv[i] = 0.0;
    for (int i = 0; i < m; ++i) inv[i * m + i] = 1.0;
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (fabs(a[r * m + col]) > fabs(a[piv * m + col])) piv = r;
        if (fabs(a[piv * m + col]) < 1e-300) return -1;
        if (piv != col)
            for (int k = 0; k < m; ++k) {
                double t = a[col * m + k]; a[col * m + k] = a[piv * m + k]; a[piv * m + k] = t;
                t = inv[col * m + k]; inv[col * m + k] = inv[piv * m + k]; inv[piv * m + k] = t;
            }
        double d = a[col * m + col];
        for (int k = 0; k < m; ++k) { a[col * m + k] /= d; inv[col * m + k] /= d; }
        for (int r = 0; r < m; ++r) {
            if (r == col) continue;
            double fct = a[r * m + col];
            if (fct == 0.0) continue;
            for (int k = 0; k < m; ++k) {
                a[r * m + k] -= fct * a[col * m + k];
                inv[r * m + k] -= fct * inv[col * m + k];
            }
        }
    }
    return 0;
}

/* Dense coarsest operator alpha I - D L_H; for alpha = 0 the pseudo-inverse
 * (A + e e^T/m)^{-1} - e e^T/m, which maps onto and acts on mean-zero vectors. */
static int build_coarse_inverse(ora_mg* mg) {
    int L = mg->nlev - 1;
    int nx = mg->nx[L], ny = mg->ny[L], nz = mg->nz[L];
    int m = nx * ny * nz;
    double s = mg->D / (mg->h[L] * mg->h[L]);
    double* a = (double*)calloc((size_t)m * m, sizeof(double));
    mg->cinv = (double*)calloc((size_t)m * m, sizeof(double));
    mg->ncoarse = m;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int row = (z * ny + y) * nx + x;
                a[row * m + row] += mg->alpha + 6.0 * s;
                int nb[6] = {(z * ny + y) * nx + wrapi(x - 1, nx), (z * ny + y) * nx + wrapi(x + 1, nx),
                             (z * ny + wrapi(y - 1, ny)) * nx + x, (z * ny + wrapi(y + 1, ny)) * nx + x,
                             (wrapi(z - 1, nz) * ny + y) * nx + x, (wrapi(z + 1, nz) * ny + y) * nx + x};
                for (int k = 0; k < 6; ++k) a[row * m + nb[k]] -= s;
            }
    if (mg->alpha == 0.0)
        for (int i = 0; i < m * m; ++i) a[i] += 1.0 / m;
    int rc = gauss_jordan(m, a, mg->cinv);
    if (mg->alpha == 0.0)
        for (int i = 0; i < m * m; ++i) mg->cinv[i] -= 1.0 / m;
    free(a);
    return rc;
}

ora_mg* ora_mg_create(int nx, int ny, int nz, double h, double D, double alpha) {
    ora_mg* mg = (ora_mg*)calloc(1, sizeof(ora_mg));
    int dims[3 * ORA_MAX_LEVELS];
    mg->nlev = ora_mg_levels(nx, ny, nz, dims);
    mg->D = D;
    mg->alpha = alpha;
    mg->nu1 = 2;
    mg->nu2 = 2;
    for (int l = 0; l < mg->nlev; ++l) {
        mg->nx[l] = dims[3 * l]; mg->ny[l] = dims[3 * l + 1]; mg->nz[l] = dims[3 * l + 2];
        mg->h[l] = h * (double)(1 << l);
        size_t n = (size_t)mg->nx[l] * mg->ny[l] * mg->nz[l];
        mg->u[l] = (double*)calloc(n, sizeof(double));
        mg->f[l] = (double*)calloc(n, sizeof(double));
        mg->r[l] = (double*)calloc(n, sizeof(double));
    }
    if (build_coarse_inverse(mg) != 0) { fprintf(stderr, "oracle: singular coarse operator\n"); }
    return mg;
}

void ora_mg_destroy(ora_mg* mg) {
    if (!mg) return;
    for (int l = 0; l < mg->nlev; ++l) { free(mg->u[l]); free(mg->f[l]); free(mg->r[l]); }
    free(mg->cinv);
    free(mg);
}

static void vcycle_level(ora_mg* mg, int l) {
    int nx = mg->nx[l], ny = mg->ny[l], nz = mg->nz[l];
    size_t n = (size_t)nx * ny * nz;
    double* u = mg->u[l];
    const double* f = mg->f[l];
    if (l == mg->nlev - 1) {
        int m = mg->ncoarse;
        for (int i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int j = 0; j < m; ++j) acc += mg->cinv[(size_t)i * m + j] * f[j];
            u[i] = acc;
        }
        return;
    }
    memset(u, 0, n * sizeof(double));
    for (int s = 0; s < mg->nu1; ++s) {
        ora_gs_color(nx, ny, nz, mg->h[l], mg->D, mg->alpha, u, f, 0);
        ora_gs_color(nx, ny, nz, mg->h[l], mg->D, mg->alpha, u, f, 1);
    }
    ora_residual(nx, ny, nz, mg->h[l], mg->D, mg->alpha, u, f, mg->r[l]);
    ora_restrict(nx, ny, nz, mg->r[l], mg->f[l + 1]);
    vcycle_level(mg, l + 1);
    ora_prolong_add(nx, ny, nz, mg->u[l + 1], u);
    for (int s = 0; s < mg->nu2; ++s) {
        ora_gs_color(nx, ny, nz, mg->h[l], mg->D, mg->alpha, u, f, 1);
        ora_gs_color(nx, ny, nz, mg->h[l], mg->D, mg->alpha, u, f, 0);
    }
}

/* u = MG(f): one V(nu1, nu2) cycle from a zero initial guess. */
void ora_mg_vcycle(ora_mg* mg, const double* f, double* u) {
    size_t n = (size_t)mg->nx[0] * mg->ny[0] * mg->nz[0];
    memcpy(mg->f[0], f, n * sizeof(double));
    vcycle_level(mg, 0);
    memcpy(u, mg->u[0], n * sizeof(double));
}

/* Stand-alone V-cycle for tests: creates and frees its own hierarchy. */
void ora_vcycle(int nx, int ny, int nz, double h, double D, double alpha, const double* f, double* u) {
    ora_mg* mg = ora_mg_create(nx, ny, nz, h, D, alpha);
    ora_mg_vcycle(mg, f, u);
    ora_mg_destroy(mg);
}

/* Dense coarsest-grid solve for tests: u = A_H^{+} f on the coarsest level of (nx,ny,nz). */
int ora_coarse_solve(int nx, int ny, int nz, double h, double D, double alpha, const double* f, double* u,
                     int* cdims) {
    ora_mg* mg = ora_mg_create(nx, ny, nz, h, D, alpha);
    int L = mg->nlev - 1;
    int m = mg->ncoarse;
    for (int i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc += mg->cinv[(size_t)i * m + j] * f[j];
        u[i] = acc;
    }
    if (cdims) { cdims[0] = mg->nx[L]; cdims[1] = mg->ny[L]; cdims[2] = mg->nz[L]; }
    ora_mg_destroy(mg);
    return m;
}

/* ------------------------------------------------------------------ */
/* Vector helpers (sequential sums: deterministic).                    */
/* ------------------------------------------------------------------ */

static double vdot(size_t n, const double* a, const double* b) {
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}
static double vsum(size_t n, const double* a) {
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i];
    return s;
}

/* ------------------------------------------------------------------ */
/* Preconditioned CG for B c = g (B = alpha I - D L [+ S kappa J]).    */
/* ------------------------------------------------------------------ */

typedef struct {
    const ora_problem* P;
    double alpha;
    int with_blobs;     /* 1: B includes S kappa J; 0: A only */
    double eBe;         /* e^T B e for the alpha = 0 constant-mode correction */
    ora_mg* mg;
} ora_op;

static void op_apply(const ora_op* op, const double* x, double* y) {
    const ora_problem* P = op->P;
    if (op->with_blobs) ora_apply_B(P, op->alpha, x, y);
    else ora_apply_A(P->nx, P->ny, P->nz, P->h, P->D, op->alpha, x, y);
}

/* z = M^{-1} r. alpha > 0: one V-cycle. alpha = 0: P MG(P r) plus, when the
 * operator has blobs, the exact constant-mode part e (e^T r)/(e^T B e). */
static void op_precond(const ora_op* op, const double* r, double* z, double* tmp, int* vcycles) {
    const ora_problem* P = op->P;
    size_t n = (size_t)P->nx * P->ny * P->nz;
    if (op->alpha > 0.0) {
        ora_mg_vcycle(op->mg, r, z);
        ++*vcycles;
        return;
    }
    double rs = vsum(n, r);
    double rm = rs / (double)n;
    for (size_t i = 0; i < n; ++i) tmp[i] = r[i] - rm;
    ora_mg_vcycle(op->mg, tmp, z);
    ++*vcycles;
    double zm = vsum(n, z) / (double)n;
    double add = op->with_blobs ? rs / op->eBe : 0.0;
    for (size_t i = 0; i < n; ++i) z[i] = z[i] - zm + add;
}

/* PCG from the initial guess in x. Stops when ||r|| <= rtol ||g|| (recursive
 * residual); returns 0 on convergence, 1 otherwise. */
static int pcg(const ora_op* op, const double* g, double* x, double rtol, int maxit, ora_stats* st) {
    const ora_problem* P = op->P;
    size_t n = (size_t)P->nx * P->ny * P->nz;
    double* r = (double*)malloc(n * sizeof(double));
    double* z = (double*)malloc(n * sizeof(double));
    double* p = (double*)malloc(n * sizeof(double));
    double* q = (double*)malloc(n * sizeof(double));
    double* t = (double*)malloc(n * sizeof(double));
    op_apply(op, x, q);
    for (size_t i = 0; i < n; ++i) r[i] = g[i] - q[i];
    double gn = sqrt(vdot(n, g, g));
    if (gn == 0.0) gn = 1.0;
    double rn = sqrt(vdot(n, r, r));
    int it = 0, rc = 1;
    if (rn <= rtol * gn) rc = 0;
    if (rc) {
        op_precond(op, r, z, t, &st->vcycles);
        memcpy(p, z, n * sizeof(double));
        double rz = vdot(n, r, z);
        for (it = 1; it <= maxit; ++it) {
            op_apply(op, p, q);
            double pq = vdot(n, p, q);
            double a = rz / pq;
            for (size_t i = 0; i < n; ++i) { x[i] += a * p[i]; r[i] -= a * q[i]; }
            rn = sqrt(vdot(n, r, r));
            if (rn <= rtol * gn) { rc = 0; break; }
            op_precond(op, r, z, t, &st->vcycles);
            double rz2 = vdot(n, r, z);
            double b = rz2 / rz;
            rz = rz2;
            for (size_t i = 0; i < n; ++i) p[i] = z[i] + b * p[i];
        }
        if (it > maxit) it = maxit;
    }
    st->iters += it;
    st->rel_resid = rn / gn;
    free(r); free(z); free(p); free(q); free(t);
    return rc;
}

static double total_kappa(const ora_problem* P) {
    double s = 0.0;
    if (P->kappa) for (int i = 0; i < P->N; ++i) s += P->kappa[i];
    return s;
}

/* (alpha I - D L + S kappa J) c = f, c holds the initial guess on entry. */
int ora_solve_reactive(const ora_problem* P, double alpha, const double* f, double* c,
                       double rtol, int maxit, ora_stats* st) {
    memset(st, 0, sizeof(*st));
    size_t n = (size_t)P->nx * P->ny * P->nz;
    double sk = total_kappa(P);
    if (alpha == 0.0 && sk <= 0.0) return -4;
    ora_op op;
    op.P = P;
    op.alpha = alpha;
    op.with_blobs = 1;
    op.eBe = alpha * (double)n + sk / (P->h * P->h * P->h);
    op.mg = ora_mg_create(P->nx, P->ny, P->nz, P->h, P->D, alpha);
    int rc = pcg(&op, f, c, rtol, maxit, st);
    ora_mg_destroy(op.mg);
    return rc;
}

/* One backward-Euler step: (I/dt - D L + S kappa J) c^{n+1} = c^n/dt + f. */
int ora_step(const ora_problem* P, double dt, const double* f, double* c, double rtol, int maxit,
             ora_stats* st) {
    size_t n = (size_t)P->nx * P->ny * P->nz;
    double* g = (double*)malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) g[i] = f[i] + c[i] / dt;
    int rc = ora_solve_reactive(P, 1.0 / dt, g, c, rtol, maxit, st);
    free(g);
    return rc;
}

/* u = A^+ g by PCG (mean-zero u for alpha = 0; g is projected first). */
static int poisson(const ora_op* op, const double* g, double* u, double rtol, int maxit, ora_stats* st) {
    const ora_problem* P = op->P;
    size_t n = (size_t)P->nx * P->ny * P->nz;
    double* gp = (double*)malloc(n * sizeof(double));
    memcpy(gp, g, n * sizeof(double));
    if (op->alpha == 0.0) {
        double m = vsum(n, gp) / (double)n;
        for (size_t i = 0; i < n; ++i) gp[i] -= m;
    }
    memset(u, 0, n * sizeof(double));
    ora_stats s2;
    memset(&s2, 0, sizeof(s2));
    int rc = pcg(op, gp, u, rtol, maxit, &s2);
    if (op->alpha == 0.0) {
        double m = vsum(n, u) / (double)n;
        for (size_t i = 0; i < n; ++i) u[i] -= m;
    }
    st->inner_iters += s2.iters;
    st->vcycles += s2.vcycles;
    free(gp);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Absorbing blobs: Schur-complement GMRES(restart) with MGS.          */
/* ------------------------------------------------------------------ */

typedef struct {
    const ora_problem* P;
    ora_op op;
    double inner_rtol;
    int inner_maxit;
    int project;      /* alpha = 0: work on mean-zero N-vectors */
    double* grid1;
    double* grid2;
    ora_stats* st;
} schur_ctx;

static void nproject(int N, double* v) {
    double m = 0.0;
    for (int i = 0; i < N; ++i) m += v[i];
    m /= (double)N;
    for (int i = 0; i < N; ++i) v[i] -= m;
}

/* y = [P] J A^+ S [P] x */
static void schur_apply(schur_ctx* sc, const double* x, double* y) {
    const ora_problem* P = sc->P;
    int N = P->N;
    double* xp = (double*)malloc(sizeof(double) * N);
    memcpy(xp, x, sizeof(double) * N);
    if (sc->project) nproject(N, xp);
    ora_spread(P, xp, sc->grid1);
    poisson(&sc->op, sc->grid1, sc->grid2, sc->inner_rtol, sc->inner_maxit, sc->st);
    ora_interp(P, sc->grid2, y);
    if (sc->project) nproject(N, y);
    free(xp);
}

/* GMRES(m) with modified Gram-Schmidt and Givens rotations for G x = b. */
/* Stops when ||b - G x|| <= atol (an absolute tolerance chosen by the caller). */
static int gmres(schur_ctx* sc, const double* b, double* x, double atol, int restart, int maxit,
                 int* iters, double* resnorm) {
    int N = sc->P->N;
    int m = restart;
    double* V = (double*)calloc((size_t)(m + 1) * N, sizeof(double));
    double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double));
    double* cs = (double*)calloc(m, sizeof(double));
    double* sn = (double*)calloc(m, sizeof(double));
    double* gvec = (double*)calloc(m + 1, sizeof(double));
    double* w = (double*)calloc(N, sizeof(double));
    double* yv = (double*)calloc(m, sizeof(double));
    int total = 0, rc = 1;
    double res = 0.0;
    for (;;) {
        int any = 0;
        for (int i = 0; i < N; ++i) any |= (x[i] != 0.0);
        if (any) {
            schur_apply(sc, x, w);
            for (int i = 0; i < N; ++i) V[i] = b[i] - w[i];
        } else {
            for (int i = 0; i < N; ++i) V[i] = b[i];
        }
        double beta = sqrt(vdot(N, V, V));
        res = beta;
        if (res <= atol) { rc = 0; break; }
        if (total >= maxit) break;
        for (int i = 0; i < N; ++i) V[i] /= beta;
        memset(gvec, 0, sizeof(double) * (m + 1));
        gvec[0] = beta;
        int k;
        for (k = 0; k < m && total < maxit; ++k) {
            ++total;
            double* vk1 = V + (size_t)(k + 1) * N;
            schur_apply(sc, V + (size_t)k * N, vk1);
            for (int j = 0; j <= k; ++j) {
                double hj = vdot(N, vk1, V + (size_t)j * N);
                H[j * m + k] = hj;
                for (int i = 0; i < N; ++i) vk1[i] -= hj * V[(size_t)j * N + i];
            }
            double hk1 = sqrt(vdot(N, vk1, vk1));
            H[(k + 1) * m + k] = hk1;
            if (hk1 != 0.0)
                for (int i = 0; i < N; ++i) vk1[i] /= hk1;
            for (int j = 0; j < k; ++j) {
                double a = H[j * m + k], bb = H[(j + 1) * m + k];
                H[j * m + k] = cs[j] * a + sn[j] * bb;
                H[(j + 1) * m + k] = -sn[j] * a + cs[j] * bb;
            }
            double a = H[k * m + k], bb = H[(k + 1) * m + k];
            double den = sqrt(a * a + bb * bb);
            cs[k] = den == 0.0 ? 1.0 : a / den;
            sn[k] = den == 0.0 ? 0.0 : bb / den;
            H[k * m + k] = den;
            H[(k + 1) * m + k] = 0.0;
            gvec[k + 1] = -sn[k] * gvec[k];
            gvec[k] = cs[k] * gvec[k];
            res = fabs(gvec[k + 1]);
            if (res <= atol || hk1 == 0.0) { ++k; break; }
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = gvec[i];
            for (int j = i + 1; j < k; ++j) s -= H[i * m + j] * yv[j];
            yv[i] = s / H[i * m + i];
        }
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < N; ++i) x[i] += yv[j] * V[(size_t)j * N + i];
        if (total >= maxit) break;
    }
    *iters = total;
    *resnorm = res;
    free(V); free(H); free(cs); free(sn); free(gvec); free(w); free(yv);
    return rc;
}

/* [alpha I - D L, S; J, 0][c; lam] = [f; 0].
 * alpha = 0: lam = lam_bar 1 + lam_t with lam_bar = h^3 sum(f)/N,
 *   b = J A^+ (f - S lam_bar 1),  P G P lam_t = P b,
 *   c = A^+ (f - S lam) + cbar with cbar = mean(-J A^+(f - S lam)).
 * alpha > 0: G lam = J A^{-1} f, c = A^{-1}(f - S lam). */
int ora_solve_absorbing(const ora_problem* P, double alpha, const double* f, double* c, double* lam,
                        double rtol, double inner_rtol, int restart, int maxit, ora_stats* st) {
    memset(st, 0, sizeof(*st));
    int N = P->N;
    if (N <= 0) return -1;
    size_t n = (size_t)P->nx * P->ny * P->nz;
    double h3 = P->h * P->h * P->h;
    schur_ctx sc;
    sc.P = P;
    sc.op.P = P;
    sc.op.alpha = alpha;
    sc.op.with_blobs = 0;
    sc.op.eBe = 0.0;
    sc.op.mg = ora_mg_create(P->nx, P->ny, P->nz, P->h, P->D, alpha);
    sc.inner_rtol = inner_rtol;
    sc.inner_maxit = 200;
    sc.project = alpha == 0.0;
    sc.grid1 = (double*)malloc(n * sizeof(double));
    sc.grid2 = (double*)malloc(n * sizeof(double));
    sc.st = st;
    double* g = (double*)malloc(n * sizeof(double));
    double* b = (double*)malloc(sizeof(double) * N);
    double lbar = 0.0;
    memcpy(g, f, n * sizeof(double));
    if (alpha == 0.0) {
        lbar = h3 * vsum(n, f) / (double)N;
        double* ones = (double*)malloc(sizeof(double) * N);
        for (int i = 0; i < N; ++i) ones[i] = -lbar;
        ora_spread_add(P, ones, g);
        free(ones);
    }
    poisson(&sc.op, g, sc.grid2, inner_rtol, sc.inner_maxit, st);
    ora_interp(P, sc.grid2, b);
    if (sc.project) nproject(N, b);
    double* lt = (double*)calloc(N, sizeof(double));
    int iters = 0;
    double rr = 0.0;
    /* The saddle-point residual is measured against ||f||; its constraint block is
     * the Schur residual, so GMRES stops at half the target on that scale and the
     * final Poisson solve below takes the other half. */
    double fnorm = sqrt(vdot(n, f, f));
    int rc = gmres(&sc, b, lt, 0.5 * rtol * fnorm, restart, maxit, &iters, &rr);
    st->iters = iters;
    st->rel_resid = fnorm > 0.0 ? rr / fnorm : rr;
    if (sc.project) nproject(N, lt);
    for (int i = 0; i < N; ++i) lam[i] = lbar + lt[i];
    /* c = A^+ (f - S lam) (+ cbar) */
    memcpy(g, f, n * sizeof(double));
    double* nl = (double*)malloc(sizeof(double) * N);
    for (int i = 0; i < N; ++i) nl[i] = -lam[i];
    ora_spread_add(P, nl, g);
    free(nl);
    poisson(&sc.op, g, c, inner_rtol < 0.5 * rtol ? inner_rtol : 0.5 * rtol, sc.inner_maxit, st);
    if (alpha == 0.0) {
        ora_interp(P, c, b);
        double cb = 0.0;
        for (int i = 0; i < N; ++i) cb -= b[i];
        cb /= (double)N;
        for (size_t i = 0; i < n; ++i) c[i] += cb;
    }
    free(g); free(b); free(lt); free(sc.grid1); free(sc.grid2);
    ora_mg_destroy(sc.op.mg);
    return rc;
}

/* u = A^+ g by MG-preconditioned CG to relative tolerance rtol (one inner solve
 * of the absorbing method; used to time a bounded sample of it). */
int ora_solve_poisson(const ora_problem* P, double alpha, const double* g, double* u, double rtol, int maxit,
                      ora_stats* st) {
    memset(st, 0, sizeof(*st));
    ora_op op;
    op.P = P;
    op.alpha = alpha;
    op.with_blobs = 0;
    op.eBe = 0.0;
    op.mg = ora_mg_create(P->nx, P->ny, P->nz, P->h, P->D, alpha);
    int rc = poisson(&op, g, u, rtol, maxit, st);
    ora_mg_destroy(op.mg);
    return rc;
}

/* Number of OpenMP threads the oracle runs with (1 when built without OpenMP). */
int ora_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads of later calls (no effect without OpenMP). */
void ora_set_num_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
