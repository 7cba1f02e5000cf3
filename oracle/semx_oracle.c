/*
 * semx FP64 CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, double-precision implementation of the spectral-element
 * elastic operator and its explicit time loop, written from the paper
 * ("High-Order Spectral Element Methods for Wave Propagation on ARM Multicore
 * CPU with SME", Sec. II-B) so that the HIP library can be checked against it.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this library.  It shares no code, header or table with the HIP path.
 *
 * Every loop follows the definition it cites, in the paper's notation
 * (i,j,k local GLL indices along xi, eta, zeta; N = n-1 the polynomial
 * degree).  Parallelism is OpenMP over elements only; assembly is a serial
 * loop in element order, so every result is bitwise reproducible for any
 * thread count.
 *
 * Conventions shared with the caller (plain data, no arithmetic):
 *   - element-local point q = i + n*(j + n*k), i fastest;
 *   - ibool[e*n^3 + q]   global node of local point q of element e;
 *   - elem_vert[e*8 + v] vertex of corner v = a + 2b + 4c, corner
 *     (a,b,c) in {0,1}^3 sits at (xi,eta,zeta) = (2a-1, 2b-1, 2c-1);
 *   - vectors over global nodes are [nglob][3] (component fastest);
 *   - per-point geometry gam[(e*n^3+q)*9 + 3*d + b] = d xi_d / d x_b and
 *     jac[e*n^3+q] = det J.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXN 16

#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the oracle's parallel loops use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Legendre polynomial P_N(x) and its first derivative by the three-term
 * recurrence (k+1)P_{k+1} = (2k+1) x P_k - k P_{k-1}.
 * ------------------------------------------------------------------------- */
static void legendre(int N, double x, double *p, double *dp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (N == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;  /* P'_{k+1} = P'_{k-1} + (2k+1) P_k */
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *p = p1; *dp = d1;
}

/* ---------------------------------------------------------------------------
 * GLL nodes and weights (Sec. II-B: the interpolation points are the
 * Gauss-Lobatto-Legendre points).  xi_0 = -1, xi_N = +1; the interior nodes
 * are the zeros of P'_N, found by Newton's method on P'_N starting from the
 * Chebyshev-Gauss-Lobatto points.  Quadrature weights
 * w_a = 2 / (N (N+1) P_N(xi_a)^2).  Returns 0, or -1 for n outside [2, 16].
 * ------------------------------------------------------------------------- */
int orc_gll(int n, double *xi, double *w)
{
    if (n < 2 || n > ORC_MAXN) return -1;
    int N = n - 1;
    xi[0] = -1.0; xi[N] = 1.0;
    for (int a = 1; a < N; ++a) {
        double x = -cos(M_PI * a / N);
        for (int it = 0; it < 100; ++it) {
            /* Newton on g(x) = P'_N(x); g'(x) from Legendre's ODE:
             * (1-x^2) P''_N = 2x P'_N - N(N+1) P_N. */
            double p, dp;
            legendre(N, x, &p, &dp);
            double d2p = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
            double dx = dp / d2p;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[a] = x;
    }
    /* enforce the exact symmetry xi_{N-a} = -xi_a */
    for (int a = 0; a < n / 2; ++a) {
        double s = 0.5 * (xi[N - a] - xi[a]);
        xi[a] = -s; xi[N - a] = s;
    }
    if (n % 2 == 1) xi[N / 2] = 0.0;
    for (int a = 0; a < n; ++a) {
        double p, dp;
        legendre(N, xi[a], &p, &dp);
        w[a] = 2.0 / (N * (N + 1.0) * p * p);
    }
    return 0;
}

/* Lagrange basis l_a(x) by the product formula of Sec. II-B. */
void orc_lagrange(int n, const double *xi, double x, double *l)
{
    for (int a = 0; a < n; ++a) {
        double num = 1.0, den = 1.0;
        for (int m = 0; m < n; ++m) {
            if (m == a) continue;
            num *= (x - xi[m]);
            den *= (xi[a] - xi[m]);
        }
        l[a] = num / den;
    }
}

/* Derivative l'_b(x) of the product formula (product rule, term by term). */
void orc_lagrange_deriv(int n, const double *xi, double x, double *dl)
{
    for (int b = 0; b < n; ++b) {
        double den = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != b) den *= (xi[b] - xi[m]);
        double s = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == b) continue;
            double term = 1.0;
            for (int l = 0; l < n; ++l)
                if (l != b && l != m) term *= (x - xi[l]);
            s += term;
        }
        dl[b] = s / den;
    }
}

/* Differentiation matrix D[a*n+b] = l'_b(xi_a): the (N+1)x(N+1) matrix whose
 * product with a 1-D line of nodal values gives the reference derivative at
 * the nodes (Sec. II-B, xi-derivative equation and the remark after it). */
void orc_dmatrix(int n, const double *xi, double *D)
{
    for (int a = 0; a < n; ++a) orc_lagrange_deriv(n, xi, xi[a], D + a * n);
}

/* ---------------------------------------------------------------------------
 * Trilinear (8-node) geometry.  x(xi,eta,zeta) = sum_v N_v x_v with
 * N_v = (1 + s_a xi)(1 + s_b eta)(1 + s_c zeta)/8, s = 2a-1.  At every GLL
 * point: J_{ab} = d x_a / d xi_b analytically, det J, and Gamma = J^{-1} by
 * cofactors (row d of Gamma = gradient of reference coordinate d).
 * Returns 0, or -1 if some det J <= 0.
 * ------------------------------------------------------------------------- */
int orc_geometry(int n, int64_t nspec, const int32_t *elem_vert, const double *vert,
                 double *gam, double *jac, double *xyz)
{
    double xi[ORC_MAXN], w[ORC_MAXN];
    if (orc_gll(n, xi, w)) return -2;
    const int n3 = n * n * n;
    int bad = 0;
#pragma omp parallel for reduction(| : bad) schedule(static)
    for (int64_t e = 0; e < nspec; ++e) {
        for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double r[3] = {xi[i], xi[j], xi[k]};
            double J[3][3] = {{0}}, x[3] = {0};
            for (int v = 0; v < 8; ++v) {
                double s[3] = {(v & 1) ? 1.0 : -1.0, (v & 2) ? 1.0 : -1.0, (v & 4) ? 1.0 : -1.0};
                double f[3] = {1.0 + s[0] * r[0], 1.0 + s[1] * r[1], 1.0 + s[2] * r[2]};
                double Nv = f[0] * f[1] * f[2] / 8.0;
                double dN[3] = {s[0] * f[1] * f[2] / 8.0, f[0] * s[1] * f[2] / 8.0, f[0] * f[1] * s[2] / 8.0};
                const double *xv = vert + 3 * (int64_t)elem_vert[8 * e + v];
                for (int a = 0; a < 3; ++a) {
                    x[a] += Nv * xv[a];
                    for (int b = 0; b < 3; ++b) J[a][b] += xv[a] * dN[b];
                }
            }
            double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                       - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                       + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            if (!(det > 0.0)) bad = 1;
            /* inverse by cofactors: Gamma[d][b] = cof(J)[b][d] / det */
            double G[3][3];
            G[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
            G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
            G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
            G[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
            G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
            G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
            G[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
            G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
            G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
            int64_t p = e * n3 + i + n * (j + n * k);
            for (int d = 0; d < 3; ++d)
                for (int b = 0; b < 3; ++b) gam[9 * p + 3 * d + b] = G[d][b];
            jac[p] = det;
            if (xyz)
                for (int a = 0; a < 3; ++a) xyz[3 * p + a] = x[a];
        }
    }
    return bad ? -1 : 0;
}

/* Lumped GLL mass (Sec. II-B: the mass matrix is diagonal when integrated at
 * the GLL nodes): M_g = sum over (e,i,j,k) with ibool = g of
 * rho * w_i w_j w_k * det J.  Serial, element order. */
void orc_mass(int n, int64_t nspec, int64_t nglob, const int32_t *ibool,
              const double *jac, const double *rho, double *mass)
{
    double xi[ORC_MAXN], w[ORC_MAXN];
    orc_gll(n, xi, w);
    const int n3 = n * n * n;
    memset(mass, 0, sizeof(double) * nglob);
    for (int64_t e = 0; e < nspec; ++e)
        for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int64_t p = e * n3 + i + n * (j + n * k);
            mass[ibool[p]] += rho[p] * w[i] * w[j] * w[k] * jac[p];
        }
}

/* ---------------------------------------------------------------------------
 * Internal force f = -K u (Sec. II-B, weak form; the stiffness term applied
 * matrix-free as three forward and three transpose small contractions).
 * For each element and each local point (i,j,k):
 *   1. reference derivatives  du_c/dxi   = sum_a D_ia u_c(a,j,k),
 *                             du_c/deta  = sum_a D_ja u_c(i,a,k),
 *                             du_c/dzeta = sum_a D_ka u_c(i,j,a);
 *   2. physical gradient g_cb = sum_d (du_c/dxi_d) Gamma_db;
 *   3. isotropic Hooke stress sigma_cb = lambda tr(g) delta_cb + mu (g_cb + g_bc);
 *   4. weighted fluxes Phi_cd = w_i w_j w_k det J sum_b sigma_cb Gamma_db;
 *   5. F_c(i,j,k) = -[sum_a D_ai Phi_c0(a,j,k) + sum_a D_aj Phi_c1(i,a,k)
 *                     + sum_a D_ak Phi_c2(i,j,a)];
 *   6. f[ibool(e,i,j,k)][c] += F_c(i,j,k).
 * Steps 1-5 run per element in parallel into a private buffer; step 6 is a
 * serial loop in element order.
 * ------------------------------------------------------------------------- */
static void element_force(int n, const double *D, const double *w, int64_t e,
                          const int32_t *ibool, const double *gam, const double *jac,
                          const double *lam, const double *mu, const double *u,
                          double *ue, double *phi, double *Fe)
{
    const int n3 = n * n * n;
    for (int q = 0; q < n3; ++q)
        for (int c = 0; c < 3; ++c) ue[3 * q + c] = u[3 * (int64_t)ibool[e * n3 + q] + c];
    for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
        int q = i + n * (j + n * k);
        int64_t p = e * n3 + q;
        double du[3][3]; /* du[c][d] = d u_c / d xi_d */
        for (int c = 0; c < 3; ++c) {
            double s0 = 0, s1 = 0, s2 = 0;
            for (int a = 0; a < n; ++a) {
                s0 += D[i * n + a] * ue[3 * (a + n * (j + n * k)) + c];
                s1 += D[j * n + a] * ue[3 * (i + n * (a + n * k)) + c];
                s2 += D[k * n + a] * ue[3 * (i + n * (j + n * a)) + c];
            }
            du[c][0] = s0; du[c][1] = s1; du[c][2] = s2;
        }
        const double *G = gam + 9 * p;
        double g[3][3];
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                g[c][b] = du[c][0] * G[0 * 3 + b] + du[c][1] * G[1 * 3 + b] + du[c][2] * G[2 * 3 + b];
        double tr = g[0][0] + g[1][1] + g[2][2];
        double sig[3][3];
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                sig[c][b] = (c == b ? lam[p] * tr : 0.0) + mu[p] * (g[c][b] + g[b][c]);
        double W = w[i] * w[j] * w[k] * jac[p];
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d)
                phi[9 * q + 3 * c + d] = W * (sig[c][0] * G[3 * d + 0] + sig[c][1] * G[3 * d + 1] + sig[c][2] * G[3 * d + 2]);
    }
    for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
        int q = i + n * (j + n * k);
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int a = 0; a < n; ++a) {
                s += D[a * n + i] * phi[9 * (a + n * (j + n * k)) + 3 * c + 0];
                s += D[a * n + j] * phi[9 * (i + n * (a + n * k)) + 3 * c + 1];
                s += D[a * n + k] * phi[9 * (i + n * (j + n * a)) + 3 * c + 2];
            }
            Fe[3 * q + c] = -s;
        }
    }
}

void orc_force(int n, int64_t nspec, int64_t nglob, const int32_t *ibool,
               const double *gam, const double *jac, const double *lam, const double *mu,
               const double *u, double *f)
{
    double xi[ORC_MAXN], w[ORC_MAXN], D[ORC_MAXN * ORC_MAXN];
    orc_gll(n, xi, w);
    orc_dmatrix(n, xi, D);
    const int n3 = n * n * n;
    double *Fe = (double *)malloc(sizeof(double) * 3 * n3 * (size_t)nspec);
#pragma omp parallel
    {
        double *ue = (double *)malloc(sizeof(double) * 3 * n3);
        double *phi = (double *)malloc(sizeof(double) * 9 * n3);
#pragma omp for schedule(static)
        for (int64_t e = 0; e < nspec; ++e)
            element_force(n, D, w, e, ibool, gam, jac, lam, mu, u, ue, phi, Fe + 3 * n3 * e);
        free(ue); free(phi);
    }
    memset(f, 0, sizeof(double) * 3 * nglob);
    for (int64_t e = 0; e < nspec; ++e)
        for (int q = 0; q < n3; ++q)
            for (int c = 0; c < 3; ++c)
                f[3 * (int64_t)ibool[e * n3 + q] + c] += Fe[3 * (n3 * e + q) + c];
    free(Fe);
}

/* ---------------------------------------------------------------------------
 * Point force injection and receiver interpolation via the tensor-product
 * interpolation of Sec. II-B: a point at reference coordinates
 * (xi_s, eta_s, zeta_s) in element e_s couples to node (i,j,k) of that
 * element with weight l_i(xi_s) l_j(eta_s) l_k(zeta_s).
 * ------------------------------------------------------------------------- */
static void point_weights(int n, const double *xi, const double *r, double *wt)
{
    double lx[ORC_MAXN], ly[ORC_MAXN], lz[ORC_MAXN];
    orc_lagrange(n, xi, r[0], lx);
    orc_lagrange(n, xi, r[1], ly);
    orc_lagrange(n, xi, r[2], lz);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) wt[i + n * (j + n * k)] = lx[i] * ly[j] * lz[k];
}

static double dot3n(int64_t nglob, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t g = 0; g < 3 * nglob; ++g) s += a[g] * b[g];
    return s;
}

/* ---------------------------------------------------------------------------
 * Explicit second-order Newmark (beta = 0, gamma = 1/2) time loop with the
 * diagonal mass, as used for the paper's wave-propagation runs:
 *   u^0 = v^0 = 0,  a^0 = M^{-1} f_src(t_0);
 *   for n = 0..nt-1:
 *     u <- u + dt v + dt^2/2 a;   v <- v + dt/2 a;
 *     f <- -K u + f_src(t_{n+1}); a <- M^{-1} f;   v <- v + dt/2 a;
 *     seis[r][c][n] = sum_q l_q(x_r) u_c(ibool(e_r, q)).
 * Source s: f_src,c = stf[s][m] * dir[s][c] * l_q(x_s) at the nodes of
 * element src_elem[s]; stf has nt+1 samples per source, sample m at t_m.
 * If energy is non-NULL: energy[n] = E^{n+1/2} =
 *   1/2 |u^{n+1}-u^n|_M^2 / dt^2 + 1/2 (u^{n+1})^T K u^n,
 * and work[n] = 1/2 (u^{n+1} - u^{n-1})^T f_src(t_n) for n >= 1 (work[0]=0),
 * so that energy[n] - energy[n-1] = work[n] holds up to rounding.
 * If uhist is non-NULL it receives u^0..u^nt ([nt+1][nglob][3]).
 * ------------------------------------------------------------------------- */
int orc_forward(int n, int64_t nspec, int64_t nglob, const int32_t *ibool,
                const double *gam, const double *jac, const double *lam, const double *mu,
                const double *rho, double dt, int64_t nt,
                int nsrc, const int32_t *src_elem, const double *src_xi, const double *src_dir,
                const double *stf, int nrec, const int32_t *rec_elem, const double *rec_xi,
                double *seis, double *energy, double *work, double *uhist)
{
    double xi[ORC_MAXN], w[ORC_MAXN];
    if (orc_gll(n, xi, w)) return -2;
    const int n3 = n * n * n;
    size_t nv = 3 * (size_t)nglob;
    double *mass = (double *)malloc(sizeof(double) * nglob);
    double *u = (double *)calloc(nv, sizeof(double));
    double *v = (double *)calloc(nv, sizeof(double));
    double *a = (double *)calloc(nv, sizeof(double));
    double *f = (double *)calloc(nv, sizeof(double));
    double *fint_old = (double *)calloc(nv, sizeof(double)); /* -K u^n */
    double *uold = (double *)calloc(nv, sizeof(double));     /* u^{n-1} */
    double *fsrc = (double *)calloc(nv, sizeof(double));
    double *swt = (double *)malloc(sizeof(double) * n3 * (nsrc > 0 ? nsrc : 1));
    double *rwt = (double *)malloc(sizeof(double) * n3 * (nrec > 0 ? nrec : 1));
    orc_mass(n, nspec, nglob, ibool, jac, rho, mass);
    for (int s = 0; s < nsrc; ++s) point_weights(n, xi, src_xi + 3 * s, swt + n3 * s);
    for (int r = 0; r < nrec; ++r) point_weights(n, xi, rec_xi + 3 * r, rwt + n3 * r);

#define BUILD_FSRC(m)                                                                  \
    do {                                                                               \
        memset(fsrc, 0, sizeof(double) * nv);                                          \
        for (int s = 0; s < nsrc; ++s)                                                 \
            for (int q = 0; q < n3; ++q)                                               \
                for (int c = 0; c < 3; ++c)                                            \
                    fsrc[3 * (int64_t)ibool[(int64_t)src_elem[s] * n3 + q] + c] +=     \
                        stf[(size_t)s * (nt + 1) + (m)] * src_dir[3 * s + c] * swt[n3 * s + q]; \
    } while (0)

    /* a^0 = M^{-1} (f_src(t_0) - K u^0), u^0 = 0 */
    BUILD_FSRC(0);
    for (int64_t g = 0; g < nglob; ++g)
        for (int c = 0; c < 3; ++c) a[3 * g + c] = fsrc[3 * g + c] / mass[g];
    if (uhist) memcpy(uhist, u, sizeof(double) * nv);
    double *unew_minus_uold = NULL;
    if (energy) unew_minus_uold = (double *)malloc(sizeof(double) * nv);

    for (int64_t it = 0; it < nt; ++it) {
        /* keep u^n and -K u^n for the energy bookkeeping */
        double *un = NULL;
        if (energy) {
            un = (double *)malloc(sizeof(double) * nv);
            memcpy(un, u, sizeof(double) * nv);
        }
        for (size_t g = 0; g < nv; ++g) {
            u[g] += dt * v[g] + 0.5 * dt * dt * a[g];
            v[g] += 0.5 * dt * a[g];
        }
        if (energy) {
            /* source work of step it: 1/2 (u^{n+1} - u^{n-1})^T f_src^n, n = it */
            if (it >= 1) {
                BUILD_FSRC(it);
                for (size_t g = 0; g < nv; ++g) unew_minus_uold[g] = u[g] - uold[g];
                work[it] = 0.5 * dot3n(nglob, unew_minus_uold, fsrc);
            } else {
                work[it] = 0.0;
            }
        }
        orc_force(n, nspec, nglob, ibool, gam, jac, lam, mu, u, f);
        if (energy) {
            double kin = 0.0;
            for (int64_t g = 0; g < nglob; ++g)
                for (int c = 0; c < 3; ++c) {
                    double d = (u[3 * g + c] - un[3 * g + c]) / dt;
                    kin += 0.5 * mass[g] * d * d;
                }
            /* (u^{n+1})^T K u^n = -(u^{n+1})^T fint(u^n) */
            double pot = -0.5 * dot3n(nglob, u, fint_old);
            energy[it] = kin + pot;
            memcpy(fint_old, f, sizeof(double) * nv);
            memcpy(uold, un, sizeof(double) * nv);
            free(un);
        }
        BUILD_FSRC(it + 1);
        for (int64_t g = 0; g < nglob; ++g)
            for (int c = 0; c < 3; ++c) {
                f[3 * g + c] += fsrc[3 * g + c];
                a[3 * g + c] = f[3 * g + c] / mass[g];
                v[3 * g + c] += 0.5 * dt * a[3 * g + c];
            }
        for (int r = 0; r < nrec; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int q = 0; q < n3; ++q)
                    s += rwt[n3 * r + q] * u[3 * (int64_t)ibool[(int64_t)rec_elem[r] * n3 + q] + c];
                seis[((size_t)r * 3 + c) * nt + it] = s;
            }
        if (uhist) memcpy(uhist + nv * (it + 1), u, sizeof(double) * nv);
    }
#undef BUILD_FSRC
    free(mass); free(u); free(v); free(a); free(f); free(fint_old); free(uold);
    free(fsrc); free(swt); free(rwt); free(unew_minus_uold);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Discrete adjoint of the Newmark run above (exact gradient of a seismogram
 * misfit with respect to lambda, mu and rho at every element-local point).
 *
 * The run is, for n >= 1, the central-difference recursion
 *   r^{n+1} = M (u^{n+1} - 2u^n + u^{n-1}) + dt^2 K u^n - dt^2 f_src^n = 0,
 * started by r^1 = M u^1 - dt^2/2 f_src^0 = 0 (u^0 = 0), and seis[.][.][n-1]
 * = R u^n.  Given gseis = d chi / d seis ([nrec][3][nt]), the adjoint fields
 * psi^m solve, for m = nt .. 1 with psi^{nt+1} = psi^{nt+2} = 0,
 *   M psi^m = R^T gseis(m) + M (2 psi^{m+1} - psi^{m+2}) - dt^2 K psi^{m+1},
 * and since K is linear in (lambda, mu) and M in rho (Sec. II-B weak form
 * with the lumped GLL mass), with W_q = w_i w_j w_k det J:
 *   dchi/dlambda_q = -dt^2 sum_{n=1}^{nt-1} W_q div psi^{n+1} div u^n,
 *   dchi/dmu_q     = -dt^2 sum_{n=1}^{nt-1} 2 W_q eps(psi^{n+1}) : eps(u^n),
 *   dchi/drho_q    = - sum_{n=1}^{nt-1} W_q psi^{n+1}.(u^{n+1} - 2u^n + u^{n-1})
 *                    - W_q psi^1 . u^1            (all at node ibool(q)).
 * The forward history is recomputed here in full (small problems only).
 * ------------------------------------------------------------------------- */

/* grad[q][c][b] = d u_c / d x_b at every local point of element e */
static void element_grad(int n, const double *D, int64_t e, const int32_t *ibool,
                         const double *gam, const double *u, double *ue, double *grad)
{
    const int n3 = n * n * n;
    for (int q = 0; q < n3; ++q)
        for (int c = 0; c < 3; ++c) ue[3 * q + c] = u[3 * (int64_t)ibool[e * n3 + q] + c];
    for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
        int q = i + n * (j + n * k);
        const double *G = gam + 9 * (e * n3 + q);
        for (int c = 0; c < 3; ++c) {
            double d0 = 0, d1 = 0, d2 = 0;
            for (int a = 0; a < n; ++a) {
                d0 += D[i * n + a] * ue[3 * (a + n * (j + n * k)) + c];
                d1 += D[j * n + a] * ue[3 * (i + n * (a + n * k)) + c];
                d2 += D[k * n + a] * ue[3 * (i + n * (j + n * a)) + c];
            }
            for (int b = 0; b < 3; ++b)
                grad[9 * q + 3 * c + b] = d0 * G[b] + d1 * G[3 + b] + d2 * G[6 + b];
        }
    }
}

int orc_adjoint(int n, int64_t nspec, int64_t nglob, const int32_t *ibool,
                const double *gam, const double *jac, const double *lam, const double *mu,
                const double *rho, double dt, int64_t nt,
                int nsrc, const int32_t *src_elem, const double *src_xi, const double *src_dir,
                const double *stf, int nrec, const int32_t *rec_elem, const double *rec_xi,
                const double *gseis, double *g_lam, double *g_mu, double *g_rho)
{
    double xi[ORC_MAXN], w[ORC_MAXN], D[ORC_MAXN * ORC_MAXN];
    if (orc_gll(n, xi, w)) return -2;
    orc_dmatrix(n, xi, D);
    const int n3 = n * n * n;
    const size_t nv = 3 * (size_t)nglob;
    double *seis = (double *)malloc(sizeof(double) * (nrec > 0 ? nrec : 1) * 3 * nt);
    double *uh = (double *)malloc(sizeof(double) * nv * (nt + 1));
    int rc = orc_forward(n, nspec, nglob, ibool, gam, jac, lam, mu, rho, dt, nt, nsrc, src_elem,
                         src_xi, src_dir, stf, nrec, rec_elem, rec_xi, seis, NULL, NULL, uh);
    free(seis);
    if (rc) { free(uh); return rc; }
    double *mass = (double *)malloc(sizeof(double) * nglob);
    orc_mass(n, nspec, nglob, ibool, jac, rho, mass);
    double *rwt = (double *)malloc(sizeof(double) * n3 * (nrec > 0 ? nrec : 1));
    for (int r = 0; r < nrec; ++r) point_weights(n, xi, rec_xi + 3 * r, rwt + n3 * r);
    double *p0 = (double *)calloc(nv, sizeof(double)); /* psi^{m+2} */
    double *p1 = (double *)calloc(nv, sizeof(double)); /* psi^{m+1} */
    double *p2 = (double *)calloc(nv, sizeof(double)); /* psi^m */
    double *kf = (double *)calloc(nv, sizeof(double)); /* -K psi^{m+1} */
    double *gsrc = (double *)calloc(nv, sizeof(double));
    memset(g_lam, 0, sizeof(double) * nspec * n3);
    memset(g_mu, 0, sizeof(double) * nspec * n3);
    memset(g_rho, 0, sizeof(double) * nspec * n3);
    for (int64_t m = nt; m >= 1; --m) {
        /* adjoint source R^T gseis(m), seismogram sample m-1 */
        memset(gsrc, 0, sizeof(double) * nv);
        for (int r = 0; r < nrec; ++r)
            for (int q = 0; q < n3; ++q)
                for (int c = 0; c < 3; ++c)
                    gsrc[3 * (int64_t)ibool[(int64_t)rec_elem[r] * n3 + q] + c] +=
                        rwt[n3 * r + q] * gseis[((size_t)r * 3 + c) * nt + (m - 1)];
        orc_force(n, nspec, nglob, ibool, gam, jac, lam, mu, p1, kf);
        for (int64_t g = 0; g < nglob; ++g)
            for (int c = 0; c < 3; ++c) {
                size_t t = 3 * g + c;
                p2[t] = 2.0 * p1[t] - p0[t] + (dt * dt * kf[t] + gsrc[t]) / mass[g];
            }
        /* gradient terms pairing psi^{m+1} (p1) with u^m, for 1 <= m <= nt-1 */
        if (m <= nt - 1) {
            const double *um = uh + nv * m;
            const double *up = uh + nv * (m + 1);
            const double *uo = uh + nv * (m - 1);
#pragma omp parallel
            {
                double *ue = (double *)malloc(sizeof(double) * 3 * n3);
                double *gp = (double *)malloc(sizeof(double) * 9 * n3);
                double *gu = (double *)malloc(sizeof(double) * 9 * n3);
#pragma omp for schedule(static)
                for (int64_t e = 0; e < nspec; ++e) {
                    element_grad(n, D, e, ibool, gam, p1, ue, gp);
                    element_grad(n, D, e, ibool, gam, um, ue, gu);
                    for (int k = 0; k < n; ++k)
                    for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) {
                        int q = i + n * (j + n * k);
                        int64_t p = e * n3 + q;
                        double W = w[i] * w[j] * w[k] * jac[p];
                        const double *A = gp + 9 * q, *B = gu + 9 * q;
                        double divp = A[0] + A[4] + A[8], divu = B[0] + B[4] + B[8];
                        double ee = 0.0;
                        for (int c = 0; c < 3; ++c)
                            for (int b = 0; b < 3; ++b)
                                ee += 0.5 * (A[3 * c + b] + A[3 * b + c]) * 0.5 * (B[3 * c + b] + B[3 * b + c]);
                        g_lam[p] += -dt * dt * W * divp * divu;
                        g_mu[p] += -dt * dt * 2.0 * W * ee;
                        int64_t gq = ibool[p];
                        double acc = 0.0;
                        for (int c = 0; c < 3; ++c)
                            acc += p1[3 * gq + c] * (up[3 * gq + c] - 2.0 * um[3 * gq + c] + uo[3 * gq + c]);
                        g_rho[p] += -W * acc;
                    }
                }
                free(ue); free(gp); free(gu);
            }
        }
        double *tmp = p0; p0 = p1; p1 = p2; p2 = tmp;
    }
    /* p1 now holds psi^1: the start-up term -W psi^1 . u^1 */
    {
        const double *u1 = uh + nv * 1;
        for (int64_t e = 0; e < nspec; ++e)
            for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int64_t p = e * n3 + i + n * (j + n * k);
                double W = w[i] * w[j] * w[k] * jac[p];
                int64_t gq = ibool[p];
                double acc = 0.0;
                for (int c = 0; c < 3; ++c) acc += p1[3 * gq + c] * u1[3 * gq + c];
                g_rho[p] += -W * acc;
            }
    }
    free(uh); free(mass); free(rwt); free(p0); free(p1); free(p2); free(kf); free(gsrc);
    return 0;
}
