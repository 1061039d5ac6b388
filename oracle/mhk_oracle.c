/*
 * Reference CPU implementation of the kernel-split potential evaluation for
 * the 2D modified Helmholtz equation (-Lap + alpha^2) u = f, G = K0(alpha r)/2pi.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the GPU
 * library is checked.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code with the GPU path: no headers, tables or helpers.
 *
 * What it computes, per target x (Section 2.1 of the paper, "Decomposition
 * of volume and layer potentials"):
 *   S[sigma](x) = S_H + sum_{j=1..J} S_{L,D}^{(j)} + S_{L,A}
 *   D[mu](x)    = D_H + sum_{j=1..J} D_{L,D}^{(j)} + D_{L,A}
 *   V[f](x)     = V_H + V_L
 * The history part (t > delta) and the dyadic levels are summed DIRECTLY in
 * real space over every source (no NUFFT, no cell lists, no truncation
 * radius), so that a difference to the fast method measures only the fast
 * method's own approximations (Fourier truncation, periodic images, window
 * error, level cut-off radius, rounding).
 *
 * Precision: FP64 throughout; the closed forms of the local expansions
 * (Lemmas 4.1, 4.5, 4.8 and their corollaries) are evaluated in __float128
 * because their defining expressions cancel for small c2 = alpha*sqrt(delta*).
 *
 * Readings of the paper that this file follows (each one is pinned by a
 * test under tests/):
 *  - incomplete Bessel convention K_nu(x,y) = int_1^inf s^(nu-1) e^(-xs-y/s) ds
 *    (difference kernels of eqs. (diffker_s), (diffker_dlp));
 *  - Z in Lemma 4.1 carries a factor c2: Z = 4 c2 exp(-c1^2/4-c2^2)/sqrt(pi);
 *  - rho in Lemmas 4.1/4.5 is +1 for targets inside Omega and -1 outside
 *    (i.e. measured along the inward normal);
 *  - local terms are kept through first order in delta* (Section 4.1: error
 *    O(delta*^{3/2})); V uses delta in place of delta* (Section 4.2);
 *  - dyadic level j uses every panel bisected j times, geometry and density
 *    at the child nodes interpolated with the parent's degree-15 polynomial;
 *  - V at exterior targets closer than sqrt(delta)(12+2 alpha sqrt(delta))
 *    to the boundary has no formula in the paper (Lemma 4.8 holds inside);
 *    it is taken from the complement domain, which contains the target:
 *    V_L = delta f0 [(1 - e^{-c2^2})/c2^2 - W0/4] with f0 the value of f at
 *    the closest boundary point (panel interpolation of f at the boundary
 *    nodes, the on-surface entries of f_trg); NaN when those are not given.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <quadmath.h>

#define OR_NGL 16          /* Gauss-Legendre nodes per boundary panel        */
#define OR_QN 20           /* nodes of the composite rule for u-integrals    */

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1] by Newton iteration on P_n                 */
/* ------------------------------------------------------------------------ */
static void or_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        long double t = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = t;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
                p0 = p1; p1 = p2;
            }
            /* p1 = P_n(t), p0 = P_{n-1}(t) */
            long double dp = n * (t * p1 - p0) / (t * t - 1.0L);
            long double dt = p1 / dp;
            t -= dt;
            if (fabsl(dt) < 1e-19L) break;
        }
        long double p0 = 1.0L, p1 = t;
        for (int k = 2; k <= n; ++k) {
            long double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
            p0 = p1; p1 = p2;
        }
        long double dp = n * (t * p1 - p0) / (t * t - 1.0L);
        /* ascending order */
        x[n - 1 - i] = (double)t;
        w[n - 1 - i] = (double)(2.0L / ((1.0L - t * t) * dp * dp));
    }
}

static double g_qx[OR_QN], g_qw[OR_QN];
static double g_bx[OR_NGL], g_bw[OR_NGL];
static int g_init = 0;

static void or_init(void)
{
    if (g_init) return;
    or_gauss_legendre(OR_QN, g_qx, g_qw);
    or_gauss_legendre(OR_NGL, g_bx, g_bw);
    g_init = 1;
}

void or_gl_rule(int n, double *x, double *w) { or_gauss_legendre(n, x, w); }

/* ------------------------------------------------------------------------ */
/* Time integrals of the heat kernel H(t,x) = exp(-|x|^2/4t - alpha^2 t)/4pi t
 * (eq. (H_ker)).  With t = T e^{-u} every piece becomes
 *     I_p(a,b;lo,hi) = int_lo^hi exp(-a e^u - b e^{-u} + p u) du,
 * a = r^2/(4T), b = alpha^2 T.  The integrand is below e^-745 where
 * a e^u > 745 or b e^-u > 745, so the range is clipped there.  Composite
 * Gauss-Legendre with panels no wider than the integrand's peak width.      */
/* ------------------------------------------------------------------------ */
static double or_uint(double a, double b, double lo, double hi, int p)
{
    if (a > 0.0) { double c = log(745.0 / a); if (c < hi) hi = c; }
    if (b > 0.0) { double c = log(b / 745.0); if (c > lo) lo = c; }
    if (!(hi > lo)) return 0.0;
    double L = 3.0 / sqrt(1.0 + 2.0 * sqrt(a * b));
    if (L > 1.0) L = 1.0;
    int m = (int)ceil((hi - lo) / L);
    if (m < 1) m = 1;
    double h = (hi - lo) / m, s = 0.0;
    for (int i = 0; i < m; ++i) {
        double c = lo + (i + 0.5) * h, ps = 0.0;
        for (int q = 0; q < OR_QN; ++q) {
            double u = c + 0.5 * h * g_qx[q];
            ps += g_qw[q] * exp(-a * exp(u) - b * exp(-u) + p * u);
        }
        s += 0.5 * h * ps;
    }
    return s;
}

/* Both p=0 and p=1 integrals with one set of exponentials. */
static void or_uint2(double a, double b, double lo, double hi, double *i0, double *i1)
{
    *i0 = 0.0; *i1 = 0.0;
    if (a > 0.0) { double c = log(745.0 / a); if (c < hi) hi = c; }
    if (b > 0.0) { double c = log(b / 745.0); if (c > lo) lo = c; }
    if (!(hi > lo)) return;
    double L = 3.0 / sqrt(1.0 + 2.0 * sqrt(a * b));
    if (L > 1.0) L = 1.0;
    int m = (int)ceil((hi - lo) / L);
    if (m < 1) m = 1;
    double h = (hi - lo) / m, s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < m; ++i) {
        double c = lo + (i + 0.5) * h, p0 = 0.0, p1 = 0.0;
        for (int q = 0; q < OR_QN; ++q) {
            double u = c + 0.5 * h * g_qx[q];
            double eu = exp(u);
            double e = g_qw[q] * exp(-a * eu - b / eu);
            p0 += e; p1 += e * eu;
        }
        s0 += 0.5 * h * p0; s1 += 0.5 * h * p1;
    }
    *i0 = s0; *i1 = s1;
}

#define OR_PI 3.14159265358979323846
#define OR_LN4 1.38629436111989061883

/* History kernel G^H(r) = int_delta^inf H dt  (eq. (sl_sh), t > delta). */
double or_GH(double r, double alpha, double delta)
{
    or_init();
    return or_uint(r * r / (4.0 * delta), alpha * alpha * delta, -INFINITY, 0.0, 0) / (4.0 * OR_PI);
}

/* History factor of the double layer: the normal derivative of H in the
 * source variable is nu'.(x-x')/(2t) H, so D_H = sum w mu nu.(x-x') GHD(r)
 * with GHD(r) = int_delta^inf H/(2t) dt. */
double or_GHD(double r, double alpha, double delta)
{
    or_init();
    return or_uint(r * r / (4.0 * delta), alpha * alpha * delta, -INFINITY, 0.0, 1) / (8.0 * OR_PI * delta);
}

/* Real-space (Ewald) part G^R(r, d) = int_0^d H dt  (eqs. (equiv_split), (ewald_real)). */
double or_GR(double r, double alpha, double d)
{
    or_init();
    return or_uint(r * r / (4.0 * d), alpha * alpha * d, 0.0, INFINITY, 0) / (4.0 * OR_PI);
}

/* Difference kernels of level j: time interval [delta/4^j, delta/4^(j-1)]
 * (eqs. (diffker_s), (diffker_dlp)).  With T = delta_j = delta/4^(j-1) the
 * interval is u in [0, ln 4]. */
double or_KS(double r, double alpha, double delta, int j)
{
    or_init();
    double dj = delta / pow(4.0, j - 1);
    return or_uint(r * r / (4.0 * dj), alpha * alpha * dj, 0.0, OR_LN4, 0) / (4.0 * OR_PI);
}

double or_KD(double r, double alpha, double delta, int j)
{
    or_init();
    double dj = delta / pow(4.0, j - 1);
    return or_uint(r * r / (4.0 * dj), alpha * alpha * dj, 0.0, OR_LN4, 1) / (8.0 * OR_PI * dj);
}

/* ------------------------------------------------------------------------ */
/* Local expansion coefficients (Lemma 4.1, 4.5, 4.8), in __float128.        */
/* out: [0]Phi- [1]Phi+ [2]Z [3..6]P0..P3 [7,8]Q0,Q1 [9..13]U0..U4          */
/*      [14]lambda [15]W0 [16]W1                                             */
/* ------------------------------------------------------------------------ */
void or_local_coeffs(double c1d, double c2d, double *out)
{
    __float128 c1 = c1d, c2 = c2d;
    __float128 em = expq(-c1 * c2), ep = expq(c1 * c2);
    __float128 phim = em * erfcq(c1 / 2 - c2) - ep * erfcq(c1 / 2 + c2);
    __float128 phip = em * erfcq(c1 / 2 - c2) + ep * erfcq(c1 / 2 + c2);
    __float128 Z = 4 * c2 * expq(-c1 * c1 / 4 - c2 * c2) / sqrtq(M_PIq);
    __float128 cm[5];
    cm[0] = 1; for (int m = 1; m < 5; ++m) cm[m] = cm[m - 1] * c1;
    out[0] = (double)phim; out[1] = (double)phip; out[2] = (double)Z;
    for (int m = 0; m < 4; ++m) out[3 + m] = (double)(cm[m] * phim / c2);
    for (int m = 0; m < 2; ++m)
        out[7 + m] = (double)(cm[m] * ((phim - Z) / (c2 * c2 * c2) + c1 * phip / (c2 * c2)));
    for (int m = 0; m < 5; ++m) out[9 + m] = (double)(cm[m] * phip);
    __float128 e2 = expq(-c2 * c2);
    __float128 lam = e2 * erfcq(c1 / 2);
    __float128 W0 = (4 - 4 * e2 + 2 * lam - phip) / (c2 * c2);
    __float128 P1 = c1 * phim / c2;
    __float128 W1 = (2 * W0 - P1 + 4 * (lam - 2 * e2)) / (c2 * c2);
    out[14] = (double)lam; out[15] = (double)W0; out[16] = (double)W1;
}

/* ------------------------------------------------------------------------ */
/* Panel polynomials.  A function sampled at the 16 Gauss-Legendre nodes of
 * a panel is the degree-15 polynomial with Legendre coefficients
 * c_k = (2k+1)/2 sum_i w_i P_k(t_i) f_i (exact by Gauss-Legendre
 * orthogonality).  Values and t-derivatives from the Legendre recurrences.  */
/* ------------------------------------------------------------------------ */
static void or_legendre_all(double t, double *P, double *dP, double *ddP)
{
    P[0] = 1.0; dP[0] = 0.0; ddP[0] = 0.0;
    P[1] = t;   dP[1] = 1.0; ddP[1] = 0.0;
    for (int k = 1; k < OR_NGL - 1; ++k) {
        P[k + 1] = ((2 * k + 1) * t * P[k] - k * P[k - 1]) / (k + 1);
        dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
        ddP[k + 1] = ddP[k - 1] + (2 * k + 1) * dP[k];
    }
}

static void or_coeffs(const double *f, int stride, double *c)
{
    double P[OR_NGL], dP[OR_NGL], ddP[OR_NGL];
    for (int k = 0; k < OR_NGL; ++k) c[k] = 0.0;
    for (int i = 0; i < OR_NGL; ++i) {
        or_legendre_all(g_bx[i], P, dP, ddP);
        for (int k = 0; k < OR_NGL; ++k) c[k] += g_bw[i] * P[k] * f[i * stride];
    }
    for (int k = 0; k < OR_NGL; ++k) c[k] *= (2 * k + 1) / 2.0;
}

static void or_eval_poly(const double *c, double t, double *v, double *d1, double *d2)
{
    double P[OR_NGL], dP[OR_NGL], ddP[OR_NGL];
    or_legendre_all(t, P, dP, ddP);
    double a = 0, b = 0, e = 0;
    for (int k = 0; k < OR_NGL; ++k) { a += c[k] * P[k]; b += c[k] * dP[k]; e += c[k] * ddP[k]; }
    if (v) *v = a;
    if (d1) *d1 = b;
    if (d2) *d2 = e;
}

/* P_k and their first four t-derivatives, by the recurrences
 * P_{k+1}^{(m)} = P_{k-1}^{(m)} + (2k+1) P_k^{(m-1)}.                        */
static void or_legendre_d4(double t, double D[5][OR_NGL])
{
    double dP[OR_NGL], ddP[OR_NGL];
    or_legendre_all(t, D[0], dP, ddP);
    for (int k = 0; k < OR_NGL; ++k) { D[1][k] = dP[k]; D[2][k] = ddP[k]; }
    for (int m = 3; m <= 4; ++m) {
        D[m][0] = 0.0; D[m][1] = 0.0;
        for (int k = 1; k < OR_NGL - 1; ++k) D[m][k + 1] = D[m][k - 1] + (2 * k + 1) * D[m - 1][k];
    }
}

/* Taylor coefficients F_0..F_4 in tau = t - t* of the panel polynomial c. */
static void or_taylor(const double *c, double D[5][OR_NGL], double F[5])
{
    static const double fact[5] = {1, 1, 2, 6, 24};
    for (int m = 0; m <= 4; ++m) {
        double a = 0.0;
        for (int k = 0; k < OR_NGL; ++k) a += c[k] * D[m][k];
        F[m] = a / fact[m];
    }
}

/* Local data at a boundary point in the tangent-line parameterisation of
 * Section 4.1: xi along the unit tangent T0 (increasing t), the boundary the
 * graph eta = gamma(xi) along the inward normal N0, gamma(xi) = kappa0 xi^2/2
 * + g3 xi^3/6 + g4 xi^4/24 + ...  Derivatives in xi of a function on the
 * boundary follow from its Taylor series in tau = t - t* and the reversion of
 * xi(tau) = c1 tau + c2 tau^2 + c3 tau^3 + c4 tau^4, i.e.
 * tau = b1 xi + b2 xi^2 + b3 xi^3 + b4 xi^4.                                  */
typedef struct {
    double T0x, T0y, N0x, N0y;      /* unit tangent and inward normal            */
    double b[5];                    /* reversion coefficients b1..b4 (b[0] = 0)   */
    double kh, g3, g4;              /* second, third, fourth xi-derivative of the graph */
} or_tl;

/* d^m/dxi^m, m = 0..4, of a function with Taylor coefficients F in tau */
static void or_xi_derivs(const or_tl *L, const double F[5], double d[5])
{
    const double b1 = L->b[1], b2 = L->b[2], b3 = L->b[3], b4 = L->b[4];
    const double g1 = F[1] * b1;
    const double g2 = F[1] * b2 + F[2] * b1 * b1;
    const double g3 = F[1] * b3 + F[2] * 2.0 * b1 * b2 + F[3] * b1 * b1 * b1;
    const double g4 = F[1] * b4 + F[2] * (b2 * b2 + 2.0 * b1 * b3) + F[3] * 3.0 * b1 * b1 * b2 + F[4] * b1 * b1 * b1 * b1;
    d[0] = F[0]; d[1] = g1; d[2] = 2.0 * g2; d[3] = 6.0 * g3; d[4] = 24.0 * g4;
}

static void or_tangent_line(const double *cx, const double *cy, double D[5][OR_NGL], or_tl *L)
{
    double X[5], Y[5];
    or_taylor(cx, D, X);
    or_taylor(cy, D, Y);
    const double sp = sqrt(X[1] * X[1] + Y[1] * Y[1]);
    L->T0x = X[1] / sp; L->T0y = Y[1] / sp;
    L->N0x = -L->T0y; L->N0y = L->T0x;          /* inward for a counter-clockwise curve */
    double c[5], e[5];
    for (int m = 0; m <= 4; ++m) {
        c[m] = X[m] * L->T0x + Y[m] * L->T0y;
        e[m] = X[m] * L->N0x + Y[m] * L->N0y;
    }
    c[0] = 0.0; e[0] = 0.0; e[1] = 0.0;
    const double c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4];
    L->b[0] = 0.0;
    L->b[1] = 1.0 / c1;
    L->b[2] = -c2 / (c1 * c1 * c1);
    L->b[3] = (2.0 * c2 * c2 - c1 * c3) / pow(c1, 5);
    L->b[4] = (5.0 * c1 * c2 * c3 - c1 * c1 * c4 - 5.0 * c2 * c2 * c2) / pow(c1, 7);
    double h[5];
    or_xi_derivs(L, e, h);
    L->kh = h[2]; L->g3 = h[3]; L->g4 = h[4];
}

/* ------------------------------------------------------------------------ */
/* Problem description                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double alpha, delta;        /* kernel parameter and history split        */
    int J;                      /* dyadic levels, delta* = delta/4^J         */
    int parts;                  /* bit 0 history, bit 1 levels, bit 2 local  */
    /* boundary: n_panels*16 nodes, panel-contiguous, counter-clockwise      */
    int64_t n_panels;
    const double *bx, *by, *bnx, *bny, *bw, *bkappa;
    const int64_t *panel_prev, *panel_next;
    /* volume quadrature */
    int64_t n_vol;
    const double *vx, *vy, *vw;
    /* off-surface targets */
    int64_t n_trg;
    const double *tx, *ty;
    const int8_t *inside;
    int on_surface;             /* 1: boundary nodes appended as targets     */
    /* densities */
    const double *sigma, *mu, *f_vol, *f_trg;   /* f_trg: n_trg (+n_B)        */
    /* local expansions kept to first order (1, Section 4.1) or to the
     * printed second-order terms (2): then f_jet holds the gradient and the
     * Hessian of f at the targets, [5][n_trg (+n_B)] = f_x, f_y, f_xx, f_xy,
     * f_yy (Lemma 4.8 and its corollaries need f_eta, f_eta eta, f_xi xi) */
    int local_order;
    const double *f_jet;
} or_problem;

/* ------------------------------------------------------------------------ */
/* Dyadic refinement (Section 4.2): every panel bisected j times; child
 * nodes carry interpolated x, y, speed, normal (renormalised), sigma, mu;
 * child weight = w_GL * speed * 2^-j.                                        */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t n; double *x, *y, *nx, *ny, *w, *s, *m; } or_level;

static void or_refine(const or_problem *P, int j, or_level *L)
{
    int64_t nch = (int64_t)1 << j;
    int64_t n = P->n_panels * nch * OR_NGL;
    L->n = n;
    L->x = malloc(sizeof(double) * n); L->y = malloc(sizeof(double) * n);
    L->nx = malloc(sizeof(double) * n); L->ny = malloc(sizeof(double) * n);
    L->w = malloc(sizeof(double) * n); L->s = malloc(sizeof(double) * n);
    L->m = malloc(sizeof(double) * n);
    double scale = 1.0 / (double)nch;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P->n_panels; ++p) {
        double cx[OR_NGL], cy[OR_NGL], cnx[OR_NGL], cny[OR_NGL], csp[OR_NGL], cs[OR_NGL], cm[OR_NGL];
        double sp[OR_NGL];
        const int64_t o = p * OR_NGL;
        for (int i = 0; i < OR_NGL; ++i) sp[i] = P->bw[o + i] / g_bw[i];
        or_coeffs(P->bx + o, 1, cx); or_coeffs(P->by + o, 1, cy);
        or_coeffs(P->bnx + o, 1, cnx); or_coeffs(P->bny + o, 1, cny);
        or_coeffs(sp, 1, csp);
        if (P->sigma) or_coeffs(P->sigma + o, 1, cs); else memset(cs, 0, sizeof cs);
        if (P->mu) or_coeffs(P->mu + o, 1, cm); else memset(cm, 0, sizeof cm);
        for (int64_t c = 0; c < nch; ++c) {
            for (int k = 0; k < OR_NGL; ++k) {
                double t = -1.0 + (2.0 * c + 1.0 + g_bx[k]) * scale;
                int64_t q = (p * nch + c) * OR_NGL + k;
                double vnx, vny, vsp;
                or_eval_poly(cx, t, &L->x[q], NULL, NULL);
                or_eval_poly(cy, t, &L->y[q], NULL, NULL);
                or_eval_poly(cnx, t, &vnx, NULL, NULL);
                or_eval_poly(cny, t, &vny, NULL, NULL);
                double nn = sqrt(vnx * vnx + vny * vny);
                L->nx[q] = vnx / nn; L->ny[q] = vny / nn;
                or_eval_poly(csp, t, &vsp, NULL, NULL);
                L->w[q] = g_bw[k] * vsp * scale;
                or_eval_poly(cs, t, &L->s[q], NULL, NULL);
                or_eval_poly(cm, t, &L->m[q], NULL, NULL);
            }
        }
    }
}

static void or_level_free(or_level *L)
{
    free(L->x); free(L->y); free(L->nx); free(L->ny); free(L->w); free(L->s); free(L->m);
}

/* Exported: refined nodes of level j (for tests). Arrays of n_panels*2^j*16. */
int or_refine_level(const or_problem *P, int j, double *x, double *y, double *nx, double *ny,
                    double *w, double *s, double *m)
{
    or_init();
    or_level L;
    or_refine(P, j, &L);
    memcpy(x, L.x, sizeof(double) * L.n); memcpy(y, L.y, sizeof(double) * L.n);
    memcpy(nx, L.nx, sizeof(double) * L.n); memcpy(ny, L.ny, sizeof(double) * L.n);
    memcpy(w, L.w, sizeof(double) * L.n); memcpy(s, L.s, sizeof(double) * L.n);
    memcpy(m, L.m, sizeof(double) * L.n);
    or_level_free(&L);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Closest boundary point (Section 3.2): nearest node by brute force (lowest
 * index on ties) selects a panel; the squared distance to that panel's
 * polynomial and to its two neighbours' is minimised over t in [-1,1] and
 * the best of the three is kept.  On each panel the minimisation is
 * Newton's method on d/dt |x - gamma(t)|^2 = 0, started from the nearest of
 * the panel's two end points and 16 nodes, safeguarded as the reading of the
 * paper's "Newton" that always ends at a local minimum: a step that does not
 * decrease the distance is halved, and where the squared distance is not
 * convex a fixed step of 1/4 downhill replaces the Newton step; Newton steps
 * below 1e-6 where it is convex are taken as they are (the distance is flat
 * below its rounding there) and end the iteration once one is below 1e-12,
 * after one more Newton step; a damped step below 1e-15 also ends it.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t panel; double t, x0, y0, r;
    double tx, ty;      /* gamma'(t)   */
    double txx, tyy;    /* gamma''(t)  */
} or_cp;

static double or_d2(const double *cx, const double *cy, double t, double px, double py)
{
    double x, y;
    or_eval_poly(cx, t, &x, NULL, NULL);
    or_eval_poly(cy, t, &y, NULL, NULL);
    return (x - px) * (x - px) + (y - py) * (y - py);
}

/* returns 1 when the iteration converged */
static int or_panel_min(const double *cx, const double *cy, const double *nx, const double *ny,
                        double px, double py, double *tbest, double *d2best)
{
    /* start: the nearest of the end point -1, the nodes, the end point +1 */
    double bt = -1.0, bd = or_d2(cx, cy, -1.0, px, py);
    for (int i = 0; i < OR_NGL; ++i) {
        double d = (nx[i] - px) * (nx[i] - px) + (ny[i] - py) * (ny[i] - py);
        if (d < bd) { bd = d; bt = g_bx[i]; }
    }
    {
        double d = or_d2(cx, cy, 1.0, px, py);
        if (d < bd) { bd = d; bt = 1.0; }
    }
    double t = bt, phi = or_d2(cx, cy, t, px, py);
    int conv = 0;
    for (int it = 0; it < 60; ++it) {
        double x, y, x1, y1, x2, y2;
        or_eval_poly(cx, t, &x, &x1, &x2);
        or_eval_poly(cy, t, &y, &y1, &y2);
        double g = (x - px) * x1 + (y - py) * y1;
        double h = x1 * x1 + y1 * y1 + (x - px) * x2 + (y - py) * y2;
        double step = h > 0.0 ? -g / h : (g > 0.0 ? -0.25 : 0.25);
        double tn = fmin(1.0, fmax(-1.0, t + step));
        if (h > 0.0 && fabs(step) < 1e-6) {
            /* near a minimum the distance is flat below its rounding: plain
               Newton steps, driven by the derivative */
            /* quadratic convergence: after a step below 1e-12 the error is at
               the rounding level */
            double moved = fabs(tn - t);
            t = tn;
            if (moved < 1e-12) {
                /* one more Newton step brings t to the rounding level also
                   where the convergence is slow */
                or_eval_poly(cx, t, &x, &x1, &x2);
                or_eval_poly(cy, t, &y, &y1, &y2);
                double h2 = x1 * x1 + y1 * y1 + (x - px) * x2 + (y - py) * y2;
                if (h2 > 0.0) t = fmin(1.0, fmax(-1.0, t - ((x - px) * x1 + (y - py) * y1) / h2));
                conv = 1;
                break;
            }
            continue;
        }
        double dn = phi;
        for (int k = 0; k <= 52; ++k) {
            dn = or_d2(cx, cy, tn, px, py);
            if (dn <= phi) break;
            step *= 0.5;
            tn = fmin(1.0, fmax(-1.0, t + step));
        }
        double moved = fabs(tn - t);
        if (dn <= phi) { t = tn; phi = dn; }
        if (moved < 1e-15) { conv = 1; break; }
    }
    phi = or_d2(cx, cy, t, px, py);
    *tbest = t;
    *d2best = phi;
    return conv;
}

static void or_closest(const or_problem *P, double px, double py, or_cp *cp)
{
    int64_t nb = P->n_panels * OR_NGL, best = 0;
    double bd = INFINITY;
    for (int64_t i = 0; i < nb; ++i) {
        double dx = px - P->bx[i], dy = py - P->by[i];
        double d = dx * dx + dy * dy;
        if (d < bd) { bd = d; best = i; }
    }
    int64_t p0 = best / OR_NGL;
    int64_t cand[3] = { p0, P->panel_prev[p0], P->panel_next[p0] };
    double dbest = INFINITY;
    for (int c = 0; c < 3; ++c) {
        int64_t p = cand[c];
        double cx[OR_NGL], cy[OR_NGL], t, d2;
        or_coeffs(P->bx + p * OR_NGL, 1, cx);
        or_coeffs(P->by + p * OR_NGL, 1, cy);
        or_panel_min(cx, cy, P->bx + p * OR_NGL, P->by + p * OR_NGL, px, py, &t, &d2);
        if (d2 < dbest) {
            dbest = d2;
            cp->panel = p; cp->t = t;
            or_eval_poly(cx, t, &cp->x0, &cp->tx, &cp->txx);
            or_eval_poly(cy, t, &cp->y0, &cp->ty, &cp->tyy);
        }
    }
    cp->r = sqrt((px - cp->x0) * (px - cp->x0) + (py - cp->y0) * (py - cp->y0));
}

/* Exported closest point for tests: out = panel, t, x0, y0, r */
int or_closest_point(const or_problem *P, double px, double py, double *out)
{
    or_init();
    or_cp cp;
    or_closest(P, px, py, &cp);
    out[0] = (double)cp.panel; out[1] = cp.t; out[2] = cp.x0; out[3] = cp.y0; out[4] = cp.r;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Local parts (Lemmas 4.1, 4.5, 4.8; Corollaries 4.4, 4.7, 4.10, 4.11) to
 * first order in delta* (order 1, as Section 4.1 keeps them) or with the
 * printed second-order terms (order 2).                                       */
/* ------------------------------------------------------------------------ */
typedef struct { double S, D; } or_sd;

/* Boundary data at the closest point for the second-order terms: the graph
 * derivatives g3, g4 of the tangent-line parameterisation and the
 * xi-derivatives s[0..4], m[0..4] of sigma and mu. */
typedef struct { double g3, g4, s[5], m[5]; } or_bjet;

/* (2 erf(c2) - 4 c2 e^{-c2^2}/sqrt(pi)) / c2^3, the c1 = 0 value of Q0 */
static __float128 or_q0_on(__float128 c2)
{
    return (2 * erfq(c2) - 4 * c2 * expq(-c2 * c2) / sqrtq(M_PIq)) / (c2 * c2 * c2);
}

/* (1 - (1 + c2^2) e^{-c2^2}) / c2^4 */
static __float128 or_v2(__float128 c2)
{
    __float128 a = c2 * c2;
    return (-expm1q(-a) - a * expq(-a)) / (a * a);
}

/* Off-surface, layer potentials: x0 data given. */
static or_sd or_local_layer(double r, double rho, double ds, double alpha, double kappa0, double sigma0,
                            double mu0, double mu0pp, int order, const or_bjet *J)
{
    or_sd o = { 0.0, 0.0 };
    double sq = sqrt(ds);
    double c2 = alpha * sq;
    if (r >= sq * (12.0 + 2.0 * c2)) return o;       /* Remark 4.3 */
    double c[17];
    or_local_coeffs(r / sq, c2, c);
    double P0 = c[3], P1 = c[4], U0 = c[9], U1 = c[10], U2 = c[11];
    o.S = sq * sigma0 * P0 / 4.0 + ds * rho * kappa0 * sigma0 * P1 / 8.0;
    o.D = -rho * mu0 * U0 / 4.0 - sq * kappa0 * mu0 * (P0 + U1) / 8.0
          - ds * (rho * mu0pp * P1 / 8.0 + 3.0 * rho * kappa0 * kappa0 * mu0 * (P1 + U2) / 32.0);
    if (order >= 2) {
        const double P2 = c[5], P3 = c[6], Q0 = c[7], Q1 = c[8], U3 = c[12], U4 = c[13];
        const double k = kappa0, g3 = J->g3, g4 = J->g4;
        const double s1 = J->s[1], s2 = J->s[2], m1 = J->m[1], m2 = J->m[2], m4 = J->m[4];
        const double d32 = ds * sq, d2 = ds * ds;
        /* eq. (slp_local1), delta*^{3/2} and delta*^2 terms */
        o.S += d32 * (k * k * sigma0 / 32.0 * (Q0 + 3.0 * P2) + s2 / 8.0 * Q0)
               + d2 * rho * (k * k * k * sigma0 / 64.0 * (-3.0 * Q1 + 5.0 * P3)
                             + (3.0 * k * s2 / 16.0 + s1 * g3 / 8.0 + sigma0 * g4 / 32.0) * Q1);
        /* eq. (dlp_local1), delta*^{3/2} and delta*^2 terms.  Reading: the
         * gamma'''' term of the delta*^{3/2} bracket is -mu0 g4 (3 Q0 + P2)/32;
         * the printed lemma groups it with the kappa^3 term under
         * (3 Q0 - U3).  The series expansion of the local integral (tangent-
         * line coordinates, Gaussian moments in xi) gives the form used
         * here, both agree at c1 = 0 (Corollary 4.7), and only this form
         * converges at order 5/2 against brute-force quadrature. */
        o.D += d32 * (5.0 * k * k * k * mu0 / 64.0 * (3.0 * Q0 - U3) - mu0 * g4 / 32.0 * (3.0 * Q0 + P2)
                      + 3.0 * k * m2 / 16.0 * (-Q0 - P2) + m1 * g3 / 8.0 * (-2.0 * Q0 - P2))
               + d2 * (35.0 * rho * k * k * k * k * mu0 / 512.0 * (9.0 * Q1 + 2.0 * P3 - U4)
                       - rho * m4 / 32.0 * Q1 - 15.0 * rho * k * k * m2 / 64.0 * (Q1 + P3))
               - d2 * (5.0 * rho * k * m1 * g3 / 16.0 * (2.0 * Q1 + P3)
                       + (5.0 * rho * k * mu0 * g4 / 64.0 + 5.0 * rho * mu0 * g3 * g3 / 96.0) * (3.0 * Q1 + P3));
    }
    return o;
}

/* On-surface layer potentials (Corollaries 4.4 and 4.7). */
static or_sd or_local_layer_on(double ds, double alpha, double kappa0, double sigma0, double mu0, int order,
                               const or_bjet *J)
{
    or_sd o;
    __float128 sq = sqrtq((__float128)ds), c2 = alpha * sq;
    __float128 e = erfq(c2) / c2;
    o.S = (double)(sq * sigma0 * e / 2);
    o.D = (double)(-sq * kappa0 * mu0 * e / 4);
    if (order >= 2) {
        const __float128 q = or_q0_on(c2) * sq * sq * sq, k = kappa0;
        o.S += (double)(q * (k * k * sigma0 / 32 + (__float128)J->s[2] / 8));
        o.D += (double)(q * (15 * k * k * k * mu0 / 64 - 3 * (__float128)mu0 * J->g4 / 32
                             - 3 * k * (__float128)J->m[2] / 16 - (__float128)J->m[1] * J->g3 / 4));
    }
    return o;
}

/* f and its derivatives at the target in the frame of the closest point:
 * f_eta along the inward normal N0 and the second derivatives along N0 and
 * along the tangent T0 (Lemma 4.8); lap = f_xx + f_yy. */
typedef struct { double fe, fee, fxx, lap; } or_fjet;

/* Volume local part with delta (Lemma 4.8 / Cor. 4.10 / Cor. 4.11).
 * where: 0 interior off-surface, 1 on-surface, 2 exterior off-surface.
 * Exterior targets (the paper's lemma holds inside Omega): the local
 * integral over Omega is the whole-plane integral minus the one over the
 * complement, and the complement is a domain that contains x, so Lemma 4.8
 * applies to it; to first order, with f taken at the closest boundary
 * point (f0; the difference to f(x) is of the neglected order),
 * V_L = delta f0 [(1 - e^{-c2^2})/c2^2 - W0(c1, c2)/4].  f0 is NaN when f on
 * the boundary is unknown.  Order 2 adds the printed delta^{3/2} and
 * delta^2 terms at interior and on-surface targets; exterior targets keep
 * the first-order complement form. */
static double or_local_vol(double r, int where, double delta, double alpha, double f, double kappa0,
                           int order, const or_fjet *F)
{
    __float128 sq = sqrtq((__float128)delta), c2 = alpha * sq;
    double band = (double)(sq * (12 + 2 * c2));
    const int two = order >= 2 && where != 2;
    if (where == 1) {
        double v = (double)(delta * f * (-expm1q(-c2 * c2)) / (2 * c2 * c2));
        if (two)   /* eq. (vp_local2) */
            v += (double)(sq * sq * sq * or_q0_on(c2) * (2 * (__float128)F->fe - (__float128)f * kappa0) / 8
                          + (__float128)delta * delta * (F->fee + F->fxx) / 2 * or_v2(c2));
        return v;
    }
    if (r >= band) {
        if (where == 2) return 0.0;
        double v = (double)(delta * f * (-expm1q(-c2 * c2)) / (c2 * c2));
        if (two)   /* eq. (vp_local3) */
            v += (double)((__float128)delta * delta * F->lap * or_v2(c2));
        return v;
    }
    double c[17];
    or_local_coeffs(r / (double)sq, (double)c2, c);
    if (where == 2)
        return delta * f * ((double)(-expm1q(-c2 * c2) / (c2 * c2)) - c[15] / 4.0);
    double v = delta * f * c[15] / 4.0;
    if (two) {   /* eq. (vp_local1) */
        const double Q0 = c[7], Q1 = c[8], W1 = c[16], k = kappa0;
        v += delta * sqrt(delta) * (2.0 * F->fe - f * k) / 8.0 * Q0
             + delta * delta * ((F->fe * k / 8.0 - 3.0 * f * k * k / 32.0 - F->fee / 8.0) * Q1
                                + (F->fee + F->fxx) / 8.0 * W1);
    }
    return v;
}

/* Second-order data at the boundary point t of panel pn: the graph
 * derivatives and the xi-derivatives of sigma and mu (or_bjet), and f's
 * derivatives at the target in the frame (T0, N0) of that point (or_fjet). */
static void or_boundary_jets(const or_problem *P, const double *cs, const double *cm, int64_t pn, double t,
                             double gx, double gy, double hxx, double hxy, double hyy, or_bjet *BJ, or_fjet *FJ)
{
    double cx[OR_NGL], cy[OR_NGL], D[5][OR_NGL], F[5];
    or_coeffs(P->bx + pn * OR_NGL, 1, cx);
    or_coeffs(P->by + pn * OR_NGL, 1, cy);
    or_legendre_d4(t, D);
    or_tl L;
    or_tangent_line(cx, cy, D, &L);
    BJ->g3 = L.g3;
    BJ->g4 = L.g4;
    or_taylor(cs + pn * OR_NGL, D, F);
    or_xi_derivs(&L, F, BJ->s);
    or_taylor(cm + pn * OR_NGL, D, F);
    or_xi_derivs(&L, F, BJ->m);
    FJ->fe = gx * L.N0x + gy * L.N0y;
    FJ->fee = hxx * L.N0x * L.N0x + 2.0 * hxy * L.N0x * L.N0y + hyy * L.N0y * L.N0y;
    FJ->fxx = hxx * L.T0x * L.T0x + 2.0 * hxy * L.T0x * L.T0y + hyy * L.T0y * L.T0y;
    FJ->lap = hxx + hyy;
}

/* ------------------------------------------------------------------------ */
/* Full evaluation.  Output arrays have n_trg (+ n_B if on_surface) entries.
 * If `subset` is non-NULL only targets subset[0..n_subset) are evaluated and
 * written densely to S/D/V[0..n_subset).                                     */
/* ------------------------------------------------------------------------ */
int or_eval(const or_problem *P, const int64_t *subset, int64_t n_subset,
            double *S, double *D, double *V)
{
    or_init();
    const int64_t nb = P->n_panels * OR_NGL;
    const int64_t ntot = P->n_trg + (P->on_surface ? nb : 0);
    const int64_t nout = subset ? n_subset : ntot;
    const double alpha = P->alpha, delta = P->delta;
    const double dstar = delta / pow(4.0, P->J);

    or_level *lev = NULL;
    if ((P->parts & 2) && P->J > 0) {
        lev = malloc(sizeof(or_level) * P->J);
        for (int j = 1; j <= P->J; ++j) or_refine(P, j, &lev[j - 1]);
    }
    /* panel Legendre coefficients of sigma, mu, kappa for local terms */
    double *cs = NULL, *cm = NULL, *ck = NULL, *cf = NULL;
    /* f on the boundary nodes: the on-surface entries of f_trg */
    const double *fb = (P->on_surface && P->f_trg) ? P->f_trg + P->n_trg : NULL;
    if (P->parts & 4) {
        cs = calloc(nb, sizeof(double)); cm = calloc(nb, sizeof(double)); ck = calloc(nb, sizeof(double));
        cf = calloc(nb, sizeof(double));
        for (int64_t p = 0; p < P->n_panels; ++p) {
            if (P->sigma) or_coeffs(P->sigma + p * OR_NGL, 1, cs + p * OR_NGL);
            if (P->mu) or_coeffs(P->mu + p * OR_NGL, 1, cm + p * OR_NGL);
            or_coeffs(P->bkappa + p * OR_NGL, 1, ck + p * OR_NGL);
            if (fb) or_coeffs(fb + p * OR_NGL, 1, cf + p * OR_NGL);
        }
    }

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t o = 0; o < nout; ++o) {
        int64_t it = subset ? subset[o] : o;
        int on = it >= P->n_trg;
        int64_t ib = on ? it - P->n_trg : -1;
        double px = on ? P->bx[ib] : P->tx[it];
        double py = on ? P->by[ib] : P->ty[it];
        int inside = on ? 1 : (P->inside ? P->inside[it] != 0 : 1);
        double s = 0.0, d = 0.0, v = 0.0;

        /* history part: direct real-space sums with G^H and GHD */
        if (P->parts & 1) {
            double a4 = 1.0 / (4.0 * delta), b = alpha * alpha * delta;
            for (int64_t i = 0; i < nb; ++i) {
                double dx = px - P->bx[i], dy = py - P->by[i];
                double i0, i1;
                or_uint2((dx * dx + dy * dy) * a4, b, -INFINITY, 0.0, &i0, &i1);
                double gh = i0 / (4.0 * OR_PI), ghd = i1 / (8.0 * OR_PI * delta);
                if (P->sigma) s += P->bw[i] * P->sigma[i] * gh;
                if (P->mu) d += P->bw[i] * P->mu[i] * (P->bnx[i] * dx + P->bny[i] * dy) * ghd;
            }
            if (P->f_vol) {
                for (int64_t i = 0; i < P->n_vol; ++i) {
                    double dx = px - P->vx[i], dy = py - P->vy[i];
                    double gh = or_uint((dx * dx + dy * dy) * a4, b, -INFINITY, 0.0, 0) / (4.0 * OR_PI);
                    v += P->vw[i] * P->f_vol[i] * gh;
                }
            }
        }
        /* dyadic levels: direct sums over all refined nodes */
        if ((P->parts & 2) && P->J > 0) {
            for (int j = 1; j <= P->J; ++j) {
                const or_level *L = &lev[j - 1];
                double dj = delta / pow(4.0, j - 1);
                double a4 = 1.0 / (4.0 * dj), b = alpha * alpha * dj;
                for (int64_t q = 0; q < L->n; ++q) {
                    double dx = px - L->x[q], dy = py - L->y[q];
                    double a = (dx * dx + dy * dy) * a4;
                    if (a > 40.0) continue;      /* kernel < 1e-17 of its peak */
                    double i0, i1;
                    or_uint2(a, b, 0.0, OR_LN4, &i0, &i1);
                    s += L->w[q] * L->s[q] * i0 / (4.0 * OR_PI);
                    d += L->w[q] * L->m[q] * (L->nx[q] * dx + L->ny[q] * dy) * i1 / (8.0 * OR_PI * dj);
                }
            }
        }
        /* local asymptotic parts */
        if (P->parts & 4) {
            const int order = P->local_order >= 2 ? 2 : 1;
            double fx = P->f_trg ? P->f_trg[it] : 0.0;
            /* gradient and Hessian of f at the target (order 2) */
            double gx = 0, gy = 0, hxx = 0, hxy = 0, hyy = 0;
            if (order >= 2 && P->f_jet) {
                gx = P->f_jet[0 * ntot + it]; gy = P->f_jet[1 * ntot + it];
                hxx = P->f_jet[2 * ntot + it]; hxy = P->f_jet[3 * ntot + it]; hyy = P->f_jet[4 * ntot + it];
            }
            or_bjet BJ;
            or_fjet FJ;
            memset(&BJ, 0, sizeof BJ);
            memset(&FJ, 0, sizeof FJ);
            if (on) {
                double sg = P->sigma ? P->sigma[ib] : 0.0, mm = P->mu ? P->mu[ib] : 0.0;
                if (order >= 2)
                    or_boundary_jets(P, cs, cm, ib / OR_NGL, g_bx[ib % OR_NGL], gx, gy, hxx, hxy, hyy, &BJ, &FJ);
                or_sd l = or_local_layer_on(dstar, alpha, P->bkappa[ib], sg, mm, order, &BJ);
                s += l.S; d += l.D;
                if (P->f_trg) v += or_local_vol(0.0, 1, delta, alpha, fx, P->bkappa[ib], order, &FJ);
            } else {
                double sqs = sqrt(dstar);
                double bandS = sqs * (12.0 + 2.0 * alpha * sqs);
                or_cp cp;
                or_closest(P, px, py, &cp);
                double rho = inside ? 1.0 : -1.0;
                double P_[OR_NGL], dP[OR_NGL], ddP[OR_NGL];
                or_legendre_all(cp.t, P_, dP, ddP);
                const double *a_k = ck + cp.panel * OR_NGL;
                double kk = 0;
                for (int q = 0; q < OR_NGL; ++q) kk += a_k[q] * P_[q];
                if (order >= 2) or_boundary_jets(P, cs, cm, cp.panel, cp.t, gx, gy, hxx, hxy, hyy, &BJ, &FJ);
                if (cp.r < bandS) {
                    const double *a_s = cs + cp.panel * OR_NGL, *a_m = cm + cp.panel * OR_NGL;
                    double sg = 0, mm = 0, mt = 0, mtt = 0;
                    for (int q = 0; q < OR_NGL; ++q) {
                        sg += a_s[q] * P_[q]; mm += a_m[q] * P_[q];
                        mt += a_m[q] * dP[q]; mtt += a_m[q] * ddP[q];
                    }
                    double sp2 = cp.tx * cp.tx + cp.ty * cp.ty;
                    double tdot = cp.tx * cp.txx + cp.ty * cp.tyy;
                    double mss = (mtt - mt * tdot / sp2) / sp2;    /* arclength 2nd derivative */
                    or_sd l = or_local_layer(cp.r, rho, dstar, alpha, kk, sg, mm, mss, order, &BJ);
                    s += l.S; d += l.D;
                }
                if (P->f_trg) {
                    if (!inside) {
                        /* f at the closest boundary point (exterior targets) */
                        double f0 = NAN;
                        if (fb) {
                            f0 = 0.0;
                            for (int q = 0; q < OR_NGL; ++q) f0 += cf[cp.panel * OR_NGL + q] * P_[q];
                        }
                        fx = f0;
                    }
                    v += or_local_vol(cp.r, inside ? 0 : 2, delta, alpha, fx, kk, order, &FJ);
                }
            }
        }
        S[o] = s; D[o] = d; V[o] = v;
    }
    if (lev) { for (int j = 0; j < P->J; ++j) or_level_free(&lev[j]); free(lev); }
    free(cs); free(cm); free(ck); free(cf);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* A dyadic level of the volume potential: out[t] = sum_s q[s] K_j^S(|x_t -  */
/* y_s|) over every source, directly (the level term of V when its local     */
/* part is split in time like the layer potentials', Section 4.2).  Pairs    */
/* with r^2/(4 delta_j) > 40 (K below 1e-17 of K(0)) are skipped.            */
/* ------------------------------------------------------------------------ */
void or_level_sum_S(double alpha, double delta, int j, int64_t ns, const double *sx, const double *sy,
                    const double *q, int64_t nt, const double *tx, const double *ty, double *out)
{
    or_init();
    const double dj = delta / pow(4.0, j - 1);
    const double rmax2 = 160.0 * dj;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; ++t) {
        double acc = 0.0;
        for (int64_t s = 0; s < ns; ++s) {
            const double dx = tx[t] - sx[s], dy = ty[t] - sy[s];
            const double r2 = dx * dx + dy * dy;
            if (r2 > rmax2) continue;
            acc += q[s] * or_KS(sqrt(r2), alpha, delta, j);
        }
        out[t] = acc;
    }
}
