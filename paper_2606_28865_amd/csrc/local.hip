// Local asymptotic part (Section 4.1) and the closest boundary point
// (Section 3.2), in FP64 in both precision paths, plus the final scatter of
// the accumulated potentials to the caller's target order.
//
// For an off-surface target x the nearest boundary node is found from the
// target's closest-point cell, which lists every panel whose node bounding
// box lies within reach = (widest band + largest node gap) of the cell,
// nearest first: panels whose box is farther than the best node so far are
// skipped, so a few panels are scanned node by node.  Whenever the nearest
// node lies within reach of x (the only case in which it is used) its panel
// is in the list, so the result is the global nearest node, ties to the
// lowest index.  Its panel and the two neighbouring panels are searched for
// the closest point x0 by Newton's method on d/dt |x - gamma(t)|^2 = 0,
// started from the best of the panel's nodes and end points.  The geometry, the
// curvature and the densities are evaluated at x0 from their per-panel
// Legendre expansions.  rho = +1 for targets inside Omega, -1 outside, so
// that D jumps by -mu/2 on entering Omega (eq. (jumprel)).
#include "mhk_internal.h"

namespace mhk {

// Legendre coefficients of sigma, mu and (for the exterior volume part) f
// at the boundary nodes on every panel: c = Leg * f (FP64).  f at the
// boundary nodes is the on-surface part of f_trg ([B][nout], entries nt..).
template <typename T>
__global__ void __launch_bounds__(256) k_panel_coeffs(int64_t npan, int B, const double *__restrict__ leg,
                                                      const T *__restrict__ sigma,
                                                      const T *__restrict__ mu,
                                                      const T *__restrict__ f_trg, int64_t nout, int frows, int64_t nt,
                                                      double *__restrict__ cs, double *__restrict__ cm,
                                                      double *__restrict__ cf)
{
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tot = npan * NGL * B;
    if (id >= tot) return;
    int k = (int)(id % NGL);
    int64_t pb = id / NGL;                 // b * npan + p
    const double *row = leg + k * NGL;
    if (sigma) {
        const T *f = sigma + pb * NGL;
        double v = 0;
#pragma unroll
        for (int i = 0; i < NGL; ++i) v = fma(row[i], (double)f[i], v);
        cs[id] = v;
    }
    if (mu) {
        const T *f = mu + pb * NGL;
        double v = 0;
#pragma unroll
        for (int i = 0; i < NGL; ++i) v = fma(row[i], (double)f[i], v);
        cm[id] = v;
    }
    if (f_trg) {
        const int64_t b = pb / npan, p = pb % npan;
        const T *f = f_trg + b * frows * nout + nt + p * NGL;
        double v = 0;
#pragma unroll
        for (int i = 0; i < NGL; ++i) v = fma(row[i], (double)f[i], v);
        cf[id] = v;
    }
}

// Legendre recurrence P_{k+1} = A_k t P_k - B_k P_{k-1}, A_k = (2k+1)/(k+1),
// B_k = k/(k+1): with the loops unrolled, k is a constant and both
// coefficients fold to literals (no division on the device).

// Value and first two t-derivatives of two Legendre series at t, using the
// recurrence above with P'_{k+1} = P'_{k-1} + (2k+1) P_k and
// P''_{k+1} = P''_{k-1} + (2k+1) P'_k.
__device__ inline void leg2(const double *__restrict__ ca, const double *__restrict__ cb, double t,
                            double &a0, double &a1, double &a2, double &b0, double &b1, double &b2)
{
    double pm = 1.0, p = t, dm = 0.0, d = 1.0, em = 0.0, e = 0.0;
    a0 = ca[0] + ca[1] * t;
    a1 = ca[1];
    a2 = 0.0;
    b0 = cb[0] + cb[1] * t;
    b1 = cb[1];
    b2 = 0.0;
#pragma unroll
    for (int k = 1; k < NGL - 1; ++k) {
        const double pn = ((2.0 * k + 1.0) / (k + 1.0)) * t * p - ((double)k / (k + 1.0)) * pm;
        const double dn = dm + (2 * k + 1) * p;
        const double en = em + (2 * k + 1) * d;
        pm = p; p = pn;
        dm = d; d = dn;
        em = e; e = en;
        const double A = ca[k + 1], Bc = cb[k + 1];
        a0 = fma(A, p, a0); a1 = fma(A, d, a1); a2 = fma(A, e, a2);
        b0 = fma(Bc, p, b0); b1 = fma(Bc, d, b1); b2 = fma(Bc, e, b2);
    }
}

// Value and first two t-derivatives of one Legendre series at t.
__device__ inline void leg2s(const double *__restrict__ c, double t, double &v0, double &v1, double &v2)
{
    double pm = 1.0, p = t, dm = 0.0, d = 1.0, em = 0.0, e = 0.0;
    v0 = c[0] + c[1] * t;
    v1 = c[1];
    v2 = 0.0;
#pragma unroll
    for (int k = 1; k < NGL - 1; ++k) {
        const double pn = ((2.0 * k + 1.0) / (k + 1.0)) * t * p - ((double)k / (k + 1.0)) * pm;
        const double dn = dm + (2 * k + 1) * p;
        const double en = em + (2 * k + 1) * d;
        pm = p; p = pn;
        dm = d; d = dn;
        em = e; e = en;
        const double A = c[k + 1];
        v0 = fma(A, p, v0); v1 = fma(A, d, v1); v2 = fma(A, e, v2);
    }
}

__device__ inline double leg1(const double *__restrict__ c, double t)
{
    double pm = 1.0, p = t, v = c[0] + c[1] * t;
#pragma unroll
    for (int k = 1; k < NGL - 1; ++k) {
        const double pn = ((2.0 * k + 1.0) / (k + 1.0)) * t * p - ((double)k / (k + 1.0)) * pm;
        pm = p; p = pn;
        v = fma(c[k + 1], p, v);
    }
    return v;
}

// ---------------------------------------------------------------------------
// Second-order local expansions (local_order = 2)
// ---------------------------------------------------------------------------
// Taylor coefficients F[m] = c^(m)(t)/m!, m = 0..4, of a Legendre series at
// t, with P_{k+1}^(m) = P_{k-1}^(m) + (2k+1) P_k^(m-1) for the derivatives.
__device__ inline void leg_taylor4(const double *__restrict__ c, double t, double F[5])
{
    double pm[5] = {1.0, 0.0, 0.0, 0.0, 0.0}, p[5] = {t, 1.0, 0.0, 0.0, 0.0};
    double v[5] = {c[0] + c[1] * t, c[1], 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 1; k < NGL - 1; ++k) {
        double pn[5];
        pn[0] = ((2.0 * k + 1.0) / (k + 1.0)) * t * p[0] - ((double)k / (k + 1.0)) * pm[0];
#pragma unroll
        for (int m = 1; m < 5; ++m) pn[m] = pm[m] + (2 * k + 1) * p[m - 1];
        const double a = c[k + 1];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            pm[m] = p[m];
            p[m] = pn[m];
            v[m] = fma(a, pn[m], v[m]);
        }
    }
    F[0] = v[0];
    F[1] = v[1];
    F[2] = v[2] * 0.5;
    F[3] = v[3] * (1.0 / 6.0);
    F[4] = v[4] * (1.0 / 24.0);
}

// Derivatives d^m/dxi^m (m = 1, 2, 4; d[0] the value) of a function with
// Taylor coefficients F in tau = t - t*, where tau = b1 xi + b2 xi^2 + b3 xi^3
// + b4 xi^4 is the reversion of the tangent-line coordinate xi(tau).
__device__ inline void xi_derivs(const double F[5], double b1, double b2, double b3, double b4, double d[5])
{
    const double g1 = F[1] * b1;
    const double g2 = F[1] * b2 + F[2] * b1 * b1;
    const double g3 = F[1] * b3 + F[2] * 2.0 * b1 * b2 + F[3] * b1 * b1 * b1;
    const double g4 = F[1] * b4 + F[2] * (b2 * b2 + 2.0 * b1 * b3) + F[3] * 3.0 * b1 * b1 * b2 + F[4] * b1 * b1 * b1 * b1;
    d[0] = F[0];
    d[1] = g1;
    d[2] = 2.0 * g2;
    d[3] = 6.0 * g3;
    d[4] = 24.0 * g4;
}

// Tangent-line parameterisation of the boundary at t on a panel with
// Legendre coefficients cx, cy (Section 4.1): unit tangent T0 (increasing t),
// inward normal N0 = (-T0y, T0x) (counter-clockwise curves), the reversion
// coefficients b1..b4 of xi(tau) = (gamma(t* + tau) - gamma(t*)).T0, and the
// third and fourth xi-derivatives g3, g4 of the boundary's height
// (gamma(t* + tau) - gamma(t*)).N0 over the tangent line.
__device__ inline void tangent_line(const double *__restrict__ cx, const double *__restrict__ cy, double t,
                                    double &tx, double &ty, double b[4], double &g3, double &g4)
{
    double X[5], Y[5];
    leg_taylor4(cx, t, X);
    leg_taylor4(cy, t, Y);
    const double sp = sqrt(X[1] * X[1] + Y[1] * Y[1]);
    tx = X[1] / sp;
    ty = Y[1] / sp;
    const double nx = -ty, ny = tx;
    double c[5], e[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        c[m] = X[m] * tx + Y[m] * ty;
        e[m] = X[m] * nx + Y[m] * ny;
    }
    e[0] = 0.0;
    e[1] = 0.0;
    const double c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4];
    const double i1 = 1.0 / c1, i2 = i1 * i1, i3 = i2 * i1;
    b[0] = i1;
    b[1] = -c2 * i3;
    b[2] = (2.0 * c2 * c2 - c1 * c3) * i3 * i2;
    b[3] = (5.0 * c1 * c2 * c3 - c1 * c1 * c4 - 5.0 * c2 * c2 * c2) * i3 * i3 * i1;
    double h[5];
    xi_derivs(e, b[0], b[1], b[2], b[3], h);
    g3 = h[3];
    g4 = h[4];
}

// (2 erf(c) - 4 c e^{-c^2}/sqrt(pi))/c^3, the value of Q0 at c1 = 0
// (Corollaries 4.4, 4.7, 4.10); its Taylor series below c = 1/2, where the
// difference cancels.
__device__ inline double q0_on(double c)
{
    if (c < 0.5) {
        // (4/sqrt(pi)) sum_{n>=1} (-1)^{n+1} 2n c^{2n-2} / (n! (2n+1))
        const double x = c * c;
        double s = 0.0, term = 1.0;   // term = x^{n-1}/n!
        for (int n = 1; n <= 14; ++n) {
            term = n == 1 ? 1.0 : term * x / n;
            const double v = 2.0 * n / (2.0 * n + 1.0) * term;
            s += (n % 2 == 1) ? v : -v;
        }
        return s * 2.2567583341910251478;   // 4/sqrt(pi)
    }
    return (2.0 * erf(c) - 2.2567583341910251478 * c * exp(-c * c)) / (c * c * c);
}

// (1 - (1 + c^2) e^{-c^2})/c^4 (Corollaries 4.10, 4.11); its Taylor series
// below c = 1/2.
__device__ inline double v2_far(double c)
{
    const double x = c * c;
    if (c < 0.5) {
        // sum_{n>=2} (-1)^n (n - 1) x^{n-2} / n!
        double s = 0.0, term = 0.5;   // term = x^{n-2}/n!
        for (int n = 2; n <= 16; ++n) {
            if (n > 2) term *= x / n;
            const double v = (n - 1) * term;
            s += (n % 2 == 0) ? v : -v;
        }
        return s;
    }
    return (-expm1(-x) - x * exp(-x)) / (x * x);
}

// T: the plan's precision (accumulators, outputs); TI: the type of the
// caller's densities and f_trg (double for an FP32 plan given FP64 inputs)
template <typename T, typename TI = T>
struct LocalArgs {
    int64_t nout, nt, nb, npan;
    int B;
    int parts;
    const double *tx, *ty;
    const int8_t *tin;
    const int32_t *tidx;
    const double *bx, *by, *bk;
    const TI *sigma, *mu, *f_trg;
    const double *cs, *cm;
    const double *cf;      // Legendre coefficients of f on the boundary, or NULL
    const double *geo;     // per-plan local geometry (k_local_geom)
    const int32_t *gpan;
    const uint8_t *gflag;
    const double *pcx, *pcy, *pck, *ends, *gl_t;
    const int32_t *prev, *next, *cand, *cell_start;
    const double *pbox, *cbox;
    int32_t *noconv;
    double cell, ox, oy, reach;
    int ncx, ncy;
    double alpha, delta, dstar, band_s, band_v;
    int frows;             // rows of f_trg per density: 1 (f) or 6 (f and its gradient and Hessian)
    const T *acc;          // [3][B][nout]: S, D, V in sorted order (history part)
    const T *lev;          // [2][B][nout]: S, D of the level sums, or null
    const T *vlev;         // [B][nout]: the volume potential's level sums, or null
    T *out_s, *out_d, *out_v;
};

// Minimise |x - gamma_p(t)|^2 over t in [-1, 1] on panel p by Newton's
// method on d/dt, safeguarded: started from the nearest of the panel's nodes
// and end points; a step that does not decrease the distance is halved
// (bisection towards the current point), and where the distance is not
// convex (beyond a centre of curvature) a fixed step of 1/4 downhill is
// tried instead of the Newton step; Newton steps below 1e-6 where the
// distance is convex are taken as they are (there the distance is flat below
// its rounding, and the derivative decides) and end the iteration once one is
// below 1e-12, after one more Newton step.  Returns whether the iteration
// converged (that, or a damped step below 1e-15, possibly held at an end
// point).
template <typename Args>
__device__ inline bool panel_min(const Args &A, int p, double px, double py, double &tbest, double &d2best)
{
    const double *cx = A.pcx + (size_t)p * NGL, *cy = A.pcy + (size_t)p * NGL;
    // start: best of the two end points and the 16 nodes
    double ts = -1.0;
    double dx = A.ends[p * 4 + 0] - px, dy = A.ends[p * 4 + 1] - py;
    double ds = dx * dx + dy * dy;
    for (int i = 0; i < NGL; ++i) {
        dx = A.bx[(size_t)p * NGL + i] - px;
        dy = A.by[(size_t)p * NGL + i] - py;
        const double d = dx * dx + dy * dy;
        if (d < ds) { ds = d; ts = A.gl_t[i]; }
    }
    dx = A.ends[p * 4 + 2] - px;
    dy = A.ends[p * 4 + 3] - py;
    if (dx * dx + dy * dy < ds) { ds = dx * dx + dy * dy; ts = 1.0; }
    double t = ts, phi;
    {
        const double xv = leg1(cx, t) - px, yv = leg1(cy, t) - py;
        phi = xv * xv + yv * yv;
    }
    bool conv = false;
#pragma unroll 1
    for (int it = 0; it < 60; ++it) {
        double x0, x1, x2, y0, y1, y2;
        leg2(cx, cy, t, x0, x1, x2, y0, y1, y2);
        const double ex = x0 - px, ey = y0 - py;
        const double g = ex * x1 + ey * y1;
        const double h = x1 * x1 + y1 * y1 + ex * x2 + ey * y2;
        double step = h > 0.0 ? -g / h : (g > 0.0 ? -0.25 : 0.25);
        double tn = fmin(1.0, fmax(-1.0, t + step));
        if (h > 0.0 && fabs(step) < 1e-6) {
            // close to a minimum the distance is flat below its rounding:
            // plain Newton steps, driven by the derivative
            // quadratic convergence: after a step below 1e-12 the error is
            // at the rounding level (a stricter test can fail on rounding
            // noise of the step itself)
            const double moved = fabs(tn - t);
            t = tn;
            if (moved < 1e-12) {
                // one more Newton step brings t to the rounding level also
                // where the convergence is slow (small curvature of |x - gamma|^2)
                leg2(cx, cy, t, x0, x1, x2, y0, y1, y2);
                const double e2x = x0 - px, e2y = y0 - py;
                const double h2 = x1 * x1 + y1 * y1 + e2x * x2 + e2y * y2;
                if (h2 > 0.0) t = fmin(1.0, fmax(-1.0, t - (e2x * x1 + e2y * y1) / h2));
                conv = true;
                break;
            }
            continue;
        }
        double dn = phi;
#pragma unroll 1
        for (int k = 0; k <= 52; ++k) {
            const double xv = leg1(cx, tn) - px, yv = leg1(cy, tn) - py;
            dn = xv * xv + yv * yv;
            if (dn <= phi) break;
            step *= 0.5;
            tn = fmin(1.0, fmax(-1.0, t + step));
        }
        const double moved = fabs(tn - t);
        if (dn <= phi) {
            t = tn;
            phi = dn;
        }
        if (moved < 1e-15) {
            conv = true;
            break;
        }
    }
    {
        const double xv = leg1(cx, t) - px, yv = leg1(cy, t) - py;
        phi = xv * xv + yv * yv;
    }
    tbest = t;
    d2best = phi;
    return conv;
}

// Geometry of the local part, once per plan (targets and boundary are
// fixed): closest point, the density-independent coefficients of Lemmas
// 4.1, 4.5 and the factor of Lemma 4.8 / Cor. 4.10 / 4.11 per sorted
// target, so that an evaluation only combines them with the densities.
// Stored per sorted target s: pan[s] (closest panel or -1), flag[s] (bit 0:
// inside the layer band with a closest point; bit 1: exterior target inside
// the volume band) and geo[k * nout + s] for k = GEO_T, GEO_P0, ... GEO_VFAC.
enum { GEO_T, GEO_P0, GEO_P1, GEO_U0, GEO_U1, GEO_U2, GEO_KAP, GEO_MF1, GEO_MF2, GEO_VFAC, GEO_N };
// second-order plans store more per target: the coefficients of the
// delta*^{3/2} and delta*^2 layer terms (Q0, Q1, P2, P3, U3, U4; zero but Q0
// on the boundary), the reversion coefficients b1..b4 and the curve's g3, g4
// at the closest point, its unit tangent, and the factors A, B, C of the V
// terms delta^{3/2}(2 f_eta - f kappa0)/8 A + delta^2 [(f_eta kappa0/8 -
// 3 f kappa0^2/32 - f_etaeta/8) B + (f_etaeta + f_xixi)/8 C]
enum { GEO_Q0 = GEO_N, GEO_Q1, GEO_P2, GEO_P3, GEO_U3, GEO_U4, GEO_B1, GEO_B2, GEO_B3, GEO_B4, GEO_G3, GEO_G4,
       GEO_TX, GEO_TY, GEO_VA, GEO_VB, GEO_VC, GEO_N2 };
static_assert(GEO_N == LOCAL_GEO_N1 && GEO_N2 == LOCAL_GEO_N2, "local geometry layout");

// ORDER is the order of the local expansions (1 or 2); first-order plans
// get a kernel without the second-order registers.
template <int ORDER>
__global__ void __launch_bounds__(256) k_local_geom(LocalArgs<double> A, double *__restrict__ geo,
                                                    int32_t *__restrict__ pan, uint8_t *__restrict__ flag)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= A.nout) return;
    const int64_t idx = A.tidx[s];
    const double px = A.tx[s], py = A.ty[s];
    const bool inside = A.tin[s] != 0;
    const bool on = idx >= A.nt;
    const double sq = sqrt(A.dstar), c2 = A.alpha * sq;
    const double sv = sqrt(A.delta), c2v = A.alpha * sv;
    bool near_s = false, ext = false;
    double r = INFINITY;
    int pbest = -1;
    double tbest = 0.0;
    double P0 = 0, P1 = 0, U0 = 0, U1 = 0, U2 = 0, kap = 0, mss_fac1 = 0, mss_fac2 = 0;
    double vfac = 0.0;             // V local = delta * f * vfac
    if (on) {
        vfac = -expm1(-c2v * c2v) / (2.0 * c2v * c2v);          // Cor. 4.10
    } else {
        // nearest boundary node (lowest index on ties) among the nodes of the
        // cell's candidate panels, nearest panels first; a panel whose node
        // box is farther than the best node so far cannot improve on it
        const int cx = (int)floor((px - A.ox) / A.cell), cy = (int)floor((py - A.oy) / A.cell);
        double dmin = INFINITY;
        int imin = -1;
        if (cx >= 0 && cx < A.ncx && cy >= 0 && cy < A.ncy) {
            const int64_t cell = (int64_t)cy * A.ncx + cx;
            const int k0 = A.cell_start[cell], k1 = A.cell_start[cell + 1];
            for (int k = k0; k < k1; ++k) {
                const int p = A.cand[k];
                const double *bb = A.pbox + (size_t)p * 4;
                const double ex = fmax(0.0, fmax(bb[0] - px, px - bb[1]));
                const double ey = fmax(0.0, fmax(bb[2] - py, py - bb[3]));
                if (ex * ex + ey * ey > dmin) continue;
                const double *nx = A.bx + (size_t)p * NGL, *ny = A.by + (size_t)p * NGL;
#pragma unroll 4
                for (int i = 0; i < NGL; ++i) {
                    const double dx = nx[i] - px, dy = ny[i] - py;
                    const double d = dx * dx + dy * dy;
                    const int node = p * NGL + i;
                    if (d < dmin || (d == dmin && node < imin)) { dmin = d; imin = node; }
                }
            }
        }
        // the closest point lies within half a node gap of a node, so a
        // nearest node farther than band + gap puts x outside both bands
        if (imin >= 0 && sqrt(dmin) <= A.reach) {
            const int p0 = imin / NGL;
            int cand[3] = {p0, A.prev[p0], A.next[p0]};
            double d2b = INFINITY;
            bool conv = true;
#pragma unroll 1
            for (int c = 0; c < 3; ++c) {
                // a neighbouring panel whose curve box is farther than the
                // best distance so far cannot improve on it (ties are kept)
                if (c > 0) {
                    const double *bb = A.cbox + (size_t)cand[c] * 4;
                    const double ex = fmax(0.0, fmax(bb[0] - px, px - bb[1]));
                    const double ey = fmax(0.0, fmax(bb[2] - py, py - bb[3]));
                    if (ex * ex + ey * ey > d2b) continue;
                }
                double t, d2;
                const bool cv = panel_min(A, cand[c], px, py, t, d2);
                if (d2 < d2b) { d2b = d2; pbest = cand[c]; tbest = t; conv = cv; }
            }
            r = sqrt(d2b);
            // a closest point that is not a converged Newton solution is
            // only an approximation: count it where the local part uses its
            // parameter (the layer terms, the exterior volume term through f
            // at the closest point, the second-order volume terms).  The
            // first-order interior volume term needs only the distance,
            // which the safeguarded iteration has minimised; past the
            // curve's centre of curvature (volume bands wider than the
            // radius of curvature) the distance is flat in the parameter and
            // the iteration can stall without harm to it.
            const bool uses_t = r < A.band_s || (r < A.band_v && (!inside || ORDER >= 2));
            if (!conv && uses_t && A.noconv) atomicAdd(A.noconv, 1);
        }
        // volume part (Lemma 4.8 first order inside the band, Cor. 4.11
        // beyond).  Exterior targets in the band: the local integral over
        // Omega is the whole-plane one minus the one over the complement, a
        // domain that contains x, so V_L = delta f0 [(1 - e^{-c2^2})/c2^2 -
        // W0/4] with f0 = f at the closest boundary point, from the panel
        // expansion of f at the boundary nodes (NaN without them).
        if (r < A.band_v) {
            const double c1v = r / sv, a = 0.5 * c1v;
            const double em = erfcx(a - c2v), ep = erfcx(a + c2v), e0 = erfcx(a);
            const double pre = exp(-a * a - c2v * c2v);
            // W0 = (4 - 4 e^{-c2^2} + 2 lambda - Phi_+)/c2^2, lambda = e^{-c2^2} erfc(c1/2)
            const double W0 = (-4.0 * expm1(-c2v * c2v) + pre * ((e0 - em) + (e0 - ep))) / (c2v * c2v);
            if (inside) {
                vfac = 0.25 * W0;
            } else {
                vfac = -expm1(-c2v * c2v) / (c2v * c2v) - 0.25 * W0;
                ext = true;
            }
        } else {
            vfac = inside ? -expm1(-c2v * c2v) / (c2v * c2v) : 0.0;
        }
        if (r < A.band_s && pbest >= 0) {
            near_s = true;
            const double c1 = r / sq, a = 0.5 * c1;
            const double em = erfcx(a - c2), ep = erfcx(a + c2);
            const double pre = exp(-a * a - c2 * c2);
            const double phim = pre * (em - ep), phip = pre * (em + ep);
            P0 = phim / c2;
            P1 = c1 * P0;
            U0 = phip;
            U1 = c1 * U0;
            U2 = c1 * U1;
            kap = leg1(A.pck + (size_t)pbest * NGL, tbest);
            double x0, x1, x2, y0, y1, y2;
            leg2(A.pcx + (size_t)pbest * NGL, A.pcy + (size_t)pbest * NGL, tbest, x0, x1, x2, y0, y1, y2);
            const double sp2 = x1 * x1 + y1 * y1;
            // d^2/ds^2 = (d^2/dt^2 - (gamma'.gamma''/|gamma'|^2) d/dt)/|gamma'|^2
            mss_fac2 = 1.0 / sp2;
            mss_fac1 = -(x1 * x2 + y1 * y2) / (sp2 * sp2);
        }
    }
    const int64_t n = A.nout;
    if (ORDER >= 2) {
        double q0 = 0, q1 = 0, p2 = 0, p3 = 0, u3 = 0, u4 = 0, bb[4] = {0, 0, 0, 0}, g3 = 0, g4 = 0;
        double ttx = 1.0, tty = 0.0, va = 0.0, vb = 0.0, vc = 0.0;
        // the boundary point whose tangent line is used: the node itself on
        // the boundary, the closest point elsewhere
        int pp = -1;
        double tt = 0.0;
        if (on) {
            const int64_t i = idx - A.nt;
            pp = (int)(i / NGL);
            tt = A.gl_t[i % NGL];
        } else if (pbest >= 0) {
            pp = pbest;
            tt = tbest;
        }
        if (pp >= 0) {
            tangent_line(A.pcx + (size_t)pp * NGL, A.pcy + (size_t)pp * NGL, tt, ttx, tty, bb, g3, g4);
            if (!on) kap = leg1(A.pck + (size_t)pp * NGL, tt);
        }
        if (on) {
            q0 = q0_on(c2);                                   // Cor. 4.4, 4.7 (c1 = 0)
            va = q0_on(c2v);                                  // Cor. 4.10
            vc = 4.0 * v2_far(c2v);
        } else {
            if (near_s) {
                // Lemma 4.1, 4.5 coefficients at c1 = r / sqrt(delta*)
                const double c1 = r / sq, a = 0.5 * c1;
                const double em = erfcx(a - c2), ep = erfcx(a + c2);
                const double pre = exp(-a * a - c2 * c2);
                const double phim = pre * (em - ep), phip = pre * (em + ep);
                const double z = 1.1283791670955125739 * 2.0 * c2 * pre;   // 4 c2 e^{-c1^2/4 - c2^2}/sqrt(pi)
                q0 = (phim - z) / (c2 * c2 * c2) + c1 * phip / (c2 * c2);
                q1 = c1 * q0;
                p2 = c1 * c1 * phim / c2;
                p3 = c1 * p2;
                u3 = c1 * c1 * c1 * phip;
                u4 = c1 * u3;
            }
            if (inside && r < A.band_v) {
                // Lemma 4.8 coefficients at c1 = r / sqrt(delta)
                const double c1 = r / sv, a = 0.5 * c1;
                const double em = erfcx(a - c2v), ep = erfcx(a + c2v), e0 = erfcx(a);
                const double pre = exp(-a * a - c2v * c2v);
                const double phim = pre * (em - ep), phip = pre * (em + ep);
                const double z = 1.1283791670955125739 * 2.0 * c2v * pre;
                const double w0 = (-4.0 * expm1(-c2v * c2v) + pre * ((e0 - em) + (e0 - ep))) / (c2v * c2v);
                const double lam = pre * e0;                  // e^{-c2^2} erfc(c1/2)
                va = (phim - z) / (c2v * c2v * c2v) + c1 * phip / (c2v * c2v);
                vb = c1 * va;
                vc = (2.0 * w0 - c1 * phim / c2v + 4.0 * (lam - 2.0 * exp(-c2v * c2v))) / (c2v * c2v);
            } else if (inside) {
                vc = 8.0 * v2_far(c2v);                       // Cor. 4.11
            }
        }
        geo[GEO_Q0 * n + s] = q0;
        geo[GEO_Q1 * n + s] = q1;
        geo[GEO_P2 * n + s] = p2;
        geo[GEO_P3 * n + s] = p3;
        geo[GEO_U3 * n + s] = u3;
        geo[GEO_U4 * n + s] = u4;
        geo[GEO_B1 * n + s] = bb[0];
        geo[GEO_B2 * n + s] = bb[1];
        geo[GEO_B3 * n + s] = bb[2];
        geo[GEO_B4 * n + s] = bb[3];
        geo[GEO_G3 * n + s] = g3;
        geo[GEO_G4 * n + s] = g4;
        geo[GEO_TX * n + s] = ttx;
        geo[GEO_TY * n + s] = tty;
        geo[GEO_VA * n + s] = va;
        geo[GEO_VB * n + s] = vb;
        geo[GEO_VC * n + s] = vc;
    }
    geo[GEO_T * n + s] = tbest;
    geo[GEO_P0 * n + s] = P0;
    geo[GEO_P1 * n + s] = P1;
    geo[GEO_U0 * n + s] = U0;
    geo[GEO_U1 * n + s] = U1;
    geo[GEO_U2 * n + s] = U2;
    geo[GEO_KAP * n + s] = kap;
    geo[GEO_MF1 * n + s] = mss_fac1;
    geo[GEO_MF2 * n + s] = mss_fac2;
    geo[GEO_VFAC * n + s] = vfac;
    pan[s] = pbest;
    flag[s] = (uint8_t)((near_s ? 1 : 0) | (ext ? 2 : 0));
}

// Local part of an evaluation from the per-plan geometry, added to the
// accumulated history and level sums, and the scatter to the caller's order.
template <typename T, typename TI, int ORDER>
__global__ void __launch_bounds__(256) k_local(LocalArgs<T, TI> A)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= A.nout) return;
    const int64_t idx = A.tidx[s];
    const bool inside = A.tin[s] != 0;
    const bool on = idx >= A.nt;
    const bool do_local = (A.parts & MHK_PART_LOCAL) != 0;
    const bool ws = A.out_s != nullptr, wd = A.out_d != nullptr, wv = A.out_v != nullptr;
    const double sq = sqrt(A.dstar), c2 = A.alpha * sq;
    const double rho = inside ? 1.0 : -1.0;
    const int64_t n = A.nout;
    const uint8_t fl = A.gflag[s];
    const bool near_s = (fl & 1) != 0, ext = (fl & 2) != 0;
    const int pbest = A.gpan[s];
    const double vfac = do_local && wv ? A.geo[GEO_VFAC * n + s] : 0.0;
    double tbest = 0.0, P0 = 0, P1 = 0, U0 = 0, U1 = 0, U2 = 0, kap = 0, mss_fac1 = 0, mss_fac2 = 0;
    if (do_local && (near_s || ext)) tbest = A.geo[GEO_T * n + s];
    if (do_local && near_s && (ws || wd)) {
        P0 = A.geo[GEO_P0 * n + s];
        P1 = A.geo[GEO_P1 * n + s];
        kap = A.geo[GEO_KAP * n + s];
        if (wd) {
            U0 = A.geo[GEO_U0 * n + s];
            U1 = A.geo[GEO_U1 * n + s];
            U2 = A.geo[GEO_U2 * n + s];
            mss_fac1 = A.geo[GEO_MF1 * n + s];
            mss_fac2 = A.geo[GEO_MF2 * n + s];
        }
    }

    // second order: coefficients, tangent-line data and the boundary point
    // (the node itself on the boundary, the closest point elsewhere)
    const bool o2 = do_local && ORDER >= 2;
    double q0 = 0, q1 = 0, p2 = 0, p3 = 0, u3 = 0, u4 = 0, bb[4] = {0, 0, 0, 0}, g3 = 0, g4 = 0;
    double ttx = 1.0, tty = 0.0, va = 0, vb = 0, vc = 0, kap2 = 0.0, tt2 = 0.0;
    int pp2 = -1;
    if (o2) {
        q0 = A.geo[GEO_Q0 * n + s]; q1 = A.geo[GEO_Q1 * n + s];
        p2 = A.geo[GEO_P2 * n + s]; p3 = A.geo[GEO_P3 * n + s];
        u3 = A.geo[GEO_U3 * n + s]; u4 = A.geo[GEO_U4 * n + s];
        bb[0] = A.geo[GEO_B1 * n + s]; bb[1] = A.geo[GEO_B2 * n + s];
        bb[2] = A.geo[GEO_B3 * n + s]; bb[3] = A.geo[GEO_B4 * n + s];
        g3 = A.geo[GEO_G3 * n + s]; g4 = A.geo[GEO_G4 * n + s];
        ttx = A.geo[GEO_TX * n + s]; tty = A.geo[GEO_TY * n + s];
        va = A.geo[GEO_VA * n + s]; vb = A.geo[GEO_VB * n + s]; vc = A.geo[GEO_VC * n + s];
        if (on) {
            const int64_t i = idx - A.nt;
            pp2 = (int)(i / NGL);
            tt2 = A.gl_t[i % NGL];
            kap2 = A.bk[i];
        } else {
            pp2 = pbest;
            tt2 = A.geo[GEO_T * n + s];
            kap2 = A.geo[GEO_KAP * n + s];
        }
    }
    const double d32 = A.dstar * sq, d2 = A.dstar * A.dstar;

#pragma unroll 1
    for (int b = 0; b < A.B; ++b) {
        const size_t ob = (size_t)b * A.nout + idx;
        const size_t ab = (size_t)b * A.nout + s;
        if (ws) {
            double v = (double)A.acc[(size_t)0 * A.B * A.nout + ab];
            if (A.lev) v += (double)A.lev[ab];
            if (do_local) {
                if (on) {
                    const int64_t i = idx - A.nt;
                    v += sq * (double)A.sigma[(size_t)b * A.nb + i] * erf(c2) / (2.0 * c2);        // Cor. 4.4
                } else if (near_s) {
                    const double sg = leg1(A.cs + ((size_t)b * A.npan + pbest) * NGL, tbest);
                    v += sq * sg * P0 * 0.25 + A.dstar * rho * kap * sg * P1 * 0.125;     // Lemma 4.1
                }
                if (o2 && (on || near_s) && pp2 >= 0) {
                    // delta*^{3/2} and delta*^2 terms of Lemma 4.1 (Cor. 4.4 on the boundary)
                    double F[5], d[5];
                    leg_taylor4(A.cs + ((size_t)b * A.npan + pp2) * NGL, tt2, F);
                    xi_derivs(F, bb[0], bb[1], bb[2], bb[3], d);
                    const double s0 = on ? (double)A.sigma[(size_t)b * A.nb + (idx - A.nt)] : d[0];
                    const double k = kap2;
                    v += d32 * (k * k * s0 / 32.0 * (q0 + 3.0 * p2) + d[2] / 8.0 * q0) +
                         d2 * rho * (k * k * k * s0 / 64.0 * (-3.0 * q1 + 5.0 * p3) +
                                     (3.0 * k * d[2] / 16.0 + d[1] * g3 / 8.0 + s0 * g4 / 32.0) * q1);
                }
            }
            A.out_s[ob] = (T)v;
        }
        if (wd) {
            double v = (double)A.acc[(size_t)1 * A.B * A.nout + ab];
            if (A.lev) v += (double)A.lev[(size_t)A.B * A.nout + ab];
            if (do_local) {
                if (on) {
                    const int64_t i = idx - A.nt;
                    v -= sq * A.bk[i] * (double)A.mu[(size_t)b * A.nb + i] * erf(c2) / (4.0 * c2);  // Cor. 4.7
                } else if (near_s) {
                    double m0, m1, m2;
                    leg2s(A.cm + ((size_t)b * A.npan + pbest) * NGL, tbest, m0, m1, m2);
                    const double mss = mss_fac2 * m2 + mss_fac1 * m1;
                    v += -rho * m0 * U0 * 0.25 - sq * kap * m0 * (P0 + U1) * 0.125                // Lemma 4.5
                         - A.dstar * (rho * mss * P1 * 0.125 + 3.0 * rho * kap * kap * m0 * (P1 + U2) / 32.0);
                }
                if (o2 && (on || near_s) && pp2 >= 0) {
                    // delta*^{3/2} and delta*^2 terms of Lemma 4.5 (Cor. 4.7 on
                    // the boundary); the gamma'''' term of the delta*^{3/2}
                    // bracket multiplies (3 Q0 + P2) (the series of the local
                    // integral; the kappa^3 term keeps (3 Q0 - U3))
                    double F[5], d[5];
                    leg_taylor4(A.cm + ((size_t)b * A.npan + pp2) * NGL, tt2, F);
                    xi_derivs(F, bb[0], bb[1], bb[2], bb[3], d);
                    const double m0 = on ? (double)A.mu[(size_t)b * A.nb + (idx - A.nt)] : d[0];
                    const double k = kap2;
                    v += d32 * (5.0 * k * k * k * m0 / 64.0 * (3.0 * q0 - u3) - m0 * g4 / 32.0 * (3.0 * q0 + p2) +
                                3.0 * k * d[2] / 16.0 * (-q0 - p2) + d[1] * g3 / 8.0 * (-2.0 * q0 - p2)) +
                         d2 * (35.0 * rho * k * k * k * k * m0 / 512.0 * (9.0 * q1 + 2.0 * p3 - u4) -
                               rho * d[4] / 32.0 * q1 - 15.0 * rho * k * k * d[2] / 64.0 * (q1 + p3)) -
                         d2 * (5.0 * rho * k * d[1] * g3 / 16.0 * (2.0 * q1 + p3) +
                               (5.0 * rho * k * m0 * g4 / 64.0 + 5.0 * rho * m0 * g3 * g3 / 96.0) * (3.0 * q1 + p3));
                }
            }
            A.out_d[ob] = (T)v;
        }
        if (wv) {
            double v = (double)A.acc[(size_t)2 * A.B * A.nout + ab];
            if (A.vlev) v += (double)A.vlev[ab];
            if (do_local) {
                // f (and with second order its gradient and Hessian) at the target
                const TI *fr = A.f_trg + (size_t)b * A.frows * A.nout + idx;
                double f;
                if (ext)
                    f = A.cf ? leg1(A.cf + ((size_t)b * A.npan + pbest) * NGL, tbest) : NAN;
                else
                    f = (double)fr[0];
                v += A.delta * f * vfac;
                if (o2 && !ext) {
                    // delta^{3/2} and delta^2 terms of Lemma 4.8 (Cor. 4.10 on the
                    // boundary, Cor. 4.11 far from it): f's derivatives along
                    // the inward normal N0 = (-t_y, t_x) and the tangent t
                    const size_t nn = (size_t)A.nout;
                    const double fx = (double)fr[nn], fy = (double)fr[2 * nn];
                    const double fxx = (double)fr[3 * nn], fxy = (double)fr[4 * nn], fyy = (double)fr[5 * nn];
                    const double nx = -tty, ny = ttx;
                    const double fe = fx * nx + fy * ny;
                    const double fee = fxx * nx * nx + 2.0 * fxy * nx * ny + fyy * ny * ny;
                    const double fxi = fxx * ttx * ttx + 2.0 * fxy * ttx * tty + fyy * tty * tty;
                    const double k = kap2;
                    v += A.delta * sqrt(A.delta) * (2.0 * fe - f * k) / 8.0 * va +
                         A.delta * A.delta * ((fe * k / 8.0 - 3.0 * f * k * k / 32.0 - fee / 8.0) * vb +
                                              (fee + fxi) / 8.0 * vc);
                }
            }
            A.out_v[ob] = (T)v;
        }
    }
}

__global__ void k_zero(uint32_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_fill_int(int *p, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t *)p, n);
    return hipGetLastError();
}

hipError_t launch_fill(mhk_plan *P, void *p, int64_t n)
{
    const int64_t words = n * (int64_t)P->es / 4;
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, P->stream, (uint32_t *)p, words);
    return hipGetLastError();
}

template <typename T>
static hipError_t panel_coeffs(mhk_plan *P, const void *sigma, const void *mu, const void *f_bnd)
{
    const int64_t tot = P->npan * NGL * P->bat;
    hipLaunchKernelGGL(k_panel_coeffs<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, P->stream, P->npan,
                       P->bat, P->loc.leg, (const T *)sigma, (const T *)mu, (const T *)f_bnd, P->nout,
                       P->p.local_order >= 2 ? 6 : 1, P->nt,
                       P->loc.csig, P->loc.cmu, P->loc.cf);
    return hipGetLastError();
}

// the densities as the caller gives them: FP64 for FP64 plans and for FP32
// plans created with in64
hipError_t launch_panel_coeffs(mhk_plan *P, const void *sigma, const void *mu, const void *f_bnd)
{
    return (P->p.prec == MHK_FP64 || P->p.in64) ? panel_coeffs<double>(P, sigma, mu, f_bnd)
                                                : panel_coeffs<float>(P, sigma, mu, f_bnd);
}

template <typename T, typename TI>
static void fill_args(mhk_plan *P, LocalArgs<T, TI> &A)
{
    A.nout = P->nout;
    A.nt = P->nt;
    A.nb = P->nb;
    A.npan = P->npan;
    A.B = P->bat;
    A.parts = MHK_PART_ALL;
    A.tx = P->tx;
    A.ty = P->ty;
    A.tin = P->tin;
    A.tidx = P->tidx;
    A.bx = P->bx;
    A.by = P->by;
    A.bk = P->bk;
    A.sigma = nullptr;
    A.mu = nullptr;
    A.f_trg = nullptr;
    A.cs = P->loc.csig;
    A.cm = P->loc.cmu;
    A.cf = nullptr;
    A.geo = P->loc.geo;
    A.gpan = P->loc.gpan;
    A.gflag = P->loc.gflag;
    A.pcx = P->loc.cx;
    A.pcy = P->loc.cy;
    A.pck = P->loc.ck;
    A.ends = P->loc.ends;
    A.gl_t = P->loc.gl_t;
    A.prev = P->loc.prev;
    A.next = P->loc.next;
    A.cand = P->loc.cand;
    A.cell_start = P->loc.cell_start;
    A.pbox = P->loc.pbox;
    A.cbox = P->loc.cbox;
    A.noconv = P->loc.noconv;
    A.reach = P->loc.reach;
    A.cell = P->loc.cell;
    A.ox = P->loc.ox;
    A.oy = P->loc.oy;
    A.ncx = P->loc.ncx;
    A.ncy = P->loc.ncy;
    A.alpha = P->p.alpha;
    A.delta = P->delta_v;                 // V's local part: delta, or delta* with volume levels
    A.dstar = P->dstar;
    A.band_s = P->info.band_layer;
    A.band_v = P->info.band_volume;
    A.frows = P->p.local_order >= 2 ? 6 : 1;
    A.acc = (const T *)P->acc;
    A.lev = nullptr;
    A.vlev = nullptr;
    A.out_s = A.out_d = A.out_v = nullptr;
}

hipError_t launch_local_geom(mhk_plan *P, hipStream_t st)
{
    if (P->nout == 0) return hipSuccess;
    LocalArgs<double> A;
    fill_args(P, A);
    const dim3 grid((unsigned)((P->nout + 255) / 256));
    if (P->p.local_order >= 2)
        hipLaunchKernelGGL(k_local_geom<2>, grid, dim3(256), 0, st, A, P->loc.geo, P->loc.gpan, P->loc.gflag);
    else
        hipLaunchKernelGGL(k_local_geom<1>, grid, dim3(256), 0, st, A, P->loc.geo, P->loc.gpan, P->loc.gflag);
    return hipGetLastError();
}

template <typename T, typename TI>
static hipError_t local_t(mhk_plan *P, int parts, const void *sigma, const void *mu, const void *f_trg,
                          void *out_s, void *out_d, void *out_v, bool have_fb, bool have_lev, bool have_vlev)
{
    LocalArgs<T, TI> A;
    fill_args(P, A);
    A.lev = have_lev ? (const T *)P->acc_lev : nullptr;
    A.vlev = have_vlev ? (const T *)P->acc_vlev : nullptr;
    A.parts = parts;
    A.sigma = (const TI *)sigma;
    A.mu = (const TI *)mu;
    A.f_trg = (const TI *)f_trg;
    A.cf = have_fb ? P->loc.cf : nullptr;
    A.out_s = (T *)out_s;
    A.out_d = (T *)out_d;
    A.out_v = (T *)out_v;
    const dim3 grid((unsigned)((P->nout + 255) / 256));
    if (P->p.local_order >= 2)
        hipLaunchKernelGGL((k_local<T, TI, 2>), grid, dim3(256), 0, P->stream, A);
    else
        hipLaunchKernelGGL((k_local<T, TI, 1>), grid, dim3(256), 0, P->stream, A);
    return hipGetLastError();
}

hipError_t launch_local(mhk_plan *P, int parts, const void *sigma, const void *mu, const void *f_trg,
                        void *out_s, void *out_d, void *out_v, bool have_fb, bool have_lev, bool have_vlev)
{
    if (P->p.prec == MHK_FP64)
        return local_t<double, double>(P, parts, sigma, mu, f_trg, out_s, out_d, out_v, have_fb, have_lev, have_vlev);
    if (P->p.in64)
        return local_t<float, double>(P, parts, sigma, mu, f_trg, out_s, out_d, out_v, have_fb, have_lev, have_vlev);
    return local_t<float, float>(P, parts, sigma, mu, f_trg, out_s, out_d, out_v, have_fb, have_lev, have_vlev);
}

// FP32 copies of FP64 inputs (FP32 plans with in64): n values, rounded once
__global__ void __launch_bounds__(256) k_round32(const double *__restrict__ x, float *__restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

hipError_t launch_round32(mhk_plan *P, const void *x, void *y, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_round32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, P->stream, (const double *)x,
                       (float *)y, n);
    return hipGetLastError();
}

}  // namespace mhk
