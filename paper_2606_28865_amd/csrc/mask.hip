// Inside/outside mask of the targets when the caller passes none.
//
// The paper takes the domain Omega as given; a target's side decides which
// local expansions apply (the sign rho of Section 3.2, Lemma 4.8 inside and
// the complement form outside).  The mask is the parity of the crossings of
// a ray in +x with the closed curves, computed in two steps:
//
//  * the polygon through each panel's end points and its 16 nodes (18
//    vertices per panel, closed along each curve): a target's ray crosses an
//    edge when the edge's y-range holds the target's y (half-open, so a
//    vertex is counted once) and the crossing lies to its right;
//  * the lune between an edge and the arc of the panel's degree-15
//    interpolant that it spans: a target inside such a lune is on the other
//    side of the curve than of the polygon, so its parity flips.  A target
//    is tested against a lune only when its distance from the edge's chord
//    is below a bound of the arc's deviation from the chord (set at plan
//    creation) and its projection falls on the chord; the arc's point over
//    the target's projection is found by bisection in the panel parameter
//    with the interpolant in barycentric form.
//
// Edges are listed per horizontal strip (each edge in every strip its
// y-range, widened by its deviation bound, meets), so a target visits the
// few edges of its own strip.  One thread per target.
#include "mhk_internal.h"

namespace mhk {

// x(t), y(t) of panel p from its nodal values, second barycentric form with
// the weights lam of the Gauss-Legendre nodes tn
__device__ inline void bary_eval(const double *__restrict__ tn, const double *__restrict__ lam,
                                 const double *__restrict__ px, const double *__restrict__ py, double t, double &x,
                                 double &y)
{
    double nx = 0, ny = 0, den = 0;
    for (int i = 0; i < NGL; ++i) {
        const double d = t - tn[i];
        if (d == 0.0) {
            x = px[i];
            y = py[i];
            return;
        }
        const double c = lam[i] / d;
        nx = fma(c, px[i], nx);
        ny = fma(c, py[i], ny);
        den += c;
    }
    x = nx / den;
    y = ny / den;
}

__global__ void __launch_bounds__(256) k_inside(MaskArgs A, int8_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const double px = A.tx[i], py = A.ty[i];
    int par = 0;
    if (py >= A.ylo && py < A.yhi) {
        const int s = min(A.nstrip - 1, max(0, (int)((py - A.ylo) * A.hinv)));
        for (int k = A.strip_start[s]; k < A.strip_start[s + 1]; ++k) {
            const int e = A.strip_edge[k];
            const double x0 = A.edge[e * 4 + 0], y0 = A.edge[e * 4 + 1];
            const double x1 = A.edge[e * 4 + 2], y1 = A.edge[e * 4 + 3];
            if ((y0 > py) != (y1 > py)) {
                const double xc = x0 + (py - y0) * (x1 - x0) / (y1 - y0);
                if (xc > px) par ^= 1;
            }
            const double sag = A.sag[e];
            if (!(sag > 0.0)) continue;
            const double ex = x1 - x0, ey = y1 - y0;
            const double l2 = ex * ex + ey * ey;
            const double u = ((px - x0) * ex + (py - y0) * ey) / l2;
            if (!(u > 0.0 && u < 1.0)) continue;
            const double il = rsqrt(l2);
            const double v = (ex * (py - y0) - ey * (px - x0)) * il;
            if (fabs(v) > sag) continue;
            // the arc's point whose projection on the chord is u: the
            // projection grows from 0 at t_a to 1 at t_b
            const int p = A.edge_pan[e];
            const double *bx = A.bx + (size_t)p * NGL, *by = A.by + (size_t)p * NGL;
            double ta = A.edge_t[e * 2 + 0], tb = A.edge_t[e * 2 + 1];
            double ax = x0, ay = y0;
            for (int it = 0; it < 64 && tb - ta > 1e-16; ++it) {
                const double tm = 0.5 * (ta + tb);
                bary_eval(A.gl_t, A.lam, bx, by, tm, ax, ay);
                const double um = ((ax - x0) * ex + (ay - y0) * ey) / l2;
                if (um < u)
                    ta = tm;
                else
                    tb = tm;
            }
            bary_eval(A.gl_t, A.lam, bx, by, 0.5 * (ta + tb), ax, ay);
            const double w = (ex * (ay - y0) - ey * (ax - x0)) * il;
            // between the chord and the arc: same side as the arc, nearer the chord
            if ((v > 0.0 && w > v) || (v < 0.0 && w < v)) par ^= 1;
        }
    }
    out[i] = (int8_t)par;
}

hipError_t dev_inside_mask(const MaskArgs &A, int8_t *out, hipStream_t st)
{
    if (A.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inside, dim3((unsigned)((A.n + 255) / 256)), dim3(256), 0, st, A, out);
    return hipGetLastError();
}

}  // namespace mhk
