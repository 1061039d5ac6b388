// Dyadic levels of the volume potential (Section 4.2 applied to V).
//
// The local part of V is split in time like the layer potentials': a
// first-order expansion over [0, delta*] (delta* = delta/4^J) plus, for
// j = 1..J, the level term
//   V_j(x) = sum_q w_q f(y_q) K_j^S(|x - y_q|)
// over a volume quadrature fine enough for the level's kernel (the volume and
// single-layer difference kernels are the same, so the level-j table of the
// layer potentials serves).  The level-j quadrature refines every triangle of
// the volume rule (nodes in groups of six): its reference triangle
// T0 = {s, t >= 0, s + t <= 1} is split into 4^j congruent triangles, each
// carrying the reference rule (s_i, t_i, W_i); the triangle's map x(s, t) is
// the quadratic in (s, t) through its six nodes (exact for straight
// triangles); a node is x at a mapped rule point and its weight
// W_i |det Dx| / (2 4^j).  f at a level node is the quadratic through the
// six nodal values of its own triangle (for slivers, whose quadratic is
// ill-determined, that of the triangle holding the nearest usable node, as
// f at the targets).
//
// Plan creation builds the level nodes, sorts them by cells of side R_j/4
// and lists per target wavefront the nodes within R_j (the same device
// binning as the layer levels); an evaluation forms q = w f per node and
// density and runs the level-sum kernel on them (single-layer sums only).
#include "mhk_internal.h"

namespace mhk {

// positions, weights and cell keys of the level-j nodes (unsorted), node
// q = (triangle, sub-triangle, rule point) in that order
__global__ void __launch_bounds__(256) k_vnodes(int64_t ntri, int j, VRule M, const double *__restrict__ vx,
                                                const double *__restrict__ vy, double ox, double oy, double cell,
                                                int64_t ncx, int64_t ncy, double *__restrict__ cx,
                                                double *__restrict__ cy, double *__restrict__ cw,
                                                uint32_t *__restrict__ key, int32_t *__restrict__ val)
{
    const int n = 1 << j;
    const int64_t nsub = (int64_t)n * n;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ntri * nsub * 6) return;
    const int i = (int)(q % 6);
    const int64_t sub = (q / 6) % nsub, k = q / (6 * nsub);
    // sub-triangle: the n(n+1)/2 upright ones row by row (row b holds n - b),
    // then the n(n-1)/2 inverted ones (row b holds n - 1 - b)
    const int64_t nup = (int64_t)n * (n + 1) / 2;
    double s, t;
    if (sub < nup) {
        int64_t r = sub, b = 0;
        while (r >= n - b) { r -= n - b; ++b; }
        s = (r + M.s[i]) / n;
        t = (b + M.t[i]) / n;
    } else {
        int64_t r = sub - nup, b = 0;
        while (r >= n - 1 - b) { r -= n - 1 - b; ++b; }
        s = (r + 1 - M.s[i]) / n;
        t = (b + 1 - M.t[i]) / n;
    }
    double ax[6], ay[6];
    for (int m = 0; m < 6; ++m) {
        double u = 0, v = 0;
        for (int l = 0; l < 6; ++l) {
            u = fma(M.rinv[m * 6 + l], vx[k * 6 + l], u);
            v = fma(M.rinv[m * 6 + l], vy[k * 6 + l], v);
        }
        ax[m] = u;
        ay[m] = v;
    }
    const double x = ax[0] + ax[1] * s + ax[2] * t + ax[3] * s * s + ax[4] * s * t + ax[5] * t * t;
    const double y = ay[0] + ay[1] * s + ay[2] * t + ay[3] * s * s + ay[4] * s * t + ay[5] * t * t;
    const double xs = ax[1] + 2 * ax[3] * s + ax[4] * t, xt = ax[2] + ax[4] * s + 2 * ax[5] * t;
    const double ys = ay[1] + 2 * ay[3] * s + ay[4] * t, yt = ay[2] + ay[4] * s + 2 * ay[5] * t;
    cx[q] = x;
    cy[q] = y;
    cw[q] = fabs(xs * yt - xt * ys) * M.W[i] / (2.0 * (double)nsub);
    const int64_t ix = min(ncx - 1, max((int64_t)0, (int64_t)floor((x - ox) / cell)));
    const int64_t iy = min(ncy - 1, max((int64_t)0, (int64_t)floor((y - oy) / cell)));
    key[q] = (uint32_t)(iy * ncx + ix);
    val[q] = (int32_t)q;
}

__global__ void __launch_bounds__(256) k_vgather(int64_t n, int64_t per_tri, const int32_t *__restrict__ order,
                                                 const double *__restrict__ cx, const double *__restrict__ cy,
                                                 const double *__restrict__ cw, double *__restrict__ sx,
                                                 double *__restrict__ sy, double *__restrict__ sw,
                                                 int32_t *__restrict__ parent)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t q = order[s];
    sx[s] = cx[q];
    sy[s] = cy[q];
    sw[s] = cw[q];
    parent[s] = (int32_t)(q / per_tri);
}

// strengths q = w f of the level nodes for every density: f from the
// quadratic of the node's own volume triangle (of the nearest usable node's
// triangle for slivers)
template <typename TF, typename T>
__global__ void __launch_bounds__(256) k_vlevel_q(int64_t n, int B, const double *__restrict__ sx,
                                                  const double *__restrict__ sy, const double *__restrict__ sw,
                                                  const int32_t *__restrict__ tri, const double *__restrict__ minv,
                                                  const double *__restrict__ tc, int64_t nv,
                                                  const TF *__restrict__ fv, T *__restrict__ q)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t t = tri[s];
    const double h = tc[t * 3 + 2];
    const double X = (sx[s] - tc[t * 3 + 0]) / h, Y = (sy[s] - tc[t * 3 + 1]) / h;
    const double m[6] = {1.0, X, Y, X * X, X * Y, Y * Y};
    // interpolation weights of the six nodal values at the node
    double L[6];
    for (int i = 0; i < 6; ++i) {
        double v = 0;
        for (int k = 0; k < 6; ++k) v = fma(m[k], minv[((size_t)t * 6 + k) * 6 + i], v);
        L[i] = v;
    }
    const double w = sw[s];
    for (int b = 0; b < B; ++b) {
        const TF *f = fv + (size_t)b * nv + (size_t)t * 6;
        double v = 0;
        for (int i = 0; i < 6; ++i) v = fma(L[i], (double)f[i], v);
        q[(size_t)b * n + s] = (T)(w * v);
    }
}

hipError_t dev_vlevel_nodes(int64_t ntri, int j, const VRule &M, const double *vx, const double *vy, double ox,
                            double oy, double cell, int64_t ncx, int64_t ncy, double *sx, double *sy, double *sw,
                            int32_t *parent, int32_t *cell_start, hipStream_t st)
{
    const int64_t n = ntri * ((int64_t)1 << (2 * j)) * 6;
    double *t[3] = {};
    uint32_t *key = nullptr;
    int32_t *val = nullptr;
    hipError_t e = hipSuccess;
    for (auto &p : t)
        if (e == hipSuccess) e = hipMallocAsync((void **)&p, sizeof(double) * std::max<int64_t>(1, n), st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&key, sizeof(uint32_t) * std::max<int64_t>(1, n), st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&val, sizeof(int32_t) * std::max<int64_t>(1, n), st);
    if (e == hipSuccess && n > 0) {
        hipLaunchKernelGGL(k_vnodes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ntri, j, M, vx, vy, ox, oy,
                           cell, ncx, ncy, t[0], t[1], t[2], key, val);
        e = hipGetLastError();
    }
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < ncx * ncy) ++bits;
    if (e == hipSuccess) e = dev_sort_pairs(key, val, n, bits, st);
    if (e == hipSuccess && n > 0) {
        hipLaunchKernelGGL(k_vgather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, n / ntri, val, t[0],
                           t[1], t[2], sx, sy, sw, parent);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = dev_cell_starts(key, n, ncx * ncy, cell_start, st);
    for (auto p : t)
        if (p) (void)hipFreeAsync(p, st);
    if (key) (void)hipFreeAsync(key, st);
    if (val) (void)hipFreeAsync(val, st);
    return e;
}

hipError_t launch_vlevel_q(mhk_plan *P, hipStream_t st, int j, const void *f_vol)
{
    VLevel &V = P->vlev[j - 1];
    const dim3 grid((unsigned)((V.n_src + 255) / 256));
    const bool in_d = P->p.prec == MHK_FP64 || P->p.in64;
    if (P->p.prec == MHK_FP64)
        hipLaunchKernelGGL((k_vlevel_q<double, double>), grid, dim3(256), 0, st, V.n_src, P->bat, V.sx, V.sy, V.sw,
                           V.tri, P->fj.minv, P->fj.tc, P->nv, (const double *)f_vol, (double *)V.q);
    else if (in_d)
        hipLaunchKernelGGL((k_vlevel_q<double, float>), grid, dim3(256), 0, st, V.n_src, P->bat, V.sx, V.sy, V.sw,
                           V.tri, P->fj.minv, P->fj.tc, P->nv, (const double *)f_vol, (float *)V.q);
    else
        hipLaunchKernelGGL((k_vlevel_q<float, float>), grid, dim3(256), 0, st, V.n_src, P->bat, V.sx, V.sy, V.sw,
                           V.tri, P->fj.minv, P->fj.tc, P->nv, (const float *)f_vol, (float *)V.q);
    return hipGetLastError();
}

}  // namespace mhk
