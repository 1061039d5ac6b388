// f and its derivatives at the targets from the volume quadrature.
//
// The local part of V (Lemma 4.8, Corollary 4.11) needs f at the target,
// and its second-order terms the gradient and Hessian; the volume
// quadrature (Section 3.1) carries f only at its nodes, which come in
// consecutive groups of six per triangle (the 6-point rule of a background
// or cut triangle).  f near a target is the quadratic that interpolates f at
// the six nodes of one triangle:
//  * per triangle (plan creation): centroid c of the six nodes, scale h (the
//    largest node distance from c), the 6 x 6 matrix of the monomials
//    1, X, Y, X^2, XY, Y^2 of the scaled coordinates (X, Y) = (x - c)/h at
//    the nodes, inverted by Gauss-Jordan elimination with partial pivoting;
//    a shape measure (the smaller eigenvalue of the nodes' scaled second
//    moments) below THIN_MIN marks a sliver, whose nearly collinear nodes
//    leave the quadratic ill-determined across it: not used;
//  * per target that needs f (inside the domain, or a boundary node): the
//    triangle of the nearest node of a usable triangle (ties to the lowest
//    node index), from a cell list of those nodes searched ring by ring;
//  * per evaluation: the coefficients (inverse times the six nodal values)
//    and f, f_x, f_y, f_xx, f_xy, f_yy at the target, written where the
//    caller's f_trg would be ([batch][rows][n_out], caller order).
#include "mhk_internal.h"

namespace mhk {

constexpr int FJ_GROUP = 6;
constexpr double THIN_MIN = 1e-3;

__global__ void __launch_bounds__(256) k_tri_setup(int64_t ntri, const double *__restrict__ vx,
                                                   const double *__restrict__ vy, double *__restrict__ minv,
                                                   double *__restrict__ tc, uint8_t *__restrict__ good)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntri) return;
    double x[FJ_GROUP], y[FJ_GROUP];
    double cx = 0, cy = 0;
    for (int i = 0; i < FJ_GROUP; ++i) {
        x[i] = vx[t * FJ_GROUP + i];
        y[i] = vy[t * FJ_GROUP + i];
        cx += x[i];
        cy += y[i];
    }
    cx /= FJ_GROUP;
    cy /= FJ_GROUP;
    double h2 = 0;
    for (int i = 0; i < FJ_GROUP; ++i) h2 = fmax(h2, (x[i] - cx) * (x[i] - cx) + (y[i] - cy) * (y[i] - cy));
    const double h = sqrt(h2);
    double M[FJ_GROUP][2 * FJ_GROUP];
    double a = 0, b = 0, c = 0;
    for (int i = 0; i < FJ_GROUP; ++i) {
        const double X = (x[i] - cx) / h, Y = (y[i] - cy) / h;
        a += X * X;
        b += X * Y;
        c += Y * Y;
        const double row[FJ_GROUP] = {1.0, X, Y, X * X, X * Y, Y * Y};
        for (int k = 0; k < FJ_GROUP; ++k) {
            M[i][k] = row[k];
            M[i][FJ_GROUP + k] = (i == k) ? 1.0 : 0.0;
        }
    }
    a /= FJ_GROUP;
    b /= FJ_GROUP;
    c /= FJ_GROUP;
    const double thin = 0.5 * (a + c) - sqrt(0.25 * (a - c) * (a - c) + b * b);
    bool ok = h > 0.0 && thin >= THIN_MIN;
    // Gauss-Jordan with partial pivoting on [A | I]
    for (int col = 0; col < FJ_GROUP && ok; ++col) {
        int piv = col;
        for (int r = col + 1; r < FJ_GROUP; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (fabs(M[piv][col]) < 1e-13) {
            ok = false;
            break;
        }
        if (piv != col)
            for (int k = 0; k < 2 * FJ_GROUP; ++k) {
                const double tmp = M[col][k];
                M[col][k] = M[piv][k];
                M[piv][k] = tmp;
            }
        const double inv = 1.0 / M[col][col];
        for (int k = 0; k < 2 * FJ_GROUP; ++k) M[col][k] *= inv;
        for (int r = 0; r < FJ_GROUP; ++r) {
            if (r == col) continue;
            const double f = M[r][col];
            for (int k = 0; k < 2 * FJ_GROUP; ++k) M[r][k] -= f * M[col][k];
        }
    }
    // coefficients c = Minv f6: row k of the inverse in minv[t][k][0..5]
    for (int k = 0; k < FJ_GROUP; ++k)
        for (int i = 0; i < FJ_GROUP; ++i) minv[(t * FJ_GROUP + k) * FJ_GROUP + i] = ok ? M[k][FJ_GROUP + i] : 0.0;
    tc[t * 3 + 0] = cx;
    tc[t * 3 + 1] = cy;
    tc[t * 3 + 2] = h;
    good[t] = ok ? 1 : 0;
}

// cell key of every node of a usable triangle; nodes of other triangles get
// the key past the last cell (sorted to the end, never searched)
__global__ void __launch_bounds__(256) k_fj_keys(int64_t nv, const double *__restrict__ vx,
                                                 const double *__restrict__ vy, const uint8_t *__restrict__ good,
                                                 double ox, double oy, double cell, int64_t ncx, int64_t ncy,
                                                 uint32_t *__restrict__ key, int32_t *__restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    uint32_t k = (uint32_t)(ncx * ncy);
    if (good[i / FJ_GROUP]) {
        const int64_t ix = min(ncx - 1, max((int64_t)0, (int64_t)floor((vx[i] - ox) / cell)));
        const int64_t iy = min(ncy - 1, max((int64_t)0, (int64_t)floor((vy[i] - oy) / cell)));
        k = (uint32_t)(iy * ncx + ix);
    }
    key[i] = k;
    val[i] = (int32_t)i;
}

// Per sorted target: the triangle of the nearest usable node (-1 where f is
// not needed: exterior off-surface targets).  Rings of cells around the
// target's cell are searched until the best distance is below the ring's
// reach (every node not yet seen is at least r cells away); the grid covers
// the targets, so the bound holds.
__global__ void __launch_bounds__(256) k_fj_nearest(int64_t nout, int64_t nt, const double *__restrict__ tx,
                                                    const double *__restrict__ ty, const int8_t *__restrict__ tin,
                                                    const int32_t *__restrict__ tidx, const double *__restrict__ vx,
                                                    const double *__restrict__ vy, const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ start, double ox, double oy,
                                                    double cell, int64_t ncx, int64_t ncy,
                                                    int32_t *__restrict__ tri)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nout) return;
    const bool need = tin[s] != 0 || tidx[s] >= nt;
    if (!need) {
        tri[s] = -1;
        return;
    }
    const double px = tx[s], py = ty[s];
    const int64_t cx = min(ncx - 1, max((int64_t)0, (int64_t)floor((px - ox) / cell)));
    const int64_t cy = min(ncy - 1, max((int64_t)0, (int64_t)floor((py - oy) / cell)));
    double best = INFINITY;
    int32_t bi = INT32_MAX;
    const int64_t rmax = max(ncx, ncy);
    for (int64_t r = 0; r <= rmax; ++r) {
        for (int64_t iy = cy - r; iy <= cy + r; ++iy) {
            if (iy < 0 || iy >= ncy) continue;
            const bool edge_row = iy == cy - r || iy == cy + r;
            for (int64_t ix = cx - r; ix <= cx + r; ix += (edge_row || r == 0) ? 1 : 2 * r) {
                if (ix < 0 || ix >= ncx) continue;
                const int64_t c = iy * ncx + ix;
                for (int32_t k = start[c]; k < start[c + 1]; ++k) {
                    const int32_t i = perm[k];
                    const double dx = vx[i] - px, dy = vy[i] - py;
                    const double d2 = dx * dx + dy * dy;
                    if (d2 < best || (d2 == best && i < bi)) {
                        best = d2;
                        bi = i;
                    }
                }
            }
        }
        const double reach = (double)r * cell;
        if (best < reach * reach) break;
    }
    tri[s] = bi == INT32_MAX ? -1 : bi / FJ_GROUP;
}

// f (rows = 1) or f and its gradient and Hessian (rows = 6) at every target,
// [b][rows][nout] in caller order; zero where f is not needed
template <typename TF>
__global__ void __launch_bounds__(256) k_fjets(int64_t nout, int B, int rows, const double *__restrict__ tx,
                                               const double *__restrict__ ty, const int32_t *__restrict__ tidx,
                                               const int32_t *__restrict__ tri, const double *__restrict__ minv,
                                               const double *__restrict__ tc, int64_t nv, const TF *__restrict__ fv,
                                               TF *__restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nout) return;
    const int64_t idx = tidx[s];
    const int32_t t = tri[s];
    double X = 0, Y = 0, h = 1;
    if (t >= 0) {
        h = tc[t * 3 + 2];
        X = (tx[s] - tc[t * 3 + 0]) / h;
        Y = (ty[s] - tc[t * 3 + 1]) / h;
    }
    for (int b = 0; b < B; ++b) {
        double j[6] = {0, 0, 0, 0, 0, 0};
        if (t >= 0) {
            double f6[FJ_GROUP], c[FJ_GROUP];
            for (int i = 0; i < FJ_GROUP; ++i) f6[i] = (double)fv[(size_t)b * nv + (size_t)t * FJ_GROUP + i];
            for (int k = 0; k < FJ_GROUP; ++k) {
                double v = 0;
                for (int i = 0; i < FJ_GROUP; ++i) v = fma(minv[((size_t)t * FJ_GROUP + k) * FJ_GROUP + i], f6[i], v);
                c[k] = v;
            }
            j[0] = c[0] + c[1] * X + c[2] * Y + c[3] * X * X + c[4] * X * Y + c[5] * Y * Y;
            j[1] = (c[1] + 2 * c[3] * X + c[4] * Y) / h;
            j[2] = (c[2] + c[4] * X + 2 * c[5] * Y) / h;
            j[3] = 2 * c[3] / (h * h);
            j[4] = c[4] / (h * h);
            j[5] = 2 * c[5] / (h * h);
        }
        for (int r = 0; r < rows; ++r) out[((size_t)b * rows + r) * nout + idx] = (TF)j[r];
    }
}

hipError_t dev_fj_setup(int64_t ntri, const double *vx, const double *vy, double *minv, double *tc, uint8_t *good,
                        hipStream_t st)
{
    if (ntri <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri_setup, dim3((unsigned)((ntri + 255) / 256)), dim3(256), 0, st, ntri, vx, vy, minv, tc,
                       good);
    return hipGetLastError();
}

// cell list of the nodes of usable triangles (kept by the plan: the level
// nodes of the volume potential are located with it too) and each sorted
// target's triangle
hipError_t dev_fj_nearest(mhk_plan *P, const double *vx, const double *vy, const uint8_t *good, double ox,
                          double oy, double cell, int64_t ncx, int64_t ncy, int32_t *tri, hipStream_t st)
{
    FJets &F = P->fj;
    const int64_t nv = P->nv;
    uint32_t *key = nullptr;
    hipError_t e = hipMallocAsync((void **)&key, sizeof(uint32_t) * nv, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fj_keys, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, nv, vx, vy, good, ox, oy,
                           cell, ncx, ncy, key, F.perm);
        e = hipGetLastError();
    }
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) <= ncx * ncy) ++bits;
    if (e == hipSuccess) e = dev_sort_pairs(key, F.perm, nv, bits, st);
    // starts of the ncx * ncy cells and of the unusable tail
    if (e == hipSuccess) e = dev_cell_starts(key, nv, ncx * ncy + 1, F.start, st);
    F.ox = ox;
    F.oy = oy;
    F.cell = cell;
    F.ncx = ncx;
    F.ncy = ncy;
    if (e == hipSuccess && P->nout > 0) {
        hipLaunchKernelGGL(k_fj_nearest, dim3((unsigned)((P->nout + 255) / 256)), dim3(256), 0, st, P->nout, P->nt,
                           P->tx, P->ty, P->tin, P->tidx, vx, vy, F.perm, F.start, ox, oy, cell, ncx, ncy, tri);
        e = hipGetLastError();
    }
    if (key) (void)hipFreeAsync(key, st);
    return e;
}

// the triangle of the nearest usable node for arbitrary points (the level
// nodes of the volume potential), with the cell list above; the points must
// lie in the box the cells cover
__global__ void __launch_bounds__(256) k_fj_nearest_pts(int64_t n, const double *__restrict__ px_,
                                                        const double *__restrict__ py_,
                                                        const int32_t *__restrict__ parent,
                                                        const uint8_t *__restrict__ good,
                                                        const double *__restrict__ vx, const double *__restrict__ vy,
                                                        const int32_t *__restrict__ perm,
                                                        const int32_t *__restrict__ start, double ox, double oy,
                                                        double cell, int64_t ncx, int64_t ncy,
                                                        int32_t *__restrict__ tri)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    // a point of a usable triangle keeps it
    if (parent && good[parent[s]]) {
        tri[s] = parent[s];
        return;
    }
    const double px = px_[s], py = py_[s];
    const int64_t cx = min(ncx - 1, max((int64_t)0, (int64_t)floor((px - ox) / cell)));
    const int64_t cy = min(ncy - 1, max((int64_t)0, (int64_t)floor((py - oy) / cell)));
    double best = INFINITY;
    int32_t bi = INT32_MAX;
    const int64_t rmax = max(ncx, ncy);
    for (int64_t r = 0; r <= rmax; ++r) {
        for (int64_t iy = cy - r; iy <= cy + r; ++iy) {
            if (iy < 0 || iy >= ncy) continue;
            const bool edge_row = iy == cy - r || iy == cy + r;
            for (int64_t ix = cx - r; ix <= cx + r; ix += (edge_row || r == 0) ? 1 : 2 * r) {
                if (ix < 0 || ix >= ncx) continue;
                const int64_t c = iy * ncx + ix;
                for (int32_t k = start[c]; k < start[c + 1]; ++k) {
                    const int32_t i = perm[k];
                    const double dx = vx[i] - px, dy = vy[i] - py;
                    const double d2 = dx * dx + dy * dy;
                    if (d2 < best || (d2 == best && i < bi)) {
                        best = d2;
                        bi = i;
                    }
                }
            }
        }
        const double reach = (double)r * cell;
        if (best < reach * reach) break;
    }
    tri[s] = bi == INT32_MAX ? 0 : bi / FJ_GROUP;
}

hipError_t dev_fj_nearest_pts(mhk_plan *P, int64_t n, const double *px, const double *py, const int32_t *parent,
                              const double *vx, const double *vy, int32_t *tri, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const FJets &F = P->fj;
    hipLaunchKernelGGL(k_fj_nearest_pts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, px, py, parent,
                       F.good, vx, vy, F.perm, F.start, F.ox, F.oy, F.cell, F.ncx, F.ncy, tri);
    return hipGetLastError();
}

hipError_t launch_fjets(mhk_plan *P, const void *f_vol, void *out)
{
    const int rows = P->p.local_order >= 2 ? 6 : 1;
    const dim3 grid((unsigned)((P->nout + 255) / 256));
    if (P->p.prec == MHK_FP64 || P->p.in64)
        hipLaunchKernelGGL(k_fjets<double>, grid, dim3(256), 0, P->stream, P->nout, P->bat, rows, P->tx, P->ty,
                           P->tidx, P->fj.tri, P->fj.minv, P->fj.tc, P->nv, (const double *)f_vol, (double *)out);
    else
        hipLaunchKernelGGL(k_fjets<float>, grid, dim3(256), 0, P->stream, P->nout, P->bat, rows, P->tx, P->ty,
                           P->tidx, P->fj.tri, P->fj.minv, P->fj.tc, P->nv, (const float *)f_vol, (float *)out);
    return hipGetLastError();
}

}  // namespace mhk
