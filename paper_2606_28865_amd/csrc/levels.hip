// Dyadic difference-kernel levels (Section 4.2, eqs. (sld), (dld)).
//
// Level j sums, for every target x,
//   S_j(x) = sum_q w_q sigma_q K_j^S(|x - x_q|),
//   D_j(x) = sum_q w_q mu_q nu_q.(x - x_q) K_j^D(|x - x_q|),
// over the child nodes q of the panels bisected j times.  The kernels are
// read from a piecewise-polynomial table in a = r^2/(4 delta_j) held in LDS;
// pairs with a >= a_max are below the requested accuracy and skipped.
//
// Work decomposition: a workgroup owns 256 consecutive targets of the Morton
// order, takes the bounding box of their cells (cells of side R_j) and walks
// the sources of the 3x3-extended box row by row.  Sources are staged through
// LDS in blocks of 256 and read back by broadcast, so every source is loaded
// from HBM once per workgroup, and each lane keeps its target's sums in
// registers: no atomics, deterministic summation order.
#include "mhk_internal.h"

namespace mhk {

// Child-node strengths of level j for the current densities: q_S = w sigma,
// q_Dx = w nu_x mu, q_Dy = w nu_y mu, with sigma, mu at the child node
// interpolated from the parent panel's 16 nodal values.
__global__ void __launch_bounds__(256) k_level_q(int64_t n_src, int nch, int B, int64_t nb,
                                                 const int32_t *__restrict__ code,
                                                 const double *__restrict__ T,
                                                 const double *__restrict__ sw,
                                                 const double *__restrict__ swx,
                                                 const double *__restrict__ swy,
                                                 const double *__restrict__ sigma,
                                                 const double *__restrict__ mu,
                                                 double *__restrict__ q)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_src) return;
    int c = code[s];
    int k = c % NGL;
    int pc = c / NGL;
    int child = pc % nch;
    int64_t panel = pc / nch;
    const double *row = T + ((size_t)child * NGL + k) * NGL;
    double r[NGL];
#pragma unroll
    for (int i = 0; i < NGL; ++i) r[i] = row[i];
    const double w = sw[s], wx = swx[s], wy = swy[s];
    for (int b = 0; b < B; ++b) {
        if (sigma) {
            const double *f = sigma + (size_t)b * nb + panel * NGL;
            double v = 0;
#pragma unroll
            for (int i = 0; i < NGL; ++i) v = fma(r[i], f[i], v);
            q[((size_t)0 * B + b) * n_src + s] = w * v;
        }
        if (mu) {
            const double *f = mu + (size_t)b * nb + panel * NGL;
            double v = 0;
#pragma unroll
            for (int i = 0; i < NGL; ++i) v = fma(r[i], f[i], v);
            q[((size_t)1 * B + b) * n_src + s] = wx * v;
            q[((size_t)2 * B + b) * n_src + s] = wy * v;
        }
    }
}

struct LevelArgs {
    int64_t nout, n_src;
    const double *tx, *ty;
    double ox, oy, cell, inv4d, a_max, seg_inv;
    int ncx, ncy, nseg, B, b0, nbh;
    const int32_t *cell_start;
    const double *sx, *sy, *q, *tab;
    double *acc_s, *acc_d;     // [B][nout] each (sorted order)
    int want_s, want_d;
};

template <int BCH>
__global__ void __launch_bounds__(LV_BLOCK) k_level_sums(LevelArgs A)
{
    extern __shared__ double lds[];
    double *s_tab = lds;                                  // [nseg][TAB_NC][2]
    double *s_x = lds + (size_t)A.nseg * TAB_NC * 2;      // [LV_BLOCK]
    double *s_y = s_x + LV_BLOCK;
    double *s_q = s_y + LV_BLOCK;                         // [3*BCH][LV_BLOCK]
    __shared__ int bbox[4];

    const int tid = threadIdx.x;
    for (int i = tid; i < A.nseg * TAB_NC * 2; i += LV_BLOCK) s_tab[i] = A.tab[i];
    if (tid == 0) {
        bbox[0] = 0x7fffffff; bbox[1] = -1; bbox[2] = 0x7fffffff; bbox[3] = -1;
    }
    __syncthreads();

    const int64_t t = (int64_t)blockIdx.x * LV_BLOCK + tid;
    const bool active = t < A.nout;
    double x = 0, y = 0;
    if (active) {
        x = A.tx[t];
        y = A.ty[t];
        int cx = (int)floor((x - A.ox) / A.cell);
        int cy = (int)floor((y - A.oy) / A.cell);
        cx = min(max(cx, 0), A.ncx - 1);
        cy = min(max(cy, 0), A.ncy - 1);
        atomicMin(&bbox[0], cx);
        atomicMax(&bbox[1], cx);
        atomicMin(&bbox[2], cy);
        atomicMax(&bbox[3], cy);
    }
    __syncthreads();
    const int x0 = max(bbox[0] - 1, 0), x1 = min(bbox[1] + 1, A.ncx - 1);
    const int y0 = max(bbox[2] - 1, 0), y1 = min(bbox[3] + 1, A.ncy - 1);

    double S[BCH], D[BCH];
#pragma unroll
    for (int b = 0; b < BCH; ++b) S[b] = D[b] = 0.0;

    for (int cy = y0; cy <= y1; ++cy) {
        const int s0 = A.cell_start[(int64_t)cy * A.ncx + x0];
        const int s1 = A.cell_start[(int64_t)cy * A.ncx + x1 + 1];
        for (int c0 = s0; c0 < s1; c0 += LV_BLOCK) {
            const int m = min(LV_BLOCK, s1 - c0);
            __syncthreads();
            if (tid < m) {
                const int64_t s = c0 + tid;
                s_x[tid] = A.sx[s];
                s_y[tid] = A.sy[s];
#pragma unroll
                for (int b = 0; b < BCH; ++b) {
                    if (b < A.nbh) {
                        const int bb = A.b0 + b;
                        s_q[(0 * BCH + b) * LV_BLOCK + tid] = A.want_s ? A.q[((size_t)0 * A.B + bb) * A.n_src + s] : 0.0;
                        s_q[(1 * BCH + b) * LV_BLOCK + tid] = A.want_d ? A.q[((size_t)1 * A.B + bb) * A.n_src + s] : 0.0;
                        s_q[(2 * BCH + b) * LV_BLOCK + tid] = A.want_d ? A.q[((size_t)2 * A.B + bb) * A.n_src + s] : 0.0;
                    }
                }
            }
            __syncthreads();
            if (active) {
                for (int i = 0; i < m; ++i) {
                    const double dx = x - s_x[i], dy = y - s_y[i];
                    const double a = (dx * dx + dy * dy) * A.inv4d;
                    if (a < A.a_max) {
                        const double f = a * A.seg_inv;
                        const int sg = (int)f;
                        const double v = 2.0 * (f - sg) - 1.0;
                        const double2 *c = reinterpret_cast<const double2 *>(s_tab) + sg * TAB_NC;
                        double2 cc = c[TAB_NC - 1];
                        double ks = cc.x, kd = cc.y;
#pragma unroll
                        for (int k = TAB_NC - 2; k >= 0; --k) {
                            cc = c[k];
                            ks = fma(ks, v, cc.x);
                            kd = fma(kd, v, cc.y);
                        }
#pragma unroll
                        for (int b = 0; b < BCH; ++b) {
                            S[b] = fma(s_q[(0 * BCH + b) * LV_BLOCK + i], ks, S[b]);
                            const double nd = fma(s_q[(1 * BCH + b) * LV_BLOCK + i], dx,
                                                  s_q[(2 * BCH + b) * LV_BLOCK + i] * dy);
                            D[b] = fma(nd, kd, D[b]);
                        }
                    }
                }
            }
        }
    }
    if (active) {
#pragma unroll
        for (int b = 0; b < BCH; ++b) {
            if (b < A.nbh) {
                const size_t o = (size_t)(A.b0 + b) * A.nout + t;
                if (A.want_s) A.acc_s[o] += S[b];
                if (A.want_d) A.acc_d[o] += D[b];
            }
        }
    }
}

hipError_t launch_level_densities(mhk_plan *P, int j, const double *sigma, const double *mu)
{
    Level &L = P->lev[j - 1];
    const int64_t n = L.n_src;
    dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_level_q, grid, dim3(256), 0, P->stream, n, L.nchild, P->p.batch, P->nb, L.code,
                       L.interp, L.sw, L.swx, L.swy, sigma, mu, L.q);
    return hipGetLastError();
}

hipError_t launch_level_sums(mhk_plan *P, int j, bool want_s, bool want_d)
{
    Level &L = P->lev[j - 1];
    const int B = P->p.batch;
    LevelArgs A;
    A.nout = P->nout;
    A.n_src = L.n_src;
    A.tx = P->tx;
    A.ty = P->ty;
    A.ox = L.ox;
    A.oy = L.oy;
    A.cell = L.cell;
    A.inv4d = L.inv4d;
    A.a_max = L.a_max;
    A.seg_inv = L.seg_inv;
    A.ncx = L.ncx;
    A.ncy = L.ncy;
    A.nseg = L.nseg;
    A.B = B;
    A.cell_start = L.cell_start;
    A.sx = L.sx;
    A.sy = L.sy;
    A.q = L.q;
    A.tab = L.tab;
    A.acc_s = P->acc;                                  // component 0: S
    A.acc_d = P->acc + (size_t)B * P->nout;            // component 1: D
    A.want_s = want_s;
    A.want_d = want_d;
    const size_t lds = sizeof(double) * ((size_t)L.nseg * TAB_NC * 2 + (2 + 3 * LV_BCH) * LV_BLOCK);
    dim3 grid((unsigned)((P->nout + LV_BLOCK - 1) / LV_BLOCK));
    for (int b0 = 0; b0 < B; b0 += LV_BCH) {
        A.b0 = b0;
        A.nbh = min(LV_BCH, B - b0);
        if (A.nbh == 1)
            hipLaunchKernelGGL(k_level_sums<1>, grid, dim3(LV_BLOCK), lds, P->stream, A);
        else
            hipLaunchKernelGGL(k_level_sums<LV_BCH>, grid, dim3(LV_BLOCK), lds, P->stream, A);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mhk
