// Dyadic difference-kernel levels (Section 4.2, eqs. (sld), (dld)).
//
// Level j sums, for every target x,
//   S_j(x) = sum_q w_q sigma_q K_j^S(|x - x_q|),
//   D_j(x) = sum_q w_q mu_q nu_q.(x - x_q) K_j^D(|x - x_q|),
// over the child nodes q of the panels bisected j times.  The kernels come
// from one piecewise-polynomial table of K_j^S in a = r^2/(4 delta_j) held in
// LDS: Horner's rule gives the polynomial and its derivative together, and
// K_j^D is a constant times dK_j^S/da, applied once per target at the end
// (the table reads, which bound the loop, serve both kernels).  Pairs with
// a >= a_max are below the requested accuracy and skipped.
//
// Work decomposition: a wavefront owns 64 consecutive targets of the Morton
// order.  At plan time the cells (side R_j/4) that can hold a source within
// R_j of one of its targets are turned into a short list of ranges of the
// cell-sorted sources.  The wavefront reads its ranges and then, range by
// range, 64 sources at a time with vector loads (lane l holds source l) and
// hands each source to all lanes with readlane; each lane keeps its target's
// sums in registers: no atomics, no barriers in the loop, deterministic
// summation order.  The kernel table sits in LDS (shared by the wavefronts of
// a workgroup) with a padded segment stride so that the per-lane gathers of
// different segments spread over the LDS banks.
//
// Precision: T = double (FP64 path) or float (FP32 path).  In the FP32 path
// the separation x - x_q is formed in FP64 from FP64 positions and rounded
// once, so that its relative error is that of one rounding even when the
// separation is far smaller than the coordinates; the table (degree 7), the
// kernel evaluation and the accumulation are FP32.
#include "mhk_internal.h"

namespace mhk {

// Child-node strengths of level j for the current densities: q_S = w sigma,
// q_Dx = w nu_x mu, q_Dy = w nu_y mu, with sigma, mu at the child node
// interpolated from the parent panel's 16 nodal values.
template <typename T>
__global__ void __launch_bounds__(256) k_level_q(int64_t n_src, int nch, int B, int64_t nb,
                                                 const int32_t *__restrict__ code,
                                                 const double *__restrict__ Tm,
                                                 const double *__restrict__ sw,
                                                 const double *__restrict__ swx,
                                                 const double *__restrict__ swy,
                                                 const T *__restrict__ sigma,
                                                 const T *__restrict__ mu,
                                                 T *__restrict__ q)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_src) return;
    int c = code[s];
    int k = c % NGL;
    int pc = c / NGL;
    int child = pc % nch;
    int64_t panel = pc / nch;
    const double *row = Tm + ((size_t)child * NGL + k) * NGL;
    double r[NGL];
#pragma unroll
    for (int i = 0; i < NGL; ++i) r[i] = row[i];
    const double w = sw[s], wx = swx[s], wy = swy[s];
    for (int b = 0; b < B; ++b) {
        if (sigma) {
            const T *f = sigma + (size_t)b * nb + panel * NGL;
            double v = 0;
#pragma unroll
            for (int i = 0; i < NGL; ++i) v = fma(r[i], (double)f[i], v);
            q[((size_t)0 * B + b) * n_src + s] = (T)(w * v);
        }
        if (mu) {
            const T *f = mu + (size_t)b * nb + panel * NGL;
            double v = 0;
#pragma unroll
            for (int i = 0; i < NGL; ++i) v = fma(r[i], (double)f[i], v);
            q[((size_t)1 * B + b) * n_src + s] = (T)(wx * v);
            q[((size_t)2 * B + b) * n_src + s] = (T)(wy * v);
        }
    }
}

template <typename T>
struct LevelArgs {
    int64_t nout, n_src;
    const double *tx, *ty;
    double inv4d, a_max, seg_inv, d_scale;
    int nseg, B;
    const int32_t *blk_ofs, *blk_rng, *wave_order;
    const double *sx, *sy;
    const T *q, *tab;
    T *acc_s, *acc_d;     // [B][nout] each (sorted order)
    int want_s, want_d;
    int init;             // store (first level) instead of add
};


// Value of lane k (wave-uniform k) for the whole wave.
__device__ inline double bcast(double v, int k)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}
__device__ inline float bcast(float v, int k)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// x - floor(x) for x >= 0 (exact), one instruction
__device__ inline double frac_part(double x) { return __builtin_amdgcn_fract(x); }
__device__ inline float frac_part(float x) { return __builtin_amdgcn_fractf(x); }

template <int BCH, typename T, int NC, int STRIDE>
__global__ void __launch_bounds__(LV_BLOCK) k_level_sums(LevelArgs<T> A)
{
    extern __shared__ double lds[];
    T *s_tab = reinterpret_cast<T *>(lds);                // [nseg][STRIDE]
    const int tid = threadIdx.x;
    for (int i = tid; i < A.nseg * STRIDE; i += LV_BLOCK) s_tab[i] = A.tab[i];
    __syncthreads();

    // one wavefront = LV_TPW consecutive targets with their own source ranges
    // (the wave number is wave-uniform); lane l holds targets l, l + 64, ...
    const int wave = __builtin_amdgcn_readfirstlane(A.wave_order[blockIdx.x * (LV_BLOCK / LV_WAVE) + tid / LV_WAVE]);
    double x[LV_TPL], y[LV_TPL];
    int64_t t[LV_TPL];
#pragma unroll
    for (int i = 0; i < LV_TPL; ++i) {
        t[i] = (int64_t)wave * LV_TPW + i * LV_WAVE + (tid % LV_WAVE);
        x[i] = y[i] = 0.0;
        if (t[i] < A.nout) {
            x[i] = A.tx[t[i]];
            y[i] = A.ty[t[i]];
        }
    }
    const int b0 = blockIdx.y * BCH, nbh = min(BCH, A.B - b0);
    // segment coordinate f = a seg_inv = r^2 inv4d seg_inv in one product
    const T fscale = (T)(A.inv4d * A.seg_inv), f_max = (T)(A.a_max * A.seg_inv);
    T S[LV_TPL][BCH], D[LV_TPL][BCH];
#pragma unroll
    for (int i = 0; i < LV_TPL; ++i)
#pragma unroll
        for (int b = 0; b < BCH; ++b) S[i][b] = D[i][b] = (T)0;
    const T *qs[BCH], *qx[BCH], *qy[BCH];
#pragma unroll
    for (int b = 0; b < BCH; ++b) {
        const int bb = b0 + min(b, nbh - 1);
        qs[b] = A.q + ((size_t)0 * A.B + bb) * A.n_src;
        qx[b] = A.q + ((size_t)1 * A.B + bb) * A.n_src;
        qy[b] = A.q + ((size_t)2 * A.B + bb) * A.n_src;
    }

    // source k of the lanes' batch against the lane's targets; the source's
    // strengths are handed over only where some lane is in range
    auto pair = [&](int k, double sxv, double syv, const T *lqs, const T *lqx, const T *lqy) {
#pragma unroll
        for (int i = 0; i < LV_TPL; ++i) {
            const T dx = (T)(x[i] - sxv), dy = (T)(y[i] - syv);
            const T f = (dx * dx + dy * dy) * fscale;
            if (f < f_max) {
                const int sg = (int)f;
                const T v = (T)2 * frac_part(f) - (T)1;
                const T *c = s_tab + __umul24((unsigned)sg, (unsigned)STRIDE);
                // p(v) and p'(v) by Horner's rule (K_j^S and, up to the
                // factor d_scale, K_j^D); the derivative's first step is c_7
                T kd = c[NC - 1];
                T ks = fma(kd, v, c[NC - 2]);
#pragma unroll
                for (int m = NC - 3; m >= 0; --m) {
                    kd = fma(kd, v, ks);
                    ks = fma(ks, v, c[m]);
                }
#pragma unroll
                for (int b = 0; b < BCH; ++b) {
                    const T qsv = bcast(lqs[b], k), qxv = bcast(lqx[b], k), qyv = bcast(lqy[b], k);
                    S[i][b] = fma(qsv, ks, S[i][b]);
                    D[i][b] = fma(fma(qxv, dx, qyv * dy), kd, D[i][b]);
                }
            }
        }
    };
    // The wave's ranges and, per range, its sources 64 at a time are read
    // with vector loads, lane l holding item l, and handed to the whole wave
    // one by one with readlane: no scalar loads are in flight in the loop,
    // so the waits for the kernel-table reads from LDS (which share their
    // counter with scalar loads) never wait for source data.
    const int lane = tid % LV_WAVE;
    const int r0 = A.blk_ofs[wave], r1 = A.blk_ofs[wave + 1];
    for (int rb = r0; rb < r1; rb += LV_WAVE) {
        int my_s0 = 0, my_s1 = 0;
        if (rb + lane < r1) {
            my_s0 = A.blk_rng[2 * (rb + lane)];
            my_s1 = A.blk_rng[2 * (rb + lane) + 1];
        }
        const int rcnt = min(LV_WAVE, r1 - rb);
        for (int ri = 0; ri < rcnt; ++ri) {
            const int s0 = __builtin_amdgcn_readlane(my_s0, ri), s1 = __builtin_amdgcn_readlane(my_s1, ri);
            for (int base = s0; base < s1; base += LV_WAVE) {
                const int sl = min(base + lane, s1 - 1);
                const double lx = A.sx[sl], ly = A.sy[sl];
                T lqs[BCH], lqx[BCH], lqy[BCH];
#pragma unroll
                for (int b = 0; b < BCH; ++b) {
                    lqs[b] = A.want_s ? qs[b][sl] : (T)0;
                    lqx[b] = A.want_d ? qx[b][sl] : (T)0;
                    lqy[b] = A.want_d ? qy[b][sl] : (T)0;
                }
                const int cnt = __builtin_amdgcn_readfirstlane(min(LV_WAVE, s1 - base));   // wave-uniform: scalar loop test
                for (int k = 0; k < cnt; ++k) pair(k, bcast(lx, k), bcast(ly, k), lqs, lqx, lqy);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < LV_TPL; ++i) {
        if (t[i] < A.nout) {
#pragma unroll
            for (int b = 0; b < BCH; ++b) {
                if (b < nbh) {
                    const size_t o = (size_t)(b0 + b) * A.nout + t[i];
                    const T s = S[i][b], d = D[i][b] * (T)A.d_scale;
                    if (A.want_s) A.acc_s[o] = A.init ? s : A.acc_s[o] + s;
                    if (A.want_d) A.acc_d[o] = A.init ? d : A.acc_d[o] + d;
                }
            }
        }
    }
}

template <typename T>
static hipError_t level_q(mhk_plan *P, hipStream_t st, int j, const void *sigma, const void *mu)
{
    Level &L = P->lev[j - 1];
    const int64_t n = L.n_src;
    dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_level_q<T>, grid, dim3(256), 0, st, n, L.nchild, P->p.batch, P->nb, L.code,
                       L.interp, L.sw, L.swx, L.swy, (const T *)sigma, (const T *)mu, (T *)L.q);
    return hipGetLastError();
}

hipError_t launch_level_densities(mhk_plan *P, hipStream_t st, int j, const void *sigma, const void *mu)
{
    return P->p.prec == MHK_FP64 ? level_q<double>(P, st, j, sigma, mu) : level_q<float>(P, st, j, sigma, mu);
}

template <typename T, int NC, int STRIDE>
static hipError_t level_sums(mhk_plan *P, hipStream_t st, int j, bool want_s, bool want_d, bool init)
{
    Level &L = P->lev[j - 1];
    const int B = P->p.batch;
    LevelArgs<T> A;
    A.nout = P->nout;
    A.n_src = L.n_src;
    A.tx = P->tx;
    A.ty = P->ty;
    A.inv4d = L.inv4d;
    A.a_max = L.a_max;
    A.seg_inv = L.seg_inv;
    A.d_scale = level_d_scale(L);
    A.nseg = L.nseg;
    A.B = B;
    A.blk_ofs = L.blk_ofs;
    A.blk_rng = L.blk_rng;
    A.wave_order = L.wave_order;
    A.sx = L.sx;
    A.sy = L.sy;
    A.q = (const T *)L.q;
    A.tab = (const T *)L.tab_dev;
    A.acc_s = (T *)P->acc_lev;                              // component 0: S
    A.acc_d = (T *)P->acc_lev + (size_t)B * P->nout;        // component 1: D
    A.want_s = want_s;
    A.want_d = want_d;
    A.init = init;
    const int bch = B == 1 ? 1 : LV_BCH;
    dim3 grid((unsigned)((P->nout + LV_BLOCK * LV_TPL - 1) / (LV_BLOCK * LV_TPL)), (unsigned)((B + bch - 1) / bch));
    const size_t lds = sizeof(T) * (size_t)L.nseg * STRIDE;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (bch == 1) {
        if (lds > 64 * 1024)
            (void)hipFuncSetAttribute((const void *)k_level_sums<1, T, NC, STRIDE>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_level_sums<1, T, NC, STRIDE>), grid, dim3(LV_BLOCK), lds, st, A);
    } else {
        if (lds > 64 * 1024)
            (void)hipFuncSetAttribute((const void *)k_level_sums<LV_BCH, T, NC, STRIDE>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((k_level_sums<LV_BCH, T, NC, STRIDE>), grid, dim3(LV_BLOCK), lds, st, A);
    }
    return hipGetLastError();
}

hipError_t launch_level_sums(mhk_plan *P, hipStream_t st, int j, bool want_s, bool want_d, bool init)
{
    if (P->p.prec == MHK_FP64) return level_sums<double, TAB_NC, TAB_STRIDE>(P, st, j, want_s, want_d, init);
    return level_sums<float, TABF_NC, TABF_STRIDE>(P, st, j, want_s, want_d, init);
}

}  // namespace mhk
