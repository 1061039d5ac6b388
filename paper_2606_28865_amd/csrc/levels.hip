// Dyadic difference-kernel levels (Section 4.2, eqs. (sld), (dld)).
//
// Level j sums, for every target x,
//   S_j(x) = sum_q w_q sigma_q K_j^S(|x - x_q|),
//   D_j(x) = sum_q w_q mu_q nu_q.(x - x_q) K_j^D(|x - x_q|),
// over the child nodes q of the panels bisected j times.  The kernels come
// from one piecewise-polynomial table of K_j^S in a = r^2/(4 delta_j) held in
// LDS: Horner's rule gives the polynomial and its derivative together, and
// K_j^D is a constant times dK_j^S/da, applied once per target at the end
// (the table reads serve both kernels).  Pairs with a >= a_max are below
// the requested accuracy and skipped (a lane beyond it reads the table's
// zero segment).  Target and source coordinates are scaled by sqrt(seg_inv / (4 delta_j)),
// so that the squared separation is the segment coordinate a seg_inv itself;
// the double-layer sum is rescaled once per target.
//
// Work decomposition: a wavefront owns 64 consecutive targets of the Morton
// order, one per lane, and a flat list (built at plan time) of the sources
// within R_j of its targets' bounding box.  It reads the list 64 sources at
// a time with vector loads (lane l holds source l) -- the next batch is
// loaded while the current one is summed -- and hands each source to all
// lanes with readlane; each lane keeps its target's sums in registers: no
// atomics, no barriers in the loop, deterministic summation order.  Sources
// are taken two at a time with no branch per lane, and a pair of sources out
// of range of every lane is skipped as a whole.  The two polynomial
// evaluations are independent, so their table reads and multiply-adds
// interleave.  The kernel table sits in LDS (shared by the wavefronts of a
// workgroup) in rows of 48 bytes, an odd multiple of 16, read as aligned
// 16-byte loads, so that neighbouring segments fall in different bank
// groups.
//
// Precision: T = double (FP64 path) or float (FP32 path).  In the FP32 path
// the separation x - x_q is formed in FP64 from FP64 positions and rounded
// once, so that its relative error is that of one rounding even when the
// separation is far smaller than the coordinates; the table (degree 7), the
// kernel evaluation and the accumulation are FP32.  The FP64 path keeps its
// table's three highest coefficients, each below 4e-8 of K_j(0), as floats
// and starts Horner's rule over them in FP32 (52 bytes of table per pair
// instead of 64); the rest is FP64.
#include <type_traits>

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
    double pscale;        // sqrt(inv4d seg_inv): coordinates scaled by it give f = a seg_inv = |dx|^2
    int nseg, B;
    const int32_t *wave_ofs, *wave_src, *wave_order;
    const double *sx, *sy;
    const T *q, *tab;
    T *acc_s, *acc_d;     // [B][nout] each (sorted order)
    int want_s, want_d;
    int init;             // store (first level) instead of add
    int64_t n_wave;       // wavefront lists (persistent launch: work items n_wave x density chunks)
    int *counter;         // persistent launch: next work item, zero at the launch
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

// One batch of up to 64 sources held one per lane: positions and strengths.
template <typename T, int BCH>
struct SrcBatch {
    double x, y;
    T qs[BCH], qx[BCH], qy[BCH];
};

// Source k of a batch against the lane's target: separation, table segment
// (the zero segment out of range), local variable.
template <typename T>
struct PairGeo {
    T dx, dy, v;
    const T *c;          // the segment's row
    const float *c7;     // FP64 table: the segment's c_7
};

template <typename T, int STRIDE>
__device__ inline PairGeo<T> pair_geo(double x, double y, double sxv, double syv, T f_max, T f_zero,
                                      const T *s_tab, const float *s_c7, bool &in)
{
    PairGeo<T> g;
    g.dx = (T)(x - sxv);
    g.dy = (T)(y - syv);
    // coordinates are scaled so that |dx|^2 is the segment coordinate
    // f = a seg_inv; a pair beyond the cut-off reads the zero segment f_zero
    // (at v = -1), which adds exactly nothing
    const T f = g.dx * g.dx + g.dy * g.dy;
    in = f < f_max;
    const T fc = in ? f : f_zero;
    const int sg = (int)fc;
    g.v = (T)2 * frac_part(fc) - (T)1;
    g.c = s_tab + __umul24((unsigned)sg, (unsigned)STRIDE);
    if constexpr (std::is_same<T, double>::value) g.c7 = s_c7 + sg;
    return g;
}

// p(v) and p'(v) of a table segment by Horner's rule for two sources at
// once (K_j^S and, up to the factor d_scale, K_j^D); the derivative's first
// step is c_7.  FP32 table: eight floats.
__device__ inline void horner2(const PairGeo<float> &g0, const PairGeo<float> &g1, float &ks0, float &kd0,
                               float &ks1, float &kd1)
{
    kd0 = g0.c[TAB_NC - 1];
    kd1 = g1.c[TAB_NC - 1];
    ks0 = fmaf(kd0, g0.v, g0.c[TAB_NC - 2]);
    ks1 = fmaf(kd1, g1.v, g1.c[TAB_NC - 2]);
#pragma unroll
    for (int m = TAB_NC - 3; m >= 0; --m) {
        kd0 = fmaf(kd0, g0.v, ks0);
        kd1 = fmaf(kd1, g1.v, ks1);
        ks0 = fmaf(ks0, g0.v, g0.c[m]);
        ks1 = fmaf(ks1, g1.v, g1.c[m]);
    }
}

// FP64 table row (48 bytes, 16-byte aligned): c_0..c_4 as doubles and c_5,
// c_6 as two floats, read as three 16-byte LDS loads; c_7 (float) from the
// array after the rows.  The high part goes through Horner's rule in FP32
// and the result continues in FP64 (the same order as the plan's accuracy
// check of the table).
struct Row64 {
    double c[TAB_NC64];
    float c5, c6, c7;
};
__device__ inline Row64 load_row(const PairGeo<double> &g)
{
    const double2 *r = reinterpret_cast<const double2 *>(g.c);
    const double2 a = r[0], b = r[1], h = r[2];
    Row64 w;
    w.c[0] = a.x;
    w.c[1] = a.y;
    w.c[2] = b.x;
    w.c[3] = b.y;
    w.c[4] = h.x;
    w.c5 = __int_as_float(__double2loint(h.y));
    w.c6 = __int_as_float(__double2hiint(h.y));
    w.c7 = *g.c7;
    return w;
}
__device__ inline void horner_hi(const Row64 &w, double v, float &ks, float &kd)
{
    const float vf = (float)v;
    kd = w.c7;
    ks = fmaf(kd, vf, w.c6);
    kd = fmaf(kd, vf, ks);
    ks = fmaf(ks, vf, w.c5);
}
__device__ inline void horner2(const PairGeo<double> &g0, const PairGeo<double> &g1, double &ks0, double &kd0,
                               double &ks1, double &kd1)
{
    const Row64 w0 = load_row(g0), w1 = load_row(g1);
    float hs0, hd0, hs1, hd1;
    horner_hi(w0, g0.v, hs0, hd0);
    horner_hi(w1, g1.v, hs1, hd1);
    ks0 = hs0;
    kd0 = hd0;
    ks1 = hs1;
    kd1 = hd1;
#pragma unroll
    for (int m = TAB_NC64 - 1; m >= 0; --m) {
        kd0 = fma(kd0, g0.v, ks0);
        kd1 = fma(kd1, g1.v, ks1);
        ks0 = fma(ks0, g0.v, w0.c[m]);
        ks1 = fma(ks1, g1.v, w1.c[m]);
    }
}
__device__ inline void horner1(const PairGeo<float> &g, float &ks, float &kd)
{
    kd = g.c[TAB_NC - 1];
    ks = fmaf(kd, g.v, g.c[TAB_NC - 2]);
#pragma unroll
    for (int m = TAB_NC - 3; m >= 0; --m) {
        kd = fmaf(kd, g.v, ks);
        ks = fmaf(ks, g.v, g.c[m]);
    }
}
__device__ inline void horner1(const PairGeo<double> &g, double &ks, double &kd)
{
    const Row64 w = load_row(g);
    float hs, hd;
    horner_hi(w, g.v, hs, hd);
    ks = hs;
    kd = hd;
#pragma unroll
    for (int m = TAB_NC64 - 1; m >= 0; --m) {
        kd = fma(kd, g.v, ks);
        ks = fma(ks, g.v, w.c[m]);
    }
}

// One work item: the LV_WAVE targets of wavefront list `wave` against its
// candidate sources, for the densities of chunk `chunk` (BCH of them).
template <int BCH, typename T, int STRIDE>
__device__ inline void level_item(const LevelArgs<T> &A, const T *s_tab, const float *s_c7, int lane, int wave,
                                  int chunk)
{
    const int64_t t = (int64_t)wave * LV_WAVE + lane;
    const double ps = A.pscale;
    double x = 0.0, y = 0.0;
    if (t < A.nout) {
        x = A.tx[t] * ps;
        y = A.ty[t] * ps;
    }
    const int b0 = chunk * BCH, nbh = min(BCH, A.B - b0);
    const T f_max = (T)(A.a_max * A.seg_inv), f_zero = (T)A.nseg;
    T S[BCH], D[BCH];
    // FP32 path: the sums of each batch of 64 sources are added into FP64
    // totals (a volume level sums thousands of nodes per target, where one
    // running FP32 sum would lose about sqrt(N) roundings)
    double S64[BCH], D64[BCH];
#pragma unroll
    for (int b = 0; b < BCH; ++b) S[b] = D[b] = (T)0, S64[b] = D64[b] = 0.0;
    // strengths of density b0 + b: q[c][b0 + b][s] for c = S, D_x, D_y
    const size_t fstride = (size_t)A.B * A.n_src;
    const T *q0 = A.q + (size_t)b0 * A.n_src;
    // lane l of a batch holds source l of the list; lanes past its end hold a
    // far-away source of zero strength
    auto load = [&](int pos, int end, SrcBatch<T, BCH> &sb) {
        if (pos < end) {
            const int s = A.wave_src[pos];
            sb.x = A.sx[s] * ps;
            sb.y = A.sy[s] * ps;
#pragma unroll
            for (int b = 0; b < BCH; ++b) {
                const T *qb = q0 + (size_t)min(b, nbh - 1) * A.n_src + s;
                sb.qs[b] = A.want_s ? qb[0] : (T)0;
                sb.qx[b] = A.want_d ? qb[fstride] : (T)0;
                sb.qy[b] = A.want_d ? qb[2 * fstride] : (T)0;
            }
        } else {
            sb.x = sb.y = 1e30;
#pragma unroll
            for (int b = 0; b < BCH; ++b) sb.qs[b] = sb.qx[b] = sb.qy[b] = (T)0;
        }
    };
    auto accumulate = [&](const SrcBatch<T, BCH> &sb, int k, const PairGeo<T> &g, T ks, T kd) {
#pragma unroll
        for (int b = 0; b < BCH; ++b) {
            const T qsv = bcast(sb.qs[b], k), qxv = bcast(sb.qx[b], k), qyv = bcast(sb.qy[b], k);
            S[b] = fma(qsv, ks, S[b]);
            D[b] = fma(fma(qxv, g.dx, qyv * g.dy), kd, D[b]);
        }
    };
    const int c0 = A.wave_ofs[wave], c1 = A.wave_ofs[wave + 1];
    SrcBatch<T, BCH> cur, nxt;
    load(c0 + lane, c1, cur);
    for (int base = c0; base < c1; base += LV_WAVE) {
        load(base + LV_WAVE + lane, c1, nxt);            // next batch in flight while this one is summed
        const int cnt = __builtin_amdgcn_readfirstlane(min(LV_WAVE, c1 - base));
        if (BCH == 1) {
            for (int k = 0; k < cnt; k += 2) {
                // sources k and k + 1 (past the batch's end: a lane holding
                // the far-away source of zero strength)
                bool in0, in1;
                const PairGeo<T> g0 = pair_geo<T, STRIDE>(x, y, bcast(cur.x, k), bcast(cur.y, k), f_max, f_zero,
                                                          s_tab, s_c7, in0);
                const PairGeo<T> g1 = pair_geo<T, STRIDE>(x, y, bcast(cur.x, k + 1), bcast(cur.y, k + 1), f_max,
                                                          f_zero, s_tab, s_c7, in1);
                if (__ballot(in0 || in1) == 0) continue;
                T ks0, kd0, ks1, kd1;
                horner2(g0, g1, ks0, kd0, ks1, kd1);
                accumulate(cur, k, g0, ks0, kd0);
                accumulate(cur, k + 1, g1, ks1, kd1);
            }
        } else {
            // several densities: the strengths of one source already fill
            // the registers, so one source at a time
            for (int k = 0; k < cnt; ++k) {
                bool in0;
                const PairGeo<T> g0 = pair_geo<T, STRIDE>(x, y, bcast(cur.x, k), bcast(cur.y, k), f_max, f_zero,
                                                          s_tab, s_c7, in0);
                if (__ballot(in0) == 0) continue;
                T ks0, kd0;
                horner1(g0, ks0, kd0);
                accumulate(cur, k, g0, ks0, kd0);
            }
        }
        if constexpr (std::is_same<T, float>::value) {
#pragma unroll
            for (int b = 0; b < BCH; ++b) {
                S64[b] += (double)S[b];
                D64[b] += (double)D[b];
                S[b] = D[b] = 0.0f;
            }
        }
        cur = nxt;
    }
    if constexpr (std::is_same<T, float>::value) {
#pragma unroll
        for (int b = 0; b < BCH; ++b) {
            S[b] = (float)S64[b];
            D[b] = (float)(D64[b] * A.d_scale);
        }
    } else {
#pragma unroll
        for (int b = 0; b < BCH; ++b) D[b] *= A.d_scale;
    }
    if (t < A.nout) {
#pragma unroll
        for (int b = 0; b < BCH; ++b) {
            if (b < nbh) {
                const size_t o = (size_t)(b0 + b) * A.nout + t;
                const T s = S[b], d = D[b];
                if (A.want_s) A.acc_s[o] = A.init ? s : A.acc_s[o] + s;
                if (A.want_d) A.acc_d[o] = A.init ? d : A.acc_d[o] + d;
            }
        }
    }
}

// The kernel table is loaded into LDS once per workgroup.  PERSIST = false:
// one work item per wavefront (wave list from the launch position, density
// chunk from blockIdx.y).  PERSIST = true: a grid sized to fill the device
// once; every wavefront takes work items (list-major: the density chunks of
// one list follow each other, so its candidates stay in cache) from a
// counter in device memory, zeroed before the launch, until none is left --
// the exit every wavefront reaches.
template <int BCH, typename T, int STRIDE, int NB, bool PERSIST>
__global__ void __launch_bounds__(NB) k_level_sums(LevelArgs<T> A)
{
    extern __shared__ double lds[];
    T *s_tab = reinterpret_cast<T *>(lds);                // [nseg + 1][STRIDE], the last segment zero
    const int tid = threadIdx.x;
    for (int i = tid; i < (A.nseg + 1) * STRIDE; i += NB) s_tab[i] = i < A.nseg * STRIDE ? A.tab[i] : (T)0;
    // FP64 table: c_7 of every segment (the zero segment's last) after the rows
    float *s_c7 = nullptr;
    if constexpr (std::is_same<T, double>::value) {
        s_c7 = reinterpret_cast<float *>(s_tab + (A.nseg + 1) * STRIDE);
        const float *g7 = reinterpret_cast<const float *>(A.tab + (size_t)A.nseg * STRIDE);
        for (int i = tid; i <= A.nseg; i += NB) s_c7[i] = i < A.nseg ? g7[i] : 0.0f;
    }
    __syncthreads();
    const int lane = tid % LV_WAVE;
    if (!PERSIST) {
        // the wave number is wave-uniform
        const int wave = __builtin_amdgcn_readfirstlane(A.wave_order[blockIdx.x * (NB / LV_WAVE) + tid / LV_WAVE]);
        level_item<BCH, T, STRIDE>(A, s_tab, s_c7, lane, wave, blockIdx.y);
        return;
    }
    const int nchunk = (A.B + BCH - 1) / BCH;
    const int64_t nitems = A.n_wave * nchunk;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(A.counter, 1);
        item = __builtin_amdgcn_readfirstlane(__shfl(item, 0));
        if (item >= nitems) break;
        const int wave = __builtin_amdgcn_readfirstlane(A.wave_order[item / nchunk]);
        level_item<BCH, T, STRIDE>(A, s_tab, s_c7, lane, wave, item % nchunk);
    }
}

// LDS bytes of a level's table: the rows of nseg + 1 segments (the last zero)
// and, FP64, their c_7 as floats
template <typename T, int STRIDE>
static size_t level_lds(int nseg)
{
    size_t b = sizeof(T) * (size_t)(nseg + 1) * STRIDE;
    if (std::is_same<T, double>::value) b += sizeof(float) * (size_t)(nseg + 2);
    return b;
}

template <typename T>
static hipError_t level_q(mhk_plan *P, hipStream_t st, int j, const void *sigma, const void *mu)
{
    Level &L = P->lev[j - 1];
    const int64_t n = L.n_src;
    dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_level_q<T>, grid, dim3(256), 0, st, n, L.nchild, P->bat, P->nb, L.code,
                       L.interp, L.sw, L.swx, L.swy, (const T *)sigma, (const T *)mu, (T *)L.q);
    return hipGetLastError();
}

hipError_t launch_level_densities(mhk_plan *P, hipStream_t st, int j, const void *sigma, const void *mu)
{
    return P->p.prec == MHK_FP64 ? level_q<double>(P, st, j, sigma, mu) : level_q<float>(P, st, j, sigma, mu);
}

template <int BCH, typename T, int STRIDE, int NB, bool PERSIST>
static void level_launch(const LevelArgs<T> &A, dim3 grid, size_t lds, hipStream_t st)
{
    const void *fn = (const void *)k_level_sums<BCH, T, STRIDE, NB, PERSIST>;
    if (lds > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (PERSIST) {
        // as many workgroups as are resident at once, at most one per item
        int per_cu = 0, dev = 0, ncu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NB, lds) != hipSuccess || per_cu < 1) per_cu = 1;
        const int64_t items = A.n_wave * grid.y;
        const int64_t wg = std::min<int64_t>((int64_t)per_cu * std::max(ncu, 1), (items + NB / LV_WAVE - 1) / (NB / LV_WAVE));
        grid = dim3((unsigned)std::max<int64_t>(1, wg), 1u);
    }
    hipLaunchKernelGGL((k_level_sums<BCH, T, STRIDE, NB, PERSIST>), grid, dim3(NB), lds, st, A);
}

template <int BCH, typename T, int STRIDE>
static void level_launch_nb(int nb, bool persist, const LevelArgs<T> &A, int64_t nwave, size_t lds, hipStream_t st,
                            int nbatch)
{
    // exactly nwave wavefronts (the lists are padded to whole workgroups of
    // either shape), the batch in chunks of BCH along y
    const dim3 grid((unsigned)(nwave / (nb / LV_WAVE)), (unsigned)nbatch);
    if (nb == 512) {
        if (persist) level_launch<BCH, T, STRIDE, 512, true>(A, grid, lds, st);
        else level_launch<BCH, T, STRIDE, 512, false>(A, grid, lds, st);
    } else {
        if (persist) level_launch<BCH, T, STRIDE, 256, true>(A, grid, lds, st);
        else level_launch<BCH, T, STRIDE, 256, false>(A, grid, lds, st);
    }
}

template <typename T, int STRIDE>
static hipError_t level_sums(mhk_plan *P, hipStream_t st, int j, bool want_s, bool want_d, bool init)
{
    Level &L = P->lev[j - 1];
    const int B = P->bat;
    LevelArgs<T> A;
    A.nout = P->nout;
    A.n_src = L.n_src;
    A.tx = P->tx;
    A.ty = P->ty;
    A.inv4d = L.inv4d;
    A.a_max = L.a_max;
    A.seg_inv = L.seg_inv;
    A.pscale = sqrt(L.inv4d * L.seg_inv);
    A.d_scale = level_d_scale(L) / A.pscale;       // D was summed over scaled separations
    A.nseg = L.nseg;
    A.B = B;
    A.wave_ofs = L.wave_ofs;
    A.wave_src = L.wave_src;
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
    // densities per pass: the plan's lv_bch, or fewer for a smaller batch
    // (rounded up to an instantiated size; missing densities of the last
    // pass are skipped)
    const int want = std::min(B, P->p.lv_bch);
    const int bch = want <= 1 ? 1 : want <= 2 ? 2 : want <= 4 ? 4 : 8;
    const int nby = (B + bch - 1) / bch;
    const size_t lds = level_lds<T, STRIDE>(L.nseg);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int nb = P->p.lv_block;
    const bool pers = P->p.lv_persist != 0;
    A.n_wave = L.n_wave;
    A.counter = P->lv_counter;
    if (pers) {
        const hipError_t e = launch_fill_int(P->lv_counter, 1, st);
        if (e != hipSuccess) return e;
    }
    switch (bch) {
    case 1: level_launch_nb<1, T, STRIDE>(nb, pers, A, L.n_wave, lds, st, nby); break;
    case 2: level_launch_nb<2, T, STRIDE>(nb, pers, A, L.n_wave, lds, st, nby); break;
    case 4: level_launch_nb<4, T, STRIDE>(nb, pers, A, L.n_wave, lds, st, nby); break;
    default: level_launch_nb<8, T, STRIDE>(nb, pers, A, L.n_wave, lds, st, nby); break;
    }
    return hipGetLastError();
}

// the volume potential's level j: the same kernel table, the volume level
// nodes as sources (single-layer sums only), into acc_vlev
template <typename T, int STRIDE>
static hipError_t level_sums_v(mhk_plan *P, hipStream_t st, int j, bool init)
{
    Level &L = P->lev[j - 1];
    VLevel &V = P->vlev[j - 1];
    const int B = P->bat;
    LevelArgs<T> A;
    A.nout = P->nout;
    A.n_src = V.n_src;
    A.tx = P->tx;
    A.ty = P->ty;
    A.inv4d = L.inv4d;
    A.a_max = L.a_max;
    A.seg_inv = L.seg_inv;
    A.pscale = sqrt(L.inv4d * L.seg_inv);
    A.d_scale = level_d_scale(L) / A.pscale;       // D was summed over scaled separations
    A.nseg = L.nseg;
    A.B = B;
    A.wave_ofs = V.wave_ofs;
    A.wave_src = V.wave_src;
    A.wave_order = V.wave_order;
    A.sx = V.sx;
    A.sy = V.sy;
    A.q = (const T *)V.q;
    A.tab = (const T *)L.tab_dev;
    A.acc_s = (T *)P->acc_vlev;
    A.acc_d = (T *)P->acc_vlev;            // not written (want_d = 0)
    A.want_s = 1;
    A.want_d = 0;
    A.init = init;
    const int want = std::min(B, P->p.lv_bch);
    const int bch = want <= 1 ? 1 : want <= 2 ? 2 : want <= 4 ? 4 : 8;
    const int nby = (B + bch - 1) / bch;
    const size_t lds = level_lds<T, STRIDE>(L.nseg);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int nb = P->p.lv_block;
    const bool pers = P->p.lv_persist != 0;
    A.n_wave = V.n_wave;
    A.counter = P->lv_counter;
    if (pers) {
        const hipError_t e = launch_fill_int(P->lv_counter, 1, st);
        if (e != hipSuccess) return e;
    }
    switch (bch) {
    case 1: level_launch_nb<1, T, STRIDE>(nb, pers, A, V.n_wave, lds, st, nby); break;
    case 2: level_launch_nb<2, T, STRIDE>(nb, pers, A, V.n_wave, lds, st, nby); break;
    case 4: level_launch_nb<4, T, STRIDE>(nb, pers, A, V.n_wave, lds, st, nby); break;
    default: level_launch_nb<8, T, STRIDE>(nb, pers, A, V.n_wave, lds, st, nby); break;
    }
    return hipGetLastError();
}

hipError_t launch_level_sums_v(mhk_plan *P, hipStream_t st, int j, bool init)
{
    if (P->p.prec == MHK_FP64) return level_sums_v<double, TAB_STRIDE>(P, st, j, init);
    return level_sums_v<float, TABF_STRIDE>(P, st, j, init);
}

hipError_t launch_level_sums(mhk_plan *P, hipStream_t st, int j, bool want_s, bool want_d, bool init)
{
    if (P->p.prec == MHK_FP64) return level_sums<double, TAB_STRIDE>(P, st, j, want_s, want_d, init);
    return level_sums<float, TABF_STRIDE>(P, st, j, want_s, want_d, init);
}

}  // namespace mhk
