// Device-side binning of plan creation: cell keys, stable sorts and the
// lists built from them (level cells and per-wavefront candidate lists,
// spreading-tile lists, target tiles).
//
// Every list is built in two passes over the same loops -- count, exclusive
// scan of the counts, fill -- so that its order is fixed by the sorted
// orders alone (no atomics decide a position), and plan creation gives the
// same buffers on every run.
//
// Sorting is a stable least-significant-digit radix sort of 32-bit keys
// with 32-bit values, 8 bits per pass: per 2048-element block a digit
// histogram, one exclusive scan over (digit, block), then a scatter in
// which each element's rank among the equal digits before it in its block
// comes from ballots (wavefront) and per-wavefront digit counts in LDS.
// Stability makes the result the sort by (key, input position).
#include "mhk_internal.h"

namespace mhk {

constexpr int BT = 256;                // threads per block of the binning kernels
constexpr int RS_ITEMS = 8;            // elements per thread and pass of the radix sort
constexpr int RS_TILE = BT * RS_ITEMS; // elements per radix-sort block
constexpr int SC_ITEMS = 8;            // elements per thread of the scan
constexpr int SC_TILE = BT * SC_ITEMS;

static inline unsigned nblocks(int64_t n, int64_t per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

// ---------------------------------------------------------------------------
// Radix sort
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BT) k_rs_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                int32_t *__restrict__ counts, int nblk)
{
    __shared__ int h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int64_t i = base + r * BT + tid;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    counts[(int64_t)tid * nblk + blockIdx.x] = h[tid];
}

// offs: exclusive scan of counts in (digit, block) order, i.e. the first
// output position of each digit of each block.
__global__ void __launch_bounds__(BT) k_rs_scatter(const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                                   uint32_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                   int64_t n, int shift, const int32_t *__restrict__ offs, int nblk)
{
    __shared__ int run[256];          // next output position of each digit
    __shared__ int wc[BT / 64][256];  // per-wavefront digit counts of a round, then their prefix
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    run[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
#pragma unroll
        for (int w = 0; w < BT / 64; ++w) wc[w][tid] = 0;
        __syncthreads();
        const int64_t i = base + r * BT + tid;
        const bool valid = i < n;
        const uint32_t k = valid ? kin[i] : 0u;
        const int32_t v = valid ? vin[i] : 0;
        const int d = (int)((k >> shift) & 255u);
        // lanes of this wavefront holding the same digit
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const int rank = __popcll(m & below);
        if (valid && rank == 0) wc[wv][d] = __popcll(m);
        __syncthreads();
        {
            // thread tid = digit: positions of its elements per wavefront
            int acc = run[tid];
#pragma unroll
            for (int w = 0; w < BT / 64; ++w) {
                const int c = wc[w][tid];
                wc[w][tid] = acc;
                acc += c;
            }
            run[tid] = acc;
        }
        __syncthreads();
        if (valid) {
            const int pos = wc[wv][d] + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32 counts: out[i] = sum_{k<i} in[k], out[n] = total
// (int32; the int64 total is also stored in *total so that the caller can
// reject lists beyond 2^31 entries).
// ---------------------------------------------------------------------------
__device__ inline int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t &total)
{
    // sh: BT entries
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < BT; off <<= 1) {
        const int64_t t = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    total = sh[BT - 1];
    const int64_t incl = sh[tid];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(BT) k_scan_partial(const int32_t *__restrict__ in, int64_t n,
                                                     int64_t *__restrict__ bsum)
{
    __shared__ int64_t sh[BT];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < SC_ITEMS; ++r)
        if (base + r < n) s += in[base + r];
    int64_t tot;
    (void)block_excl_scan(s, sh, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// one workgroup: exclusive scan of the block sums in place, total at the end
__global__ void __launch_bounds__(BT) k_scan_top(int64_t *__restrict__ bsum, int64_t nb, int64_t *__restrict__ total)
{
    __shared__ int64_t sh[BT];
    const int64_t per = (nb + BT - 1) / BT;
    const int64_t b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += bsum[b];
    int64_t tot;
    int64_t acc = block_excl_scan(s, sh, tot);
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t v = bsum[b];
        bsum[b] = acc;
        acc += v;
    }
    if (threadIdx.x == 0) *total = tot;
}

__global__ void __launch_bounds__(BT) k_scan_apply(const int32_t *__restrict__ in, int64_t n,
                                                   const int64_t *__restrict__ bsum, int32_t *__restrict__ out)
{
    __shared__ int64_t sh[BT];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    int32_t v[SC_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < SC_ITEMS; ++r) {
        v[r] = base + r < n ? in[base + r] : 0;
        s += v[r];
    }
    int64_t tot;
    int64_t acc = block_excl_scan(s, sh, tot) + bsum[blockIdx.x];
#pragma unroll
    for (int r = 0; r < SC_ITEMS; ++r) {
        if (base + r < n) out[base + r] = (int32_t)acc;
        acc += v[r];
    }
    if (base + SC_ITEMS >= n && base < n) out[n] = (int32_t)acc;   // the block holding the last element
    if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}

// first index of each key in a sorted key array: start[c] for c in [0, nkeys],
// the lower bound of c by binary search (one thread per cell)
__global__ void __launch_bounds__(BT) k_cell_starts(const uint32_t *__restrict__ keys, int64_t n, int64_t nkeys,
                                                    int32_t *__restrict__ start)
{
    for (int64_t c = (int64_t)blockIdx.x * BT + threadIdx.x; c <= nkeys; c += (int64_t)gridDim.x * BT) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)keys[mid] < c)
                lo = mid + 1;
            else
                hi = mid;
        }
        start[c] = (int32_t)lo;
    }
}

__global__ void __launch_bounds__(BT) k_iota(int32_t *__restrict__ v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

hipError_t dev_sort_pairs(uint32_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t st)
{
    if (n <= 1 || bits <= 0) return hipSuccess;
    const int passes = (std::min(bits, 32) + 7) / 8;
    const int nblk = (int)nblocks(n, RS_TILE);
    uint32_t *k2 = nullptr;
    int32_t *v2 = nullptr, *cnt = nullptr, *off = nullptr;
    int64_t *bsum = nullptr, *tot = nullptr;
    const int64_t m = 256 * (int64_t)nblk;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(hipMallocAsync((void **)&k2, sizeof(uint32_t) * n, st));
    chk(hipMallocAsync((void **)&v2, sizeof(int32_t) * n, st));
    chk(hipMallocAsync((void **)&cnt, sizeof(int32_t) * m, st));
    chk(hipMallocAsync((void **)&off, sizeof(int32_t) * (m + 1), st));
    chk(hipMallocAsync((void **)&bsum, sizeof(int64_t) * nblocks(m, SC_TILE), st));
    chk(hipMallocAsync((void **)&tot, sizeof(int64_t), st));
    if (e == hipSuccess) {
        uint32_t *ka = keys, *kb = k2;
        int32_t *va = vals, *vb = v2;
        for (int p = 0; p < passes && e == hipSuccess; ++p) {
            hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(BT), 0, st, ka, n, 8 * p, cnt, nblk);
            const unsigned sb = nblocks(m, SC_TILE);
            hipLaunchKernelGGL(k_scan_partial, dim3(sb), dim3(BT), 0, st, cnt, m, bsum);
            hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BT), 0, st, bsum, (int64_t)sb, tot);
            hipLaunchKernelGGL(k_scan_apply, dim3(sb), dim3(BT), 0, st, cnt, m, bsum, off);
            hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(BT), 0, st, ka, va, kb, vb, n, 8 * p, off, nblk);
            chk(hipGetLastError());
            std::swap(ka, kb);
            std::swap(va, vb);
        }
        if (e == hipSuccess && ka != keys) {
            chk(hipMemcpyAsync(keys, ka, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
            chk(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
        }
    }
    for (void *p : {(void *)k2, (void *)v2, (void *)cnt, (void *)off, (void *)bsum, (void *)tot})
        if (p) (void)hipFreeAsync(p, st);
    return e;
}

hipError_t dev_scan(const int32_t *in, int32_t *out, int64_t n, int64_t *total, hipStream_t st)
{
    const unsigned sb = nblocks(n, SC_TILE);
    int64_t *bsum = nullptr;
    hipError_t e = hipMallocAsync((void **)&bsum, sizeof(int64_t) * sb, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_partial, dim3(sb), dim3(BT), 0, st, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BT), 0, st, bsum, (int64_t)sb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3(sb), dim3(BT), 0, st, in, n, bsum, out);
    e = hipGetLastError();
    (void)hipFreeAsync(bsum, st);
    return e;
}

hipError_t dev_cell_starts(const uint32_t *keys, int64_t n, int64_t nkeys, int32_t *start, hipStream_t st)
{
    const unsigned nbk = (unsigned)std::min<int64_t>(65536, nblocks(nkeys + 1, BT));
    hipLaunchKernelGGL(k_cell_starts, dim3(nbk), dim3(BT), 0, st, keys, n, nkeys, start);
    return hipGetLastError();
}

hipError_t dev_iota(int32_t *v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(nblocks(n, BT)), dim3(BT), 0, st, v, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Targets: Morton keys of cells of side hh (16 bits per axis) and the
// gathered sorted arrays
// ---------------------------------------------------------------------------
__device__ inline uint32_t spread16(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__global__ void __launch_bounds__(BT) k_target_keys(const double *__restrict__ x, const double *__restrict__ y,
                                                    int64_t n, double ox, double oy, double hh,
                                                    uint32_t *__restrict__ key, int32_t *__restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    const double fx = fmax(0.0, floor((x[i] - ox) / hh)), fy = fmax(0.0, floor((y[i] - oy) / hh));
    const uint32_t ix = (uint32_t)fmin(fx, 65535.0), iy = (uint32_t)fmin(fy, 65535.0);
    key[i] = spread16(ix) | (spread16(iy) << 1);
    val[i] = (int32_t)i;
}

__global__ void __launch_bounds__(BT) k_target_gather(const double *__restrict__ x, const double *__restrict__ y,
                                                      const int8_t *__restrict__ in, const int32_t *__restrict__ idx,
                                                      int64_t n, double *__restrict__ sx, double *__restrict__ sy,
                                                      int8_t *__restrict__ sin, int32_t *__restrict__ sidx)
{
    const int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (s >= n) return;
    const int32_t i = idx[s];
    sx[s] = x[i];
    sy[s] = y[i];
    sin[s] = in[i];
    sidx[s] = i;
}

hipError_t dev_sort_targets(const double *x, const double *y, const int8_t *in, int64_t n, double ox, double oy,
                            double hh, double *sx, double *sy, int8_t *sin, int32_t *sidx, hipStream_t st)
{
    uint32_t *key = nullptr;
    int32_t *val = nullptr;
    hipError_t e = hipMallocAsync((void **)&key, sizeof(uint32_t) * std::max<int64_t>(1, n), st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&val, sizeof(int32_t) * std::max<int64_t>(1, n), st);
    if (e == hipSuccess && n > 0) {
        hipLaunchKernelGGL(k_target_keys, dim3(nblocks(n, BT)), dim3(BT), 0, st, x, y, n, ox, oy, hh, key, val);
        e = hipGetLastError();
        if (e == hipSuccess) e = dev_sort_pairs(key, val, n, 32, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_target_gather, dim3(nblocks(n, BT)), dim3(BT), 0, st, x, y, in, val, n, sx, sy, sin,
                               sidx);
            e = hipGetLastError();
        }
    }
    if (key) (void)hipFreeAsync(key, st);
    if (val) (void)hipFreeAsync(val, st);
    return e;
}

// ---------------------------------------------------------------------------
// Dyadic levels: child nodes, their cells, per-wavefront candidate lists
// ---------------------------------------------------------------------------
// Child node q = (panel p, child c, node k): position, normal (renormalised)
// and speed from the parent's 16 nodal values through the interpolation row
// Tm[c][k][:]; weight w_GL,k speed / 2^j; cell key of side `cell`.
__global__ void __launch_bounds__(BT) k_child_nodes(int64_t n_src, int nch, const double *__restrict__ Tm,
                                                    const double *__restrict__ bx, const double *__restrict__ by,
                                                    const double *__restrict__ bnx, const double *__restrict__ bny,
                                                    const double *__restrict__ bw, const double *__restrict__ glw,
                                                    double ox, double oy, double cell, int64_t ncx, int64_t ncy,
                                                    double *__restrict__ cx, double *__restrict__ cy,
                                                    double *__restrict__ cw, double *__restrict__ cwx,
                                                    double *__restrict__ cwy, uint32_t *__restrict__ key,
                                                    int32_t *__restrict__ val)
{
    const int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (q >= n_src) return;
    const int k = (int)(q % NGL);
    const int64_t pc = q / NGL;
    const int c = (int)(pc % nch);
    const int64_t o = (pc / nch) * NGL;
    const double *row = Tm + ((int64_t)c * NGL + k) * NGL;
    double x = 0, y = 0, nx = 0, ny = 0, s = 0;
    for (int i = 0; i < NGL; ++i) {
        const double r = row[i];
        x += r * bx[o + i];
        y += r * by[o + i];
        nx += r * bnx[o + i];
        ny += r * bny[o + i];
        s += r * (bw[o + i] / glw[i]);
    }
    const double nn = sqrt(nx * nx + ny * ny);
    const double wq = glw[k] * s / nch;
    cx[q] = x;
    cy[q] = y;
    cw[q] = wq;
    cwx[q] = wq * nx / nn;
    cwy[q] = wq * ny / nn;
    const int64_t ix = min(ncx - 1, max((int64_t)0, (int64_t)floor((x - ox) / cell)));
    const int64_t iy = min(ncy - 1, max((int64_t)0, (int64_t)floor((y - oy) / cell)));
    key[q] = (uint32_t)(iy * ncx + ix);
    val[q] = (int32_t)q;
}

__global__ void __launch_bounds__(BT) k_child_gather(int64_t n, const int32_t *__restrict__ order,
                                                     const double *__restrict__ cx, const double *__restrict__ cy,
                                                     const double *__restrict__ cw, const double *__restrict__ cwx,
                                                     const double *__restrict__ cwy, double *__restrict__ sx,
                                                     double *__restrict__ sy, double *__restrict__ sw,
                                                     double *__restrict__ swx, double *__restrict__ swy,
                                                     int32_t *__restrict__ code)
{
    const int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (s >= n) return;
    const int32_t q = order[s];
    sx[s] = cx[q];
    sy[s] = cy[q];
    sw[s] = cw[q];
    swx[s] = cwx[q];
    swy[s] = cwy[q];
    code[s] = q;
}

// Per wavefront of 64 consecutive sorted targets: the sorted sources within
// R of the wavefront's target bounding box, from the cells (side R/4) that
// can hold a source within R of one of its targets (per cell row, a
// target's cells span its row gap g and half-width sqrt(R^2 - g^2)).  Row
// by row and cell by cell in increasing order, sources in sorted order.
// One wavefront of the launch per target wavefront; FILL = false counts,
// FILL = true writes at ofs[w].
template <bool FILL>
__global__ void __launch_bounds__(BT) k_wave_cands(const double *__restrict__ tx, const double *__restrict__ ty,
                                                   int64_t nout, int64_t nwave, double R, double R2, double ox,
                                                   double oy, double cell, int64_t ncx, int64_t ncy,
                                                   const int32_t *__restrict__ start, const double *__restrict__ sx,
                                                   const double *__restrict__ sy, int32_t *__restrict__ cnt,
                                                   const int32_t *__restrict__ ofs, int32_t *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * BT + threadIdx.x) >> 6;
    if (wave >= nwave) return;
    const int64_t t = wave * 64 + lane;
    const bool act = t < nout;
    const double x = act ? tx[t] : 0.0, y = act ? ty[t] : 0.0;
    auto col = [&](double v) { return min(ncx - 1, max((int64_t)0, (int64_t)floor((v - ox) / cell))); };
    auto row = [&](double v) { return min(ncy - 1, max((int64_t)0, (int64_t)floor((v - oy) / cell))); };
    double bx0 = act ? x : 1e300, bx1 = act ? x : -1e300, by0 = act ? y : 1e300, by1 = act ? y : -1e300;
    int64_t r0 = act ? row(y - R) : INT64_MAX, r1 = act ? row(y + R) : -1;
    const int64_t myr0 = r0, myr1 = r1;
    for (int off = 32; off > 0; off >>= 1) {
        bx0 = fmin(bx0, __shfl_xor(bx0, off));
        bx1 = fmax(bx1, __shfl_xor(bx1, off));
        by0 = fmin(by0, __shfl_xor(by0, off));
        by1 = fmax(by1, __shfl_xor(by1, off));
        r0 = min(r0, (int64_t)__shfl_xor(r0, off));
        r1 = max(r1, (int64_t)__shfl_xor(r1, off));
    }
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t n = 0;
    const int64_t base = FILL ? ofs[wave] : 0;
    for (int64_t r = r0; r <= r1; ++r) {
        // this lane's cells of row r
        bool valid = act && r >= myr0 && r <= myr1;
        int64_t c0 = INT64_MAX, c1 = -1;
        if (valid) {
            const double ylo = oy + r * cell, yhi = ylo + cell;
            const double g = fmax(0.0, fmax(ylo - y, y - yhi));
            if (g > R) {
                valid = false;
            } else {
                const double hw = sqrt(R * R - g * g);
                c0 = col(x - hw);
                c1 = col(x + hw);
            }
        }
        int64_t cmin = valid ? c0 : INT64_MAX, cmax = valid ? c1 : -1;
        for (int off = 32; off > 0; off >>= 1) {
            cmin = min(cmin, (int64_t)__shfl_xor(cmin, off));
            cmax = max(cmax, (int64_t)__shfl_xor(cmax, off));
        }
        for (int64_t c = cmin; c <= cmax; ++c) {
            if (__ballot(valid && c0 <= c && c <= c1) == 0) continue;
            const int32_t s0 = start[r * ncx + c], s1 = start[r * ncx + c + 1];
            for (int32_t sb = s0; sb < s1; sb += 64) {
                const int32_t s = sb + lane;
                bool keep = false;
                if (s < s1) {
                    const double px = sx[s], py = sy[s];
                    const double ex = fmax(0.0, fmax(bx0 - px, px - bx1));
                    const double ey = fmax(0.0, fmax(by0 - py, py - by1));
                    keep = ex * ex + ey * ey <= R2;
                }
                const uint64_t m = __ballot(keep);
                if (FILL && keep) out[base + n + __popcll(m & below)] = s;
                n += __popcll(m);
            }
        }
    }
    if (!FILL && lane == 0) cnt[wave] = (int32_t)min(n, (int64_t)INT32_MAX);
}

// key INT32_MAX - count: the stable ascending sort orders the wavefronts by
// decreasing work, ties in wavefront order
__global__ void __launch_bounds__(BT) k_wave_keys(const int32_t *__restrict__ ofs, int64_t nwave,
                                                  uint32_t *__restrict__ key, int32_t *__restrict__ val)
{
    const int64_t w = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (w >= nwave) return;
    key[w] = (uint32_t)(INT32_MAX - (ofs[w + 1] - ofs[w]));
    val[w] = (int32_t)w;
}

hipError_t dev_child_nodes(int64_t n_src, int nch, const double *Tm, const double *bx, const double *by,
                           const double *bnx, const double *bny, const double *bw, const double *glw, double ox,
                           double oy, double cell, int64_t ncx, int64_t ncy, double *sx, double *sy, double *sw,
                           double *swx, double *swy, int32_t *code, int32_t *cell_start, hipStream_t st)
{
    double *t[5] = {};
    uint32_t *key = nullptr;
    int32_t *val = nullptr;
    hipError_t e = hipSuccess;
    for (auto &p : t)
        if (e == hipSuccess) e = hipMallocAsync((void **)&p, sizeof(double) * std::max<int64_t>(1, n_src), st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&key, sizeof(uint32_t) * std::max<int64_t>(1, n_src), st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&val, sizeof(int32_t) * std::max<int64_t>(1, n_src), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_child_nodes, dim3(nblocks(n_src, BT)), dim3(BT), 0, st, n_src, nch, Tm, bx, by, bnx, bny,
                           bw, glw, ox, oy, cell, ncx, ncy, t[0], t[1], t[2], t[3], t[4], key, val);
        e = hipGetLastError();
    }
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < ncx * ncy) ++bits;
    if (e == hipSuccess) e = dev_sort_pairs(key, val, n_src, bits, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_child_gather, dim3(nblocks(n_src, BT)), dim3(BT), 0, st, n_src, val, t[0], t[1], t[2],
                           t[3], t[4], sx, sy, sw, swx, swy, code);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = dev_cell_starts(key, n_src, ncx * ncy, cell_start, st);
    for (auto p : t)
        if (p) (void)hipFreeAsync(p, st);
    if (key) (void)hipFreeAsync(key, st);
    if (val) (void)hipFreeAsync(val, st);
    return e;
}

hipError_t dev_wave_counts(const double *tx, const double *ty, int64_t nout, int64_t nwave, double R, double R2,
                           double ox, double oy, double cell, int64_t ncx, int64_t ncy, const int32_t *start,
                           const double *sx, const double *sy, int32_t *cnt, hipStream_t st)
{
    hipLaunchKernelGGL(k_wave_cands<false>, dim3(nblocks(nwave * 64, BT)), dim3(BT), 0, st, tx, ty, nout, nwave, R, R2,
                       ox, oy, cell, ncx, ncy, start, sx, sy, cnt, (const int32_t *)nullptr, (int32_t *)nullptr);
    return hipGetLastError();
}

hipError_t dev_wave_fill(const double *tx, const double *ty, int64_t nout, int64_t nwave, double R, double R2,
                         double ox, double oy, double cell, int64_t ncx, int64_t ncy, const int32_t *start,
                         const double *sx, const double *sy, const int32_t *ofs, int32_t *out, int32_t *order,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_wave_cands<true>, dim3(nblocks(nwave * 64, BT)), dim3(BT), 0, st, tx, ty, nout, nwave, R, R2,
                       ox, oy, cell, ncx, ncy, start, sx, sy, (int32_t *)nullptr, ofs, out);
    hipError_t e = hipGetLastError();
    uint32_t *key = nullptr;
    if (e == hipSuccess) e = hipMallocAsync((void **)&key, sizeof(uint32_t) * std::max<int64_t>(1, nwave), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_wave_keys, dim3(nblocks(nwave, BT)), dim3(BT), 0, st, ofs, nwave, key, order);
        e = hipGetLastError();
        if (e == hipSuccess) e = dev_sort_pairs(key, order, nwave, 31, st);
    }
    if (key) (void)hipFreeAsync(key, st);
    return e;
}

// ---------------------------------------------------------------------------
// History part: sources by spreading tile, per-tile lists, target tiles
// ---------------------------------------------------------------------------
// tile of a point, as the spreading kernels place it (32 x 32 grid points)
__device__ inline int64_t tile_index(double x, double y, double ox, double oy, double h, int64_t ntile)
{
    int64_t ix = (int64_t)floor((x - ox) / h) / TILE;
    int64_t iy = (int64_t)floor((y - oy) / h) / TILE;
    ix = min(ntile - 1, max((int64_t)0, ix));
    iy = min(ntile - 1, max((int64_t)0, iy));
    return iy * ntile + ix;
}

__global__ void __launch_bounds__(BT) k_tile_keys(const double *__restrict__ x, const double *__restrict__ y,
                                                  int64_t n, double ox, double oy, double h, int64_t ntile,
                                                  uint32_t *__restrict__ key, int32_t *__restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint32_t)tile_index(x[i], y[i], ox, oy, h, ntile);
    val[i] = (int32_t)i;
}

// sorted sources in grid coordinates, weights (with the normal for the
// double layer), original indices; bounds of the grid rows and columns
// their windows [m0, m0 + W) use (m0 = ceil(g - W/2)), by atomics into
// sup[0..3] = min x, max x (exclusive), min y, max y (exclusive)
__global__ void __launch_bounds__(BT) k_source_gather(int64_t n, const int32_t *__restrict__ order,
                                                      const double *__restrict__ x, const double *__restrict__ y,
                                                      const double *__restrict__ w, const double *__restrict__ nx,
                                                      const double *__restrict__ ny, double ox, double oy, double h,
                                                      int W, double *__restrict__ gx, double *__restrict__ gy,
                                                      double *__restrict__ gw, double *__restrict__ gwx,
                                                      double *__restrict__ gwy, int *__restrict__ sup)
{
    const int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x;
    int mx0 = INT32_MAX, mx1 = INT32_MIN, my0 = INT32_MAX, my1 = INT32_MIN;
    if (s < n) {
        const int32_t i = order[s];
        const double ax = (x[i] - ox) / h, ay = (y[i] - oy) / h;
        gx[s] = ax;
        gy[s] = ay;
        gw[s] = w[i];
        if (gwx) {
            gwx[s] = w[i] * nx[i];
            gwy[s] = w[i] * ny[i];
        }
        const int mx = (int)ceil(ax - 0.5 * W), my = (int)ceil(ay - 0.5 * W);
        mx0 = mx;
        mx1 = mx + W;
        my0 = my;
        my1 = my + W;
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx0 = min(mx0, __shfl_xor(mx0, off));
        mx1 = max(mx1, __shfl_xor(mx1, off));
        my0 = min(my0, __shfl_xor(my0, off));
        my1 = max(my1, __shfl_xor(my1, off));
    }
    if ((threadIdx.x & 63) == 0 && mx1 != INT32_MIN) {
        atomicMin(&sup[0], mx0);
        atomicMax(&sup[1], mx1);
        atomicMin(&sup[2], my0);
        atomicMax(&sup[3], my1);
    }
}

// Per tile (one wavefront each): the sorted sources whose window meets the
// tile in both axes.  A window (W <= 16 < 32 points) reaches at most the
// neighbouring tiles of its source's own tile, so the candidates are the
// sources of the 3 x 3 neighbourhood, taken in increasing tile index, i.e.
// in sorted order.
template <bool FILL>
__global__ void __launch_bounds__(BT) k_tile_lists(const double *__restrict__ gx, const double *__restrict__ gy,
                                                   const int32_t *__restrict__ tstart, int64_t ntile, int W,
                                                   int32_t *__restrict__ cnt, const int32_t *__restrict__ ofs,
                                                   int32_t *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t t = ((int64_t)blockIdx.x * BT + threadIdx.x) >> 6;
    if (t >= ntile * ntile) return;
    const int64_t tx = t % ntile, ty = t / ntile;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    auto span = [&](double g, int64_t &t0, int64_t &t1) {
        const int64_t m0 = (int64_t)ceil(g - 0.5 * W);
        t0 = max((int64_t)0, (int64_t)floor((double)m0 / TILE));
        t1 = min(ntile - 1, (int64_t)floor((double)(m0 + W - 1) / TILE));
    };
    int64_t n = 0;
    const int64_t base = FILL ? ofs[t] : 0;
    for (int64_t ny = max((int64_t)0, ty - 1); ny <= min(ntile - 1, ty + 1); ++ny)
        for (int64_t nx = max((int64_t)0, tx - 1); nx <= min(ntile - 1, tx + 1); ++nx) {
            const int32_t s0 = tstart[ny * ntile + nx], s1 = tstart[ny * ntile + nx + 1];
            for (int32_t sb = s0; sb < s1; sb += 64) {
                const int32_t s = sb + lane;
                bool keep = false;
                if (s < s1) {
                    int64_t x0, x1, y0, y1;
                    span(gx[s], x0, x1);
                    span(gy[s], y0, y1);
                    keep = x0 <= tx && tx <= x1 && y0 <= ty && ty <= y1;
                }
                const uint64_t m = __ballot(keep);
                if (FILL && keep) out[base + n + __popcll(m & below)] = s;
                n += __popcll(m);
            }
        }
    if (!FILL && lane == 0) cnt[t] = (int32_t)n;
}

// Sort the sources (x, y, w and, for the boundary, nx, ny) by tile and
// count their tile lists: gx.. and idx get the sorted arrays, lofs the
// list offsets (exclusive scan; lofs[nt2] = total, also in *total), tstart
// the tile starts of the sorted sources (temporary, freed by the caller)
hipError_t dev_sources_by_tile(const double *x, const double *y, const double *w, const double *nx, const double *ny,
                               int64_t n, double ox, double oy, double h, int64_t ntile, int W, double *gx, double *gy,
                               double *gw, double *gwx, double *gwy, int32_t *idx, int *sup, int32_t *lofs,
                               int32_t **tstart_out, int64_t *total, hipStream_t st)
{
    const int64_t nt2 = ntile * ntile;
    uint32_t *key = nullptr;
    int32_t *cnt = nullptr, *tstart = nullptr;
    hipError_t e = hipMallocAsync((void **)&key, sizeof(uint32_t) * std::max<int64_t>(1, n), st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&cnt, sizeof(int32_t) * nt2, st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&tstart, sizeof(int32_t) * (nt2 + 1), st);
    if (e == hipSuccess && n > 0) {
        hipLaunchKernelGGL(k_tile_keys, dim3(nblocks(n, BT)), dim3(BT), 0, st, x, y, n, ox, oy, h, ntile, key, idx);
        e = hipGetLastError();
        int bits = 1;
        while (bits < 32 && ((int64_t)1 << bits) < nt2) ++bits;
        if (e == hipSuccess) e = dev_sort_pairs(key, idx, n, bits, st);
        if (e == hipSuccess) {
            // idx holds the sorted order (the original index of each sorted source)
            hipLaunchKernelGGL(k_source_gather, dim3(nblocks(n, BT)), dim3(BT), 0, st, n, idx, x, y, w, nx, ny, ox,
                               oy, h, W, gx, gy, gw, gwx, gwy, sup);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = dev_cell_starts(key, n, nt2, tstart, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_tile_lists<false>, dim3(nblocks(nt2 * 64, BT)), dim3(BT), 0, st, gx, gy, tstart, ntile,
                           W, cnt, (const int32_t *)nullptr, (int32_t *)nullptr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = dev_scan(cnt, lofs, nt2, total, st);
    if (key) (void)hipFreeAsync(key, st);
    if (cnt) (void)hipFreeAsync(cnt, st);
    if (e == hipSuccess) {
        *tstart_out = tstart;
    } else if (tstart) {
        (void)hipFreeAsync(tstart, st);
    }
    return e;
}

hipError_t dev_tile_fill(const double *gx, const double *gy, const int32_t *tstart, int64_t ntile, int W,
                         const int32_t *lofs, int32_t *list, hipStream_t st)
{
    const int64_t nt2 = ntile * ntile;
    hipLaunchKernelGGL(k_tile_lists<true>, dim3(nblocks(nt2 * 64, BT)), dim3(BT), 0, st, gx, gy, tstart, ntile, W,
                       (int32_t *)nullptr, lofs, list);
    return hipGetLastError();
}

// Targets (sorted, tiles contiguous): flag the first target of each tile
// run; bounds of the grid rows and columns of their interpolation windows
// into win[0..3] as for the sources
__global__ void __launch_bounds__(BT) k_target_tile_flags(const double *__restrict__ tx, const double *__restrict__ ty,
                                                          int64_t n, double ox, double oy, double h, int64_t ntile,
                                                          int W, int32_t *__restrict__ flag, int *__restrict__ win)
{
    const int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x;
    int mx0 = INT32_MAX, mx1 = INT32_MIN, my0 = INT32_MAX, my1 = INT32_MIN;
    if (s < n) {
        // tile index without clamping, as the run boundaries are formed
        const int64_t t = ((int64_t)floor((ty[s] - oy) / h) / TILE) * ntile + (int64_t)floor((tx[s] - ox) / h) / TILE;
        int64_t tp = -1;
        if (s > 0) tp = ((int64_t)floor((ty[s - 1] - oy) / h) / TILE) * ntile + (int64_t)floor((tx[s - 1] - ox) / h) / TILE;
        flag[s] = (s == 0 || t != tp) ? 1 : 0;
        const double gx = (tx[s] - ox) / h, gy = (ty[s] - oy) / h;
        const int mx = (int)ceil(gx - 0.5 * W), my = (int)ceil(gy - 0.5 * W);
        mx0 = mx;
        mx1 = mx + W;
        my0 = my;
        my1 = my + W;
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx0 = min(mx0, __shfl_xor(mx0, off));
        mx1 = max(mx1, __shfl_xor(mx1, off));
        my0 = min(my0, __shfl_xor(my0, off));
        my1 = max(my1, __shfl_xor(my1, off));
    }
    if ((threadIdx.x & 63) == 0 && mx1 != INT32_MIN) {
        atomicMin(&win[0], mx0);
        atomicMax(&win[1], mx1);
        atomicMin(&win[2], my0);
        atomicMax(&win[3], my1);
    }
}

__global__ void __launch_bounds__(BT) k_target_tile_runs(const double *__restrict__ tx, const double *__restrict__ ty,
                                                         int64_t n, double ox, double oy, double h, int64_t ntile,
                                                         const int32_t *__restrict__ flag,
                                                         const int32_t *__restrict__ pos, int32_t *__restrict__ xy,
                                                         int32_t *__restrict__ rng)
{
    const int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (s >= n) return;
    if (flag[s]) {
        const int64_t t = ((int64_t)floor((ty[s] - oy) / h) / TILE) * ntile + (int64_t)floor((tx[s] - ox) / h) / TILE;
        xy[pos[s]] = (int32_t)t;
        rng[pos[s]] = (int32_t)s;
    }
    if (s == n - 1) rng[pos[n]] = (int32_t)n;
}

// flags and scan of the target tile runs: *runs_dev receives the number of
// runs; pos (n + 1 entries) is allocated here and freed by the caller
hipError_t dev_target_tiles_count(const double *tx, const double *ty, int64_t n, double ox, double oy, double h,
                                  int64_t ntile, int W, int *win, int32_t **flag_out, int32_t **pos_out,
                                  int64_t *runs_dev, hipStream_t st)
{
    int32_t *flag = nullptr, *pos = nullptr;
    hipError_t e = hipMallocAsync((void **)&flag, sizeof(int32_t) * std::max<int64_t>(1, n), st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&pos, sizeof(int32_t) * (n + 1), st);
    if (e == hipSuccess && n > 0) {
        hipLaunchKernelGGL(k_target_tile_flags, dim3(nblocks(n, BT)), dim3(BT), 0, st, tx, ty, n, ox, oy, h, ntile, W,
                           flag, win);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = dev_scan(flag, pos, n, runs_dev, st);
    if (e != hipSuccess) {
        if (flag) (void)hipFreeAsync(flag, st);
        if (pos) (void)hipFreeAsync(pos, st);
        return e;
    }
    *flag_out = flag;
    *pos_out = pos;
    return hipSuccess;
}

hipError_t dev_target_tiles_fill(const double *tx, const double *ty, int64_t n, double ox, double oy, double h,
                                 int64_t ntile, const int32_t *flag, const int32_t *pos, int32_t *xy, int32_t *rng,
                                 hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_target_tile_runs, dim3(nblocks(n, BT)), dim3(BT), 0, st, tx, ty, n, ox, oy, h, ntile, flag,
                       pos, xy, rng);
    return hipGetLastError();
}

}  // namespace mhk
