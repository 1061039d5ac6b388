// History part (Section 5): type-1 NUFFT of the quadrature sources, the
// multiplier of eq. (sh_fourier), type-2 NUFFT at the targets.
//
//   spread    g_m = sum_j q_j phi(x_m - x_j) on a periodic fine grid of step h
//             (q = w sigma, w' f, w nu_x mu, w nu_y mu: eqs. (disrete_sigma_hat),
//             (rhs_vol) and the D transform of Section 5.1);
//   FFT       rocFFT real-to-complex, in place;
//   multiply  c_l = (h^4/P^2) m(k_l) G_l / phihat(k_l)^2 for S and V, and
//             (h^4/P^2) m(k_l) (-i k_l . G_l) / phihat(k_l)^2 for D, where
//             m(k) = exp(-delta(alpha^2 + |k|^2))/(alpha^2 + |k|^2) (eq. (sh))
//             and c_l = 0 outside the square |k_x|, |k_y| <= k_max;
//   FFT       rocFFT complex-to-real, in place;
//   interp    u(x) = sum_m phi(x - x_m) U_m.
//
// Spreading: one workgroup owns one 32x32 tile of the fine grid and one
// density of the batch; it adds the windows of the sources that meet the
// tile (listed per tile at plan time) into LDS with LDS atomics and writes
// the tile once: every grid value is written exactly once, with no global
// atomics.
// Interpolation: one workgroup per non-empty target tile stages the tile plus
// its window halo of the three result grids in LDS with coalesced row reads.
#include "mhk_internal.h"

namespace mhk {

// threads per interpolation / spreading workgroup: a busy tile holds a few
// hundred targets, one per thread; the tiles that hold volume sources hold
// a couple of thousand (source, tile) pairs and are a small part of the
// grid, so their workgroups take 512 threads (measured 4.42 against 4.57 ms
// per bench step with 256; 1024 was slower)
constexpr int HB = 256;
constexpr int SB = 512;

template <typename T>
struct SpreadArgs {
    int64_t n, field, nb, nv;
    int ntile, B;
    int tbx0, tby0, ntbx;  // the launch covers tiles tbx0.. (ntbx per row) x tby0..: the box of the sources' windows
    double beta;
    const double *bgx, *bgy, *bw, *bwx, *bwy;
    const int32_t *bidx, *blofs, *blist;
    const double *vgx, *vgy, *vw;
    const int32_t *vidx, *vlofs, *vlist;
    const T *sigma, *mu, *f_vol;
    const T *wcoef;
    T *grid;               // [4][B][field]: S, V, Dx, Dy sources
};

// Window values phi(z_k), z_k = (m0 + k - g) 2/W, at the W grid points from
// m0 = ceil(g - W/2), from the per-point polynomials in t = 2(m0 - g + W/2) - 1
// (degree W + 3; the offset is formed in FP64).
// Window values at the W grid points of both axes of one source.  The
// window is even, so point W-1-k at offset t is point k at -t: with the
// polynomial of point k split into even and odd parts, p_k(t) = E(t^2) +
// t O(t^2), the pair is E +- t O, and half the polynomials serve all W
// points.  The coefficients are loaded with scalar loads inside the
// caller's loop (the empty asm keeps the compiler from hoisting all of them
// into vector registers), and each is used for both axes.
template <int W, typename T>
__device__ inline void window_weights2(double gx, double gy, const T *__restrict__ cf, int &mx0, int &my0, T *wx,
                                       T *wy)
{
    constexpr int D = W + 3;           // degree
    constexpr int NE = D / 2 + 1;      // even coefficients c_0, c_2, ...
    constexpr int NO = (D + 1) / 2;    // odd coefficients c_1, c_3, ...
    typedef const __attribute__((address_space(4))) T *ConstPtr;   // scalar-loadable
    ConstPtr cc = (ConstPtr)cf;
    asm volatile("" : "+s"(cc));
    mx0 = (int)ceil(gx - 0.5 * W);
    my0 = (int)ceil(gy - 0.5 * W);
    const T tx = (T)(2.0 * ((double)mx0 - gx + 0.5 * W) - 1.0);
    const T ty = (T)(2.0 * ((double)my0 - gy + 0.5 * W) - 1.0);
    const T sx = tx * tx, sy = ty * ty;
#pragma unroll
    for (int k = 0; k < (W + 1) / 2; ++k) {
        // the next point's coefficients are loaded only after this point's
        // inputs exist, which keeps 16 (not 8 W) coefficients live in SGPRs
        if (k > 0) asm volatile("" : "+s"(cc) : "v"(wx[k - 1]), "v"(wy[k - 1]));
        ConstPtr c = cc + k * (D + 1);
        T ex = c[2 * (NE - 1)], ey = ex;
#pragma unroll
        for (int j = NE - 2; j >= 0; --j) {
            ex = fma(ex, sx, c[2 * j]);
            ey = fma(ey, sy, c[2 * j]);
        }
        T ox = c[2 * (NO - 1) + 1], oy = ox;
#pragma unroll
        for (int j = NO - 2; j >= 0; --j) {
            ox = fma(ox, sx, c[2 * j + 1]);
            oy = fma(oy, sy, c[2 * j + 1]);
        }
        wx[k] = fma(tx, ox, ex);
        wy[k] = fma(ty, oy, ey);
        if (W - 1 - k != k) {
            wx[W - 1 - k] = fma(-tx, ox, ex);
            wy[W - 1 - k] = fma(-ty, oy, ey);
        }
    }
}

// One workgroup per (tile, density), four passes over one LDS buffer: V from
// the volume sources, then S, D_x, D_y from the boundary sources.  Each pass
// takes the plan's list of the sources whose window meets the tile (one
// source per thread, every lane busy) and adds the part of its w x w window
// inside the tile (row and column tests; the column tests are formed once
// per source).  The buffer has a margin of w - 1 points around the tile, so
// that every address is the source's window corner plus an immediate
// offset; the tile's interior is then written once, so every grid value is
// written exactly once, with no global atomics.  (Adding whole windows into
// the margin instead of testing costs more: at w = 12 a listed source lies
// ~45% outside the tile.)  The accumulators are FP64 at both precisions: LDS atomic adds of
// FP64 run at more than twice the rate of FP32 ones, and the sums lose
// nothing before the single rounding on the way out.
template <int W, typename T>
__global__ void __launch_bounds__(SB) k_spread(SpreadArgs<T> A)
{
    constexpr int PAD = W - 1, PT = TILE + 2 * PAD;
    __shared__ double acc[PT * PT];
    const int tile = (A.tby0 + (int)blockIdx.x / A.ntbx) * A.ntile + A.tbx0 + (int)blockIdx.x % A.ntbx;
    const int b = blockIdx.y, tid = threadIdx.x;
    const int x0 = (tile % A.ntile) * TILE, y0 = (tile / A.ntile) * TILE;
    const size_t fs = (size_t)A.B * A.field;
    T *gS = A.grid + (size_t)b * A.field, *gV = gS + fs, *gX = gV + fs, *gY = gX + fs;
    for (int ph = 0; ph < 4; ++ph) {
        T *out = ph == 0 ? gV : ph == 1 ? gS : ph == 2 ? gX : gY;
        const bool vol = ph == 0;
        const bool want = vol ? A.f_vol != nullptr : ph == 1 ? A.sigma != nullptr : A.mu != nullptr;
        const int32_t *lofs = vol ? A.vlofs : A.blofs, *list = vol ? A.vlist : A.blist;
        const int e0 = want ? lofs[tile] : 0, e1 = want ? lofs[tile + 1] : 0;
        if (e0 == e1) {
            for (int i = tid; i < TILE * TILE; i += SB)
                out[(size_t)(y0 + i / TILE) * (A.n + 2) + x0 + (i % TILE)] = (T)0;
            continue;
        }
        for (int i = tid; i < PT * PT; i += SB) acc[i] = 0.0;
        __syncthreads();
        for (int e = e0 + tid; e < e1; e += SB) {
            const int s = list[e];
            const double gx = vol ? A.vgx[s] : A.bgx[s], gy = vol ? A.vgy[s] : A.bgy[s];
            int mx0, my0;
            T wx[W], wy[W];
            window_weights2<W, T>(gx, gy, A.wcoef, mx0, my0, wx, wy);
            mx0 -= x0;
            my0 -= y0;
            // listed sources meet the tile; the test keeps every write inside
            // the buffer whatever the list holds
            if (mx0 <= -W || mx0 >= TILE || my0 <= -W || my0 >= TILE) continue;
            T q;
            if (vol) {
                q = (T)(A.vw[s] * (double)A.f_vol[(size_t)b * A.nv + A.vidx[s]]);
            } else {
                const int i = A.bidx[s];
                q = ph == 1 ? (T)(A.bw[s] * (double)A.sigma[(size_t)b * A.nb + i])
                            : (T)((ph == 2 ? A.bwx[s] : A.bwy[s]) * (double)A.mu[(size_t)b * A.nb + i]);
            }
            double *base = acc + (my0 + PAD) * PT + (mx0 + PAD);
            bool col[W];
#pragma unroll
            for (int kx = 0; kx < W; ++kx) col[kx] = (unsigned)(mx0 + kx) < (unsigned)TILE;
#pragma unroll
            for (int ky = 0; ky < W; ++ky) {
                if ((unsigned)(my0 + ky) >= (unsigned)TILE) continue;
                const T qy = q * wy[ky];
#pragma unroll
                for (int kx = 0; kx < W; ++kx)
                    if (col[kx]) atomicAdd(base + ky * PT + kx, (double)(qy * wx[kx]));
            }
        }
        __syncthreads();
        for (int i = tid; i < TILE * TILE; i += SB)
            out[(size_t)(y0 + i / TILE) * (A.n + 2) + x0 + (i % TILE)] =
                (T)acc[(i / TILE + PAD) * PT + PAD + (i % TILE)];
        __syncthreads();
    }
}

// Fourier multiplier on the half spectrum [n][n/2+1] of each field; the
// multiplier is formed in FP64 in both precision paths (it peaks at 1/alpha^2
// near k = 0).
template <typename T>
__global__ void __launch_bounds__(256) k_multiply(int64_t n, int B, int64_t field, T *grid,
                                                  const double *__restrict__ fac, double c, double alpha2,
                                                  double dk, const double *__restrict__ mtab, int lmax)
{
    const int64_t nh = n / 2 + 1;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n * nh * B) return;
    const int64_t lx = id % nh;
    const int64_t ly = (id / nh) % n;
    const int b = (int)(id / (nh * n));
    const int64_t fy = ly <= n / 2 ? ly : ly - n;
    const double ax = fac[lx], ay = fac[fy < 0 ? -fy : fy];
    const size_t fs = (size_t)B * field / 2;                  // complex values per field group
    typedef typename Vec2<T>::type T2;
    T2 *F = reinterpret_cast<T2 *>(grid) + (size_t)b * (field / 2) + ly * nh + lx;
    T2 zS = {0, 0}, zV = {0, 0}, zD = {0, 0};
    double M = 0.0;
    if (mtab) {
        if (lx <= lmax && fy >= -lmax && fy <= lmax) M = mtab[(fy + lmax) * (lmax + 1) + lx];
    } else if (ax != 0.0 && ay != 0.0) {
        const double kx = dk * lx, ky = dk * fy;
        M = c * ax * ay / (alpha2 + kx * kx + ky * ky);
    }
    if (M != 0.0) {
        const double kx = dk * lx, ky = dk * fy;
        const T2 s = F[0], v = F[fs], gx = F[2 * fs], gy = F[3 * fs];
        zS.x = (T)(M * s.x); zS.y = (T)(M * s.y);
        zV.x = (T)(M * v.x); zV.y = (T)(M * v.y);
        // -i (kx Gx + ky Gy)
        const double re = kx * gx.x + ky * gy.x, im = kx * gx.y + ky * gy.y;
        zD.x = (T)(M * im); zD.y = (T)(-M * re);
    }
    F[0] = zS;
    F[fs] = zV;
    F[2 * fs] = zD;
}

// ---------------------------------------------------------------------------
// Column transforms fused with the multiplier.  After the row transforms
// (real-to-complex along x, below), every column l_x of the half spectrum is
// an independent length-n sequence along y; the multiplier is applied between
// the forward and the inverse column transforms, so one workgroup takes a
// column from HBM into LDS, transforms it, multiplies, transforms back and
// writes it: the 2D transforms' two column passes, their transposes and the
// multiplier pass become one read and one write of each column.  Columns
// with l_x beyond the multiplier's support are neither written by the
// forward row transforms nor touched here; the inverse row transforms take
// them as zero.
//
// Transforms: self-sorting (Stockham) passes of radix 8, 9, 6, 4, 2, 3 or 5 on the
// LDS copy; each pass reads every butterfly's inputs into registers, waits,
// and writes the outputs in place.  Twiddles e^{-2 pi i m/n} come from a
// table (conjugated for the inverse); both directions are unnormalised, like
// the rocFFT row transforms.
// ---------------------------------------------------------------------------
constexpr int CT = 512;            // threads per column workgroup

template <typename T2>
__device__ inline T2 c2(decltype(T2::x) x, decltype(T2::x) y)
{
    T2 r;
    r.x = x;
    r.y = y;
    return r;
}
template <typename T2> __device__ inline T2 cadd(T2 a, T2 b) { return c2<T2>(a.x + b.x, a.y + b.y); }
template <typename T2> __device__ inline T2 csub(T2 a, T2 b) { return c2<T2>(a.x - b.x, a.y - b.y); }
template <typename T2> __device__ inline T2 cmul(T2 a, T2 b)
{
    return c2<T2>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T2> __device__ inline T2 cscale(T2 a, decltype(T2::x) s) { return c2<T2>(a.x * s, a.y * s); }
// -i z (forward) or +i z (inverse)
template <bool INV, typename T2> __device__ inline T2 rot(T2 z)
{
    return INV ? c2<T2>(-z.y, z.x) : c2<T2>(z.y, -z.x);
}

// DFT of R points, y_k = sum_t x_t e^{-+2 pi i t k / R}
template <int R, bool INV, typename T2> __device__ inline void dft(T2 *x)
{
    typedef decltype(T2::x) T;
    if constexpr (R == 2) {
        const T2 a = x[0];
        x[0] = cadd(a, x[1]);
        x[1] = csub(a, x[1]);
    } else if constexpr (R == 3) {
        const T c = (T)-0.5, s = (T)0.86602540378443864676;
        const T2 a = cadd(x[1], x[2]), d = csub(x[1], x[2]);
        const T2 r = cadd(x[0], cscale(a, c)), i = rot<INV>(cscale(d, s));
        x[0] = cadd(x[0], a);
        x[1] = cadd(r, i);
        x[2] = csub(r, i);
    } else if constexpr (R == 4) {
        const T2 t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]), t2 = cadd(x[1], x[3]), t3 = rot<INV>(csub(x[1], x[3]));
        x[0] = cadd(t0, t2);
        x[2] = csub(t0, t2);
        x[1] = cadd(t1, t3);
        x[3] = csub(t1, t3);
    } else if constexpr (R == 6) {
        // two DFTs of 3 on the even and odd points, combined with w6^k
        T2 e[3] = {x[0], x[2], x[4]}, o[3] = {x[1], x[3], x[5]};
        dft<3, INV>(e);
        dft<3, INV>(o);
        const T h = (T)0.86602540378443864676;
        // w6 = e^{-+ i pi/3} = 1/2 -+ i sqrt(3)/2, w6^2 = -1/2 -+ i sqrt(3)/2
        const T sg = INV ? (T)1 : (T)-1;
        const T2 o1 = c2<T2>((T)0.5 * o[1].x - sg * h * o[1].y, (T)0.5 * o[1].y + sg * h * o[1].x);
        const T2 o2 = c2<T2>((T)-0.5 * o[2].x - sg * h * o[2].y, (T)-0.5 * o[2].y + sg * h * o[2].x);
        x[0] = cadd(e[0], o[0]);
        x[3] = csub(e[0], o[0]);
        x[1] = cadd(e[1], o1);
        x[4] = csub(e[1], o1);
        x[2] = cadd(e[2], o2);
        x[5] = csub(e[2], o2);
    } else if constexpr (R == 9) {
        // three DFTs of 3 on the points t = 3u + r, twiddles w9^(r k), then
        // DFTs of 3 across r
        T2 a[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            a[r][0] = x[r];
            a[r][1] = x[r + 3];
            a[r][2] = x[r + 6];
            dft<3, INV>(a[r]);
        }
        const T c1 = (T)0.76604444311897803520, s1 = (T)0.64278760968653932632;   // 2 pi / 9
        const T c2v = (T)0.17364817766693034885, s2 = (T)0.98480775301220805936;  // 4 pi / 9
        const T c4 = (T)-0.93969262078590838405, s4 = (T)0.34202014332566873304;  // 8 pi / 9
        const T sg = INV ? (T)1 : (T)-1;
        auto tw9 = [&](T2 z, T c, T sn) { return c2<T2>(c * z.x - sg * sn * z.y, c * z.y + sg * sn * z.x); };
        a[1][1] = tw9(a[1][1], c1, s1);     // w9^1
        a[1][2] = tw9(a[1][2], c2v, s2);    // w9^2
        a[2][1] = tw9(a[2][1], c2v, s2);    // w9^2
        a[2][2] = tw9(a[2][2], c4, s4);     // w9^4
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            T2 b[3] = {a[0][k], a[1][k], a[2][k]};
            dft<3, INV>(b);
            x[k] = b[0];
            x[k + 3] = b[1];
            x[k + 6] = b[2];
        }
    } else if constexpr (R == 8) {
        // two DFTs of 4 on the even and odd points, combined with w8^k
        T2 e[4] = {x[0], x[2], x[4], x[6]}, o[4] = {x[1], x[3], x[5], x[7]};
        dft<4, INV>(e);
        dft<4, INV>(o);
        const T h = (T)0.70710678118654752440;
        // w8^k o_k, w8 = e^{-+ i pi/4}
        const T2 o1 = INV ? c2<T2>(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                          : c2<T2>(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
        const T2 o2 = rot<INV>(o[2]);
        const T2 o3 = INV ? c2<T2>(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                          : c2<T2>(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
        x[0] = cadd(e[0], o[0]);
        x[4] = csub(e[0], o[0]);
        x[1] = cadd(e[1], o1);
        x[5] = csub(e[1], o1);
        x[2] = cadd(e[2], o2);
        x[6] = csub(e[2], o2);
        x[3] = cadd(e[3], o3);
        x[7] = csub(e[3], o3);
    } else {
        static_assert(R == 5, "radix");
        const T c1 = (T)0.30901699437494742410, c2v = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        const T2 a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]), a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
        const T2 r1 = cadd(x[0], cadd(cscale(a1, c1), cscale(a2, c2v)));
        const T2 r2 = cadd(x[0], cadd(cscale(a1, c2v), cscale(a2, c1)));
        const T2 i1 = rot<INV>(cadd(cscale(b1, s1), cscale(b2, s2)));
        const T2 i2 = rot<INV>(csub(cscale(b1, s2), cscale(b2, s1)));
        x[0] = cadd(x[0], cadd(a1, a2));
        x[1] = cadd(r1, i1);
        x[4] = csub(r1, i1);
        x[2] = cadd(r2, i2);
        x[3] = csub(r2, i2);
    }
}

// One radix-R pass of a length-N transform held in LDS by NT threads (N <=
// NMAX); Ns = product of the radices of the passes before it.  The twiddle
// table holds e^{-2 pi i m / (N ts)}, read at stride ts.
template <int R, bool INV, int NT, int NMAX, typename T2>
__device__ inline void fft_pass(T2 *buf, const double2 *__restrict__ tw, int ts, int N, int Ns)
{
    typedef decltype(T2::x) T;
    constexpr int MB = (NMAX / R + NT - 1) / NT;
    const int nb = N / R, step = N / (Ns * R) * ts;
    T2 v[MB][R];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int j = threadIdx.x + i * NT;
        if (j < nb) {
            // one twiddle load per butterfly (issued before the LDS reads),
            // w^t by repeated products in FP64 (R - 2 roundings of 1e-16),
            // each rounded once to the transform's precision
            double2 w = make_double2(1.0, 0.0);
            if (Ns > 1) {
                w = tw[(j % Ns) * step];
                if (INV) w.y = -w.y;
            }
#pragma unroll
            for (int t = 0; t < R; ++t) v[i][t] = buf[j + t * nb];
            if (Ns > 1) {
                double2 wt = w;
#pragma unroll
                for (int t = 1; t < R; ++t) {
                    v[i][t] = cmul(v[i][t], c2<T2>((T)wt.x, (T)wt.y));
                    if (t + 1 < R) wt = cmul(wt, w);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int j = threadIdx.x + i * NT;
        if (j < nb) {
            dft<R, INV>(v[i]);
            const int k = j % Ns, o = (j - k) * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) buf[o + t * Ns] = v[i][t];
        }
    }
    __syncthreads();
}

template <bool INV, int NT, int NMAX, typename T2>
__device__ inline void lds_fft(T2 *buf, const double2 *tw, int ts, int N, const int8_t *radix, int npass)
{
    int Ns = 1;
    for (int p = 0; p < npass; ++p) {
        const int r = radix[p];
        if (r == 8) fft_pass<8, INV, NT, NMAX>(buf, tw, ts, N, Ns);
        else if (r == 9) fft_pass<9, INV, NT, NMAX>(buf, tw, ts, N, Ns);
        else if (r == 6) fft_pass<6, INV, NT, NMAX>(buf, tw, ts, N, Ns);
        else if (r == 4) fft_pass<4, INV, NT, NMAX>(buf, tw, ts, N, Ns);
        else if (r == 2) fft_pass<2, INV, NT, NMAX>(buf, tw, ts, N, Ns);
        else if (r == 3) fft_pass<3, INV, NT, NMAX>(buf, tw, ts, N, Ns);
        else fft_pass<5, INV, NT, NMAX>(buf, tw, ts, N, Ns);
        Ns *= r;
    }
}

// ---------------------------------------------------------------------------
// Row transforms (x direction), real to complex and back, one row per
// workgroup, in place on the padded rows: the n reals of a row are n/2
// complex points z_m = x_2m + i x_2m+1, transformed in LDS (length n/2,
// twiddles of the length-n table at stride 2) and untangled:
//   X_k = (Z_k + conj Z_{n/2-k})/2 - i e^{-2 pi i k/n} (Z_k - conj Z_{n/2-k})/2,
// k = 0..n/2; the inverse forms Z_k = (X_k + conj X_{n/2-k}) + i e^{2 pi i k/n}
// (X_k - conj X_{n/2-k}) and transforms back (unnormalised, as the column
// transforms).
// ---------------------------------------------------------------------------
constexpr int RT = 256;            // threads per row workgroup

template <typename T>
struct RowArgs {
    int64_t n;
    int r0, nrow;                  // rows r0 .. r0 + nrow - 1 of every field of the launch
    int m0, m1;                    // forward: complex points [m0, m1) of a row are read, the others are zero;
                                   // inverse: complex points [m0, m1) are written back
    int ncol;                      // half-spectrum entries k < ncol can be nonzero after the multiplier
    int npass;
    int8_t radix[COL_MAXPASS];     // of n/2
    T *grid;                       // rows of n + 2 reals, consecutive
    const double2 *tw;             // e^{-2 pi i m / n}, FP64 at both precisions
};

template <bool INV, typename T, int NMAX>
__global__ void __launch_bounds__(RT) k_rows(RowArgs<T> A)
{
    typedef typename Vec2<T>::type T2;
    extern __shared__ double lds_row[];
    T2 *buf = reinterpret_cast<T2 *>(lds_row);
    const int n = (int)A.n, h = n / 2;
    const size_t slot = blockIdx.x / A.nrow, row = A.r0 + blockIdx.x % A.nrow;
    T2 *c = reinterpret_cast<T2 *>(A.grid + (slot * (size_t)n + row) * (size_t)(n + 2));   // h + 1 complex
    const int tid = threadIdx.x;
    if (!INV) {
        // the row is zero outside the sources' windows
        const T2 zero = c2<T2>((T)0, (T)0);
        for (int m = tid; m < h; m += RT) buf[m] = m >= A.m0 && m < A.m1 ? c[m] : zero;
        __syncthreads();
        lds_fft<false, RT, NMAX / 2>(buf, A.tw, 2, h, A.radix, A.npass);
        // only the columns that the multiplier keeps are read again
        for (int k = tid; k < A.ncol; k += RT) {
            const T2 zk = buf[k == h ? 0 : k], zc = buf[k == 0 ? 0 : h - k];
            const double2 wd64 = A.tw[k];                                    // e^{-2 pi i k/n}
            const T2 w = c2<T2>((T)wd64.x, (T)wd64.y);
            const T2 sp = c2<T2>(zk.x + zc.x, zk.y - zc.y);                  // Z_k + conj Z_{h-k}
            const T2 dm = c2<T2>(zk.x - zc.x, zk.y + zc.y);                  // Z_k - conj Z_{h-k}
            const T2 wd = cmul(w, dm);
            c[k] = c2<T2>((T)0.5 * (sp.x + wd.y), (T)0.5 * (sp.y - wd.x));   // (sp - i w dm)/2
        }
    } else {
        // entries k >= ncol are zero (the column transforms leave them unwritten)
        const T2 zero = c2<T2>((T)0, (T)0);
        for (int k = tid; k < h; k += RT) {
            const T2 a = k < A.ncol ? c[k] : zero, bb = h - k < A.ncol ? c[h - k] : zero;
            const T2 sp = c2<T2>(a.x + bb.x, a.y - bb.y);                    // X_k + conj X_{h-k}
            const T2 dm = c2<T2>(a.x - bb.x, a.y + bb.y);                    // X_k - conj X_{h-k}
            const double2 wd64 = A.tw[k];
            const T2 wd = cmul(c2<T2>((T)wd64.x, (T)-wd64.y), dm);           // e^{+2 pi i k/n} dm
            buf[k] = c2<T2>(sp.x - wd.y, sp.y + wd.x);                       // sp + i wd
        }
        __syncthreads();
        lds_fft<true, RT, NMAX / 2>(buf, A.tw, 2, h, A.radix, A.npass);
        // only the points the interpolation windows use
        for (int m = A.m0 + tid; m < A.m1; m += RT) c[m] = buf[m];
    }
}

template <typename T>
struct ColArgs {
    int64_t n, field;
    int B, ncol, npass;
    int iy0, iy1;          // rows [iy0, iy1) of the input columns can be nonzero (the sources' windows)
    int oy0, oy1;          // rows [oy0, oy1) of the output columns are written (the targets' windows)
    int8_t radix[COL_MAXPASS];
    T *grid;
    const double2 *tw;             // e^{-2 pi i m / n}, FP64 at both precisions
    const double *fac, *mtab;
    double c, alpha2, dk;
    int lmax;
};

// One workgroup per (column, density, output): 0 S, 1 V, 2 D (from the D_x
// and D_y spectra: -i (k_x Gx + k_y Gy) M, as two transforms whose results
// are added).
template <typename T, int NMAX>
__global__ void __launch_bounds__(CT) k_columns(ColArgs<T> A)
{
    typedef typename Vec2<T>::type T2;
    extern __shared__ double lds_col[];
    T2 *buf = reinterpret_cast<T2 *>(lds_col);
    const int n = (int)A.n, nh = n / 2 + 1;
    // consecutive columns on one XCD (workgroups are dealt to the 8 XCDs in
    // turn), so that neighbouring columns share the XCD's L2 lines; only the
    // columns l_x < ncol that the multiplier keeps (the inverse row
    // transforms take the others as zero)
    const int per = (A.ncol + 7) / 8;
    const int lx = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (lx >= A.ncol) return;
    const int b = blockIdx.y, grp = blockIdx.z;
    const size_t fs = (size_t)A.B * (A.field / 2);              // complex values per slot
    T2 *base = reinterpret_cast<T2 *>(A.grid) + (size_t)b * (A.field / 2) + lx;
    T2 *out = base + (size_t)grp * fs;
    const double ax = A.fac[lx];
    const double kx = A.dk * lx;
    auto mult = [&](int ly) -> double {
        const int fy = ly <= n / 2 ? ly : ly - n;
        if (A.mtab) {
            if (lx <= A.lmax && fy >= -A.lmax && fy <= A.lmax) return A.mtab[(fy + A.lmax) * (A.lmax + 1) + lx];
            return 0.0;
        }
        const double ay = A.fac[fy < 0 ? -fy : fy];
        if (ax == 0.0 || ay == 0.0) return 0.0;
        const double ky = A.dk * fy;
        return A.c * ax * ay / (A.alpha2 + kx * kx + ky * ky);
    };
    const int nparts = grp == 2 ? 2 : 1;
    for (int part = 0; part < nparts; ++part) {
        const T2 *in = base + (size_t)(grp == 2 ? 2 + part : grp) * fs;
        const T2 zero = c2<T2>((T)0, (T)0);
        for (int y = threadIdx.x; y < n; y += CT) buf[y] = y >= A.iy0 && y < A.iy1 ? in[(size_t)y * nh] : zero;
        __syncthreads();
        lds_fft<false, CT, NMAX>(buf, A.tw, 1, n, A.radix, A.npass);
        for (int ly = threadIdx.x; ly < n; ly += CT) {
            const double M = mult(ly);
            const T2 z = buf[ly];
            if (grp < 2) {
                buf[ly] = c2<T2>((T)(M * z.x), (T)(M * z.y));
            } else {
                // -i k M z with k = k_x (part 0) or k_y (part 1)
                const int fy = ly <= n / 2 ? ly : ly - n;
                const double kM = (part == 0 ? kx : A.dk * fy) * M;
                buf[ly] = c2<T2>((T)(kM * z.y), (T)(-kM * z.x));
            }
        }
        __syncthreads();
        lds_fft<true, CT, NMAX>(buf, A.tw, 1, n, A.radix, A.npass);
        // part 0 of D writes its column, part 1 adds to it (same thread, same
        // rows: no other thread touches these values)
        for (int y = A.oy0 + threadIdx.x; y < A.oy1; y += CT) {
            T2 v = buf[y];
            if (part == 1) v = cadd(out[(size_t)y * nh], v);
            out[(size_t)y * nh] = v;
        }
        __syncthreads();
    }
}

template <typename T>
struct InterpArgs {
    int64_t n, field, nout;
    int ntile, B;
    double beta, ox, oy, h;
    const int32_t *tile_xy, *tile_rng;
    const double *tx, *ty;
    const T *grid;         // [3][B][field]: S, V, D results
    const T *wcoef;
    T *acc;                // [3][B][nout]: S, D, V
    int want_s, want_d, want_v;
};

template <int W, typename T>
__global__ void __launch_bounds__(HB) k_interp(InterpArgs<T> A)
{
    constexpr int RS = TILE + W + 2;
    __shared__ T reg[3][RS * RS];
    const int t = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const int tile = A.tile_xy[t];
    const int tx = tile % A.ntile, ty = tile / A.ntile;
    const int rx0 = tx * TILE - W / 2 - 1, ry0 = ty * TILE - W / 2 - 1;
    const size_t fs = (size_t)A.B * A.field;
    const T *g0 = A.grid + (size_t)b * A.field;
    for (int i = tid; i < RS * RS; i += HB) {
        // the staged region exceeds the grid by less than one period
        int gy = ry0 + i / RS, gx = rx0 + i % RS;
        gy += gy < 0 ? (int)A.n : gy >= A.n ? -(int)A.n : 0;
        gx += gx < 0 ? (int)A.n : gx >= A.n ? -(int)A.n : 0;
        const size_t o = (size_t)gy * (A.n + 2) + gx;
        reg[0][i] = A.want_s ? g0[o] : (T)0;
        reg[1][i] = A.want_v ? g0[fs + o] : (T)0;
        reg[2][i] = A.want_d ? g0[2 * fs + o] : (T)0;
    }
    __syncthreads();
    const int s0 = A.tile_rng[t], s1 = A.tile_rng[t + 1];
    for (int s = s0 + tid; s < s1; s += HB) {
        const double gx = (A.tx[s] - A.ox) / A.h, gy = (A.ty[s] - A.oy) / A.h;
        int mx0, my0;
        T wx[W], wy[W];
        window_weights2<W, T>(gx, gy, A.wcoef, mx0, my0, wx, wy);
        const int lx = min(max(mx0 - rx0, 0), RS - W), ly = min(max(my0 - ry0, 0), RS - W);
        T uS = 0, uV = 0, uD = 0;
#pragma unroll 1
        for (int ky = 0; ky < W; ++ky) {
            const int o = (ly + ky) * RS + lx;
            T rS = 0, rV = 0, rD = 0;
#pragma unroll
            for (int kx = 0; kx < W; ++kx) {
                rS = fma(wx[kx], reg[0][o + kx], rS);
                rV = fma(wx[kx], reg[1][o + kx], rV);
                rD = fma(wx[kx], reg[2][o + kx], rD);
            }
            uS = fma(wy[ky], rS, uS);
            uV = fma(wy[ky], rV, uV);
            uD = fma(wy[ky], rD, uD);
        }
        const size_t ob = (size_t)b * A.nout + s, cs = (size_t)A.B * A.nout;
        if (A.want_s) A.acc[ob] = uS;
        if (A.want_d) A.acc[cs + ob] = uD;
        if (A.want_v) A.acc[2 * cs + ob] = uV;
    }
}

// History kernel G^H(r) = int_delta^inf H(t, r) dt (eq. (sl_sh)) by composite
// 16-point Gauss-Legendre in u with t = delta e^{-u}, u in (-inf, 0]:
//   G^H = (1/4pi) int exp(-a e^u - b e^{-u}) du,  a = r^2/(4 delta), b = alpha^2 delta,
// truncated where the exponent is below -700; panels narrower than the
// width 1/sqrt(2 sqrt(ab)) of the integrand's peak.
__device__ double history_kernel(double r, double alpha, double delta, const double *__restrict__ gt,
                                 const double *__restrict__ gw)
{
    const double a = r * r / (4.0 * delta), b = alpha * alpha * delta;
    double lo = log(b / 700.0), hi = 0.0;
    if (a > 0.0) hi = fmin(hi, log(700.0 / a));
    if (!(hi > lo)) return 0.0;
    const double width = 1.0 / sqrt(1.0 + 2.0 * sqrt(a * b));
    int m = (int)ceil((hi - lo) / (0.5 * width));
    m = max(1, min(m, 2000));
    const double hp = (hi - lo) / m;
    double s = 0.0;
    for (int p = 0; p < m; ++p) {
        const double c = lo + (p + 0.5) * hp;
        double ps = 0.0;
        for (int q = 0; q < 16; ++q) {
            const double u = c + 0.5 * hp * gt[q];
            ps = fma(gw[q], exp(-a * exp(u) - b * exp(-u)), ps);
        }
        s += ps;
    }
    return s * 0.5 * hp / (4.0 * M_PI);
}

// Samples of the smoothly truncated history kernel on the quarter grid
// x = mx h, y = my h, 0 <= mx, my < M (the kernel is even in x and y and
// zero for |x| or |y| >= M h): h^2 G^H(r) chi(x) chi(y), chi(s) =
// erfc((s - rmid) slope)/2, row-major [my][mx].
__global__ void __launch_bounds__(256) k_trunc_samples(double *buf, int64_t M, double h, double alpha,
                                                       double delta, double rmid, double slope,
                                                       const double *__restrict__ gt,
                                                       const double *__restrict__ gw)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= M * M) return;
    const int64_t my = id / M, mx = id % M;
    const double x = mx * h, y = my * h;
    buf[id] = h * h * history_kernel(sqrt(x * x + y * y), alpha, delta, gt, gw) * 0.25 * erfc((x - rmid) * slope) *
              erfc((y - rmid) * slope);
}

// One separable step of the cosine transform of the even samples:
//   out[a][b] = sum_{k < K} c_k cos(2 pi a k / n) in[b][k],  c_0 = 1, c_k = 2,
// for a < NA, b < NB (the +-k pairs of the even sequence folded into c_k).
// Tiles of 64 x 64 outputs per 256-thread workgroup, 4 x 4 per thread, the
// cosine factors (from a table of cos(2 pi m / n) at m = a k mod n) and the
// input staged through LDS 32 values of k at a time.
constexpr int CS_T = 64, CS_K = 32;
__global__ void __launch_bounds__(256) k_cos_step(const double *__restrict__ in, int64_t K, int64_t NA, int64_t NB,
                                                  int n, const double *__restrict__ costab, double *__restrict__ out)
{
    __shared__ double ca[CS_K][CS_T + 1];
    __shared__ double ib[CS_K][CS_T + 1];
    const int tid = threadIdx.x;
    const int64_t a0 = (int64_t)blockIdx.x * CS_T, b0 = (int64_t)blockIdx.y * CS_T;
    const int ta = tid / 16, tb = tid % 16;
    double acc[4][4] = {};
    for (int64_t k0 = 0; k0 < K; k0 += CS_K) {
        for (int e = tid; e < CS_K * CS_T; e += 256) {
            const int kk = e / CS_T, aa = e % CS_T;
            const int64_t k = k0 + kk, a = a0 + aa;
            double v = 0.0;
            if (k < K && a < NA) v = (k == 0 ? 1.0 : 2.0) * costab[(int)((a * k) % n)];
            ca[kk][aa] = v;
        }
        for (int e = tid; e < CS_K * CS_T; e += 256) {
            const int bb = e / CS_K, kk = e % CS_K;
            const int64_t k = k0 + kk, b = b0 + bb;
            ib[kk][bb] = (k < K && b < NB) ? in[b * K + k] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < CS_K; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                av[i] = ca[kk][ta + 16 * i];
                bv[i] = ib[kk][tb + 16 * i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t a = a0 + ta + 16 * i, b = b0 + tb + 16 * j;
            if (a < NA && b < NB) out[a * NB + b] = acc[i][j];
        }
}

// Multiplier table on the kept modes |l_x|, |l_y| <= lmax from the cosine
// transform tr[l_y][l_x] (l >= 0; the kernel's transform is real and even).
__global__ void __launch_bounds__(256) k_trunc_table(const double *__restrict__ tr, int lmax,
                                                     const double *__restrict__ phi2inv, double c,
                                                     double *__restrict__ mtab)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = lmax + 1;
    if (id >= (2 * (int64_t)lmax + 1) * w) return;
    const int64_t lx = id % w, fy = id / w - lmax, ly = fy < 0 ? -fy : fy;
    mtab[id] = c * tr[ly * w + lx] * phi2inv[lx] * phi2inv[ly];
}

hipError_t launch_trunc_kernel_samples(double *buf, int64_t M, double h, double alpha, double delta, double rmid,
                                       double slope, const double *gl_t, const double *gl_w, hipStream_t s)
{
    const int64_t tot = M * M;
    hipLaunchKernelGGL(k_trunc_samples, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, buf, M, h, alpha,
                       delta, rmid, slope, gl_t, gl_w);
    return hipGetLastError();
}

hipError_t launch_cos_step(const double *in, int64_t K, int64_t NA, int64_t NB, int n, const double *costab,
                           double *out, hipStream_t s)
{
    dim3 grid((unsigned)((NA + CS_T - 1) / CS_T), (unsigned)((NB + CS_T - 1) / CS_T));
    hipLaunchKernelGGL(k_cos_step, grid, dim3(256), 0, s, in, K, NA, NB, n, costab, out);
    return hipGetLastError();
}

hipError_t launch_trunc_table(const double *tr, int lmax, const double *phi2inv, double c, double *mtab,
                              hipStream_t s)
{
    const int64_t tot = (2 * (int64_t)lmax + 1) * (lmax + 1);
    hipLaunchKernelGGL(k_trunc_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, tr, lmax, phi2inv, c,
                       mtab);
    return hipGetLastError();
}

template <int W, typename T>
static hipError_t spread_w(mhk_plan *P, const SpreadArgs<T> &A)
{
    const History &G = P->hist;
    // column path: only the tiles of the sources' windows (the transforms
    // read nothing else); rocFFT's 2D transforms read the whole grid
    const int nty = G.colpath ? (G.sy1 - 1) / TILE - A.tby0 + 1 : A.ntile;
    dim3 grid((unsigned)(A.ntbx * nty), (unsigned)A.B);
    hipLaunchKernelGGL((k_spread<W, T>), grid, dim3(SB), 0, P->stream, A);
    return hipGetLastError();
}

template <int W, typename T>
static hipError_t interp_w(mhk_plan *P, const InterpArgs<T> &A)
{
    if (P->hist.n_ttiles == 0) return hipSuccess;
    dim3 grid((unsigned)P->hist.n_ttiles, (unsigned)A.B);
    hipLaunchKernelGGL((k_interp<W, T>), grid, dim3(HB), 0, P->stream, A);
    return hipGetLastError();
}

#define MHK_W_SWITCH(w, F, T, ...)              \
    switch (w) {                                \
    case 4: return F<4, T>(__VA_ARGS__);        \
    case 5: return F<5, T>(__VA_ARGS__);        \
    case 6: return F<6, T>(__VA_ARGS__);        \
    case 7: return F<7, T>(__VA_ARGS__);        \
    case 8: return F<8, T>(__VA_ARGS__);        \
    case 9: return F<9, T>(__VA_ARGS__);        \
    case 10: return F<10, T>(__VA_ARGS__);      \
    case 11: return F<11, T>(__VA_ARGS__);      \
    case 12: return F<12, T>(__VA_ARGS__);      \
    case 13: return F<13, T>(__VA_ARGS__);      \
    case 14: return F<14, T>(__VA_ARGS__);      \
    case 15: return F<15, T>(__VA_ARGS__);      \
    case 16: return F<16, T>(__VA_ARGS__);      \
    default: return hipErrorInvalidValue;       \
    }

template <typename T>
static hipError_t spread_t(mhk_plan *P, const void *sigma, const void *mu, const void *f_vol)
{
    const History &G = P->hist;
    SpreadArgs<T> A;
    A.n = G.n;
    A.field = G.field;
    A.nb = P->nb;
    A.nv = P->nv;
    A.ntile = G.ntile;
    A.B = P->bat;
    A.tbx0 = G.colpath ? G.sx0 / TILE : 0;
    A.tby0 = G.colpath ? G.sy0 / TILE : 0;
    A.ntbx = G.colpath ? (G.sx1 - 1) / TILE - A.tbx0 + 1 : G.ntile;
    A.beta = G.beta;
    A.bgx = G.bgx; A.bgy = G.bgy; A.bw = G.bw; A.bwx = G.bwx; A.bwy = G.bwy;
    A.bidx = G.bidx; A.blofs = G.blofs; A.blist = G.blist;
    A.vgx = G.vgx; A.vgy = G.vgy; A.vw = G.vw; A.vidx = G.vidx; A.vlofs = G.vlofs; A.vlist = G.vlist;
    A.sigma = (const T *)sigma;
    A.mu = (const T *)mu;
    A.f_vol = (const T *)f_vol;
    A.grid = (T *)G.grid;
    A.wcoef = (const T *)G.wcoef;
    MHK_W_SWITCH(G.w, spread_w, T, P, A);
}

hipError_t launch_spread(mhk_plan *P, const void *sigma, const void *mu, const void *f_vol)
{
    return P->p.prec == MHK_FP64 ? spread_t<double>(P, sigma, mu, f_vol) : spread_t<float>(P, sigma, mu, f_vol);
}

template <typename T>
static hipError_t multiply_t(mhk_plan *P)
{
    const History &G = P->hist;
    const int64_t tot = G.n * (G.n / 2 + 1) * P->bat;
    hipLaunchKernelGGL(k_multiply<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, P->stream, G.n,
                       P->bat, G.field, (T *)G.grid, G.fac, G.mult_c, P->p.alpha * P->p.alpha,
                       2.0 * M_PI / G.period, G.trunc ? G.mtab : nullptr, G.lmax);
    return hipGetLastError();
}

template <typename T>
static hipError_t columns_t(mhk_plan *P)
{
    const History &G = P->hist;
    ColArgs<T> A;
    A.n = G.n;
    A.field = G.field;
    A.B = P->bat;
    A.ncol = G.ncol;
    A.npass = G.npass;
    for (int i = 0; i < COL_MAXPASS; ++i) A.radix[i] = G.radix[i];
    A.grid = (T *)G.grid;
    A.tw = (const double2 *)G.tw;
    A.fac = G.fac;
    A.mtab = G.trunc ? G.mtab : nullptr;
    A.c = G.mult_c;
    A.alpha2 = P->p.alpha * P->p.alpha;
    A.dk = 2.0 * M_PI / G.period;
    A.lmax = G.lmax;
    A.iy0 = G.sy0;
    A.iy1 = G.sy1;
    A.oy0 = G.ty0;
    A.oy1 = G.ty1;
    const size_t lds = sizeof(typename Vec2<T>::type) * (size_t)G.n;
    // register arrays sized for the longest column of the launch
    const void *fn = G.n <= COL_NMAX / 2 ? (const void *)k_columns<T, COL_NMAX / 2> : (const void *)k_columns<T, COL_NMAX>;
    if (lds > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (G.ncol == 0) return hipSuccess;     // the multiplier is zero everywhere
    dim3 grid((unsigned)(((G.ncol + 7) / 8) * 8), (unsigned)P->bat, 3u);
    if (G.n <= COL_NMAX / 2)
        hipLaunchKernelGGL((k_columns<T, COL_NMAX / 2>), grid, dim3(CT), lds, P->stream, A);
    else
        hipLaunchKernelGGL((k_columns<T, COL_NMAX>), grid, dim3(CT), lds, P->stream, A);
    return hipGetLastError();
}

template <bool INV, typename T>
static hipError_t rows_t(mhk_plan *P)
{
    const History &G = P->hist;
    RowArgs<T> A;
    A.n = G.n;
    A.ncol = G.ncol;
    A.npass = G.rnpass;
    for (int i = 0; i < COL_MAXPASS; ++i) A.radix[i] = G.rradix[i];
    A.grid = (T *)G.grid;
    A.tw = (const double2 *)G.tw;
    // forward: the rows and columns of the sources' windows; inverse: those
    // of the targets' windows
    A.r0 = INV ? G.ty0 : G.sy0;
    A.nrow = INV ? G.ty1 - G.ty0 : G.sy1 - G.sy0;
    A.m0 = (INV ? G.tx0 : G.sx0) / 2;
    A.m1 = ((INV ? G.tx1 : G.sx1) + 1) / 2;
    const size_t lds = sizeof(typename Vec2<T>::type) * (size_t)(G.n / 2);
    const int64_t rows = (INV ? 3 : 4) * (int64_t)P->bat * A.nrow;
    if (rows <= 0) return hipSuccess;
    if (G.n <= COL_NMAX / 2)
        hipLaunchKernelGGL((k_rows<INV, T, COL_NMAX / 2>), dim3((unsigned)rows), dim3(RT), lds, P->stream, A);
    else
        hipLaunchKernelGGL((k_rows<INV, T, COL_NMAX>), dim3((unsigned)rows), dim3(RT), lds, P->stream, A);
    return hipGetLastError();
}

hipError_t launch_rows(mhk_plan *P, bool inverse)
{
    if (P->p.prec == MHK_FP64) return inverse ? rows_t<true, double>(P) : rows_t<false, double>(P);
    return inverse ? rows_t<true, float>(P) : rows_t<false, float>(P);
}

hipError_t launch_columns(mhk_plan *P)
{
    return P->p.prec == MHK_FP64 ? columns_t<double>(P) : columns_t<float>(P);
}

hipError_t launch_multiply(mhk_plan *P)
{
    return P->p.prec == MHK_FP64 ? multiply_t<double>(P) : multiply_t<float>(P);
}

template <typename T>
static hipError_t interp_t(mhk_plan *P, bool want_s, bool want_d, bool want_v)
{
    const History &G = P->hist;
    InterpArgs<T> A;
    A.n = G.n;
    A.field = G.field;
    A.nout = P->nout;
    A.ntile = G.ntile;
    A.B = P->bat;
    A.beta = G.beta;
    A.ox = G.ox;
    A.oy = G.oy;
    A.h = G.h;
    A.tile_xy = G.ttile_xy;
    A.tile_rng = G.ttile_rng;
    A.tx = P->tx;
    A.ty = P->ty;
    A.grid = (const T *)G.grid;
    A.wcoef = (const T *)G.wcoef;
    A.acc = (T *)P->acc;
    A.want_s = want_s;
    A.want_d = want_d;
    A.want_v = want_v;
    MHK_W_SWITCH(G.w, interp_w, T, P, A);
}

hipError_t launch_interp(mhk_plan *P, bool want_s, bool want_d, bool want_v)
{
    return P->p.prec == MHK_FP64 ? interp_t<double>(P, want_s, want_d, want_v)
                                 : interp_t<float>(P, want_s, want_d, want_v);
}

}  // namespace mhk
