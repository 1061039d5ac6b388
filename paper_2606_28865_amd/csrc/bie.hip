// Boundary integral equations of Section 3.2 on the device: the dense Nystrom
// matrix of the double-layer operator, its matrix-vector product, restarted
// GMRES, and the Dirichlet and Neumann solves that combine them with the
// potential evaluation of a plan.
//
// Layout: K is N_B x ld row-major FP64 (ld = N_B rounded up to even, the pad
// column zero), 2 GiB at N_B = 16384 and 34 GiB at 65536, resident in HBM for
// the life of the object.  The product y = (shift I + K) x streams K once per
// call (HBM bound: 8 N_B^2 bytes); every other GMRES step is O(N_B m).
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "mhk_internal.h"

struct mhk_nystrom {
    int64_t n = 0, ld = 0;
    double alpha = 0;
    hipStream_t stream = nullptr;
    double *K = nullptr;
    // GMRES workspace (grown on demand)
    int m_cap = 0;
    int nblk = 0;
    double *V = nullptr;        // [m_cap + 1][n] Krylov basis
    double *wv = nullptr;       // [n]
    double *rv = nullptr;       // [n] residual / right-hand side
    double *part = nullptr;     // [(m_cap + 1) nblk] partial sums
    double *hd = nullptr;       // [2 (m_cap + 1) + 1] h (two passes) and |w|^2
    double *yd = nullptr;       // [m_cap] least-squares solution
    double *hh = nullptr;       // pinned host mirror of hd / yd
    // scratch of the Dirichlet and Neumann solves, [2][work_n]
    double *work = nullptr;
    int64_t work_n = 0;
    int64_t ws_bytes = 0;       // GMRES workspace
    double ms_assemble = 0;
    int64_t bytes() const { return (int64_t)sizeof(double) * (n * ld + 2 * work_n) + ws_bytes; }
};

namespace mhk {

#define BIE_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            set_error(std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_)); \
            return MHK_EHIP;                                                              \
        }                                                                                 \
    } while (0)

#define BIE_TRY(x)                        \
    do {                                  \
        mhk_status s_ = (x);              \
        if (s_ != MHK_OK) return s_;      \
    } while (0)

constexpr int BT = 256;         // threads per block of the vector kernels
constexpr int GV_ROWS = 8;      // rows of K per block of the product

// K_1(z), z > 0, by the trapezoidal rule on K_1(z) = int_0^inf exp(-z cosh t)
// cosh t dt (Trefethen and Weideman, SIAM Review 56 (2014), Section 5), written
// as e^{-z} int exp(-2 z sinh^2(t/2)) cosh t dt.  The integrand is analytic
// in the strip |Im t| < pi/2; the step min(0.2, 0.7/sqrt(z)) keeps the
// discretisation error below 1e-16 relative for large z, where the integrand
// narrows to width 1/sqrt(z), and the sum stops where the terms fall below
// e^{-45} of the first.  Relative error below 1e-15 for z in [1e-6, 700].
__device__ double bessel_k1(double z)
{
    const double h = fmin(0.2, 0.7 / sqrt(z));
    const int n = (int)ceil(acosh(1.0 + 45.0 / z) / h);
    double s = 0.5;
    for (int k = 1; k <= n; ++k) {
        const double t = k * h, sh = sinh(0.5 * t);
        s += exp(-2.0 * z * sh * sh) * cosh(t);
    }
    return h * s * exp(-z);
}

// K_ij = w_j alpha/(2 pi) K_1(alpha r) (x_i - x_j).nu_j / r for i != j and
// K_ii = -w_i kappa_i/(4 pi) (Section 3.2, with the diagonal limit of eq.
// (dlp_diag_limit)).  One block row i per blockIdx.x, columns along threads.
__global__ void __launch_bounds__(BT) k_nys_assemble(int64_t n, int64_t ld, double alpha, const double *x,
                                                     const double *y, const double *nx, const double *ny,
                                                     const double *w, const double *kap, double *K)
{
    const int64_t i = blockIdx.x;
    const int64_t j = (int64_t)blockIdx.y * BT + threadIdx.x;
    if (j >= ld) return;
    double v = 0.0;
    if (j < n) {
        if (j == i) {
            v = -w[i] * kap[i] / (4.0 * M_PI);
        } else {
            const double dx = x[i] - x[j], dy = y[i] - y[j];
            const double r = sqrt(dx * dx + dy * dy);
            v = w[j] * alpha / (2.0 * M_PI) * bessel_k1(alpha * r) * (dx * nx[j] + dy * ny[j]) / r;
        }
    }
    K[i * ld + j] = v;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// y = shift x + K x; GV_ROWS rows per block, column pairs along the threads
// (rows are 16-byte aligned since ld is even); fixed reduction order.
__global__ void __launch_bounds__(BT) k_gemv(int64_t n, int64_t ld, const double *__restrict__ K, double shift,
                                             const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t r0 = (int64_t)blockIdx.x * GV_ROWS;
    const int tid = threadIdx.x;
    double acc[GV_ROWS];
#pragma unroll
    for (int r = 0; r < GV_ROWS; ++r) acc[r] = 0.0;
    for (int64_t c = 2 * (int64_t)tid; c < n; c += 2 * BT) {
        const double x0 = x[c], x1 = (c + 1 < n) ? x[c + 1] : 0.0;
#pragma unroll
        for (int r = 0; r < GV_ROWS; ++r) {
            if (r0 + r < n) {
                const double2 k = *reinterpret_cast<const double2 *>(K + (r0 + r) * ld + c);
                acc[r] = fma(k.x, x0, acc[r]);
                acc[r] = fma(k.y, x1, acc[r]);
            }
        }
    }
    __shared__ double red[GV_ROWS][BT / 64];
#pragma unroll
    for (int r = 0; r < GV_ROWS; ++r) {
        const double s = wave_sum(acc[r]);
        if ((tid & 63) == 0) red[r][tid >> 6] = s;
    }
    __syncthreads();
    if (tid < GV_ROWS && r0 + tid < n) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < BT / 64; ++q) s += red[tid][q];
        y[r0 + tid] = fma(shift, x[r0 + tid], s);
    }
}

__device__ inline double block_sum(double v, double *sh)
{
    const int tid = threadIdx.x;
    v = wave_sum(v);
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < BT / 64; ++q) s += sh[q];
    __syncthreads();
    return s;
}

// part[i nblk + b] = partial dot product of basis vector i with w over the
// b-th slice of the index range; grid (nblk, count)
__global__ void __launch_bounds__(BT) k_dots(int64_t n, const double *__restrict__ V, const double *__restrict__ w,
                                             int nblk, double *__restrict__ part)
{
    __shared__ double sh[BT / 64];
    const int i = blockIdx.y;
    const double *v = V + (int64_t)i * n;
    double s = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < n; t += (int64_t)nblk * BT) s = fma(v[t], w[t], s);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[(int64_t)i * nblk + blockIdx.x] = s;
}

// out[i] = sum_b part[i nblk + b], one block per i, fixed order
__global__ void __launch_bounds__(BT) k_reduce(const double *__restrict__ part, int nblk, double *__restrict__ out)
{
    __shared__ double sh[BT / 64];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += BT) s += part[(int64_t)i * nblk + b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[i] = s;
}

// w -= sum_{i < count} h[i] V_i
__global__ void __launch_bounds__(BT) k_orth(int64_t n, const double *__restrict__ V, int count,
                                             const double *__restrict__ h, double *__restrict__ w)
{
    const int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (t >= n) return;
    double s = w[t];
    for (int i = 0; i < count; ++i) s = fma(-h[i], V[(int64_t)i * n + t], s);
    w[t] = s;
}

// v = w / sqrt(nrm2) (zero when the norm vanishes: breakdown, v unused)
__global__ void __launch_bounds__(BT) k_normalize(int64_t n, const double *__restrict__ w,
                                                  const double *__restrict__ nrm2, double *__restrict__ v)
{
    const int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (t >= n) return;
    const double s = *nrm2;
    v[t] = s > 0.0 ? w[t] / sqrt(s) : 0.0;
}

// x += sum_{i < count} y[i] V_i
__global__ void __launch_bounds__(BT) k_combine(int64_t n, const double *__restrict__ V, int count,
                                                const double *__restrict__ yv, double *__restrict__ x)
{
    const int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (t >= n) return;
    double s = x[t];
    for (int i = 0; i < count; ++i) s = fma(yv[i], V[(int64_t)i * n + t], s);
    x[t] = s;
}

__global__ void __launch_bounds__(BT) k_fill(int64_t n, double v, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (t < n) out[t] = v;
}

// out = a p + b q (out may alias p or q)
__global__ void __launch_bounds__(BT) k_axpby(int64_t n, double a, const double *p, double b, const double *q,
                                              double *out)
{
    const int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (t >= n) return;
    out[t] = a * p[t] + (q ? b * q[t] : 0.0);
}

// Dirichlet: u = V + D[mu] at the targets, the interior limit V + D[mu] - mu/2
// on the boundary nodes (jump relation, eq. (jumprel)).
__global__ void __launch_bounds__(BT) k_dirichlet_u(int64_t nt, int64_t nout, const double *__restrict__ d,
                                                    const double *__restrict__ mu, double *__restrict__ u)
{
    const int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (s >= nout) return;
    double v = u[s] + d[s];
    if (s >= nt) v -= 0.5 * mu[s - nt];
    u[s] = v;
}

// Neumann: u = V + S[g] - D[u_b] at the targets, u_b on the boundary nodes.
__global__ void __launch_bounds__(BT) k_neumann_u(int64_t nt, int64_t nout, const double *__restrict__ sg,
                                                  const double *__restrict__ d, const double *__restrict__ ub,
                                                  double *__restrict__ u)
{
    const int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (s >= nout) return;
    u[s] = s < nt ? u[s] + sg[s] - d[s] : ub[s - nt];
}

// f = alpha^2 u + F (F may be NULL): the source of one implicit-Euler step
__global__ void __launch_bounds__(BT) k_heat_source(int64_t n, double a2, const double *__restrict__ u,
                                                    const double *__restrict__ F, double *__restrict__ f)
{
    const int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (s >= n) return;
    f[s] = a2 * u[s] + (F ? F[s] : 0.0);
}

// rhs[i] = a * p[off + i] + b * q[off + i]  (q may be NULL)
__global__ void __launch_bounds__(BT) k_rhs(int64_t n, int64_t off, double a, const double *p, double b,
                                            const double *q, double *rhs)
{
    const int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (i >= n) return;
    rhs[i] = a * p[off + i] + (q ? b * q[off + i] : 0.0);
}

static inline unsigned nb_of(int64_t n) { return (unsigned)((n + BT - 1) / BT); }

// GMRES workspace: device vectors and the host mirror of the small ones.
// The object's own workspace (nys_workspace) or the fixed scratch array of
// mhk_nystrom_solve_noalloc.
struct GmresWs {
    int nblk = 0;               // blocks of the two-stage dot products
    double *V = nullptr;        // [m + 1][n] Krylov basis
    double *wv = nullptr;       // [n]
    double *rv = nullptr;       // [n] residual / right-hand side
    double *part = nullptr;     // [(m + 1) nblk] partial sums
    double *hd = nullptr;       // [2 (m + 1) + 1] h (two passes) and |w|^2
    double *yd = nullptr;       // [m] least-squares solution
    double *hh = nullptr;       // host, [2 (m + 1) + 1 + m]: mirror of hd, then y
    // host arrays of the least-squares problem: H [(m + 1) m], cs, sn, yv [m], g [m + 1]
    double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *yv = nullptr;
};

static inline int gmres_nblk(int64_t n) { return (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + BT - 1) / BT)); }

// Device buffers of a Nystrom object are allocated and freed in the order
// of its stream (hipFree would wait for every stream of the device, i.e.
// for other plans' work); an allocation is waited for on that stream before
// use, since the solves run on the plan's stream.
static mhk_status nys_alloc(mhk_nystrom *N, double **p, int64_t count)
{
    *p = nullptr;
    if (hipMallocAsync((void **)p, sizeof(double) * (size_t)std::max<int64_t>(count, 1), N->stream) != hipSuccess ||
        hipStreamSynchronize(N->stream) != hipSuccess) {
        (void)hipGetLastError();
        if (*p) (void)hipFreeAsync(*p, N->stream);
        *p = nullptr;
        set_error("device allocation of " + std::to_string(sizeof(double) * count) + " bytes failed");
        return MHK_ENOMEM;
    }
    return MHK_OK;
}

static void nys_free(mhk_nystrom *N, double **p)
{
    if (*p) (void)hipFreeAsync(*p, N->stream);
    *p = nullptr;
}

static void nys_free_ws(mhk_nystrom *N)
{
    for (double **p : {&N->V, &N->wv, &N->rv, &N->part, &N->hd, &N->yd}) nys_free(N, p);
    delete[] N->hh;
    N->hh = nullptr;
    N->ws_bytes = 0;
    N->m_cap = 0;
}

static mhk_status nys_workspace(mhk_nystrom *N, int m)
{
    if (m <= N->m_cap) return MHK_OK;
    nys_free_ws(N);
    N->nblk = gmres_nblk(N->n);
    BIE_TRY(nys_alloc(N, &N->V, (int64_t)(m + 1) * N->n));
    BIE_TRY(nys_alloc(N, &N->wv, N->n));
    BIE_TRY(nys_alloc(N, &N->rv, N->n));
    BIE_TRY(nys_alloc(N, &N->part, (int64_t)(m + 1) * N->nblk));
    BIE_TRY(nys_alloc(N, &N->hd, 2 * (m + 1) + 1));
    BIE_TRY(nys_alloc(N, &N->yd, m));
    // host mirror of the few Arnoldi values copied back per iteration
    // (pageable: pinned host memory would have to be released with
    // hipHostFree, which waits for the whole device)
    N->hh = new double[(size_t)(2 * (m + 1) + 1 + m)];
    N->m_cap = m;
    N->ws_bytes = (int64_t)sizeof(double) * ((int64_t)(m + 3) * N->n + (int64_t)(m + 1) * N->nblk + 3 * (m + 1));
    return MHK_OK;
}

// The object's own workspace as a GmresWs, with host arrays for restart m.
struct OwnWs {
    GmresWs W;
    std::vector<double> H, cs, sn, g, yv;
};

static mhk_status own_workspace(mhk_nystrom *N, int m, OwnWs &o)
{
    BIE_TRY(nys_workspace(N, m));
    o.H.assign((size_t)(m + 1) * m, 0.0);
    o.cs.assign(m, 0.0);
    o.sn.assign(m, 0.0);
    o.g.assign(m + 1, 0.0);
    o.yv.assign(m, 0.0);
    GmresWs &W = o.W;
    W.nblk = N->nblk;
    W.V = N->V; W.wv = N->wv; W.rv = N->rv; W.part = N->part; W.hd = N->hd; W.yd = N->yd; W.hh = N->hh;
    W.H = o.H.data(); W.cs = o.cs.data(); W.sn = o.sn.data(); W.g = o.g.data(); W.yv = o.yv.data();
    return MHK_OK;
}

static mhk_status nys_scratch(mhk_nystrom *N, int64_t nout)
{
    if (nout <= N->work_n) return MHK_OK;
    nys_free(N, &N->work);
    N->work_n = 0;
    BIE_TRY(nys_alloc(N, &N->work, 2 * nout));
    N->work_n = nout;
    return MHK_OK;
}

static hipError_t gemv(const mhk_nystrom *N, double shift, const double *x, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_gemv, dim3((unsigned)((N->n + GV_ROWS - 1) / GV_ROWS)), dim3(BT), 0, st, N->n, N->ld, N->K,
                       shift, x, y);
    return hipGetLastError();
}

// out[0..count) = dot products of V_0..V_{count-1} with w (device result)
static hipError_t dots(const mhk_nystrom *N, const GmresWs &W, const double *V, int count, const double *w,
                       double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_dots, dim3((unsigned)W.nblk, (unsigned)count), dim3(BT), 0, st, N->n, V, w, W.nblk,
                       W.part);
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)count), dim3(BT), 0, st, W.part, W.nblk, out);
    return hipGetLastError();
}

// host copy of a device scalar
static mhk_status fetch(mhk_nystrom *N, const double *d, int count, double *h, hipStream_t st)
{
    BIE_HIP(hipMemcpyAsync(h, d, sizeof(double) * count, hipMemcpyDeviceToHost, st));
    BIE_HIP(hipStreamSynchronize(st));
    return MHK_OK;
}

// Restarted GMRES(m) for (shift I + K) x = b, x = 0 initially; classical
// Gram-Schmidt with one re-orthogonalisation on the device, Givens rotations
// of the small Hessenberg matrix on the host.  Converged when the true
// residual |b - A x| <= tol |b| at the end of a cycle.
static mhk_status gmres(mhk_nystrom *N, const GmresWs &W, double shift, const double *b, double *x, double tol,
                        int m, int maxit, hipStream_t st, mhk_solve_info *info)
{
    const int64_t n = N->n;
    double *hh = W.hh, *h1 = W.hd, *h2 = W.hd + (m + 1), *nrm = W.hd + 2 * (m + 1);
    hipLaunchKernelGGL(k_fill, dim3(nb_of(n)), dim3(BT), 0, st, n, 0.0, x);
    BIE_HIP(hipGetLastError());
    BIE_HIP(dots(N, W, b, 1, b, nrm, st));
    double bn2;
    BIE_TRY(fetch(N, nrm, 1, &bn2, st));
    const double bnorm = sqrt(bn2);
    info->iters = 0;
    info->resid = 0.0;
    info->converged = 1;
    if (!(bnorm > 0.0)) return MHK_OK;
    if (!std::isfinite(bnorm)) {
        set_error("right-hand side is not finite");
        return MHK_EINVAL;
    }
    double *H = W.H, *cs = W.cs, *sn = W.sn, *g = W.g, *yv = W.yv;
    int total = 0;
    bool first = true;
    for (;;) {
        // r = b - A x
        if (first) {
            BIE_HIP(hipMemcpyAsync(W.rv, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        } else {
            BIE_HIP(gemv(N, shift, x, W.wv, st));
            hipLaunchKernelGGL(k_axpby, dim3(nb_of(n)), dim3(BT), 0, st, n, 1.0, b, -1.0, (const double *)W.wv,
                               W.rv);
            BIE_HIP(hipGetLastError());
        }
        first = false;
        BIE_HIP(dots(N, W, W.rv, 1, W.rv, nrm, st));
        double r2;
        BIE_TRY(fetch(N, nrm, 1, &r2, st));
        const double beta = sqrt(r2);
        info->resid = beta / bnorm;
        if (!std::isfinite(beta)) {
            set_error("GMRES residual is not finite");
            return MHK_EHIP;
        }
        if (beta <= tol * bnorm) {
            info->converged = 1;
            break;
        }
        if (total >= maxit) {
            info->converged = 0;
            break;
        }
        hipLaunchKernelGGL(k_normalize, dim3(nb_of(n)), dim3(BT), 0, st, n, (const double *)W.rv,
                           (const double *)nrm, W.V);
        BIE_HIP(hipGetLastError());
        std::fill(g, g + m + 1, 0.0);
        g[0] = beta;
        int jend = 0;
        for (int j = 0; j < m; ++j) {
            const double *vj = W.V + (int64_t)j * n;
            BIE_HIP(gemv(N, shift, vj, W.wv, st));
            BIE_HIP(dots(N, W, W.V, j + 1, W.wv, h1, st));
            hipLaunchKernelGGL(k_orth, dim3(nb_of(n)), dim3(BT), 0, st, n, (const double *)W.V, j + 1,
                               (const double *)h1, W.wv);
            BIE_HIP(dots(N, W, W.V, j + 1, W.wv, h2, st));
            hipLaunchKernelGGL(k_orth, dim3(nb_of(n)), dim3(BT), 0, st, n, (const double *)W.V, j + 1,
                               (const double *)h2, W.wv);
            BIE_HIP(dots(N, W, W.wv, 1, W.wv, nrm, st));
            hipLaunchKernelGGL(k_normalize, dim3(nb_of(n)), dim3(BT), 0, st, n, (const double *)W.wv,
                               (const double *)nrm, W.V + (int64_t)(j + 1) * n);
            BIE_HIP(hipGetLastError());
            BIE_TRY(fetch(N, W.hd, 2 * (m + 1) + 1, hh, st));
            double *col = &H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) col[i] = hh[i] + hh[(m + 1) + i];
            const double hn = sqrt(std::max(0.0, hh[2 * (m + 1)]));
            col[j + 1] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = col[i], c = col[i + 1];
                col[i] = cs[i] * a + sn[i] * c;
                col[i + 1] = -sn[i] * a + cs[i] * c;
            }
            const double den = hypot(col[j], col[j + 1]);
            cs[j] = den > 0 ? col[j] / den : 1.0;
            sn[j] = den > 0 ? col[j + 1] / den : 0.0;
            col[j] = den;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++total;
            jend = j + 1;
            if (fabs(g[j + 1]) <= tol * bnorm || total >= maxit || !(hn > 0.0)) break;
        }
        // back substitution H y = g, then x += V y
        for (int i = jend - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < jend; ++k) s -= H[(size_t)k * (m + 1) + i] * yv[k];
            const double d = H[(size_t)i * (m + 1) + i];
            yv[i] = d != 0.0 ? s / d : 0.0;
        }
        double *yh = hh + 2 * (m + 1) + 1;
        for (int i = 0; i < jend; ++i) yh[i] = yv[i];
        BIE_HIP(hipMemcpyAsync(W.yd, yh, sizeof(double) * jend, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_combine, dim3(nb_of(n)), dim3(BT), 0, st, n, (const double *)W.V, jend,
                           (const double *)W.yd, x);
        BIE_HIP(hipGetLastError());
        // the pinned buffer is reused by the next fetch: wait for the copy
        BIE_HIP(hipStreamSynchronize(st));
    }
    info->iters = total;
    return MHK_OK;
}

// Scratch of mhk_nystrom_solve_noalloc: one fixed device array of
// NOALLOC_DOUBLES doubles (32 MiB), held by every GPU the library runs on
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it stands for no device address): the address of each
// device's copy is looked up once, with that device current, and kept.
constexpr int64_t NOALLOC_DOUBLES = (int64_t)4 << 20;
constexpr int NOALLOC_MAX_RESTART = 64;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

static mhk_status scratch_base(double **out)
{
    int dev = 0;
    BIE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("device index out of the range of the scratch table");
        return MHK_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
            return MHK_EHIP;
        }
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return MHK_OK;
}

static inline int64_t round256(int64_t count) { return (count + 31) / 32 * 32; }   // doubles -> 256 B

static mhk_status check_solve(mhk_plan *P, mhk_nystrom *N, const void *g, const void *f_vol, const void *f_trg,
                              double tol, int restart, int maxit, const void *dens, const void *u)
{
    if (!P || !N || !g || !dens || !u) {
        set_error("null plan, Nystrom matrix, data or output pointer");
        return MHK_EINVAL;
    }
    if (P->p.prec != MHK_FP64 || P->p.batch != 1 || P->p.local_order >= 2) {
        set_error("the boundary integral solves need an FP64 plan with batch 1 and first-order local expansions");
        return MHK_EUNSUPPORTED;
    }
    if (P->nout != P->nt + P->nb) {
        set_error("the boundary integral solves need a plan with on-surface targets");
        return MHK_EINVAL;
    }
    if (P->nb != N->n || P->p.alpha != N->alpha) {
        set_error("plan and Nystrom matrix differ in boundary size or alpha");
        return MHK_EINVAL;
    }
    if ((f_vol == nullptr) != (f_trg == nullptr)) {
        set_error("f_vol and f_trg must be given together");
        return MHK_EINVAL;
    }
    if (f_vol && P->nv == 0) {
        set_error("volume source given but the plan has no volume nodes");
        return MHK_EINVAL;
    }
    if (!(tol > 0.0 && tol < 1.0) || restart < 1 || restart > 1000 || maxit < 1) {
        set_error("need 0 < tol < 1, 1 <= restart <= 1000, maxit >= 1");
        return MHK_EINVAL;
    }
    return MHK_OK;
}

}  // namespace mhk

using namespace mhk;

extern "C" {

mhk_status mhk_nystrom_create(double alpha, const mhk_boundary *b, void *hip_stream, mhk_nystrom **out)
{
    if (!out) {
        set_error("null output handle");
        return MHK_EINVAL;
    }
    *out = nullptr;
    if (!b || !(alpha > 0.0) || !std::isfinite(alpha) || b->n_panels < 1 || !b->x || !b->y || !b->nx || !b->ny ||
        !b->w || !b->kappa) {
        set_error("need alpha > 0 and a boundary with panels and all node arrays");
        return MHK_EINVAL;
    }
    const int64_t n = b->n_panels * NGL;
    if (n > (int64_t)1 << 20) {
        set_error("boundary too large for a dense Nystrom matrix");
        return MHK_EUNSUPPORTED;
    }
    mhk_nystrom *N = new mhk_nystrom();
    N->n = n;
    N->ld = (n + 1) / 2 * 2;
    N->alpha = alpha;
    N->stream = (hipStream_t)hip_stream;
    double *geo = nullptr;
    mhk_status st = nys_alloc(N, &N->K, n * N->ld);
    if (st == MHK_OK) st = nys_alloc(N, &geo, 6 * n);
    if (st != MHK_OK) {
        mhk_nystrom_destroy(N);
        return st;
    }
    std::vector<double> h(6 * (size_t)n);
    const double *src[6] = {b->x, b->y, b->nx, b->ny, b->w, b->kappa};
    for (int k = 0; k < 6; ++k) memcpy(&h[(size_t)k * n], src[k], sizeof(double) * n);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMemcpyAsync(geo, h.data(), sizeof(double) * 6 * n, hipMemcpyHostToDevice, N->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, N->stream);
    if (e == hipSuccess) {
        dim3 grid((unsigned)n, (unsigned)((N->ld + BT - 1) / BT));
        hipLaunchKernelGGL(k_nys_assemble, grid, dim3(BT), 0, N->stream, n, N->ld, alpha, (const double *)geo,
                           (const double *)(geo + n), (const double *)(geo + 2 * n), (const double *)(geo + 3 * n),
                           (const double *)(geo + 4 * n), (const double *)(geo + 5 * n), N->K);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, N->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(N->stream);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    nys_free(N, &geo);
    if (e != hipSuccess) {
        set_error(std::string("Nystrom assembly: ") + hipGetErrorString(e));
        mhk_nystrom_destroy(N);
        return MHK_EHIP;
    }
    N->ms_assemble = ms;
    *out = N;
    return MHK_OK;
}

mhk_status mhk_nystrom_info(const mhk_nystrom *N, mhk_nys_info *info)
{
    if (!N || !info) {
        set_error("null Nystrom matrix or info");
        return MHK_EINVAL;
    }
    info->n = N->n;
    info->alpha = N->alpha;
    info->device_bytes = N->bytes();
    info->ms_assemble = N->ms_assemble;
    return MHK_OK;
}

mhk_status mhk_nystrom_apply(mhk_nystrom *N, double shift, const double *x, double *y)
{
    if (!N || !x || !y || x == y) {
        set_error("null Nystrom matrix or vector, or x aliases y");
        return MHK_EINVAL;
    }
    BIE_HIP(gemv(N, shift, x, y, N->stream));
    return MHK_OK;
}

mhk_status mhk_nystrom_solve(mhk_nystrom *N, double shift, const double *rhs, double *x, double tol, int restart,
                             int maxit, mhk_solve_info *info)
{
    if (!N || !rhs || !x || !info || rhs == x) {
        set_error("null Nystrom matrix, vector or info, or rhs aliases x");
        return MHK_EINVAL;
    }
    if (!(tol > 0.0 && tol < 1.0) || restart < 1 || restart > 1000 || maxit < 1) {
        set_error("need 0 < tol < 1, 1 <= restart <= 1000, maxit >= 1");
        return MHK_EINVAL;
    }
    memset(info, 0, sizeof(*info));
    OwnWs o;
    BIE_TRY(own_workspace(N, restart, o));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BIE_HIP(hipEventCreate(&e0));
    BIE_HIP(hipEventCreate(&e1));
    BIE_HIP(hipEventRecord(e0, N->stream));
    mhk_status st = gmres(N, o.W, shift, rhs, x, tol, restart, maxit, N->stream, info);
    if (st == MHK_OK) {
        BIE_HIP(hipEventRecord(e1, N->stream));
        BIE_HIP(hipEventSynchronize(e1));
        float ms = 0;
        BIE_HIP(hipEventElapsedTime(&ms, e0, e1));
        info->ms_gmres = ms;
        info->ms_total = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

mhk_status mhk_nystrom_solve_noalloc(mhk_nystrom *N, double shift, const double *rhs, double *x, double tol,
                                     int restart, int maxit, mhk_solve_info *info)
{
    if (!N || !rhs || !x || !info || rhs == x) {
        set_error("null Nystrom matrix, vector or info, or rhs aliases x");
        return MHK_EINVAL;
    }
    if (!(tol > 0.0 && tol < 1.0) || restart < 1 || restart > NOALLOC_MAX_RESTART || maxit < 1) {
        set_error("need 0 < tol < 1, 1 <= restart <= " + std::to_string(NOALLOC_MAX_RESTART) + ", maxit >= 1");
        return MHK_EINVAL;
    }
    const int m = restart;
    const int64_t n = N->n;
    const int nblk = gmres_nblk(n);
    const int64_t nV = round256((int64_t)(m + 1) * n), nvec = round256(n), npart = round256((int64_t)(m + 1) * nblk),
                  nhd = round256(2 * (m + 1) + 1), nyd = round256(m);
    const int64_t need = nV + 2 * nvec + npart + nhd + nyd;
    if (need > NOALLOC_DOUBLES) {
        set_error("GMRES needs " + std::to_string(need * 8) + " bytes of scratch at N_B = " + std::to_string(n) +
                  " and restart " + std::to_string(m) + "; the fixed scratch holds " +
                  std::to_string(NOALLOC_DOUBLES * 8));
        return MHK_EINVAL;
    }
    double *base = nullptr;
    BIE_TRY(scratch_base(&base));
    GmresWs W;
    W.nblk = nblk;
    W.V = base;
    W.wv = W.V + nV;
    W.rv = W.wv + nvec;
    W.part = W.rv + nvec;
    W.hd = W.part + npart;
    W.yd = W.hd + nhd;
    // host side of the least-squares problem on the stack (restart <= 64)
    double hh[2 * (NOALLOC_MAX_RESTART + 1) + 1 + NOALLOC_MAX_RESTART];
    double H[(NOALLOC_MAX_RESTART + 1) * NOALLOC_MAX_RESTART];
    double cs[NOALLOC_MAX_RESTART], sn[NOALLOC_MAX_RESTART], g[NOALLOC_MAX_RESTART + 1], yv[NOALLOC_MAX_RESTART];
    W.hh = hh;
    W.H = H;
    W.cs = cs;
    W.sn = sn;
    W.g = g;
    W.yv = yv;
    memset(info, 0, sizeof(*info));
    const auto t0 = std::chrono::steady_clock::now();
    const mhk_status st = gmres(N, W, shift, rhs, x, tol, m, maxit, N->stream, info);
    if (st == MHK_OK) {
        // GMRES ends with the stream synchronised
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        info->ms_gmres = ms;
        info->ms_total = ms;
    }
    return st;
}

static mhk_status solve_common(mhk_plan *P, mhk_nystrom *N, int neumann, const double *g, const double *f_vol,
                               const double *f_trg, double tol, int restart, int maxit, double *dens, double *u,
                               mhk_solve_info *info)
{
    BIE_TRY(check_solve(P, N, g, f_vol, f_trg, tol, restart, maxit, dens, u));
    if (!info) {
        set_error("null solve info");
        return MHK_EINVAL;
    }
    memset(info, 0, sizeof(*info));
    hipStream_t st = P->stream;
    const int64_t nt = P->nt, nb = P->nb, nout = P->nout;
    BIE_TRY(nys_scratch(N, nout));
    OwnWs o;
    BIE_TRY(own_workspace(N, restart, o));
    double *w1 = N->work, *w2 = N->work + N->work_n;
    hipEvent_t ev[4] = {};
    for (auto &e : ev) BIE_HIP(hipEventCreate(&e));
    mhk_status rc = MHK_OK;
#define SOLVE_HIP(call)                                                                       \
    if ((call) != hipSuccess) {                                                               \
        set_error(std::string("HIP error in the boundary integral solve: ") + #call);         \
        rc = MHK_EHIP;                                                                        \
        break;                                                                                \
    }
    do {
        SOLVE_HIP(hipEventRecord(ev[0], st));
        // right-hand side: Dirichlet g - V on the boundary, Neumann V + S[g]
        if (neumann) {
            rc = mhk_eval_parts(P, MHK_PART_ALL, g, nullptr, f_vol, f_trg, w1, nullptr, f_vol ? u : nullptr);
            if (rc != MHK_OK) break;
            if (!f_vol) hipLaunchKernelGGL(k_fill, dim3(nb_of(nout)), dim3(BT), 0, st, nout, 0.0, u);
            hipLaunchKernelGGL(k_rhs, dim3(nb_of(nb)), dim3(BT), 0, st, nb, nt, 1.0, (const double *)u, 1.0,
                               (const double *)w1, o.W.rv);
        } else {
            if (f_vol) {
                rc = mhk_eval_parts(P, MHK_PART_ALL, nullptr, nullptr, f_vol, f_trg, nullptr, nullptr, u);
                if (rc != MHK_OK) break;
            } else {
                hipLaunchKernelGGL(k_fill, dim3(nb_of(nout)), dim3(BT), 0, st, nout, 0.0, u);
            }
            hipLaunchKernelGGL(k_rhs, dim3(nb_of(nb)), dim3(BT), 0, st, nb, (int64_t)0, 1.0, g, -1.0,
                               (const double *)(u + nt), o.W.rv);
        }
        SOLVE_HIP(hipGetLastError());
        SOLVE_HIP(hipEventRecord(ev[1], st));
        // GMRES on (-/+ 1/2 I + K); the right-hand side lives in the
        // residual vector, which GMRES overwrites, so it is first copied to w2
        SOLVE_HIP(hipMemcpyAsync(w2, o.W.rv, sizeof(double) * nb, hipMemcpyDeviceToDevice, st));
        rc = gmres(N, o.W, neumann ? 0.5 : -0.5, w2, dens, tol, restart, maxit, st, info);
        if (rc != MHK_OK) break;
        SOLVE_HIP(hipEventRecord(ev[2], st));
        // representation at every output
        rc = mhk_eval_parts(P, MHK_PART_ALL, nullptr, dens, nullptr, nullptr, nullptr, w2, nullptr);
        if (rc != MHK_OK) break;
        if (neumann)
            hipLaunchKernelGGL(k_neumann_u, dim3(nb_of(nout)), dim3(BT), 0, st, nt, nout, (const double *)w1,
                               (const double *)w2, (const double *)dens, u);
        else
            hipLaunchKernelGGL(k_dirichlet_u, dim3(nb_of(nout)), dim3(BT), 0, st, nt, nout, (const double *)w2,
                               (const double *)dens, u);
        SOLVE_HIP(hipGetLastError());
        SOLVE_HIP(hipEventRecord(ev[3], st));
        SOLVE_HIP(hipEventSynchronize(ev[3]));
        float a = 0, b = 0, c = 0;
        (void)hipEventElapsedTime(&a, ev[0], ev[1]);
        (void)hipEventElapsedTime(&b, ev[1], ev[2]);
        (void)hipEventElapsedTime(&c, ev[2], ev[3]);
        info->ms_eval = a + c;
        info->ms_gmres = b;
        info->ms_total = a + b + c;
    } while (0);
#undef SOLVE_HIP
    for (auto &e : ev) (void)hipEventDestroy(e);
    return rc;
}

mhk_status mhk_solve_dirichlet(mhk_plan *plan, mhk_nystrom *nys, const double *g, const double *f_vol,
                               const double *f_trg, double tol, int restart, int maxit, double *mu, double *u,
                               mhk_solve_info *info)
{
    return solve_common(plan, nys, 0, g, f_vol, f_trg, tol, restart, maxit, mu, u, info);
}

mhk_status mhk_solve_neumann(mhk_plan *plan, mhk_nystrom *nys, const double *g, const double *f_vol,
                             const double *f_trg, double tol, int restart, int maxit, double *u_b, double *u,
                             mhk_solve_info *info)
{
    return solve_common(plan, nys, 1, g, f_vol, f_trg, tol, restart, maxit, u_b, u, info);
}

mhk_status mhk_heat_step(mhk_plan *P, mhk_nystrom *N, const double *u_n, const double *F, const double *g_next,
                         double tol, int restart, int maxit, double *u_next, double *mu, mhk_solve_info *info)
{
    if (!P || !N || !u_n || !u_next || u_n == u_next) {
        set_error("null plan, Nystrom matrix or state, or u_n aliases u_next");
        return MHK_EINVAL;
    }
    if (!P->targets_are_volume) {
        set_error("the heat step needs a plan whose targets are its volume nodes, in the same order");
        return MHK_EINVAL;
    }
    BIE_TRY(check_solve(P, N, g_next, u_n, u_n, tol, restart, maxit, mu, u_next));
    const int64_t nout = P->nout;
    BIE_TRY(nys_scratch(N, nout));
    // f at the outputs (volume nodes, then boundary nodes) in the first
    // scratch half, which the Dirichlet solve leaves untouched; its first N_V
    // entries are f at the volume nodes
    double *f = N->work;
    hipLaunchKernelGGL(k_heat_source, dim3(nb_of(nout)), dim3(BT), 0, P->stream, nout, P->p.alpha * P->p.alpha,
                       u_n, F, f);
    BIE_HIP(hipGetLastError());
    return solve_common(P, N, 0, g_next, f, f, tol, restart, maxit, mu, u_next, info);
}

void mhk_nystrom_destroy(mhk_nystrom *N)
{
    if (!N) return;
    (void)hipStreamSynchronize(N->stream);
    nys_free_ws(N);
    nys_free(N, &N->K);
    nys_free(N, &N->work);
    (void)hipStreamSynchronize(N->stream);
    delete N;
}

}  // extern "C"
