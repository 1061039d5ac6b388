// Plan creation, parameter rules and evaluation driver of libmhk.
//
// Host-side work happens once per plan (geometry is static): parameter rules,
// dyadic child nodes, kernel tables, sorting of sources and targets into cell
// and tile order, the history grid and its FFT plans.  mhk_eval only enqueues
// device work on the plan's stream.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

#include <map>
#include <mutex>

#include "mhk_internal.h"

namespace mhk {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

#define MHK_HIP(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            set_error(std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_)); \
            return MHK_EHIP;                                                          \
        }                                                                             \
    } while (0)

#define MHK_FFT(call)                                                                 \
    do {                                                                              \
        rocfft_status s_ = (call);                                                    \
        if (s_ != rocfft_status_success) {                                            \
            set_error(std::string("rocFFT error ") + std::to_string((int)s_) + " in " + #call); \
            return MHK_EHIP;                                                          \
        }                                                                             \
    } while (0)

// ---------------------------------------------------------------------------
// Small numerical helpers (host)
// ---------------------------------------------------------------------------

// Gauss-Legendre nodes and weights on [-1, 1], ascending, by Newton's method
// on the Legendre polynomial P_n (three-term recurrence).
static void gauss_legendre(int n, std::vector<double> &t, std::vector<double> &w)
{
    t.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double x = cosl(M_PIl * (4 * i + 3) / (4 * n + 2));
        long double dp = 0;
        for (int it = 0; it < 64; ++it) {
            long double p0 = 1, p1 = x;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (p0 - x * p1) / (1 - x * x);
            long double dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        {
            long double p0 = 1, p1 = x;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (p0 - x * p1) / (1 - x * x);
        }
        double wi = (double)(2 / ((1 - x * x) * dp * dp));
        t[i] = -(double)x;
        t[n - 1 - i] = (double)x;
        w[i] = w[n - 1 - i] = wi;
    }
}

// Lagrange basis of the 16 Gauss-Legendre nodes at point s (barycentric form).
static void lagrange_row(const std::vector<double> &tn, const std::vector<long double> &lam,
                         double s, double *row)
{
    int n = (int)tn.size();
    for (int i = 0; i < n; ++i)
        if (s == tn[i]) {
            for (int k = 0; k < n; ++k) row[k] = (k == i);
            return;
        }
    long double den = 0;
    std::vector<long double> num(n);
    for (int i = 0; i < n; ++i) {
        num[i] = lam[i] / ((long double)s - tn[i]);
        den += num[i];
    }
    for (int i = 0; i < n; ++i) row[i] = (double)(num[i] / den);
}

// Exponential integral E1(x), x > 0 (series for x < 1, continued fraction else).
static double expint_e1(double x)
{
    if (x < 1.0) {
        double s = 0, term = 1;
        for (int k = 1; k < 60; ++k) {
            term *= -x / k;
            s += -term / k;
        }
        return -0.57721566490153286 - log(x) + s;
    }
    // Lentz's continued fraction for e^x E1(x)
    double b = x + 1, c = 1e300, d = 1 / b, h = d;
    for (int i = 1; i < 300; ++i) {
        double a = -(double)i * i;
        b += 2;
        d = 1 / (a * d + b);
        c = b + a / c;
        double del = c * d;
        h *= del;
        if (fabs(del - 1) < 1e-16) break;
    }
    return h * exp(-x);
}

// Time integral of the heat kernel over one dyadic interval in the variable u
// (t = delta_j e^{-u}, u in [0, ln 4]):
//   I_p(a, b) = int_0^{ln4} exp(-a e^u - b e^{-u}) e^{p u} du,
// so that K_j^S = I_0/(4 pi) and K_j^D = I_1/(8 pi delta_j) with
// a = r^2/(4 delta_j), b = alpha^2 delta_j (eqs. (diffker_s), (diffker_dlp)).
// Composite 16-point Gauss-Legendre on 12 panels.
struct LevelQuad {
    // nodes e^u and weights of the composite rule (12 panels of 16
    // Gauss-Legendre points on [0, ln 4]), formed once
    static constexpr int NQ = 12 * 16;
    double eu[NQ], ieu[NQ], wq[NQ];
    LevelQuad()
    {
        std::vector<double> t, w;
        gauss_legendre(16, t, w);
        const double hh = log(4.0) / 12;
        for (int p = 0; p < 12; ++p)
            for (int q = 0; q < 16; ++q) {
                const double u = hh * (p + 0.5 * (1 + t[q]));
                eu[p * 16 + q] = exp(u);
                ieu[p * 16 + q] = exp(-u);
                wq[p * 16 + q] = w[q] * 0.5 * hh;
            }
    }
    void eval(double a, double b, double &i0, double &i1) const
    {
        double s0 = 0, s1 = 0;
        for (int k = 0; k < NQ; ++k) {
            const double e = wq[k] * exp(-a * eu[k] - b * ieu[k]);
            s0 += e;
            s1 += e * eu[k];
        }
        i0 = s0;
        i1 = s1;
    }
};

// Kernel tables depend only on alpha^2 delta_j, the cut-off and the
// precision: plans created again for the same parameters (a moving geometry
// stepped in time) take them from this cache.
struct TableEntry {
    std::vector<double> tab;
    std::vector<float> tab7;
    double seg_inv = 0, tab_err = 0;
    int nseg = 0;
};
static std::mutex g_table_mu;
static std::map<std::array<uint64_t, 3>, TableEntry> g_tables;

static int64_t good_fft_size(int64_t nmin)
{
    int64_t m = (nmin + TILE - 1) / TILE;
    for (;; ++m) {
        int64_t r = m;
        for (int f : {2, 3, 5})
            while (r % f == 0) r /= f;
        if (r == 1) return m * TILE;
    }
}

static inline uint32_t spread_bits(uint32_t v)
{
    v &= 0xffff;
    v = (v | (v << 8)) & 0x00ff00ff;
    v = (v | (v << 4)) & 0x0f0f0f0f;
    v = (v | (v << 2)) & 0x33333333;
    v = (v | (v << 1)) & 0x55555555;
    return v;
}
static inline uint32_t morton(uint32_t x, uint32_t y) { return spread_bits(x) | (spread_bits(y) << 1); }


// ---------------------------------------------------------------------------
// Parameter rules
// ---------------------------------------------------------------------------
// Truncation target of the history part (multiplier cut-off and window
// width): the requested tolerance at both precisions; the FP32 rounding of
// the spreading, transforms and interpolation stays well below it.
static double hist_eps(const mhk_params &p) { return p.tol; }

static mhk_status resolve(const mhk_params *pp, mhk_info *I, mhk_params *out)
{
    if (!pp || !I) {
        set_error("null params/info");
        return MHK_EINVAL;
    }
    mhk_params p = *pp;
    if (!(p.alpha > 0) || !std::isfinite(p.alpha)) {
        set_error("alpha must be positive and finite");
        return MHK_EINVAL;
    }
    if (!(p.tol >= 1e-13 && p.tol <= 1e-3)) {
        set_error("tol must be in [1e-13, 1e-3]");
        return MHK_EINVAL;
    }
    if (p.prec != MHK_FP64 && p.prec != MHK_FP32) {
        set_error("prec must be MHK_FP64 or MHK_FP32");
        return MHK_EINVAL;
    }
    if (p.prec == MHK_FP32 && p.tol < 1e-7) {
        set_error("the FP32 path needs tol >= 1e-7");
        return MHK_EINVAL;
    }
    if (p.J < 0) p.J = 3;
    if (p.J > MAXJ) {
        set_error("J must be <= 8");
        return MHK_EINVAL;
    }
    if (p.batch < 1) {
        set_error("batch must be >= 1");
        return MHK_EINVAL;
    }
    if (!(p.delta > 0)) {
        if (!(p.dx > 0)) {
            set_error("either delta or dx must be positive");
            return MHK_EINVAL;
        }
        // Section 6.4: k_max = 0.9 k_Nyq with k_Nyq = pi/dx (eq. (k_nyq)), and
        // delta the smallest split with exp(-delta(alpha^2 + k_max^2)) = tol.
        double kmax = 0.9 * M_PI / p.dx;
        p.delta = log(1.0 / p.tol) / (kmax * kmax + p.alpha * p.alpha);
    }
    if (p.in64 != 0 && p.in64 != 1) {
        set_error("in64 must be 0 or 1");
        return MHK_EINVAL;
    }
    if (p.prec == MHK_FP64) p.in64 = 0;
    if (p.lv_block == 0) p.lv_block = 256;
    if (p.lv_block != 256 && p.lv_block != 512) {
        set_error("lv_block must be 0, 256 or 512");
        return MHK_EINVAL;
    }
    if (p.lv_persist != 0 && p.lv_persist != 1) {
        set_error("lv_persist must be 0 or 1");
        return MHK_EINVAL;
    }
    if (p.lv_bch == 0) p.lv_bch = 4;
    if (p.lv_bch != 1 && p.lv_bch != 2 && p.lv_bch != 4 && p.lv_bch != 8) {
        set_error("lv_bch must be 0, 1, 2, 4 or 8");
        return MHK_EINVAL;
    }
    if (p.local_order == 0) p.local_order = 1;
    if (p.local_order != 1 && p.local_order != 2) {
        set_error("local_order must be 0, 1 or 2");
        return MHK_EINVAL;
    }
    if (p.upsamp <= 0) p.upsamp = 2.0;
    if (p.upsamp < 1.25 || p.upsamp > 3.0) {
        set_error("upsamp must be in [1.25, 3]");
        return MHK_EINVAL;
    }
    if (p.wspread < 0 || p.wspread > MAXW || (p.wspread > 0 && p.wspread < 4)) {
        set_error("wspread must be 0 or in [4, 16]");
        return MHK_EINVAL;
    }
    memset(I, 0, sizeof(*I));
    I->alpha = p.alpha;
    I->tol = p.tol;
    I->delta = p.delta;
    I->J = p.J;
    I->delta_star = p.delta / pow(4.0, p.J);
    I->prec = p.prec;
    I->batch = p.batch;
    if (p.v_levels != 0 && p.v_levels != 1) {
        set_error("v_levels must be 0 or 1");
        return MHK_EINVAL;
    }
    if (p.v_levels && p.J < 1) {
        set_error("v_levels needs J >= 1");
        return MHK_EINVAL;
    }
    // V's local part: delta, or delta* when V has the dyadic levels too
    double sq = sqrt(I->delta_star), sv = sqrt(p.v_levels ? I->delta_star : p.delta);
    // Remark 4.3: the local layer part is negligible beyond sqrt(d*)(12 + 2 alpha sqrt(d*))
    I->band_layer = sq * (12.0 + 2.0 * p.alpha * sq);
    I->band_volume = sv * (12.0 + 2.0 * p.alpha * sv);
    // level cut-off: K_j decays like exp(-a)/a, so the sources beyond a_max =
    // ln(1/tol) + 3 add up to ~1e-3 tol of the level sum (measured on the
    // 10-body workload at tol 1e-10: 1.3e-13 of max |S_j|)
    double amax = std::min(40.5, log(1.0 / p.tol) + 3.0);
    for (int j = 1; j <= p.J; ++j) {
        double dj = p.delta / pow(4.0, j - 1);
        I->level_radius[j - 1] = sqrt(4.0 * dj * amax);
    }
    // Fourier cut-off of the history part (eqs. (kmax), (kmax_dlp)) at eps =
    // tol at both precisions (hist_eps): the truncation error is far below
    // tol relative to the potentials, and the FP32 rounding of the history
    // stages stays below it as well
    double eps = hist_eps(p), L = log(1.0 / eps), da2 = p.delta * p.alpha * p.alpha;
    if (da2 >= L) {
        I->kmax = 0;
    } else {
        double k = sqrt((L - da2) / p.delta);
        for (int it = 0; it < 50; ++it) {
            double kn = sqrt(std::max(0.0, (log(std::max(k, 1.0) / eps) - da2) / p.delta));
            if (fabs(kn - k) < 1e-12 * k) {
                k = kn;
                break;
            }
            k = kn;
        }
        I->kmax = k;
    }
    if (p.wspread == 0) {
        double ew = hist_eps(p);
        int w = (int)ceil(log(1.0 / ew) / (M_PI * sqrt(1.0 - 1.0 / p.upsamp))) + 1;
        p.wspread = std::min(MAXW, std::max(4, w));
    }
    I->wspread = p.wspread;
    if (out) *out = p;
    return MHK_OK;
}

}  // namespace mhk

using namespace mhk;

// ---------------------------------------------------------------------------
// Allocation helper
// ---------------------------------------------------------------------------
// Plan buffers are allocated and freed in the order of the plan's stream
// (stream-ordered allocation): hipFree would wait for every stream of the
// device, so destroying or building a plan would drain the work of other
// plans running beside it.
template <typename T>
static mhk_status dalloc(mhk_plan *P, T **ptr, int64_t count)
{
    *ptr = nullptr;
    if (count <= 0) count = 1;
    size_t bytes = sizeof(T) * (size_t)count;
    hipError_t e = hipMallocAsync((void **)ptr, bytes, P->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
        return MHK_ENOMEM;
    }
    P->allocs.push_back(*ptr);
    P->bytes += (int64_t)bytes;
    return MHK_OK;
}

// Host data copied into a plan buffer, in the order of the plan's stream; the
// host bytes are staged in the plan until creation has synchronised its
// stream.
template <typename T>
static mhk_status upload(mhk_plan *P, T **ptr, const T *host, int64_t count)
{
    mhk_status s = dalloc(P, ptr, count);
    if (s != MHK_OK) return s;
    if (count > 0) {
        const size_t bytes = sizeof(T) * (size_t)count;
        P->stage.emplace_back((const char *)host, (const char *)host + bytes);
        MHK_HIP(hipMemcpyAsync(*ptr, P->stage.back().data(), bytes, hipMemcpyHostToDevice, P->stream));
    }
    return MHK_OK;
}

#define TRY(x)                          \
    do {                                \
        mhk_status st_ = (x);           \
        if (st_ != MHK_OK) return st_;  \
    } while (0)

// Temporaries of plan creation, allocated and freed in the order of the
// plan's stream (hipFree would wait for the whole device, i.e. for other
// plans' work).  Host data uploaded through upload() must stay alive until
// the stream has been synchronised.
struct StreamTmp {
    hipStream_t st;
    std::vector<void *> ptrs;
    explicit StreamTmp(hipStream_t s) : st(s) {}
    StreamTmp(const StreamTmp &) = delete;
    StreamTmp &operator=(const StreamTmp &) = delete;
    ~StreamTmp()
    {
        for (void *q : ptrs) (void)hipFreeAsync(q, st);
    }
    template <typename T>
    mhk_status alloc(T **ptr, int64_t n)
    {
        *ptr = nullptr;
        if (hipMallocAsync((void **)ptr, sizeof(T) * (size_t)std::max<int64_t>(1, n), st) != hipSuccess) {
            (void)hipGetLastError();
            set_error("temporary device allocation of plan creation failed");
            return MHK_ENOMEM;
        }
        ptrs.push_back(*ptr);
        return MHK_OK;
    }
    template <typename T>
    mhk_status upload(T **ptr, const T *host, int64_t n)
    {
        TRY(alloc(ptr, n));
        if (n > 0) MHK_HIP(hipMemcpyAsync(*ptr, host, sizeof(T) * (size_t)n, hipMemcpyHostToDevice, st));
        return MHK_OK;
    }
    // device -> host copy of a few values, waiting for the stream
    template <typename T>
    mhk_status fetch(T *host, const T *dev, int64_t n)
    {
        MHK_HIP(hipMemcpyAsync(host, dev, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost, st));
        MHK_HIP(hipStreamSynchronize(st));
        return MHK_OK;
    }
};

static void free_plan(mhk_plan *P)
{
    if (!P) return;
    // uploads of a failed creation may still read the staged host bytes
    if (!P->stage.empty()) (void)hipStreamSynchronize(P->stream);
    // stream-ordered frees: after the plan's queued work, without waiting
    // for other streams
    for (void *p : P->allocs) (void)hipFreeAsync(p, P->stream);
    if (P->hist.fwd) rocfft_plan_destroy(P->hist.fwd);
    if (P->hist.inv) rocfft_plan_destroy(P->hist.inv);
    if (P->hist.exec) rocfft_execution_info_destroy(P->hist.exec);
    for (auto &e : P->ev)
        if (e) (void)hipEventDestroy(e);
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->cap) (void)hipStreamDestroy(P->cap);
    if (P->fork_ev) (void)hipEventDestroy(P->fork_ev);
    if (P->join_ev) (void)hipEventDestroy(P->join_ev);
    if (P->side) (void)hipStreamDestroy(P->side);
    delete P;
}

// rocFFT's one-time setup, once per process even when plans are created
// from several threads at a time
static std::once_flag g_rocfft_once;
static rocfft_status g_rocfft_setup = rocfft_status_success;
static rocfft_status rocfft_ready()
{
    std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
    return g_rocfft_setup;
}

// ---------------------------------------------------------------------------
// Plan construction
// ---------------------------------------------------------------------------
namespace {

struct Host {
    const mhk_boundary *b;
    const mhk_volume *v;
    const mhk_targets *t;
    std::vector<double> gl_t, gl_w;
    std::vector<long double> bary;
    std::vector<int64_t> prev, next;
    double xmin, xmax, ymin, ymax;
    // all targets (off-surface then boundary), in output order
    std::vector<double> tx, ty;
    std::vector<int8_t> tin;
    bool mask_needed = false;          // no caller mask: computed on the device
    // host side of the computed mask (kept until plan creation ends, as the
    // uploads read them asynchronously)
    std::vector<double> m_edge, m_sag, m_et, m_glt, m_lam;
    std::vector<int32_t> m_pan, m_start, m_list;
};

mhk_status check_inputs(const mhk_params *p, const mhk_boundary *b, const mhk_volume *v,
                        const mhk_targets *t)
{
    if (!p || !b) {
        set_error("params and boundary are required");
        return MHK_EINVAL;
    }
    if (b->n_panels < 1 || b->n_curves < 1 || !b->curve_panel_ofs || !b->x || !b->y || !b->nx ||
        !b->ny || !b->w || !b->kappa) {
        set_error("boundary arrays missing or empty");
        return MHK_EINVAL;
    }
    if (b->n_panels * NGL > (int64_t)1 << 26) {
        set_error("too many boundary nodes");
        return MHK_EINVAL;
    }
    if (b->curve_panel_ofs[0] != 0 || b->curve_panel_ofs[b->n_curves] != b->n_panels) {
        set_error("curve_panel_ofs must start at 0 and end at n_panels");
        return MHK_EINVAL;
    }
    for (int c = 0; c < b->n_curves; ++c)
        if (b->curve_panel_ofs[c + 1] - b->curve_panel_ofs[c] < 2) {
            set_error("every curve needs at least 2 panels");
            return MHK_EINVAL;
        }
    int64_t nb = b->n_panels * NGL;
    for (int64_t i = 0; i < nb; ++i)
        if (!std::isfinite(b->x[i]) || !std::isfinite(b->y[i]) || !std::isfinite(b->w[i]) ||
            !std::isfinite(b->nx[i]) || !std::isfinite(b->ny[i]) || !std::isfinite(b->kappa[i])) {
            set_error("non-finite boundary data");
            return MHK_EINVAL;
        }
    if (v && v->n < 0) {
        set_error("negative volume size");
        return MHK_EINVAL;
    }
    if (v && v->group != 0 && (v->group != 6 || v->n % 6 != 0)) {
        set_error("volume group must be 0 or 6 (with a multiple of 6 nodes)");
        return MHK_EINVAL;
    }
    if (v && v->n > 0) {
        if (!v->x || !v->y || !v->w || v->n > (int64_t)1 << 30) {
            set_error("volume arrays missing or too large");
            return MHK_EINVAL;
        }
        for (int64_t i = 0; i < v->n; ++i)
            if (!std::isfinite(v->x[i]) || !std::isfinite(v->y[i]) || !std::isfinite(v->w[i])) {
                set_error("non-finite volume data");
                return MHK_EINVAL;
            }
    }
    if (!t || t->n < 0 || (t->n > 0 && (!t->x || !t->y))) {
        set_error("targets missing");
        return MHK_EINVAL;
    }
    if (t->n + (t->on_surface ? nb : 0) < 1) {
        set_error("no targets");
        return MHK_EINVAL;
    }
    if (t->n + nb > (int64_t)1 << 30) {
        set_error("too many targets");
        return MHK_EINVAL;
    }
    for (int64_t i = 0; i < t->n; ++i)
        if (!std::isfinite(t->x[i]) || !std::isfinite(t->y[i])) {
            set_error("non-finite target");
            return MHK_EINVAL;
        }
    return MHK_OK;
}

void host_common(Host &H)
{
    gauss_legendre(NGL, H.gl_t, H.gl_w);
    H.bary.assign(NGL, 0);
    for (int i = 0; i < NGL; ++i) {
        long double pr = 1;
        for (int k = 0; k < NGL; ++k)
            if (k != i) pr *= ((long double)H.gl_t[i] - H.gl_t[k]);
        H.bary[i] = 1 / pr;
    }
    const mhk_boundary *b = H.b;
    H.prev.assign(b->n_panels, 0);
    H.next.assign(b->n_panels, 0);
    for (int c = 0; c < b->n_curves; ++c) {
        int64_t a = b->curve_panel_ofs[c], e = b->curve_panel_ofs[c + 1], m = e - a;
        for (int64_t q = 0; q < m; ++q) {
            H.prev[a + q] = a + (q + m - 1) % m;
            H.next[a + q] = a + (q + 1) % m;
        }
    }
    int64_t nb = b->n_panels * NGL;
    int64_t nt = H.t->n, nout = nt + (H.t->on_surface ? nb : 0);
    H.tx.resize(nout);
    H.ty.resize(nout);
    H.tin.resize(nout);
    for (int64_t i = 0; i < nt; ++i) {
        H.tx[i] = H.t->x[i];
        H.ty[i] = H.t->y[i];
        H.tin[i] = H.t->inside ? (H.t->inside[i] ? 1 : 0) : 0;
    }
    H.mask_needed = nt > 0 && !H.t->inside;
    for (int64_t i = nt; i < nout; ++i) {
        H.tx[i] = b->x[i - nt];
        H.ty[i] = b->y[i - nt];
        H.tin[i] = 1;
    }
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
    auto acc = [&](double x, double y) {
        x0 = std::min(x0, x); x1 = std::max(x1, x);
        y0 = std::min(y0, y); y1 = std::max(y1, y);
    };
    for (int64_t i = 0; i < nb; ++i) acc(b->x[i], b->y[i]);
    if (H.v)
        for (int64_t i = 0; i < H.v->n; ++i) acc(H.v->x[i], H.v->y[i]);
    for (int64_t i = 0; i < nout; ++i) acc(H.tx[i], H.ty[i]);
    H.xmin = x0; H.xmax = x1; H.ymin = y0; H.ymax = y1;
}

// Inside mask of the off-surface targets when the caller passes none: the
// polygon through every panel's end points and 16 nodes, closed along each
// curve, with a bound of each edge's arc-to-chord deviation for the lune
// correction, edges listed per horizontal strip; the kernel writes the mask
// of the first N_T entries of rin (caller order).
static mhk_status build_mask(mhk_plan *P, Host &H, StreamTmp &tmp, int8_t *rin)
{
    const mhk_boundary *b = H.b;
    const int64_t npan = b->n_panels;
    std::vector<double> row(NGL);
    auto eval = [&](int64_t p, double t, double &x, double &y) {
        lagrange_row(H.gl_t, H.bary, t, row.data());
        x = y = 0;
        for (int i = 0; i < NGL; ++i) {
            x += row[i] * b->x[p * NGL + i];
            y += row[i] * b->y[p * NGL + i];
        }
    };
    // per panel: vertices gamma(-1), nodes, gamma(1); the edges between them
    // carry lunes; gamma_p(1) -> gamma_next(-1) closes the gap between panels
    std::vector<double> &E = H.m_edge, &SG = H.m_sag, &ET = H.m_et;
    std::vector<int32_t> &EP = H.m_pan;
    std::vector<double> ends(npan * 4);
    for (int64_t p = 0; p < npan; ++p) {
        eval(p, -1.0, ends[p * 4 + 0], ends[p * 4 + 1]);
        eval(p, 1.0, ends[p * 4 + 2], ends[p * 4 + 3]);
    }
    const int64_t nedge = npan * (NGL + 2);
    E.reserve(nedge * 4);
    SG.reserve(nedge);
    ET.reserve(nedge * 2);
    EP.reserve(nedge);
    double ylo = 1e300, yhi = -1e300;
    for (int64_t p = 0; p < npan; ++p) {
        double vx[NGL + 2], vy[NGL + 2], vt[NGL + 2];
        vx[0] = ends[p * 4 + 0]; vy[0] = ends[p * 4 + 1]; vt[0] = -1.0;
        for (int i = 0; i < NGL; ++i) {
            vx[i + 1] = b->x[p * NGL + i];
            vy[i + 1] = b->y[p * NGL + i];
            vt[i + 1] = H.gl_t[i];
        }
        vx[NGL + 1] = ends[p * 4 + 2]; vy[NGL + 1] = ends[p * 4 + 3]; vt[NGL + 1] = 1.0;
        for (int k = 0; k <= NGL + 1; ++k) {
            double x0, y0, x1, y1, sag = 0.0, t0 = 0.0, t1 = 0.0;
            if (k <= NGL) {
                x0 = vx[k]; y0 = vy[k]; x1 = vx[k + 1]; y1 = vy[k + 1];
                t0 = vt[k]; t1 = vt[k + 1];
                // the arc's largest distance from the chord at 15 interior
                // points, doubled, plus a rounding margin
                const double ex = x1 - x0, ey = y1 - y0, l = std::hypot(ex, ey);
                double dev = 0.0;
                for (int m = 1; m < 16; ++m) {
                    double ax, ay;
                    eval(p, t0 + (t1 - t0) * m / 16.0, ax, ay);
                    dev = std::max(dev, std::fabs(ex * (ay - y0) - ey * (ax - x0)) / l);
                }
                sag = 2.0 * dev + 1e-14 * (std::fabs(x0) + std::fabs(y0) + l);
            } else {
                const int64_t q = H.next[p];
                x0 = vx[NGL + 1]; y0 = vy[NGL + 1]; x1 = ends[q * 4 + 0]; y1 = ends[q * 4 + 1];
            }
            E.insert(E.end(), {x0, y0, x1, y1});
            SG.push_back(sag);
            ET.push_back(t0);
            ET.push_back(t1);
            EP.push_back((int32_t)p);
            ylo = std::min(ylo, std::min(y0, y1) - sag);
            yhi = std::max(yhi, std::max(y0, y1) + sag);
        }
    }
    const int64_t ne = (int64_t)SG.size();
    const int nstrip = (int)std::max<int64_t>(1, std::min<int64_t>(1 << 20, ne / 4));
    yhi = std::nextafter(yhi, 1e300);
    const double hinv = nstrip / (yhi - ylo);
    auto strip = [&](double y) { return (int64_t)std::min<double>(nstrip - 1, std::max(0.0, std::floor((y - ylo) * hinv))); };
    std::vector<int32_t> &st = H.m_start, &li = H.m_list;
    st.assign(nstrip + 1, 0);
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t s0 = std::max<int64_t>(0, strip(std::min(E[e * 4 + 1], E[e * 4 + 3]) - SG[e]) - 1);
        const int64_t s1 = std::min<int64_t>(nstrip - 1, strip(std::max(E[e * 4 + 1], E[e * 4 + 3]) + SG[e]) + 1);
        for (int64_t s = s0; s <= s1; ++s) ++st[s + 1];
    }
    for (int s = 0; s < nstrip; ++s) st[s + 1] += st[s];
    li.assign(st[nstrip], 0);
    {
        std::vector<int32_t> fill(st.begin(), st.end() - 1);
        for (int64_t e = 0; e < ne; ++e) {
            const int64_t s0 = std::max<int64_t>(0, strip(std::min(E[e * 4 + 1], E[e * 4 + 3]) - SG[e]) - 1);
            const int64_t s1 = std::min<int64_t>(nstrip - 1, strip(std::max(E[e * 4 + 1], E[e * 4 + 3]) + SG[e]) + 1);
            for (int64_t s = s0; s <= s1; ++s) li[fill[s]++] = (int32_t)e;
        }
    }
    H.m_glt.assign(H.gl_t.begin(), H.gl_t.end());
    H.m_lam.resize(NGL);
    for (int i = 0; i < NGL; ++i) H.m_lam[i] = (double)H.bary[i];
    MaskArgs A{};
    A.n = H.t->n;
    A.ylo = ylo;
    A.yhi = yhi;
    A.hinv = hinv;
    A.nstrip = nstrip;
    double *tx = nullptr, *ty = nullptr, *edge = nullptr, *sag = nullptr, *et = nullptr, *bx = nullptr,
           *by = nullptr, *glt = nullptr, *lam = nullptr;
    int32_t *sst = nullptr, *sli = nullptr, *pan = nullptr;
    TRY(tmp.upload(&tx, H.tx.data(), A.n));
    TRY(tmp.upload(&ty, H.ty.data(), A.n));
    TRY(tmp.upload(&edge, E.data(), ne * 4));
    TRY(tmp.upload(&sag, SG.data(), ne));
    TRY(tmp.upload(&et, ET.data(), ne * 2));
    TRY(tmp.upload(&pan, EP.data(), ne));
    TRY(tmp.upload(&sst, st.data(), (int64_t)st.size()));
    TRY(tmp.upload(&sli, li.data(), (int64_t)li.size()));
    TRY(tmp.upload(&bx, b->x, npan * NGL));
    TRY(tmp.upload(&by, b->y, npan * NGL));
    TRY(tmp.upload(&glt, H.m_glt.data(), NGL));
    TRY(tmp.upload(&lam, H.m_lam.data(), NGL));
    A.tx = tx; A.ty = ty; A.edge = edge; A.sag = sag; A.edge_t = et; A.edge_pan = pan;
    A.strip_start = sst; A.strip_edge = sli; A.bx = bx; A.by = by; A.gl_t = glt; A.lam = lam;
    MHK_HIP(dev_inside_mask(A, rin, P->stream));
    return MHK_OK;
}

// Dyadic level j (Section 4.2): every panel bisected j times; child nodes are
// the 16-point Gauss-Legendre nodes of each child interval, with geometry
// interpolated by the parent's degree-15 polynomial, normals renormalised,
// and weights w_GL,child * speed * 2^-j.
mhk_status build_level(mhk_plan *P, Host &H, int j)
{
    Level &L = P->lev[j - 1];
    const mhk_boundary *b = H.b;
    const int64_t npan = b->n_panels;
    const hipStream_t st = P->stream;
    L.nchild = 1 << j;
    L.n_src = npan * L.nchild * NGL;
    L.delta_j = P->delta / pow(4.0, j - 1);
    L.inv4d = 1.0 / (4.0 * L.delta_j);
    L.radius = P->info.level_radius[j - 1];
    L.a_max = L.radius * L.radius * L.inv4d;
    const int nch = L.nchild;
    // interpolation rows: child c, node k -> 16 parent weights
    std::vector<double> T((size_t)nch * NGL * NGL);
    for (int c = 0; c < nch; ++c)
        for (int k = 0; k < NGL; ++k) {
            double s = -1.0 + (2.0 * c + 1.0 + H.gl_t[k]) / nch;
            lagrange_row(H.gl_t, H.bary, s, &T[((size_t)c * NGL + k) * NGL]);
        }
    TRY(upload(P, &L.interp, T.data(), (int64_t)T.size()));
    // cells of side R_j / LV_CDIV over the bounding box of sources and targets
    L.cell = L.radius / LV_CDIV;
    L.ox = H.xmin - 1e-9;
    L.oy = H.ymin - 1e-9;
    int64_t ncx = (int64_t)floor((H.xmax - L.ox) / L.cell) + 1;
    int64_t ncy = (int64_t)floor((H.ymax - L.oy) / L.cell) + 1;
    if (ncx * ncy > (int64_t)1 << 26) {
        set_error("level cell grid too large (delta too small for the domain)");
        return MHK_EUNSUPPORTED;
    }
    L.ncx = (int)ncx;
    L.ncy = (int)ncy;
    // child nodes (geometry interpolated from the parent panels), sorted by
    // cell on the device
    TRY(dalloc(P, &L.sx, L.n_src));
    TRY(dalloc(P, &L.sy, L.n_src));
    TRY(dalloc(P, &L.sw, L.n_src));
    TRY(dalloc(P, &L.swx, L.n_src));
    TRY(dalloc(P, &L.swy, L.n_src));
    TRY(dalloc(P, &L.code, L.n_src));
    TRY(dalloc(P, &L.cell_start, ncx * ncy + 1));
    StreamTmp tmp(st);
    double *glw = nullptr;
    TRY(tmp.upload(&glw, H.gl_w.data(), NGL));
    MHK_HIP(dev_child_nodes(L.n_src, nch, L.interp, P->bx, P->by, P->bnx, P->bny, P->bw, glw, L.ox, L.oy, L.cell,
                            ncx, ncy, L.sx, L.sy, L.sw, L.swx, L.swy, L.code, L.cell_start, st));
    // per wavefront of LV_WAVE targets: the sources within R_j of the
    // wavefront's target bounding box (flat lists, counted, scanned, then
    // filled on the device); wavefronts past the last target get empty lists
    {
        const int64_t nout = P->nout;
        // padded to whole workgroups of the larger tile shape, so that
        // either one launches exactly nwave wavefronts
        const int64_t nwave = ((nout + LV_BLOCK_MAX - 1) / LV_BLOCK_MAX) * (LV_BLOCK_MAX / LV_WAVE);
        L.n_wave = nwave;
        const double R = L.radius, R2 = R * R * (1.0 + 1e-9);
        int32_t *cnt = nullptr;
        int64_t *tot = nullptr;
        TRY(tmp.alloc(&cnt, nwave));
        TRY(tmp.alloc(&tot, 1));
        TRY(dalloc(P, &L.wave_ofs, nwave + 1));
        TRY(dalloc(P, &L.wave_order, nwave));
        MHK_HIP(dev_wave_counts(P->tx, P->ty, nout, nwave, R, R2, L.ox, L.oy, L.cell, ncx, ncy, L.cell_start, L.sx,
                                L.sy, cnt, st));
        MHK_HIP(dev_scan(cnt, L.wave_ofs, nwave, tot, st));
        int64_t total = 0;
        TRY(tmp.fetch(&total, tot, 1));
        if (total > (int64_t)INT32_MAX) {
            set_error("level candidate lists too large");
            return MHK_EUNSUPPORTED;
        }
        L.n_cand = total;
        TRY(dalloc(P, &L.wave_src, std::max<int64_t>(1, total)));
        MHK_HIP(dev_wave_fill(P->tx, P->ty, nout, nwave, R, R2, L.ox, L.oy, L.cell, ncx, ncy, L.cell_start, L.sx,
                              L.sy, L.wave_ofs, L.wave_src, L.wave_order, st));
    }
    {
        char *q = nullptr;
        TRY(dalloc(P, &q, 3 * (int64_t)P->p.batch * L.n_src * (int64_t)P->es));
        L.q = q;
    }

    // Kernel table: piecewise polynomials in a = r^2/(4 delta_j), each in the
    // local variable v in [-1, 1] of its segment; coefficients from Chebyshev
    // interpolation converted to monomials in v.  Only K_j^S is tabulated:
    // with K_j^S = cS I0(a) and K_j^D = cD I1(a), where I1 = -dI0/da (the
    // a-derivative of exp(-a e^u) brings down -e^u), K_j^D = -(1/(2 delta_j))
    // dK_j^S/da, which the level sums take from the derivative of the same
    // polynomial (one LDS table read per coefficient serves both kernels).
    // FP64 path: degree 7 on segments of 1/16 (S ~1e-15, D ~3e-13 of the
    // kernels at a = 0), c_0..c_4 stored as doubles and c_5..c_7 as floats:
    // relative to K_j(0) the high coefficients are below 4e-8, so their
    // rounding and an FP32 Horner pass over them cost ~1e-15 of K_j(0)
    // (c_4, ~2e-6, would cost ~1e-13 of K_j(0) and up to ~6e-13 of K_j^D(0)
    // through the derivative), and each pair reads 52 bytes of table
    // instead of 64.  FP32 path: degree 7 on segments of 1/4, stored as
    // floats.
    LevelQuad Q;
    const double b_j = P->p.alpha * P->p.alpha * L.delta_j;
    const double cS = 1.0 / (4.0 * M_PI), cD = 1.0 / (8.0 * M_PI * L.delta_j);
    const bool fp64 = P->p.prec == MHK_FP64;
    const int nc = fp64 ? TAB_NC : TABF_NC, stride = fp64 ? TAB_STRIDE : TABF_STRIDE;
    const double tab_tol = fp64 ? 1e-12 : 1e-8;
    std::vector<double> tab;
    std::vector<float> tab7;         // FP64 path: c_7 of each segment
    std::array<uint64_t, 3> tkey{};
    {
        uint64_t kb, ka;
        memcpy(&kb, &b_j, 8);
        memcpy(&ka, &L.a_max, 8);
        tkey = {kb, ka, (uint64_t)fp64};
    }
    bool cached = false;
    {
        std::lock_guard<std::mutex> lock(g_table_mu);
        auto it = g_tables.find(tkey);
        if (it != g_tables.end()) {
            tab = it->second.tab;
            tab7 = it->second.tab7;
            L.seg_inv = it->second.seg_inv;
            L.nseg = it->second.nseg;
            L.tab_err = it->second.tab_err;
            cached = true;
        }
    }
    // segment width halved while the table (or its derivative) misses tab_tol
    // (large alpha^2 delta_j makes K_j decay like e^{-4a})
    for (double seg_w = fp64 ? 0.0625 : 0.25; !cached; seg_w *= 0.5) {
        L.seg_inv = 1.0 / seg_w;
        L.nseg = (int)ceil(L.a_max / seg_w) + 1;
        tab.assign((size_t)L.nseg * stride, 0.0);
        tab7.assign((size_t)L.nseg, 0.0f);
        std::vector<double> node(nc);
        for (int i = 0; i < nc; ++i) node[i] = cos(M_PI * (i + 0.5) / nc);
        for (int sgi = 0; sgi < L.nseg; ++sgi) {
            double a0 = sgi * seg_w;
            std::vector<long double> f(nc);
            for (int i = 0; i < nc; ++i) {
                double a = a0 + 0.5 * seg_w * (1.0 + node[i]);
                double i0, i1;
                Q.eval(a, b_j, i0, i1);
                f[i] = i0 * cS;
            }
            // Chebyshev coefficients
            std::vector<long double> ch(nc, 0);
            for (int m = 0; m < nc; ++m) {
                long double sacc = 0;
                for (int i = 0; i < nc; ++i) sacc += f[i] * cosl(M_PIl * m * (i + 0.5L) / nc);
                ch[m] = sacc * (m == 0 ? 1.0L : 2.0L) / nc;
            }
            // T_m(v) -> monomials in v
            std::vector<long double> mono(nc, 0), tprev(nc, 0), tcur(nc, 0), tnext(nc, 0);
            tprev[0] = 1;       // T0
            tcur[1] = 1;        // T1
            for (int k = 0; k < nc; ++k) mono[k] += ch[0] * tprev[k];
            for (int k = 0; k < nc; ++k) mono[k] += ch[1] * tcur[k];
            for (int m = 2; m < nc; ++m) {
                std::fill(tnext.begin(), tnext.end(), 0.0L);
                for (int k = 0; k < nc; ++k) {
                    if (k + 1 < nc) tnext[k + 1] += 2 * tcur[k];
                    tnext[k] -= tprev[k];
                }
                for (int k = 0; k < nc; ++k) mono[k] += ch[m] * tnext[k];
                tprev = tcur;
                tcur = tnext;
            }
            double *row = &tab[(size_t)sgi * stride];
            if (fp64) {
                for (int k = 0; k < TAB_NC64; ++k) row[k] = (double)mono[k];
                const float hi[2] = {(float)mono[TAB_NC64], (float)mono[TAB_NC64 + 1]};
                memcpy(row + TAB_NC64, hi, sizeof hi);
                tab7[sgi] = (float)mono[TAB_NC - 1];
            } else {
                for (int k = 0; k < nc; ++k) row[k] = (double)mono[k];
            }
        }
        // accuracy check of the table and of its derivative against direct
        // quadrature, in the arithmetic of the device evaluation
        double k0S, k0D;
        Q.eval(0.0, b_j, k0S, k0D);
        k0S *= cS;
        k0D *= cD;
        const double dscale = level_d_scale(L);
        double emax = 0;
        for (int i = 0; i < 997; ++i) {
            double a = L.a_max * (i + 0.37) / 997.0;
            double i0, i1;
            Q.eval(a, b_j, i0, i1);
            int sgi = (int)(a * L.seg_inv);
            double v = 2.0 * (a * L.seg_inv - sgi) - 1.0;
            const double *c = &tab[(size_t)sgi * stride];
            double pS, dS;
            if (fp64) {
                // the device's order: Horner over c_7..c_5 in FP32, then c_4..c_0 in FP64
                float hi[TAB_NC - TAB_NC64];
                memcpy(hi, c + TAB_NC64, 2 * sizeof(float));
                hi[2] = tab7[sgi];
                const float vf = (float)v;
                float kd = hi[2], ks = fmaf(kd, vf, hi[1]);
                kd = fmaf(kd, vf, ks);
                ks = fmaf(ks, vf, hi[0]);
                pS = ks;
                dS = kd;
                for (int k = TAB_NC64 - 1; k >= 0; --k) {
                    dS = fma(dS, v, pS);
                    pS = fma(pS, v, c[k]);
                }
            } else {
                // the FP32 path evaluates in float; its bound (1e-8) leaves room for that
                pS = c[nc - 1];
                dS = 0;
                for (int k = nc - 2; k >= 0; --k) {
                    dS = dS * v + pS;
                    pS = pS * v + c[k];
                }
            }
            emax = std::max(emax, fabs(pS - i0 * cS) / k0S);
            emax = std::max(emax, fabs(dS * dscale - i1 * cD) / k0D);
        }
        L.tab_err = emax;
        if (emax <= tab_tol) {
            std::lock_guard<std::mutex> lock(g_table_mu);
            if (g_tables.size() >= 256) g_tables.clear();
            TableEntry &e = g_tables[tkey];
            e.tab = tab;
            e.tab7 = tab7;
            e.seg_inv = L.seg_inv;
            e.nseg = L.nseg;
            e.tab_err = emax;
            break;
        }
        if (seg_w < 0.01) {
            char msg[128];
            snprintf(msg, sizeof msg, "level kernel table not accurate: %.3e of K_j(0)", emax);
            set_error(msg);
            return MHK_EUNSUPPORTED;
        }
    }
    if (!fp64) {
        std::vector<float> tf(tab.begin(), tab.end());
        TRY(upload(P, &L.tabf, tf.data(), (int64_t)tf.size()));
        L.tab_dev = L.tabf;
        return MHK_OK;
    }
    // the rows, then c_7 of every segment as floats (two per double)
    const size_t nrow = tab.size();
    tab.resize(nrow + ((size_t)L.nseg + 1) / 2, 0.0);
    memcpy(tab.data() + nrow, tab7.data(), sizeof(float) * (size_t)L.nseg);
    TRY(upload(P, &L.tab, tab.data(), (int64_t)tab.size()));
    L.tab_dev = L.tab;
    return MHK_OK;
}

// Exponential-of-semicircle window phi(z) = exp(beta (sqrt(1 - z^2) - 1)),
// |z| < 1 (Barnett, Magland and af Klinteberg, SIAM J. Sci. Comput. 41 (2019)),
// and its Fourier transform in physical units by Gauss-Legendre quadrature.
double window_ft(double k, double half_width, double beta, const std::vector<double> &qt,
                 const std::vector<double> &qw)
{
    long double s = 0;
    for (size_t i = 0; i < qt.size(); ++i) {
        double z = qt[i];
        s += qw[i] * exp(beta * (sqrt(1.0 - z * z) - 1.0)) * cos(k * half_width * z);
    }
    return (double)(s * half_width);
}

// Multiplier table of the smoothly truncated history kernel g_T(x, y) =
// G^H(r) chi(|x|) chi(|y|), chi = 1 up to the separation bound D and 0
// beyond D + trans.  Its Fourier coefficients on the period-P grid are the
// transform of its samples of step h over the period 2P that holds its
// support without overlap, at the even modes 2l, i.e. the sums
//   T(l_x, l_y) = sum_{x, y} h^2 g_T(x, y) cos(2 pi l_x m_x / n) cos(2 pi l_y m_y / n)
// over the samples x = m_x h, y = m_y h (g_T is even, so the transform is
// real and the +-m terms pair up).  Only |l| <= lmax is kept and the
// samples vanish beyond M = ceil((D + trans)/h), so the two separable
// cosine sums over the M x M quarter grid cost O(lmax M^2) multiply-adds
// on the device (no FFT plan to build).
mhk_status build_trunc_table(mhk_plan *P, const std::vector<double> &qt, const std::vector<double> &qw)
{
    History &G = P->hist;
    const double rmid = G.trunc_d + 0.5 * G.trunc_w, slope = 11.8 / G.trunc_w;
    const double rcut = G.trunc_d + G.trunc_w;
    G.lmax = (int)floor(G.kcut * G.period / (2 * M_PI));
    if (2 * G.lmax > G.n) {
        set_error("truncated-kernel table: too many modes for the grid");
        return MHK_EUNSUPPORTED;
    }
    const int64_t M = std::min<int64_t>(G.n, (int64_t)ceil(rcut / G.h));
    const int64_t L1 = G.lmax + 1;
    std::vector<double> t16, w16;
    gauss_legendre(16, t16, w16);
    std::vector<double> phi2inv(L1);
    for (int l = 0; l <= G.lmax; ++l) {
        double k = 2 * M_PI * l / G.period;
        double ph = window_ft(k, 0.5 * G.w * G.h, G.beta, qt, qw);
        phi2inv[l] = 1.0 / (ph * ph);
    }
    std::vector<double> costab(G.n);
    for (int64_t m = 0; m < G.n; ++m) costab[m] = (double)cosl(2.0L * M_PIl * (long double)m / (long double)G.n);
    const hipStream_t st = P->stream;
    StreamTmp tmp(st);
    double *samp = nullptr, *half = nullptr, *tr = nullptr, *gt = nullptr, *gw = nullptr, *phi = nullptr,
           *ctab = nullptr;
    TRY(tmp.alloc(&samp, M * M));
    TRY(tmp.alloc(&half, L1 * M));
    TRY(tmp.alloc(&tr, L1 * L1));
    TRY(tmp.upload(&gt, t16.data(), 16));
    TRY(tmp.upload(&gw, w16.data(), 16));
    TRY(tmp.upload(&phi, phi2inv.data(), L1));
    TRY(tmp.upload(&ctab, costab.data(), G.n));
    TRY(dalloc(P, &G.mtab, (2 * (int64_t)G.lmax + 1) * L1));
    MHK_HIP(launch_trunc_kernel_samples(samp, M, G.h, P->p.alpha, P->delta, rmid, slope, gt, gw, st));
    // half[l_x][m_y] = sum_{m_x} c cos(l_x m_x) samp[m_y][m_x]
    MHK_HIP(launch_cos_step(samp, M, L1, M, (int)G.n, ctab, half, st));
    // tr[l_y][l_x] = sum_{m_y} c cos(l_y m_y) half[l_x][m_y]
    MHK_HIP(launch_cos_step(half, M, L1, L1, (int)G.n, ctab, tr, st));
    const double c = pow(G.h, 4) / (G.period * G.period);   // samples carry h^2: spectrum ~ transform
    MHK_HIP(launch_trunc_table(tr, G.lmax, phi, c, G.mtab, st));
    // the host vectors uploaded above must outlive the copies
    MHK_HIP(hipStreamSynchronize(st));
    return MHK_OK;
}

// Relative cost of rocFFT 2D transforms of size n x n (per point), measured
// on MI355X for the in-place real transforms used here: sizes above 4096
// leave the single-pass 1D kernels (x1.6 per point) and a factor 7 costs
// about x1.45.
static double fft_cost(int64_t n)
{
    double c = n <= 4096 ? 1.0 : 1.6;
    return c * (double)n * (double)n;
}

// History grid: period, step and size (shared by plan creation and the
// footprint estimate).
struct GridChoice {
    bool trunc = false;
    double h = 0, period = 0, trans = 0, Dsep = 0, sigma = 0, beta = 0;
    int64_t n = 0;
};

static mhk_status choose_grid(const mhk_params &p, const mhk_info &I, double Lx, double Ly, GridChoice &g)
{
    const double alpha = p.alpha, delta = I.delta, kc = I.kmax;
    const int W = I.wspread;
    const double eps = hist_eps(p), L = std::max(Lx, Ly);
    // image distance: the periodic images of the history kernel must be below
    // eps relative to its peak and to the mean field of a uniform source.
    double gh0 = expint_e1(alpha * alpha * delta) / (4 * M_PI);
    double m0 = exp(-delta * alpha * alpha) / (alpha * alpha);
    double thr = eps * std::min(gh0, m0 / std::max(L * L, 1e-6));
    double R = 1.0 / alpha;
    while (sqrt(M_PI / (2 * alpha * R)) * exp(-alpha * R) / (2 * M_PI) > thr) R *= 1.02;
    // Two ways to make the periodic images harmless: a period longer than the
    // extent plus the decay length R of the kernel, or a kernel cut off
    // smoothly beyond the largest source-target separation D per axis (its
    // spectrum then tabulated by FFT, in the spirit of the truncated-kernel
    // method of Vico, Greengard and Ferrando the paper cites for small
    // alpha).  The cut-off is a product of one-dimensional ones in |x| and
    // |y| (a square, not a disk: every separation has |dx| <= Lx, |dy| <= Ly,
    // and images one period away then see a separation of at least P - L >=
    // D + trans along an axis, so P = L + D + trans with D = max(Lx, Ly)
    // rather than the diagonal).  Each factor erfc((s - s_mid) 11.8/trans)/2
    // smears the spectrum by a Gaussian of width ~23.6/trans: it must stay
    // narrow against both the multiplier's own width 1/sqrt(delta) and the
    // cut-off k_max.
    g.Dsep = std::max(Lx, Ly);
    g.trans = std::max(140.0 * sqrt(delta), 160.0 / kc);
    const double per_periodic = L + R, per_trunc = L + g.Dsep + g.trans;
    g.trunc = per_trunc < 0.9 * per_periodic;
    const double P = g.trunc ? per_trunc : per_periodic;
    // oversampling: any sigma in [sigma_min, upsamp] keeps the window width W
    // (W - 1 >= ln(1/eps)/(pi sqrt(1 - 1/sigma))); among the grid sizes this
    // allows, take the cheapest FFT.
    const double q = log(1.0 / eps) / (M_PI * (W - 1));
    double smin = q < 1.0 ? 1.0 / (1.0 - q * q) : p.upsamp;
    smin = std::min(p.upsamp, std::max(1.25, smin));
    const double hmax = M_PI / (smin * kc);
    const int64_t nlo = (int64_t)ceil(P / hmax) + W + 6;
    const int64_t nhi = (int64_t)ceil((P * p.upsamp * kc / M_PI + W + 6) * 1.25);
    if (nlo > 60000) {
        set_error("history grid too large (" + std::to_string(nlo) + "^2)");
        return MHK_EUNSUPPORTED;
    }
    int64_t best = 0;
    for (int64_t n = good_fft_size(nlo); n <= std::max(nhi, good_fft_size(nlo)); n = good_fft_size(n + 1))
        if (best == 0 || fft_cost(n) < fft_cost(best)) best = n;
    g.n = best;
    g.h = std::min(hmax, P / (double)(g.n - W - 6));
    g.sigma = M_PI / (kc * g.h);
    g.period = g.n * g.h;
    g.beta = 0.97 * M_PI * (1.0 - 0.5 / g.sigma) * W;
    return MHK_OK;
}

// Grid geometry of the history part; called before the targets are sorted,
// since their order follows the grid tiles.
mhk_status history_geometry(mhk_plan *P, const Host &H)
{
    History &G = P->hist;
    G.kcut = P->info.kmax;
    G.w = P->info.wspread;
    G.ups = P->p.upsamp;
    G.active = G.kcut > 0;
    if (!G.active) return MHK_OK;
    GridChoice g;
    TRY(choose_grid(P->p, P->info, H.xmax - H.xmin, H.ymax - H.ymin, g));
    G.trunc = g.trunc;
    G.n = g.n;
    G.h = g.h;
    G.ups = g.sigma;
    G.period = g.period;
    G.beta = g.beta;
    G.ntile = (int)(G.n / TILE);
    G.field = G.n * (G.n + 2);
    G.ox = H.xmin - (G.w / 2 + 3) * G.h;
    G.oy = H.ymin - (G.w / 2 + 3) * G.h;
    G.trunc_d = g.Dsep;
    G.trunc_w = g.trans;
    P->info.period = G.period;
    P->info.n_fine = G.n;
    P->info.history_truncated = G.trunc ? 1 : 0;
    return MHK_OK;
}

mhk_status build_history(mhk_plan *P, Host &H)
{
    History &G = P->hist;
    const double alpha = P->p.alpha, delta = P->delta;
    if (!G.active) return MHK_OK;
    MHK_FFT(rocfft_ready());

    // window polynomials: phi at grid point m0 + k of a source at g, as a
    // function of t = 2(m0 - g + w/2) - 1 in [-1, 1), fitted by Chebyshev
    // interpolation and converted to monomials (Horner form, as in the
    // spreading of Barnett, Magland and af Klinteberg)
    {
        const int W = G.w, D = W + 3, nfit = 4 * (D + 1);
        std::vector<double> cf((size_t)W * (D + 1));
        double emax = 0;
        auto phi = [&](long double z) -> long double {
            return fabsl(z) < 1 ? expl((long double)G.beta * (sqrtl(1 - z * z) - 1)) : 0.0L;
        };
        for (int k = 0; k < W; ++k) {
            std::vector<long double> f(nfit), ch(D + 1, 0);
            for (int i = 0; i < nfit; ++i) {
                long double t = cosl(M_PIl * (i + 0.5L) / nfit);
                f[i] = phi(((t + 1) / 2 - W / 2.0L + k) * 2 / W);
            }
            for (int m = 0; m <= D; ++m) {
                long double acc = 0;
                for (int i = 0; i < nfit; ++i) acc += f[i] * cosl(M_PIl * m * (i + 0.5L) / nfit);
                ch[m] = acc * (m == 0 ? 1.0L : 2.0L) / nfit;
            }
            std::vector<long double> mono(D + 1, 0), tp(D + 1, 0), tc(D + 1, 0), tn(D + 1, 0);
            tp[0] = 1;
            tc[1] = 1;
            for (int j = 0; j <= D; ++j) mono[j] += ch[0] * tp[j] + ch[1] * tc[j];
            for (int m = 2; m <= D; ++m) {
                std::fill(tn.begin(), tn.end(), 0.0L);
                for (int j = 0; j <= D; ++j) {
                    if (j + 1 <= D) tn[j + 1] += 2 * tc[j];
                    tn[j] -= tp[j];
                }
                for (int j = 0; j <= D; ++j) mono[j] += ch[m] * tn[j];
                tp = tc;
                tc = tn;
            }
            for (int j = 0; j <= D; ++j) cf[(size_t)k * (D + 1) + j] = (double)mono[j];
            for (int i = 0; i <= 400; ++i) {
                double t = -1.0 + 2.0 * i / 400.0;
                double pv = 0;
                for (int j = D; j >= 0; --j) pv = pv * t + cf[(size_t)k * (D + 1) + j];
                emax = std::max(emax, fabs(pv - (double)phi(((t + 1) / 2 - W / 2.0L + k) * 2 / W)));
            }
        }
        G.wfit_err = emax;
        if (emax > std::max(P->p.prec == MHK_FP64 ? 1e-11 : 1e-6, 0.5 * P->p.tol)) {
            char msg[128];
            snprintf(msg, sizeof msg, "window polynomial fit error %.3e too large", emax);
            set_error(msg);
            return MHK_EUNSUPPORTED;
        }
        if (P->p.prec == MHK_FP64) {
            double *d = nullptr;
            TRY(upload(P, &d, cf.data(), (int64_t)cf.size()));
            G.wcoef = d;
        } else {
            std::vector<float> cff(cf.begin(), cf.end());
            float *d = nullptr;
            TRY(upload(P, &d, cff.data(), (int64_t)cff.size()));
            G.wcoef = d;
        }
    }
    // multiplier factors
    std::vector<double> qt, qw;
    gauss_legendre(160, qt, qw);
    const int64_t nh = G.n / 2 + 1;
    std::vector<double> fac(nh);
    for (int64_t l = 0; l < nh; ++l) {
        double k = 2 * M_PI * l / G.period;
        if (k > G.kcut) {
            fac[l] = 0;
            continue;
        }
        double ph = window_ft(k, 0.5 * G.w * G.h, G.beta, qt, qw);
        fac[l] = exp(-delta * k * k) / (ph * ph);
    }
    G.mult_c = pow(G.h, 4) / (G.period * G.period) * exp(-delta * alpha * alpha);
    TRY(upload(P, &G.fac, fac.data(), nh));
    if (G.trunc) TRY(build_trunc_table(P, qt, qw));
    // columns l_x that can hold a nonzero multiplier
    G.ncol = 0;
    if (G.trunc) {
        G.ncol = (int)std::min<int64_t>(nh, G.lmax + 1);
    } else {
        for (int64_t l = 0; l < nh; ++l)
            if (fac[l] != 0.0) G.ncol = (int)l + 1;
    }

    // Sources sorted by 32 x 32 tile of the grid, per-tile lists of the
    // sorted sources whose window [m0, m0 + w) (m0 = ceil(g - w/2), as the
    // spreading kernel forms it) meets the tile in both axes, and the grid
    // rows and columns the windows use; targets (already sorted with tiles
    // contiguous) as runs of tiles, and the rows and columns of their
    // interpolation windows.  All on the device; the few totals and bounds
    // the launches need come back in one wait.
    {
        const hipStream_t st = P->stream;
        StreamTmp tmp(st);
        const int64_t nb = H.b->n_panels * NGL, nv = H.v ? H.v->n : 0, nout = P->nout;
        const int64_t nt2 = (int64_t)G.ntile * G.ntile;
        const int n = (int)G.n;
        // window bounds [x0, x1) x [y0, y1): sources in bnd[0..3], targets in bnd[4..7]
        const int bnd0[8] = {n, 0, n, 0, n, 0, n, 0};
        int *bnd = nullptr;
        int64_t *tots = nullptr;   // boundary list, volume list, target tile runs
        TRY(tmp.upload(&bnd, bnd0, 8));
        TRY(tmp.alloc(&tots, 3));
        G.nbs = nb;
        TRY(dalloc(P, &G.bgx, nb));
        TRY(dalloc(P, &G.bgy, nb));
        TRY(dalloc(P, &G.bw, nb));
        TRY(dalloc(P, &G.bwx, nb));
        TRY(dalloc(P, &G.bwy, nb));
        TRY(dalloc(P, &G.bidx, nb));
        TRY(dalloc(P, &G.blofs, nt2 + 1));
        int32_t *bstart = nullptr, *vstart = nullptr, *tflag = nullptr, *tpos = nullptr;
        MHK_HIP(dev_sources_by_tile(P->bx, P->by, P->bw, P->bnx, P->bny, nb, G.ox, G.oy, G.h, G.ntile, G.w, G.bgx,
                                    G.bgy, G.bw, G.bwx, G.bwy, G.bidx, bnd, G.blofs, &bstart, tots + 0, st));
        tmp.ptrs.push_back(bstart);
        G.nvs = nv;
        double *vx = nullptr, *vy = nullptr, *vw = nullptr;
        TRY(tmp.upload(&vx, nv ? H.v->x : nullptr, nv));
        TRY(tmp.upload(&vy, nv ? H.v->y : nullptr, nv));
        TRY(tmp.upload(&vw, nv ? H.v->w : nullptr, nv));
        TRY(dalloc(P, &G.vgx, nv));
        TRY(dalloc(P, &G.vgy, nv));
        TRY(dalloc(P, &G.vw, nv));
        TRY(dalloc(P, &G.vidx, nv));
        TRY(dalloc(P, &G.vlofs, nt2 + 1));
        MHK_HIP(dev_sources_by_tile(vx, vy, vw, nullptr, nullptr, nv, G.ox, G.oy, G.h, G.ntile, G.w, G.vgx, G.vgy,
                                    G.vw, nullptr, nullptr, G.vidx, bnd, G.vlofs, &vstart, tots + 1, st));
        tmp.ptrs.push_back(vstart);
        MHK_HIP(dev_target_tiles_count(P->tx, P->ty, nout, G.ox, G.oy, G.h, G.ntile, G.w, bnd + 4, &tflag, &tpos,
                                       tots + 2, st));
        tmp.ptrs.push_back(tflag);
        tmp.ptrs.push_back(tpos);
        int64_t tot[3];
        int bh[8];
        MHK_HIP(hipMemcpyAsync(tot, tots, sizeof tot, hipMemcpyDeviceToHost, st));
        TRY(tmp.fetch(bh, bnd, 8));
        if (tot[0] > (int64_t)INT32_MAX || tot[1] > (int64_t)INT32_MAX) {
            set_error("spreading tile lists too large");
            return MHK_EUNSUPPORTED;
        }
        TRY(dalloc(P, &G.blist, std::max<int64_t>(1, tot[0])));
        TRY(dalloc(P, &G.vlist, std::max<int64_t>(1, tot[1])));
        MHK_HIP(dev_tile_fill(G.bgx, G.bgy, bstart, G.ntile, G.w, G.blofs, G.blist, st));
        MHK_HIP(dev_tile_fill(G.vgx, G.vgy, vstart, G.ntile, G.w, G.vlofs, G.vlist, st));
        G.n_ttiles = (int)tot[2];
        TRY(dalloc(P, &G.ttile_xy, std::max<int64_t>(1, tot[2])));
        TRY(dalloc(P, &G.ttile_rng, tot[2] + 1));
        MHK_HIP(dev_target_tiles_fill(P->tx, P->ty, nout, G.ox, G.oy, G.h, G.ntile, tflag, tpos, G.ttile_xy,
                                      G.ttile_rng, st));
        G.sx0 = std::max(0, bh[0]);
        G.sx1 = std::min(n, bh[1]);
        G.sy0 = std::max(0, bh[2]);
        G.sy1 = std::min(n, bh[3]);
        G.tx0 = std::max(0, bh[4]);
        G.tx1 = std::min(n, bh[5]);
        G.ty0 = std::max(0, bh[6]);
        G.ty1 = std::min(n, bh[7]);
        // the temporaries are freed in stream order; the host arrays they
        // were filled from stay alive until plan creation returns
    }
    // grids and FFT plans
    {
        char *g = nullptr;
        TRY(dalloc(P, &g, 4 * (int64_t)P->p.batch * G.field * (int64_t)P->es));
        G.grid = g;
    }
    const rocfft_precision fprec = P->p.prec == MHK_FP64 ? rocfft_precision_double : rocfft_precision_single;
    MHK_FFT(rocfft_ready());
    // column path: the column transforms in LDS need n <= COL_NMAX and
    // radices 8, 9, 6, 4, 2, 3, 5 (the grid sizes are 2^a 3^b 5^c)
    auto factor = [](int64_t m, int8_t *radix, int &np) -> bool {
        np = 0;
        while (m % 8 == 0 && np < COL_MAXPASS) { radix[np++] = 8; m /= 8; }
        while (m % 9 == 0 && np < COL_MAXPASS) { radix[np++] = 9; m /= 9; }
        if (m % 6 == 0 && np < COL_MAXPASS) { radix[np++] = 6; m /= 6; }
        while (m % 4 == 0 && np < COL_MAXPASS) { radix[np++] = 4; m /= 4; }
        for (int f : {2, 3, 5})
            while (m % f == 0 && np < COL_MAXPASS) { radix[np++] = (int8_t)f; m /= f; }
        return m == 1;
    };
    G.colpath = G.n <= COL_NMAX && G.n % 2 == 0 && factor(G.n, G.radix, G.npass) &&
                factor(G.n / 2, G.rradix, G.rnpass);
    if (G.colpath) {
        const size_t n1 = (size_t)G.n;
        // twiddles e^{-2 pi i m / n}
        std::vector<double> tw(2 * n1);
        for (size_t m = 0; m < n1; ++m) {
            const long double a = -2.0L * M_PIl * (long double)m / (long double)n1;
            tw[2 * m] = (double)cosl(a);
            tw[2 * m + 1] = (double)sinl(a);
        }
        double *d = nullptr;
        TRY(upload(P, &d, tw.data(), (int64_t)tw.size()));
        G.tw = d;
    } else {
        // rocFFT 2D transforms around k_multiply
        size_t len[2] = {(size_t)G.n, (size_t)G.n};
        size_t rstr[2] = {1, (size_t)G.n + 2}, cstr[2] = {1, (size_t)(G.n / 2 + 1)};
        size_t rdist = (size_t)G.field, cdist = (size_t)(G.field / 2);
        rocfft_plan_description df = nullptr, di = nullptr;
        MHK_FFT(rocfft_plan_description_create(&df));
        MHK_FFT(rocfft_plan_description_set_data_layout(df, rocfft_array_type_real, rocfft_array_type_hermitian_interleaved,
                                                        nullptr, nullptr, 2, rstr, rdist, 2, cstr, cdist));
        MHK_FFT(rocfft_plan_create(&G.fwd, rocfft_placement_inplace, rocfft_transform_type_real_forward,
                                   fprec, 2, len, 4 * (size_t)P->p.batch, df));
        MHK_FFT(rocfft_plan_description_create(&di));
        MHK_FFT(rocfft_plan_description_set_data_layout(di, rocfft_array_type_hermitian_interleaved, rocfft_array_type_real,
                                                        nullptr, nullptr, 2, cstr, cdist, 2, rstr, rdist));
        MHK_FFT(rocfft_plan_create(&G.inv, rocfft_placement_inplace, rocfft_transform_type_real_inverse,
                                   fprec, 2, len, 3 * (size_t)P->p.batch, di));
        rocfft_plan_description_destroy(df);
        rocfft_plan_description_destroy(di);
        size_t w1 = 0, w2 = 0;
        MHK_FFT(rocfft_plan_get_work_buffer_size(G.fwd, &w1));
        MHK_FFT(rocfft_plan_get_work_buffer_size(G.inv, &w2));
        G.work_bytes = std::max(w1, w2);
        MHK_FFT(rocfft_execution_info_create(&G.exec));
        if (G.work_bytes) {
            char *wb = nullptr;
            TRY(dalloc(P, &wb, (int64_t)G.work_bytes));
            G.work = wb;
            MHK_FFT(rocfft_execution_info_set_work_buffer(G.exec, G.work, G.work_bytes));
        }
        MHK_FFT(rocfft_execution_info_set_stream(G.exec, P->stream));
    }
    return MHK_OK;
}

mhk_status build_local(mhk_plan *P, Host &H)
{
    Local &C = P->loc;
    const mhk_boundary *b = H.b;
    const int64_t npan = b->n_panels, nb = npan * NGL;
    // Legendre coefficients c_k = (2k+1)/2 sum_i w_i P_k(t_i) f_i
    std::vector<double> leg(NGL * NGL);
    for (int i = 0; i < NGL; ++i) {
        double t = H.gl_t[i], p0 = 1, p1 = t;
        for (int k = 0; k < NGL; ++k) {
            double pk = (k == 0) ? 1.0 : (k == 1 ? t : 0.0);
            if (k >= 2) {
                double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
                pk = p2;
            }
            leg[k * NGL + i] = (2 * k + 1) / 2.0 * H.gl_w[i] * pk;
        }
    }
    auto coeffs = [&](const double *f, std::vector<double> &out) {
        out.assign(nb, 0.0);
        for (int64_t p = 0; p < npan; ++p)
            for (int k = 0; k < NGL; ++k) {
                long double s = 0;
                for (int i = 0; i < NGL; ++i) s += (long double)leg[k * NGL + i] * f[p * NGL + i];
                out[p * NGL + k] = (double)s;
            }
    };
    std::vector<double> cx, cy, ck;
    coeffs(b->x, cx);
    coeffs(b->y, cy);
    coeffs(b->kappa, ck);
    std::vector<double> ends(npan * 4);
    for (int64_t p = 0; p < npan; ++p) {
        double xm = 0, ym = 0, xp = 0, yp = 0;
        for (int k = 0; k < NGL; ++k) {
            double sgn = (k % 2) ? -1.0 : 1.0;   // P_k(-1) = (-1)^k, P_k(1) = 1
            xm += sgn * cx[p * NGL + k];
            ym += sgn * cy[p * NGL + k];
            xp += cx[p * NGL + k];
            yp += cy[p * NGL + k];
        }
        ends[p * 4 + 0] = xm; ends[p * 4 + 1] = ym; ends[p * 4 + 2] = xp; ends[p * 4 + 3] = yp;
    }
    // closest-point cells.  Any target within the larger band of the curve
    // has its nearest node within reach = band + (largest node gap); the
    // cell of side `cell` lists every panel whose node bounding box comes
    // within reach of the cell, nearest first, so the device search over
    // the list finds the global nearest node whenever it is within reach.
    double gap = 0;
    for (int64_t p = 0; p < npan; ++p) {
        for (int i = 0; i + 1 < NGL; ++i)
            gap = std::max(gap, hypot(b->x[p * NGL + i + 1] - b->x[p * NGL + i], b->y[p * NGL + i + 1] - b->y[p * NGL + i]));
        int64_t q = H.next[p];
        gap = std::max(gap, hypot(b->x[q * NGL] - b->x[p * NGL + NGL - 1], b->y[q * NGL] - b->y[p * NGL + NGL - 1]));
    }
    const double band = std::max(P->info.band_layer, P->info.band_volume);
    C.gap = gap;
    C.reach = band + gap;
    C.ox = H.xmin - 1e-9;
    C.oy = H.ymin - 1e-9;
    // cells of half the reach (a target's list then spans 2.5 reaches), at
    // most 2^22 of them
    const double ext = std::max(H.xmax - C.ox, H.ymax - C.oy);
    C.cell = std::max(0.5 * C.reach, ext / 2048.0);
    int64_t ncx = (int64_t)floor((H.xmax - C.ox) / C.cell) + 1;
    int64_t ncy = (int64_t)floor((H.ymax - C.oy) / C.cell) + 1;
    C.ncx = (int)ncx;
    C.ncy = (int)ncy;
    std::vector<double> pbox(npan * 4);
    for (int64_t p = 0; p < npan; ++p) {
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        for (int i = 0; i < NGL; ++i) {
            x0 = std::min(x0, b->x[p * NGL + i]); x1 = std::max(x1, b->x[p * NGL + i]);
            y0 = std::min(y0, b->y[p * NGL + i]); y1 = std::max(y1, b->y[p * NGL + i]);
        }
        pbox[p * 4 + 0] = x0; pbox[p * 4 + 1] = x1; pbox[p * 4 + 2] = y0; pbox[p * 4 + 3] = y1;
    }
    {
        // every (cell, panel) pair with box-to-box distance <= reach; the
        // cells a panel can reach lie in its box grown by reach
        std::vector<int32_t> start(ncx * ncy + 1, 0), cand;
        std::vector<std::array<int64_t, 2>> pairs;   // cell, panel
        auto cl = [&](double v, double o, int64_t nc) {
            return std::min<int64_t>(nc - 1, std::max<int64_t>(0, (int64_t)floor((v - o) / C.cell)));
        };
        for (int64_t p = 0; p < npan; ++p) {
            const double *bb = &pbox[p * 4];
            for (int64_t iy = cl(bb[2] - C.reach, C.oy, ncy); iy <= cl(bb[3] + C.reach, C.oy, ncy); ++iy)
                for (int64_t ix = cl(bb[0] - C.reach, C.ox, ncx); ix <= cl(bb[1] + C.reach, C.ox, ncx); ++ix) {
                    const double cx0 = C.ox + ix * C.cell, cy0 = C.oy + iy * C.cell;
                    const double ex = std::max(0.0, std::max(bb[0] - (cx0 + C.cell), cx0 - bb[1]));
                    const double ey = std::max(0.0, std::max(bb[2] - (cy0 + C.cell), cy0 - bb[3]));
                    if (ex * ex + ey * ey <= C.reach * C.reach) pairs.push_back({iy * ncx + ix, p});
                }
        }
        if (pairs.size() > ((size_t)1 << 31)) {
            set_error("closest-point cell lists too large");
            return MHK_EUNSUPPORTED;
        }
        // per cell, panels in increasing distance of their box from the cell centre
        auto dist_c = [&](int64_t c, int64_t p) {
            const double xc = C.ox + ((c % ncx) + 0.5) * C.cell, yc = C.oy + ((c / ncx) + 0.5) * C.cell;
            const double *bb = &pbox[p * 4];
            const double ex = std::max(0.0, std::max(bb[0] - xc, xc - bb[1]));
            const double ey = std::max(0.0, std::max(bb[2] - yc, yc - bb[3]));
            return ex * ex + ey * ey;
        };
        // (the distance formed once per pair, not per comparison)
        struct Key {
            int64_t cell;
            double d;
            int64_t panel;
        };
        std::vector<Key> keys(pairs.size());
        for (size_t k = 0; k < pairs.size(); ++k) keys[k] = {pairs[k][0], dist_c(pairs[k][0], pairs[k][1]), pairs[k][1]};
        std::sort(keys.begin(), keys.end(), [](const Key &a, const Key &c) {
            if (a.cell != c.cell) return a.cell < c.cell;
            return a.d != c.d ? a.d < c.d : a.panel < c.panel;
        });
        cand.resize(std::max<size_t>(1, keys.size()));
        for (size_t k = 0; k < keys.size(); ++k) {
            start[keys[k].cell + 1]++;
            cand[k] = (int32_t)keys[k].panel;
        }
        for (int64_t c = 0; c < ncx * ncy; ++c) start[c + 1] += start[c];
        TRY(upload(P, &C.cand, cand.data(), (int64_t)cand.size()));
        TRY(upload(P, &C.cell_start, start.data(), (int64_t)start.size()));
    }
    TRY(upload(P, &C.pbox, pbox.data(), npan * 4));
    {
        // box of each panel's whole curve gamma(t), t in [-1, 1]: 129
        // Chebyshev points of its Legendre series, grown by 1% of its size
        // (the curve between the points bulges far less); a neighbouring
        // panel whose box is farther than the best distance found cannot hold
        // the closest point
        std::vector<double> cbox(npan * 4);
        const int ns = 129;
        for (int64_t p = 0; p < npan; ++p) {
            double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
            for (int i = 0; i < ns; ++i) {
                const double t = -cos(M_PI * i / (ns - 1));
                double p0 = 1, p1 = t, xv = cx[p * NGL] + cx[p * NGL + 1] * t, yv = cy[p * NGL] + cy[p * NGL + 1] * t;
                for (int k = 1; k + 1 < NGL; ++k) {
                    const double p2 = ((2 * k + 1) * t * p1 - k * p0) / (k + 1);
                    p0 = p1;
                    p1 = p2;
                    xv += cx[p * NGL + k + 1] * p2;
                    yv += cy[p * NGL + k + 1] * p2;
                }
                x0 = std::min(x0, xv); x1 = std::max(x1, xv);
                y0 = std::min(y0, yv); y1 = std::max(y1, yv);
            }
            const double m = 0.01 * std::max(x1 - x0, y1 - y0) + 1e-12;
            cbox[p * 4 + 0] = x0 - m; cbox[p * 4 + 1] = x1 + m;
            cbox[p * 4 + 2] = y0 - m; cbox[p * 4 + 3] = y1 + m;
        }
        TRY(upload(P, &C.cbox, cbox.data(), npan * 4));
    }
    {
        int32_t zero = 0;
        TRY(upload(P, &C.noconv, &zero, 1));
    }
    std::vector<int32_t> prev(npan), next(npan);
    for (int64_t p = 0; p < npan; ++p) {
        prev[p] = (int32_t)H.prev[p];
        next[p] = (int32_t)H.next[p];
    }
    TRY(upload(P, &C.leg, leg.data(), NGL * NGL));
    TRY(upload(P, &C.cx, cx.data(), nb));
    TRY(upload(P, &C.cy, cy.data(), nb));
    TRY(upload(P, &C.ck, ck.data(), nb));
    TRY(upload(P, &C.ends, ends.data(), npan * 4));
    TRY(upload(P, &C.gl_t, H.gl_t.data(), NGL));
    TRY(upload(P, &C.prev, prev.data(), npan));
    TRY(upload(P, &C.next, next.data(), npan));
    TRY(dalloc(P, &C.csig, (int64_t)P->p.batch * nb));
    TRY(dalloc(P, &C.cmu, (int64_t)P->p.batch * nb));
    TRY(dalloc(P, &C.cf, (int64_t)P->p.batch * nb));
    // per-plan geometry of the local part (closest points and coefficients)
    TRY(dalloc(P, &C.geo, (P->p.local_order >= 2 ? LOCAL_GEO_N2 : LOCAL_GEO_N1) * std::max<int64_t>(P->nout, 1)));
    TRY(dalloc(P, &C.gpan, std::max<int64_t>(P->nout, 1)));
    TRY(dalloc(P, &C.gflag, std::max<int64_t>(P->nout, 1)));
    return MHK_OK;
}

// f at the targets from the volume quadrature (volume nodes in groups of
// six per triangle): per-triangle quadratic fits and each target's triangle
mhk_status build_fjets(mhk_plan *P, Host &H)
{
    FJets &F = P->fj;
    const int64_t nv = P->nv, ntri = nv / 6;
    const hipStream_t st = P->stream;
    StreamTmp tmp(st);
    double *vx = nullptr, *vy = nullptr;
    TRY(tmp.upload(&vx, H.v->x, nv));
    TRY(tmp.upload(&vy, H.v->y, nv));
    TRY(dalloc(P, &F.good, ntri));
    uint8_t *good = F.good;
    TRY(dalloc(P, &F.minv, 36 * ntri));
    TRY(dalloc(P, &F.tc, 3 * ntri));
    TRY(dalloc(P, &F.tri, P->nout));
    MHK_HIP(dev_fj_setup(ntri, vx, vy, F.minv, F.tc, good, st));
    // cells of about two node spacings over the box of nodes and targets
    const double lx = H.xmax - H.xmin, ly = H.ymax - H.ymin;
    double cell = 2.0 * sqrt(std::max(lx * ly, 1e-300) / (double)nv);
    cell = std::max(cell, std::max(lx, ly) / 4096.0);
    // the box of every point searched: nodes, targets and (volume levels)
    // the level nodes of the curved triangles' maps, which can bulge a
    // little past the nodes
    const double mg = 0.05 * std::max(lx, ly) + cell;
    const double ox = H.xmin - mg, oy = H.ymin - mg;
    const int64_t ncx = (int64_t)floor((H.xmax + mg - ox) / cell) + 1, ncy = (int64_t)floor((H.ymax + mg - oy) / cell) + 1;
    TRY(dalloc(P, &F.perm, nv));
    TRY(dalloc(P, &F.start, ncx * ncy + 2));
    MHK_HIP(dev_fj_nearest(P, vx, vy, good, ox, oy, cell, ncx, ncy, F.tri, st));
    const int rows = P->p.local_order >= 2 ? 6 : 1;
    const int64_t es_in = (P->p.prec == MHK_FP64 || P->p.in64) ? 8 : 4;
    char *fr = nullptr;
    TRY(dalloc(P, &fr, (int64_t)P->p.batch * rows * P->nout * es_in));
    F.frec = fr;
    F.active = true;
    MHK_HIP(hipStreamSynchronize(st));   // the uploads read the caller's arrays
    return MHK_OK;
}

// Dyadic levels of the volume potential: the level-j nodes of every volume
// triangle (4^j sub-triangles of its reference triangle, mapped by the
// quadratic through its six nodes), sorted by the cells of the layer level
// j, each node's triangle for f, and the per-wavefront candidate lists
mhk_status build_vlevels(mhk_plan *P, Host &H)
{
    const mhk_volume *v = H.v;
    const int64_t nv = P->nv, ntri = nv / 6;
    const hipStream_t st = P->stream;
    VRule M;
    {
        // monomials 1, s, t, s^2, st, t^2 at the rule points, inverted (Gauss-Jordan, long double)
        long double A[6][12];
        for (int i = 0; i < 6; ++i) {
            const long double s_ = v->rule[i * 3 + 0], t_ = v->rule[i * 3 + 1];
            M.s[i] = v->rule[i * 3 + 0];
            M.t[i] = v->rule[i * 3 + 1];
            M.W[i] = v->rule[i * 3 + 2];
            const long double row[6] = {1.0L, s_, t_, s_ * s_, s_ * t_, t_ * t_};
            for (int k = 0; k < 6; ++k) {
                A[i][k] = row[k];
                A[i][6 + k] = i == k ? 1.0L : 0.0L;
            }
        }
        for (int c = 0; c < 6; ++c) {
            int piv = c;
            for (int r = c + 1; r < 6; ++r)
                if (fabsl(A[r][c]) > fabsl(A[piv][c])) piv = r;
            if (fabsl(A[piv][c]) < 1e-12L) {
                set_error("volume rule: the six points do not determine a quadratic");
                return MHK_EINVAL;
            }
            for (int k = 0; k < 12; ++k) std::swap(A[c][k], A[piv][k]);
            const long double inv = 1.0L / A[c][c];
            for (int k = 0; k < 12; ++k) A[c][k] *= inv;
            for (int r = 0; r < 6; ++r)
                if (r != c) {
                    const long double f = A[r][c];
                    for (int k = 0; k < 12; ++k) A[r][k] -= f * A[c][k];
                }
        }
        // rinv[m][l]: coefficient m of the map from the node values l
        for (int m = 0; m < 6; ++m)
            for (int l = 0; l < 6; ++l) M.rinv[m * 6 + l] = (double)A[m][6 + l];
    }
    StreamTmp tmp(st);
    double *vx = nullptr, *vy = nullptr;
    TRY(tmp.upload(&vx, v->x, nv));
    TRY(tmp.upload(&vy, v->y, nv));
    {
        char *a = nullptr;
        TRY(dalloc(P, &a, (int64_t)P->p.batch * P->nout * (int64_t)P->es));
        P->acc_vlev = a;
    }
    const int64_t nout = P->nout;
    const int64_t nwave = ((nout + LV_BLOCK_MAX - 1) / LV_BLOCK_MAX) * (LV_BLOCK_MAX / LV_WAVE);
    for (int j = 1; j <= P->J; ++j) {
        const Level &L = P->lev[j - 1];
        VLevel &V = P->vlev[j - 1];
        V.n_src = ntri * ((int64_t)1 << (2 * j)) * 6;
        if (V.n_src > (int64_t)INT32_MAX) {
            set_error("volume level nodes beyond 2^31");
            return MHK_EUNSUPPORTED;
        }
        TRY(dalloc(P, &V.sx, V.n_src));
        TRY(dalloc(P, &V.sy, V.n_src));
        TRY(dalloc(P, &V.sw, V.n_src));
        TRY(dalloc(P, &V.tri, V.n_src));
        TRY(dalloc(P, &V.cell_start, (int64_t)L.ncx * L.ncy + 1));
        {
            char *q = nullptr;
            TRY(dalloc(P, &q, (int64_t)P->p.batch * V.n_src * (int64_t)P->es));
            V.q = q;
        }
        int32_t *parent = nullptr;
        TRY(tmp.alloc(&parent, V.n_src));
        MHK_HIP(dev_vlevel_nodes(ntri, j, M, vx, vy, L.ox, L.oy, L.cell, L.ncx, L.ncy, V.sx, V.sy, V.sw, parent,
                                 V.cell_start, st));
        MHK_HIP(dev_fj_nearest_pts(P, V.n_src, V.sx, V.sy, parent, vx, vy, V.tri, st));
        V.n_wave = nwave;
        const double R = L.radius, R2 = R * R * (1.0 + 1e-9);
        int32_t *cnt = nullptr;
        int64_t *tot = nullptr;
        TRY(tmp.alloc(&cnt, nwave));
        TRY(tmp.alloc(&tot, 1));
        TRY(dalloc(P, &V.wave_ofs, nwave + 1));
        TRY(dalloc(P, &V.wave_order, nwave));
        MHK_HIP(dev_wave_counts(P->tx, P->ty, nout, nwave, R, R2, L.ox, L.oy, L.cell, L.ncx, L.ncy, V.cell_start,
                                V.sx, V.sy, cnt, st));
        MHK_HIP(dev_scan(cnt, V.wave_ofs, nwave, tot, st));
        int64_t total = 0;
        TRY(tmp.fetch(&total, tot, 1));
        if (total > (int64_t)INT32_MAX) {
            set_error("volume level candidate lists too large");
            return MHK_EUNSUPPORTED;
        }
        V.n_cand = total;
        TRY(dalloc(P, &V.wave_src, std::max<int64_t>(1, total)));
        MHK_HIP(dev_wave_fill(P->tx, P->ty, nout, nwave, R, R2, L.ox, L.oy, L.cell, L.ncx, L.ncy, V.cell_start, V.sx,
                              V.sy, V.wave_ofs, V.wave_src, V.wave_order, st));
    }
    MHK_HIP(hipStreamSynchronize(st));
    return MHK_OK;
}

mhk_status create(const mhk_params *params, const mhk_boundary *b, const mhk_volume *v,
                  const mhk_targets *t, void *stream, mhk_plan *P)
{
    using clk = std::chrono::steady_clock;
    const auto t_start = clk::now();
    auto t_mark = t_start;
    // host-clock time of a phase of plan creation, into info.ms_plan[k]
    auto lap = [&](int k) {
        const auto now = clk::now();
        P->info.ms_plan[k] += std::chrono::duration<double, std::milli>(now - t_mark).count();
        t_mark = now;
    };
    TRY(check_inputs(params, b, v, t));
    TRY(resolve(params, &P->info, &P->p));
    P->es = P->p.prec == MHK_FP64 ? sizeof(double) : sizeof(float);
    P->stream = (hipStream_t)stream;
    P->J = P->p.J;
    P->delta = P->info.delta;
    P->dstar = P->info.delta_star;
    P->delta_v = P->p.v_levels ? P->dstar : P->delta;
    if (P->p.v_levels && (!v || v->n == 0 || v->group != 6 || !v->rule)) {
        set_error("v_levels needs a volume with group 6 and its rule");
        return MHK_EINVAL;
    }
    P->npan = b->n_panels;
    P->nb = b->n_panels * NGL;
    P->nv = v ? v->n : 0;
    P->nt = t->n;
    P->nout = t->n + (t->on_surface ? P->nb : 0);
    // targets that are exactly the volume nodes, in the same order (the
    // setting of elliptic marching, where u is carried at the nodes)
    P->targets_are_volume = P->nv > 0 && P->nt == P->nv &&
                            memcmp(t->x, v->x, sizeof(double) * P->nv) == 0 &&
                            memcmp(t->y, v->y, sizeof(double) * P->nv) == 0;
    Host H;
    H.b = b;
    H.v = (v && v->n > 0) ? v : nullptr;
    H.t = t;
    host_common(H);
    lap(0);

    // boundary arrays in caller order
    TRY(upload(P, &P->bx, b->x, P->nb));
    TRY(upload(P, &P->by, b->y, P->nb));
    TRY(upload(P, &P->bnx, b->nx, P->nb));
    TRY(upload(P, &P->bny, b->ny, P->nb));
    TRY(upload(P, &P->bw, b->w, P->nb));
    TRY(upload(P, &P->bk, b->kappa, P->nb));

    // history grid first: the target order follows the grid tiles
    History &G = P->hist;
    TRY(history_geometry(P, H));
    // targets sorted in Morton order of cells of one grid step (or of a virtual
    // grid of step R_J/8 when there is no history grid)
    {
        double hh, ox, oy;
        if (G.active) {
            hh = G.h;
            ox = G.ox;
            oy = G.oy;
        } else {
            double rj = P->J > 0 ? P->info.level_radius[P->J - 1] : P->info.band_layer;
            hh = std::max(rj / 8.0, std::max(H.xmax - H.xmin, H.ymax - H.ymin) / 60000.0);
            ox = H.xmin - hh;
            oy = H.ymin - hh;
        }
        const int64_t nout = P->nout;
        StreamTmp tmp(P->stream);
        double *rx = nullptr, *ry = nullptr;
        int8_t *rin = nullptr;
        TRY(tmp.upload(&rx, H.tx.data(), nout));
        TRY(tmp.upload(&ry, H.ty.data(), nout));
        TRY(tmp.upload(&rin, H.tin.data(), nout));
        if (H.mask_needed) TRY(build_mask(P, H, tmp, rin));
        TRY(dalloc(P, &P->tx, nout));
        TRY(dalloc(P, &P->ty, nout));
        TRY(dalloc(P, &P->tin, nout));
        TRY(dalloc(P, &P->tidx, nout));
        MHK_HIP(dev_sort_targets(rx, ry, rin, nout, ox, oy, hh, P->tx, P->ty, P->tin, P->tidx, P->stream));
    }
    lap(1);
    for (int j = 1; j <= P->J; ++j) TRY(build_level(P, H, j));
    lap(2);
    TRY(build_history(P, H));
    MHK_HIP(hipStreamSynchronize(P->stream));
    lap(3);
    TRY(build_local(P, H));
    if (H.v && v->group == 6) TRY(build_fjets(P, H));
    if (P->p.v_levels) TRY(build_vlevels(P, H));
    MHK_HIP(launch_local_geom(P, P->stream));
    {
        char *a = nullptr;
        TRY(dalloc(P, &a, 3 * (int64_t)P->p.batch * P->nout * (int64_t)P->es));
        P->acc = a;
        char *l = nullptr;
        TRY(dalloc(P, &l, 2 * (int64_t)P->p.batch * P->nout * (int64_t)P->es));
        P->acc_lev = l;
        if (P->p.in64) TRY(dalloc(P, &P->in32, (int64_t)P->p.batch * (2 * P->nb + P->nv)));
        TRY(dalloc(P, &P->lv_counter, 1));
    }
    for (auto &e : P->ev) MHK_HIP(hipEventCreate(&e));
    MHK_HIP(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking));
    MHK_HIP(hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming));
    MHK_HIP(hipEventCreateWithFlags(&P->join_ev, hipEventDisableTiming));
    P->info.n_boundary = P->nb;
    P->info.n_volume = P->nv;
    P->info.n_targets = P->nt;
    P->info.n_out = P->nout;
    P->info.device_bytes = P->bytes;
    // only the plan's own stream is waited for: work of other plans on other
    // streams keeps running while a plan is created
    MHK_HIP(hipStreamSynchronize(P->stream));
    P->stage.clear();
    P->stage.shrink_to_fit();
    lap(4);
    P->info.ms_plan[5] = std::chrono::duration<double, std::milli>(clk::now() - t_start).count();
    int32_t noconv = 0;
    MHK_HIP(hipMemcpy(&noconv, P->loc.noconv, sizeof(noconv), hipMemcpyDeviceToHost));
    P->info.n_noconv = noconv;
    if (noconv > 0) {
        set_error("closest-point Newton iteration did not converge for " + std::to_string(noconv) +
                  " targets inside a local band");
        return MHK_ENOCONV;
    }
    return MHK_OK;
}

mhk_status collect_timing(mhk_plan *P);   // stage times of the last timed evaluation

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *mhk_last_error(void) { return g_err.c_str(); }

mhk_status mhk_resolve_params(const mhk_params *params, mhk_info *info)
{
    return resolve(params, info, nullptr);
}

mhk_status mhk_plan_create(const mhk_params *params, const mhk_boundary *boundary,
                           const mhk_volume *volume, const mhk_targets *targets, void *hip_stream,
                           mhk_plan **out)
{
    if (!out) {
        set_error("out is NULL");
        return MHK_EINVAL;
    }
    *out = nullptr;
    mhk_plan *P = new mhk_plan();
    mhk_status s = create(params, boundary, volume, targets, hip_stream, P);
    if (s != MHK_OK) {
        free_plan(P);
        return s;
    }
    *out = P;
    return MHK_OK;
}

mhk_status mhk_plan_footprint(const mhk_params *params, const mhk_boundary *b, const mhk_volume *v,
                              const mhk_targets *t, int64_t *bytes)
{
    if (!bytes) {
        set_error("bytes is NULL");
        return MHK_EINVAL;
    }
    TRY(check_inputs(params, b, v, t));
    mhk_info I;
    mhk_params p;
    TRY(resolve(params, &I, &p));
    int64_t nb = b->n_panels * NGL, nv = v ? v->n : 0;
    int64_t nout = t->n + (t->on_surface ? nb : 0);
    int64_t B = p.batch;
    int64_t s = 0;
    s += nb * 8 * 6;                          // boundary
    s += nout * (8 * 2 + 1 + 4);              // targets
    s += 5 * B * nout * 8;                    // accumulators (history and levels)
    for (int j = 1; j <= p.J; ++j) {          // levels
        int64_t ns = nb << j;
        s += ns * (8 * 5 + 4) + 3 * B * ns * 8;
    }
    s += nb * (8 * 3 + 4) + 3 * B * nb * 8;   // local
    s += nout * ((p.local_order >= 2 ? LOCAL_GEO_N2 : LOCAL_GEO_N1) * 8 + 4 + 1);   // local geometry per target
    if (p.in64) s += B * (2 * nb + nv) * 4;   // FP32 copies of FP64 inputs
    if (v && v->group == 6)                    // f at the targets from the volume triangles
        s += (nv / 6) * 39 * 8 + nout * 4 + B * (p.local_order >= 2 ? 6 : 1) * nout * 8;
    if (I.kmax > 0) {                         // history grid
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        auto acc = [&](double x, double y) {
            x0 = std::min(x0, x); x1 = std::max(x1, x);
            y0 = std::min(y0, y); y1 = std::max(y1, y);
        };
        for (int64_t i = 0; i < nb; ++i) acc(b->x[i], b->y[i]);
        for (int64_t i = 0; i < nv; ++i) acc(v->x[i], v->y[i]);
        for (int64_t i = 0; i < t->n; ++i) acc(t->x[i], t->y[i]);
        GridChoice g;
        TRY(choose_grid(p, I, x1 - x0, y1 - y0, g));
        const int64_t es = p.prec == MHK_FP64 ? 8 : 4;
        s += 4 * B * g.n * (g.n + 2) * es * 2;   // grids + FFT work estimate
        s += (nb + nv) * (8 * 3 + 4);
        s += (nb + nv) * 4 * 4 + 2 * (int64_t)(g.n / TILE) * (g.n / TILE) * 4;   // per-tile source lists
    }
    *bytes = s;
    return MHK_OK;
}

mhk_status mhk_plan_set_timing(mhk_plan *P, int enable)
{
    if (!P) {
        set_error("plan is NULL");
        return MHK_EINVAL;
    }
    P->timing = enable != 0;
    return MHK_OK;
}

mhk_status mhk_plan_info(const mhk_plan *P, mhk_info *info)
{
    if (!P || !info) {
        set_error("plan or info is NULL");
        return MHK_EINVAL;
    }
    mhk_plan *Q = const_cast<mhk_plan *>(P);
    TRY(collect_timing(Q));
    // closest-point solves that did not converge, counted on the device by
    // the evaluations queued so far
    MHK_HIP(hipStreamSynchronize(Q->stream));
    int32_t noconv = 0;
    MHK_HIP(hipMemcpy(&noconv, Q->loc.noconv, sizeof(noconv), hipMemcpyDeviceToHost));
    Q->info.n_noconv = noconv;
    *info = Q->info;
    return MHK_OK;
}

void mhk_plan_destroy(mhk_plan *P)
{
    if (P) {
        (void)hipStreamSynchronize(P->stream);
        free_plan(P);
    }
}

}  // extern "C"

namespace {

mhk_status validate_eval(const mhk_plan *P, int parts, const void *sigma, const void *mu, const void *f_vol,
                         const void *f_trg, const void *out_s, const void *out_d, const void *out_v)
{
    if (!P) {
        set_error("plan is NULL");
        return MHK_EINVAL;
    }
    if (parts < 0 || parts > (MHK_PART_ALL | MHK_PART_GEOMETRY)) {
        set_error("invalid parts mask");
        return MHK_EINVAL;
    }
    if ((sigma && !out_s) || (mu && !out_d) || (f_vol && !out_v)) {
        set_error("an input density was given without its output array");
        return MHK_EINVAL;
    }
    if (f_vol && out_v && !f_trg && (parts & MHK_PART_LOCAL) && !P->fj.active) {
        set_error("f_trg is required with f_vol for the local part of V (unless the volume nodes come in "
                  "groups of six per triangle, from which f at the targets is reconstructed)");
        return MHK_EINVAL;
    }
    if (f_vol && P->nv == 0) {
        set_error("f_vol given but the plan has no volume nodes");
        return MHK_EINVAL;
    }
    return MHK_OK;
}

// Stage times of the last timed evaluation, read when asked for (the
// evaluation itself does not wait for them): history stages and the local
// part on the plan's stream, the level sums on the side stream, whose span
// overlaps the history part.
mhk_status collect_timing(mhk_plan *P)
{
    if (!P->t_pending) return MHK_OK;
    P->t_pending = false;
    const bool levels = P->t_levels, geom = P->t_geom;
    MHK_HIP(hipEventSynchronize(P->ev[7]));
    float ms[8] = {0}, mg = 0;
    for (int e = 1; e <= 5; ++e) MHK_HIP(hipEventElapsedTime(&ms[e], P->ev[e - 1], P->ev[e]));
    if (geom) MHK_HIP(hipEventElapsedTime(&mg, P->ev[8], P->ev[9]));
    if (levels) MHK_HIP(hipEventElapsedTime(&ms[6], geom ? P->ev[9] : P->ev[8], P->ev[6]));
    // the local part starts when both the history part and the levels are done
    float t5 = 0, t6 = 0, t7 = 0;
    MHK_HIP(hipEventElapsedTime(&t5, P->ev[0], P->ev[5]));
    if (levels) MHK_HIP(hipEventElapsedTime(&t6, P->ev[0], P->ev[6]));
    MHK_HIP(hipEventElapsedTime(&t7, P->ev[0], P->ev[7]));
    ms[7] = t7 - std::max(t5, t6);
    P->info.ms_spread = ms[1];
    P->info.ms_fft = ms[2] + ms[4];
    P->info.ms_multiply = ms[3];
    P->info.ms_interp = ms[5];
    P->info.ms_levels = ms[6];
    P->info.ms_local = ms[7];
    P->info.ms_geometry = mg;
    P->info.ms_total = t7;
    return MHK_OK;
}

// Enqueue one evaluation on P->stream (no synchronisation).
mhk_status enqueue(mhk_plan *P, int parts, const void *sigma, const void *mu, const void *f_vol, const void *f_trg,
                   void *out_s, void *out_d, void *out_v, int nbatch)
{
    // densities of this evaluation (<= the plan's batch): every launch below
    // runs over P->bat of them, with [P->bat][..] strides in the grids and
    // accumulators
    P->bat = nbatch;
    const bool ws = sigma && out_s, wd = mu && out_d, wv = f_vol && out_v;
    if (!ws && !wd && !wv) return MHK_OK;
    hipStream_t st = P->stream;
    // f (and its derivatives) at the targets from the volume quadrature when
    // the caller gives none
    if (wv && !f_trg && (parts & MHK_PART_LOCAL) && P->fj.active) {
        MHK_HIP(launch_fjets(P, f_vol, P->fj.frec));
        f_trg = P->fj.frec;
    }
    // FP32 plan given FP64 inputs: spreading and the level sums read float
    // copies (rounded once here), the local part the caller's doubles
    const void *sig_h = sigma, *mu_h = mu, *fv_h = f_vol;
    if (P->p.in64) {
        float *s32 = P->in32, *m32 = P->in32 + (size_t)nbatch * P->nb, *f32 = P->in32 + (size_t)2 * nbatch * P->nb;
        if (ws) MHK_HIP(launch_round32(P, sigma, s32, (int64_t)nbatch * P->nb));
        if (wd) MHK_HIP(launch_round32(P, mu, m32, (int64_t)nbatch * P->nb));
        if (wv) MHK_HIP(launch_round32(P, f_vol, f32, (int64_t)nbatch * P->nv));
        sig_h = s32;
        mu_h = m32;
        fv_h = f32;
    }
    const int B = P->bat;
    const int64_t nout = P->nout;
    if (P->timing) MHK_HIP(hipEventRecord(P->ev[0], st));
    // The level sums share no data with the history part: they run on the
    // side stream, forked from and joined back into the plan's stream, so the
    // two overlap (the level sums are bound by LDS and FP64 issue, the FFTs by
    // memory).  They write acc_lev; the local part adds it.
    const bool levels = (parts & MHK_PART_LEVELS) && (ws || wd) && P->J > 0;
    // the volume potential's levels (v_levels) run there too
    const bool vlevels = (parts & MHK_PART_LEVELS) && wv && P->p.v_levels;
    const bool side = levels || vlevels;
    // the local geometry (closest points, MHK_PART_GEOMETRY) depends on
    // nothing but the plan: it goes first on the side stream, beside the
    // history part, or on the plan's stream when there are no level sums
    const bool geom = (parts & MHK_PART_GEOMETRY) && (parts & MHK_PART_LOCAL);
    if (geom && !side) {
        if (P->timing) MHK_HIP(hipEventRecord(P->ev[8], st));
        MHK_HIP(launch_local_geom(P, st));
        if (P->timing) MHK_HIP(hipEventRecord(P->ev[9], st));
    }
    if (side) {
        MHK_HIP(hipEventRecord(P->fork_ev, st));
        MHK_HIP(hipStreamWaitEvent(P->side, P->fork_ev, 0));
        if (P->timing) MHK_HIP(hipEventRecord(P->ev[8], P->side));
        if (geom) {
            MHK_HIP(launch_local_geom(P, P->side));
            if (P->timing) MHK_HIP(hipEventRecord(P->ev[9], P->side));
        }
        if (levels)
            for (int j = 1; j <= P->J; ++j) {
                MHK_HIP(launch_level_densities(P, P->side, j, ws ? sig_h : nullptr, wd ? mu_h : nullptr));
                MHK_HIP(launch_level_sums(P, P->side, j, ws, wd, j == 1));
            }
        if (vlevels)
            for (int j = 1; j <= P->J; ++j) {
                MHK_HIP(launch_vlevel_q(P, P->side, j, f_vol));
                MHK_HIP(launch_level_sums_v(P, P->side, j, j == 1));
            }
        if (P->timing) MHK_HIP(hipEventRecord(P->ev[6], P->side));
        MHK_HIP(hipEventRecord(P->join_ev, P->side));
    }
    // history part writes the accumulators (or zeros them)
    bool hist = (parts & MHK_PART_HISTORY) && P->hist.active;
    if (hist) {
        MHK_HIP(launch_spread(P, ws ? sig_h : nullptr, wd ? mu_h : nullptr, wv ? fv_h : nullptr));
        if (P->timing) MHK_HIP(hipEventRecord(P->ev[1], st));
        void *buf[1] = {P->hist.grid};
        // column path: row transforms, column transforms with the
        // multiplier, inverse row transforms; else rocFFT 2D transforms
        // around the multiplier
        if (P->hist.colpath)
            MHK_HIP(launch_rows(P, false));
        else
            MHK_FFT(rocfft_execute(P->hist.fwd, buf, nullptr, P->hist.exec));
        if (P->timing) MHK_HIP(hipEventRecord(P->ev[2], st));
        MHK_HIP(P->hist.colpath ? launch_columns(P) : launch_multiply(P));
        if (P->timing) MHK_HIP(hipEventRecord(P->ev[3], st));
        if (P->hist.colpath)
            MHK_HIP(launch_rows(P, true));
        else
            MHK_FFT(rocfft_execute(P->hist.inv, buf, nullptr, P->hist.exec));
        if (P->timing) MHK_HIP(hipEventRecord(P->ev[4], st));
        MHK_HIP(launch_interp(P, ws, wd, wv));
    } else {
        MHK_HIP(launch_fill(P, P->acc, 3 * (int64_t)B * nout));
        if (P->timing)
            for (int e = 1; e <= 4; ++e) MHK_HIP(hipEventRecord(P->ev[e], st));
    }
    if (P->timing) MHK_HIP(hipEventRecord(P->ev[5], st));
    if (side) MHK_HIP(hipStreamWaitEvent(st, P->join_ev, 0));
    // f at the boundary nodes (the on-surface entries of f_trg) gives the
    // local volume part at exterior targets near the boundary
    const bool have_fb = wv && (parts & MHK_PART_LOCAL) && P->nout > P->nt;
    if ((parts & MHK_PART_LOCAL) && (ws || wd || have_fb))
        MHK_HIP(launch_panel_coeffs(P, ws ? sigma : nullptr, wd ? mu : nullptr, have_fb ? f_trg : nullptr));
    MHK_HIP(launch_local(P, parts, ws ? sigma : nullptr, wd ? mu : nullptr, wv ? f_trg : nullptr,
                         ws ? out_s : nullptr, wd ? out_d : nullptr, wv ? out_v : nullptr, have_fb, levels,
                         vlevels));
    if (P->timing) {
        MHK_HIP(hipEventRecord(P->ev[7], st));
        P->t_pending = true;
        P->t_levels = side;
        P->t_geom = geom;
    }
    return MHK_OK;
}

}  // namespace

extern "C" {

mhk_status mhk_eval_parts(mhk_plan *P, int parts, const void *sigma, const void *mu, const void *f_vol,
                          const void *f_trg, void *out_s, void *out_d, void *out_v)
{
    TRY(validate_eval(P, parts, sigma, mu, f_vol, f_trg, out_s, out_d, out_v));
    return enqueue(P, parts, sigma, mu, f_vol, f_trg, out_s, out_d, out_v, P->p.batch);
}

mhk_status mhk_plan_f_targets(mhk_plan *P, const void *f_vol, void *f_trg)
{
    if (!P || !f_vol || !f_trg) {
        set_error("plan, f_vol and f_trg are required");
        return MHK_EINVAL;
    }
    if (!P->fj.active) {
        set_error("the plan's volume nodes are not in groups of six per triangle");
        return MHK_EINVAL;
    }
    P->bat = P->p.batch;
    MHK_HIP(launch_fjets(P, f_vol, f_trg));
    return MHK_OK;
}

mhk_status mhk_eval_batch(mhk_plan *P, int nbatch, int parts, const void *sigma, const void *mu, const void *f_vol,
                          const void *f_trg, void *out_s, void *out_d, void *out_v)
{
    TRY(validate_eval(P, parts, sigma, mu, f_vol, f_trg, out_s, out_d, out_v));
    if (nbatch < 1 || nbatch > P->p.batch) {
        set_error("nbatch must be in [1, batch] of the plan");
        return MHK_EINVAL;
    }
    return enqueue(P, parts, sigma, mu, f_vol, f_trg, out_s, out_d, out_v, nbatch);
}

mhk_status mhk_plan_capture(mhk_plan *P, int parts, const void *sigma, const void *mu, const void *f_vol,
                            const void *f_trg, void *out_s, void *out_d, void *out_v)
{
    TRY(validate_eval(P, parts, sigma, mu, f_vol, f_trg, out_s, out_d, out_v));
    if (!P->cap) MHK_HIP(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
    // the work captured must not depend on work still queued on the plan's stream
    MHK_HIP(hipStreamSynchronize(P->stream));
    hipStream_t saved = P->stream;
    const bool timing = P->timing;
    P->stream = P->cap;
    P->timing = false;
    if (P->hist.exec) MHK_FFT(rocfft_execution_info_set_stream(P->hist.exec, P->cap));
    hipGraph_t g = nullptr;
    mhk_status st = MHK_OK;
    hipError_t e = hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        set_error(std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        st = MHK_EHIP;
    } else {
        st = enqueue(P, parts, sigma, mu, f_vol, f_trg, out_s, out_d, out_v, P->p.batch);
        e = hipStreamEndCapture(P->cap, &g);
        if (st == MHK_OK && e != hipSuccess) {
            set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            st = MHK_EHIP;
        }
    }
    P->stream = saved;
    P->timing = timing;
    if (P->hist.exec) MHK_FFT(rocfft_execution_info_set_stream(P->hist.exec, saved));
    if (st == MHK_OK) {
        if (P->gexec) {
            (void)hipGraphExecDestroy(P->gexec);
            P->gexec = nullptr;
        }
        e = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            P->gexec = nullptr;
            st = MHK_EHIP;
        }
    }
    if (g) (void)hipGraphDestroy(g);
    return st;
}

mhk_status mhk_plan_launch_graph(mhk_plan *P)
{
    if (!P || !P->gexec) {
        set_error("no captured graph on this plan");
        return MHK_EINVAL;
    }
    MHK_HIP(hipGraphLaunch(P->gexec, P->stream));
    return MHK_OK;
}

mhk_status mhk_eval(mhk_plan *P, const void *sigma, const void *mu, const void *f_vol, const void *f_trg,
                    void *out_S, void *out_D, void *out_V)
{
    return mhk_eval_parts(P, MHK_PART_ALL, sigma, mu, f_vol, f_trg, out_S, out_D, out_V);
}

mhk_status mhk_eval_S(mhk_plan *P, const void *sigma, void *out_S)
{
    if (!sigma || !out_S) {
        set_error("sigma and out_S are required");
        return MHK_EINVAL;
    }
    return mhk_eval_parts(P, MHK_PART_ALL, sigma, nullptr, nullptr, nullptr, out_S, nullptr, nullptr);
}

mhk_status mhk_eval_D(mhk_plan *P, const void *mu, void *out_D)
{
    if (!mu || !out_D) {
        set_error("mu and out_D are required");
        return MHK_EINVAL;
    }
    return mhk_eval_parts(P, MHK_PART_ALL, nullptr, mu, nullptr, nullptr, nullptr, out_D, nullptr);
}

mhk_status mhk_eval_V(mhk_plan *P, const void *f_vol, const void *f_trg, void *out_V)
{
    if (!f_vol || !f_trg || !out_V) {
        set_error("f_vol, f_trg and out_V are required");
        return MHK_EINVAL;
    }
    return mhk_eval_parts(P, MHK_PART_ALL, nullptr, nullptr, f_vol, f_trg, nullptr, nullptr, out_V);
}

}  // extern "C"
