// Internal declarations of libmhk (not part of the C ABI).
//
// Data layout in HBM (all arrays device-resident, owned by the plan):
//  * targets: the n_out = N_T (+ N_B) evaluation points sorted in Morton
//    order of small square cells aligned with the history grid tiles, as
//    SoA x/y (FP64), inside flag and original output index;
//  * boundary: the caller's panel-contiguous SoA arrays, plus per-panel
//    Legendre coefficients of x, y and kappa for the closest-point search;
//  * dyadic level j: the N_B 2^j child nodes of the bisected panels, sorted
//    row-major by square cells of side R_j/4, as SoA x/y/w nx/w ny/w, with a
//    code giving (panel, child, node) for the per-eval interpolation of the
//    densities, per-eval strengths q_S = w sigma, q_Dx = w nu_x mu,
//    q_Dy = w nu_y mu in the same sorted order, and per target wavefront a
//    flat list of the child nodes within R_j of its targets;
//  * history: per-tile lists of the boundary and volume sources whose windows
//    meet each 32x32 tile of the fine grid, the fine grids
//    [4][batch][n][n+2] (S, V, D_x, D_y sources, real, rows padded for
//    in-place real-to-complex FFTs; only the rows and columns of the sources'
//    and targets' windows are touched) and the 1D factors of the Fourier
//    multiplier or the truncated kernel's spectrum;
//  * local: per sorted target the closest panel, parameter and the
//    density-independent coefficients of the local expansions;
//  * f-jets and volume levels (6-node volume groups): per triangle the
//    inverse of its scaled 6x6 Vandermonde and centroid/scale, per target the
//    nearest usable triangle; per volume level the refined nodes sorted by
//    cells, with their parent triangles and wavefront lists.
// Everything is built on the device at plan creation, in stream order on the
// plan's stream.
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mhk.h"

namespace mhk {

constexpr int NGL = 16;          // Gauss-Legendre nodes per panel (Section 3.2)
constexpr int TILE = 32;         // fine-grid tile edge of spreading/interpolation
constexpr int MAXJ = 8;          // maximum number of dyadic levels
constexpr int TAB_NC = 8;        // coefficients per table segment (degree 7)
constexpr int TAB_NC64 = 5;      // FP64 path: c_0..c_4 stored as doubles, c_5..c_7 as floats
constexpr int TAB_STRIDE = 6;    // doubles per segment row: c_0..c_4 and c_5, c_6 as two floats (48 bytes);
                                 // c_7 (float) in an array of its own after the rows
                                 // (14 dwords: spreads segments over the banks)
constexpr int TABF_NC = 8;       // FP32 path: coefficients per segment (degree 7)
constexpr int TABF_STRIDE = 9;   // FP32 path: floats per segment
constexpr int COL_NMAX = 8192;   // longest history-grid column transformed in LDS
constexpr int COL_MAXPASS = 16;  // radix passes of a column transform
constexpr int LV_CDIV = 4;       // level cells are R_j / LV_CDIV wide
constexpr int MAXW = 16;         // maximum spreading window width
constexpr int LV_BLOCK_MAX = 512;  // largest level-sum workgroup (targets); 256 or 512 per plan
constexpr int LV_WAVE = 64;      // lanes per level-sum wavefront
constexpr int LOCAL_GEO_N1 = 10; // doubles of local geometry per target, first-order plans
constexpr int LOCAL_GEO_N2 = 27; // the same with the second-order terms (local_order = 2)

void set_error(const std::string &msg);

template <typename T> struct Vec2;
template <> struct Vec2<double> { typedef double2 type; };
template <> struct Vec2<float> { typedef float2 type; };

struct Level {
    double delta_j = 0;          // delta / 4^(j-1): upper end of the level's time interval
    double inv4d = 0;            // 1 / (4 delta_j)
    double a_max = 0;            // cut-off in a = r^2/(4 delta_j)
    double radius = 0;           // sqrt(4 delta_j a_max)
    double seg_inv = 0;          // segments per unit of a
    int nseg = 0;
    int nchild = 0;              // 2^j
    int64_t n_src = 0;           // N_B 2^j
    int ncx = 0, ncy = 0;
    double cell = 0, ox = 0, oy = 0;
    // device
    double *sx = nullptr, *sy = nullptr;          // sorted child nodes
    double *swx = nullptr, *swy = nullptr;        // w nu_x, w nu_y
    double *sw = nullptr;                         // w
    int32_t *code = nullptr;                      // (panel * nchild + child) * 16 + node
    int32_t *cell_start = nullptr;                // [ncx*ncy + 1]
    // per wavefront of LV_WAVE sorted targets: the sorted sources within R_j
    // of the wavefront's target bounding box, as one flat list of indices
    // (wave_src[wave_ofs[w] .. wave_ofs[w + 1]))
    int32_t *wave_ofs = nullptr;                  // [n_waves + 1]
    int32_t *wave_order = nullptr;                // wavefronts in decreasing order of candidate work
    int32_t *wave_src = nullptr;                  // [n_cand]
    int64_t n_cand = 0;
    int64_t n_wave = 0;                           // wavefronts of LV_WAVE targets (whole LV_BLOCK_MAX workgroups)
    double *interp = nullptr;                     // [nchild][16][16] parent -> child values
    double *tab = nullptr;                        // [nseg][TAB_STRIDE]: K_j^S per segment (K_j^D from its derivative)
    float *tabf = nullptr;                        // FP32 path: [nseg][TABF_STRIDE]
    void *tab_dev = nullptr;                      // the table of the plan's precision
    void *q = nullptr;                            // per eval: [3][batch][n_src], plan precision
    double tab_err = 0;                           // measured max table error / K(0)
};

// Factor taking the v-derivative of a level's K_j^S polynomial to K_j^D:
// K_j^D = -(1/(2 delta_j)) dK_j^S/da and da/dv = 1/(2 seg_inv), so
// K_j^D = -(seg_inv/delta_j) dp/dv = -4 inv4d seg_inv dp/dv.
inline double level_d_scale(const Level &L) { return -4.0 * L.inv4d * L.seg_inv; }

struct History {
    bool active = false;
    double kcut = 0, period = 0, h = 0, ox = 0, oy = 0;
    double beta = 0, ups = 2.0;
    int w = 0;
    int64_t n = 0;               // fine grid points per dimension
    int ntile = 0;               // n / TILE
    int64_t field = 0;           // doubles per padded real field: n*(n+2)
    // sorted sources (grid coordinates) and original indices
    int64_t nbs = 0, nvs = 0;
    double *bgx = nullptr, *bgy = nullptr;        // boundary nodes
    double *bw = nullptr, *bwx = nullptr, *bwy = nullptr;
    int32_t *bidx = nullptr;
    double *vgx = nullptr, *vgy = nullptr, *vw = nullptr;
    int32_t *vidx = nullptr;
    // per tile, the sorted sources whose w x w window meets the tile (a
    // source is listed in up to 4 tiles): lists [*lofs[t], *lofs[t + 1])
    int32_t *blofs = nullptr, *blist = nullptr;   // boundary: [ntile*ntile + 1], entries
    int32_t *vlofs = nullptr, *vlist = nullptr;   // volume
    // targets by tile: list of non-empty tiles and their ranges in sorted order
    int n_ttiles = 0;
    int32_t *ttile_xy = nullptr;                  // [n_ttiles] tile index ty*ntile+tx
    int32_t *ttile_rng = nullptr;                 // [n_ttiles + 1]
    // window phi_k(t), k = 0..w-1, as monomials of degree w+3 in t = 2u - 1,
    // u = m0 - g + w/2 in [0, 1): [w][w+4] in the plan precision
    void *wcoef = nullptr;
    double wfit_err = 0;
    // multiplier factors A[l] = exp(-delta k_l^2)/phihat(k_l)^2, 0 beyond kcut
    double *fac = nullptr;                        // [n/2+1]
    double mult_c = 0;                            // h^4/P^2 exp(-delta alpha^2)
    // truncated-kernel mode: the history kernel is cut off smoothly beyond the
    // largest source-target distance and its spectrum tabulated on the kept
    // modes |l_x|, |l_y| <= lmax (already divided by phihat^2, times h^4/P^2)
    bool trunc = false;
    int lmax = 0;
    double *mtab = nullptr;                       // [2 lmax + 1][lmax + 1]
    double trunc_d = 0, trunc_w = 0;              // separation bound D, transition width
    // grids
    void *grid = nullptr;                         // [4][batch][field], plan precision
    void *work = nullptr;
    size_t work_bytes = 0;
    rocfft_plan fwd = nullptr, inv = nullptr;
    rocfft_execution_info exec = nullptr;
    // column path (n <= COL_NMAX, n = 2^a 3^b 5^c, even): k_rows does the
    // row transforms and k_columns the column transforms with the
    // multiplier; otherwise fwd / inv are rocFFT 2D transforms and k_multiply
    // runs between them
    bool colpath = false;
    int ncol = 0;                                 // columns l_x that can hold a nonzero multiplier
    // column path: grid index ranges [lo, hi) holding the sources' windows
    // (spread, forward row transforms, column inputs) and the targets'
    // windows (column outputs, inverse row transforms, interpolation); the
    // grid outside them is neither written nor read
    int sx0 = 0, sx1 = 0, sy0 = 0, sy1 = 0;
    int tx0 = 0, tx1 = 0, ty0 = 0, ty1 = 0;
    int npass = 0;
    int8_t radix[COL_MAXPASS] = {};               // passes of the column transforms (length n)
    int rnpass = 0;
    int8_t rradix[COL_MAXPASS] = {};              // passes of the row transforms (length n/2)
    void *tw = nullptr;                           // [n] e^{-2 pi i m / n}, FP64
};

struct Local {
    // closest-point cells: square cells of side `cell` over the bounding
    // box; cell c lists (cand[cell_start[c] .. cell_start[c+1])) the panels
    // whose node bounding box lies within `reach` = band + largest node gap
    // of the cell, nearest first
    double cell = 0, ox = 0, oy = 0, gap = 0, reach = 0;
    int ncx = 0, ncy = 0;
    int32_t *cand = nullptr;
    double *pbox = nullptr;                       // [n_panels][4]: node bounding box xmin, xmax, ymin, ymax
    double *cbox = nullptr;                       // [n_panels][4]: box of the panel's whole curve (with a margin)
    int32_t *cell_start = nullptr;
    int32_t *noconv = nullptr;                    // device counter: closest-point solves that did not converge
    double *leg = nullptr;                        // [16][16] nodal values -> Legendre coefficients
    double *cx = nullptr, *cy = nullptr, *ck = nullptr;   // [n_panels][16]
    double *ends = nullptr;                       // [n_panels][4]: x(-1), y(-1), x(1), y(1)
    double *gl_t = nullptr;                       // [16] Gauss-Legendre abscissae
    int32_t *prev = nullptr, *next = nullptr;     // panel neighbours within each curve
    double *csig = nullptr, *cmu = nullptr;       // per eval: [batch][n_panels][16] (FP64)
    double *cf = nullptr;                         // f at the boundary nodes, same layout
    double *geo = nullptr;                        // per-plan local geometry [10][n_out] (sorted order)
    int32_t *gpan = nullptr;                      // closest panel per sorted target (-1: none)
    uint8_t *gflag = nullptr;                     // bit 0: in the layer band, bit 1: exterior in the volume band
};

}  // namespace mhk

namespace mhk {
// f at the targets from the volume quadrature (volume nodes in groups of six)
struct FJets {
    bool active = false;
    double *minv = nullptr;      // [ntri][6][6] inverse of the monomial matrix at the six nodes
    double *tc = nullptr;        // [ntri][3] centroid x, y and scale h
    int32_t *tri = nullptr;      // [n_out] sorted target -> triangle (-1: f not needed)
    void *frec = nullptr;        // per eval: [batch][rows][n_out] f (and jets), caller order, input precision
    // cell list of the nodes of usable triangles
    int32_t *perm = nullptr, *start = nullptr;
    uint8_t *good = nullptr;     // [ntri] usable triangle (not a sliver)
    double ox = 0, oy = 0, cell = 0;
    int64_t ncx = 0, ncy = 0;
};

// reference rule of the volume triangles (points (s_i, t_i) on T0, weights
// W_i) and the inverse of the monomial matrix 1, s, t, s^2, st, t^2 at the
// points (the quadratic map of a triangle from its six nodes)
struct VRule {
    double rinv[36];
    double s[6], t[6], W[6];
};

// dyadic level j of the volume potential: the level nodes sorted by cells of
// side R_j/4, their triangles for f, per-wavefront candidate lists
struct VLevel {
    int64_t n_src = 0;
    double *sx = nullptr, *sy = nullptr, *sw = nullptr;
    int32_t *tri = nullptr;
    int32_t *cell_start = nullptr;
    int32_t *wave_ofs = nullptr, *wave_src = nullptr, *wave_order = nullptr;
    int64_t n_wave = 0, n_cand = 0;
    void *q = nullptr;           // per eval: [batch][n_src], plan precision
};
}  // namespace mhk

struct mhk_plan {
    mhk_params p{};
    mhk_info info{};
    hipStream_t stream = nullptr;
    bool timing = false;
    int bat = 1;                                 // densities of the evaluation being enqueued (<= p.batch)
    int *lv_counter = nullptr;                   // work-item counter of the persistent level sums
    float *in32 = nullptr;                       // FP32 plans with in64: [batch][2 N_B + N_V] rounded inputs
    int64_t nb = 0, npan = 0, nv = 0, nt = 0, nout = 0;
    bool targets_are_volume = false;            // targets == volume nodes, same order
    int J = 3;
    double delta = 0, dstar = 0;
    // boundary (caller order)
    double *bx = nullptr, *by = nullptr, *bnx = nullptr, *bny = nullptr, *bw = nullptr, *bk = nullptr;
    // sorted targets
    double *tx = nullptr, *ty = nullptr;
    int8_t *tin = nullptr;
    int32_t *tidx = nullptr;
    // accumulators in sorted target order: [3][batch][n_out] (S, D, V), plan precision
    void *acc = nullptr;
    size_t es = 8;                               // bytes per value of the plan precision
    mhk::Level lev[mhk::MAXJ];
    mhk::History hist;
    mhk::Local loc;
    mhk::FJets fj;
    mhk::VLevel vlev[mhk::MAXJ];                // volume levels (params.v_levels)
    void *acc_vlev = nullptr;                    // [batch][n_out] their sums, sorted order
    double delta_v = 0;                          // time split of V's local part: delta, or delta* with volume levels
    std::vector<void *> allocs;                 // stream-ordered allocations on `stream`
    std::vector<std::vector<char>> stage;       // host bytes of uploads in flight during creation
    int64_t bytes = 0;
    // stage timing: ev[0..7] history stages and local part on the plan's
    // stream, ev[8] start of the side work, ev[9] end of the local geometry
    hipEvent_t ev[10] = {};
    bool t_pending = false, t_levels = false, t_geom = false;   // stage events recorded, not read yet
    hipStream_t cap = nullptr;                  // capture stream of mhk_plan_capture
    // The level sums run on a second stream beside the history part (they
    // share no data): they accumulate S and D into acc_lev, [2][batch][n_out],
    // which the local part adds.
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    void *acc_lev = nullptr;
    hipGraphExec_t gexec = nullptr;             // captured evaluation
};

namespace mhk {

// kernels launchers (defined in the .hip files); density and output pointers
// are of the plan's precision
hipError_t launch_level_densities(mhk_plan *P, hipStream_t st, int j, const void *sigma, const void *mu);
// level j's sums into acc_lev on stream st: stored when init, else added
hipError_t launch_level_sums(mhk_plan *P, hipStream_t st, int j, bool want_s, bool want_d, bool init);
hipError_t launch_panel_coeffs(mhk_plan *P, const void *sigma, const void *mu, const void *f_bnd);
hipError_t launch_local_geom(mhk_plan *P, hipStream_t st);
hipError_t launch_local(mhk_plan *P, int parts, const void *sigma, const void *mu,
                        const void *f_trg, void *out_s, void *out_d, void *out_v, bool have_fb, bool have_lev,
                        bool have_vlev);
hipError_t launch_spread(mhk_plan *P, const void *sigma, const void *mu, const void *f_vol);
hipError_t launch_multiply(mhk_plan *P);
hipError_t launch_columns(mhk_plan *P);
hipError_t launch_rows(mhk_plan *P, bool inverse);
hipError_t launch_interp(mhk_plan *P, bool want_s, bool want_d, bool want_v);
hipError_t launch_fill(mhk_plan *P, void *p, int64_t n);
hipError_t launch_fill_int(int *p, int64_t n, hipStream_t st);   // zero n ints on st (a kernel, graph-safe)
hipError_t launch_round32(mhk_plan *P, const void *x, void *y, int64_t n);
hipError_t launch_fjets(mhk_plan *P, const void *f_vol, void *out);
hipError_t dev_fj_nearest_pts(mhk_plan *P, int64_t n, const double *px, const double *py, const int32_t *parent,
                              const double *vx, const double *vy, int32_t *tri, hipStream_t st);
hipError_t dev_vlevel_nodes(int64_t ntri, int j, const VRule &M, const double *vx, const double *vy, double ox,
                            double oy, double cell, int64_t ncx, int64_t ncy, double *sx, double *sy, double *sw,
                            int32_t *parent, int32_t *cell_start, hipStream_t st);
hipError_t launch_vlevel_q(mhk_plan *P, hipStream_t st, int j, const void *f_vol);
// level j's single-layer sums over the volume level nodes into acc_vlev
hipError_t launch_level_sums_v(mhk_plan *P, hipStream_t st, int j, bool init);
hipError_t dev_fj_setup(int64_t ntri, const double *vx, const double *vy, double *minv, double *tc, uint8_t *good,
                        hipStream_t st);
hipError_t dev_fj_nearest(mhk_plan *P, const double *vx, const double *vy, const uint8_t *good, double ox,
                          double oy, double cell, int64_t ncx, int64_t ncy, int32_t *tri, hipStream_t st);
hipError_t launch_trunc_kernel_samples(double *buf, int64_t M, double h, double alpha, double delta, double rmid,
                                       double slope, const double *gl_t, const double *gl_w, hipStream_t s);
hipError_t launch_cos_step(const double *in, int64_t K, int64_t NA, int64_t NB, int n, const double *costab,
                           double *out, hipStream_t s);
hipError_t launch_trunc_table(const double *tr, int lmax, const double *phi2inv, double c, double *mtab,
                              hipStream_t s);

// Device-side binning of plan creation (bin.hip); every call is
// asynchronous on st and allocates its temporaries in the order of st.
// Stable sort of (key, value) pairs by the low `bits` bits of the keys.
hipError_t dev_sort_pairs(uint32_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t st);
// out[0..n]: exclusive prefix sums of in[0..n), out[n] the total (also in
// *total as int64, for the caller's overflow check).
hipError_t dev_scan(const int32_t *in, int32_t *out, int64_t n, int64_t *total, hipStream_t st);
// start[c], c in [0, nkeys]: first index of key c in a sorted key array.
hipError_t dev_cell_starts(const uint32_t *keys, int64_t n, int64_t nkeys, int32_t *start, hipStream_t st);
// Inside mask of n targets (caller order) from the polygon through the
// panels' end points and nodes, corrected in the lunes between its edges and
// the panels' arcs; edges listed per horizontal strip.
struct MaskArgs {
    int64_t n;
    const double *tx, *ty;
    double ylo, yhi, hinv;
    int nstrip;
    const int32_t *strip_start, *strip_edge;   // [nstrip + 1], edge indices
    const double *edge;                        // [E][4]: x0, y0, x1, y1
    const double *sag;                         // [E]: arc-to-chord bound, 0 for no lune
    const int32_t *edge_pan;                   // [E]: panel of the arc
    const double *edge_t;                      // [E][2]: panel parameters of the edge's ends
    const double *bx, *by;                     // boundary nodes [N_B]
    const double *gl_t, *lam;                  // Gauss-Legendre nodes and barycentric weights [16]
};
hipError_t dev_inside_mask(const MaskArgs &A, int8_t *out, hipStream_t st);
// Targets sorted by the Morton key of cells of side hh from (ox, oy).
hipError_t dev_sort_targets(const double *x, const double *y, const int8_t *in, int64_t n, double ox, double oy,
                            double hh, double *sx, double *sy, int8_t *sin, int32_t *sidx, hipStream_t st);
// Child nodes of a dyadic level, sorted by cells, with the cell starts.
hipError_t dev_child_nodes(int64_t n_src, int nch, const double *Tm, const double *bx, const double *by,
                           const double *bnx, const double *bny, const double *bw, const double *glw, double ox,
                           double oy, double cell, int64_t ncx, int64_t ncy, double *sx, double *sy, double *sw,
                           double *swx, double *swy, int32_t *code, int32_t *cell_start, hipStream_t st);
// Per-wavefront candidate lists of a level: counts, then (after the scan of
// the counts into ofs) the lists and the wavefronts in decreasing work.
hipError_t dev_wave_counts(const double *tx, const double *ty, int64_t nout, int64_t nwave, double R, double R2,
                           double ox, double oy, double cell, int64_t ncx, int64_t ncy, const int32_t *start,
                           const double *sx, const double *sy, int32_t *cnt, hipStream_t st);
hipError_t dev_wave_fill(const double *tx, const double *ty, int64_t nout, int64_t nwave, double R, double R2,
                         double ox, double oy, double cell, int64_t ncx, int64_t ncy, const int32_t *start,
                         const double *sx, const double *sy, const int32_t *ofs, int32_t *out, int32_t *order,
                         hipStream_t st);
// History sources by spreading tile (sorted arrays, window bounds into
// sup, list offsets into lofs) and their per-tile lists.
hipError_t dev_sources_by_tile(const double *x, const double *y, const double *w, const double *nx, const double *ny,
                               int64_t n, double ox, double oy, double h, int64_t ntile, int W, double *gx, double *gy,
                               double *gw, double *gwx, double *gwy, int32_t *idx, int *sup, int32_t *lofs,
                               int32_t **tstart_out, int64_t *total, hipStream_t st);
hipError_t dev_tile_fill(const double *gx, const double *gy, const int32_t *tstart, int64_t ntile, int W,
                         const int32_t *lofs, int32_t *list, hipStream_t st);
// Runs of equal tiles along the sorted targets, and their window bounds.
hipError_t dev_target_tiles_count(const double *tx, const double *ty, int64_t n, double ox, double oy, double h,
                                  int64_t ntile, int W, int *win, int32_t **flag_out, int32_t **pos_out,
                                  int64_t *runs_dev, hipStream_t st);
hipError_t dev_target_tiles_fill(const double *tx, const double *ty, int64_t n, double ox, double oy, double h,
                                 int64_t ntile, const int32_t *flag, const int32_t *pos, int32_t *xy, int32_t *rng,
                                 hipStream_t st);

}  // namespace mhk
