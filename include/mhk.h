/*
 * mhk.h -- C ABI of libmhk: fast evaluation of the layer potentials S[sigma],
 * D[mu] and the volume potential V[f] of the 2D modified Helmholtz equation
 * (-Lap + alpha^2) u = f, with G(x) = K0(alpha |x|)/(2 pi) (paper Section 1,
 * eqs. (mod_helm), (Greens), (vp), (slp), (dlp)), on one AMD MI355X (gfx950).
 *
 * The Green's function is split in time (Section 2.1, eqs. (ker_greens),
 * (sl_sh), (slp_dyad)): t > delta is the smooth history part, evaluated by a
 * type-1 NUFFT of the quadrature sources, the multiplier of eq. (sh_fourier)
 * and a type-2 NUFFT at the targets (Section 5); t in [delta/4^j,
 * delta/4^(j-1)], j = 1..J, are the dyadic difference-kernel levels of the
 * layer potentials, summed over locally bisected panels (Section 4.2, eqs.
 * (diffker_s), (diffker_dlp)); t < delta* = delta/4^J (delta for V) is the
 * local asymptotic part (Lemmas 4.1, 4.5, 4.8 and Corollaries 4.4, 4.7,
 * 4.10, 4.11, kept to first order as stated in Section 4.1).
 *
 * Conventions common to every call
 *  - Geometry passed to mhk_plan_create is HOST memory; the plan copies and
 *    reorders it into device buffers that it owns.  The caller may free its
 *    arrays as soon as mhk_plan_create returns.
 *  - Densities, sources and outputs passed to the eval calls are DEVICE
 *    pointers (e.g. a torch tensor's data_ptr()), contiguous, in the caller's
 *    node order, with the batch index outermost: sigma[b][N_B].  Their type
 *    is double when params.prec == MHK_FP64 and float when MHK_FP32 (inputs
 *    double for an FP32 plan with params.in64 = 1).
 *  - Eval calls are asynchronous on the stream given at plan creation; the
 *    outputs are valid once that stream has been synchronised (the plan's
 *    internal second stream, which runs the level sums, is joined back into
 *    it by an event within each eval).  A plan is not re-entrant; different
 *    plans may run concurrently on different streams.
 *  - Every call returns an mhk_status; on error nothing is enqueued and
 *    mhk_last_error() (thread-local) describes the problem.
 *  - Boundary: n_panels panels of 16 Gauss-Legendre nodes each, panel
 *    contiguous, every curve counter-clockwise with panels in increasing
 *    parameter order (Section 3.2).  nx, ny is the outward unit normal, w the
 *    quadrature weight (eq. (eq:bdry_quad), speed included) and kappa the
 *    signed curvature (positive where the curve is convex).
 *  - Target outputs: the N_T off-surface targets first, then, if
 *    targets.on_surface is set, the N_B boundary nodes as on-surface targets
 *    (D there is the direct value, i.e. the principal value of eq. (jumprel)).
 *    At exterior targets closer to the boundary than sqrt(delta)(12 + 2 alpha
 *    sqrt(delta)) the local part of V comes from the complement domain
 *    (Lemma 4.8 holds for x in Omega; the complement contains x): first
 *    order, with f at the closest boundary point interpolated from f at the
 *    boundary nodes, i.e. the on-surface entries of f_trg.  Without
 *    on-surface targets those entries are NaN.
 */
#ifndef MHK_H
#define MHK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MHK_OK = 0,
    MHK_EINVAL = -1,       /* invalid argument (message in mhk_last_error) */
    MHK_ENOMEM = -2,       /* device allocation failed / footprint too large */
    MHK_EHIP = -3,         /* HIP runtime or rocFFT error */
    MHK_EUNSUPPORTED = -4, /* valid but unsupported configuration */
    MHK_ENOCONV = -5       /* the closest-point Newton iteration (Section 3.2) did not
                              converge for a target inside a local band            */
} mhk_status;

enum { MHK_FP64 = 0, MHK_FP32 = 1 };

/* Parts of the split, for mhk_eval_parts (bit mask).  MHK_PART_GEOMETRY is
 * not a part of the split: with it, the evaluation first recomputes the
 * target geometry of the local part -- the closest boundary point of every
 * target (nearest node, then Newton on its panel and the two neighbouring
 * panels, Section 3.2) and the density-independent coefficients of Lemmas
 * 4.1, 4.5 and 4.8 -- instead of using the ones computed at plan creation.
 * The results are the same either way; the bit makes the closest-point
 * search part of the evaluation's work and time. */
enum { MHK_PART_HISTORY = 1, MHK_PART_LEVELS = 2, MHK_PART_LOCAL = 4, MHK_PART_ALL = 7,
       MHK_PART_GEOMETRY = 8 };

typedef struct {
    double alpha;    /* > 0, modified Helmholtz parameter (eq. (mod_helm))          */
    double tol;      /* requested relative accuracy, 1e-13 <= tol <= 1e-3; sets the
                        Fourier cut-off (eqs. (kmax), (kmax_dlp)), the spreading
                        window and the level cut-off radii                          */
    int prec;        /* MHK_FP64 or MHK_FP32 (FP32 spreading, FFT, interpolation
                        and level sums; the local part is always FP64)              */
    int J;           /* dyadic levels, delta* = delta/4^J (eq. (slp_dyad)); < 0: 3  */
    double delta;    /* history split; <= 0: from dx by the rule of Section 6.4:
                        k_max = 0.9 pi/dx (eq. (k_nyq)), delta = ln(1/tol)/(k_max^2
                        + alpha^2) (eq. (kmax) solved for delta)                    */
    double dx;       /* volume mesh size, used only when delta <= 0                 */
    int batch;       /* number of densities / sources per eval call, >= 1           */
    double upsamp;   /* fine-grid oversampling of the NUFFT; <= 0: 2.0              */
    int wspread;     /* spreading window width in grid points; <= 0: from tol       */
    int local_order; /* local expansions of Section 4.1: 0 or 1 keep the first-order
                        terms (error O(delta*^{3/2})), 2 adds the printed
                        delta*^{3/2} and delta*^2 terms of Lemmas 4.1, 4.5, 4.8
                        and Corollaries 4.4, 4.7, 4.10, 4.11 (error
                        O(delta*^{5/2})); with 2, f_trg carries f's gradient and
                        Hessian (see mhk_eval)                                       */
    int lv_block;    /* tile shape of the dyadic-level sums: targets per workgroup,
                        256 or 512 (0: 256); the same sums in another order       */
    int lv_bch;      /* densities per pass of the level sums for batch > 1: 1, 2, 4
                        or 8 (0: 4); each kernel-table evaluation serves them all */
    int lv_persist;  /* 1: the level sums run as one persistent launch per level (a
                        grid that fills the device once, wavefronts taking (target
                        wavefront, density chunk) items from a counter); 0: one
                        wavefront per item                                        */
    int v_levels;    /* 1: the volume potential gets the J dyadic levels too (its
                        local part split in time like the layer potentials', Section
                        4.2): V = V_H(delta) + sum_j V_j + V_L(delta*), V_j the level
                        sums of f over a level-j volume quadrature (every triangle's
                        reference triangle split into 4^j, mapped by the quadratic
                        through its six nodes, f by the reconstruction of
                        mhk_volume.group), V_L with delta* = delta/4^J in place of
                        delta (band_volume then uses delta*).  Needs volume.group = 6,
                        volume.rule and J >= 1.  0: the paper's choice, V_L at delta */
    int in64;        /* MHK_FP32 plans only: 1 = sigma, mu, f_vol, f_trg are given as
                        double; spreading and the level sums take them rounded to
                        float once, the local part (which differentiates sigma and
                        mu twice along the boundary, Lemma 4.5) reads them as
                        given.  Outputs stay float.  0 for FP64 plans.          */
} mhk_params;

typedef struct {
    int64_t n_panels;                 /* panels of 16 nodes; N_B = 16 n_panels     */
    int32_t n_curves;                 /* closed curves                              */
    const int64_t *curve_panel_ofs;   /* host [n_curves+1], panel offsets           */
    const double *x, *y, *nx, *ny, *w, *kappa;   /* host [N_B]                      */
} mhk_boundary;

typedef struct {
    int64_t n;                        /* N_V volume quadrature nodes (may be 0)     */
    const double *x, *y, *w;          /* host [N_V] nodes and weights (eq. (vol_quad)) */
    int32_t group;                    /* 0: no structure; 6: the nodes come in consecutive
                                         groups of six, the 6-point rule of one triangle
                                         each (Section 3.1).  Then f at the targets may be
                                         omitted (f_trg NULL in the eval calls): the plan
                                         takes f, and for local_order 2 its gradient and
                                         Hessian, from the quadratic through the six nodal
                                         values of the triangle holding the target's nearest
                                         node (slivers with nearly collinear nodes
                                         excluded), at targets inside the domain and at the
                                         boundary nodes                                     */
    const double *rule;               /* host [6][3] or NULL: the reference rule of the groups,
                                         (s_i, t_i, W_i) with node i of a group the image of
                                         (s_i, t_i) on {s, t >= 0, s + t <= 1} and sum W_i = 1;
                                         needed for params.v_levels                         */
} mhk_volume;

typedef struct {
    int64_t n;                        /* N_T off-surface targets (may be 0)         */
    const double *x, *y;              /* host [N_T]                                  */
    const int8_t *inside;             /* host [N_T], 1 inside Omega, 0 outside; or NULL:
                                         computed at plan creation as the parity of the
                                         crossings of a ray with the boundary curves (the
                                         polygon through each panel's end points and nodes,
                                         corrected between each edge and the panel's
                                         interpolated arc); targets on the curve itself,
                                         to rounding, may fall on either side           */
    int on_surface;                   /* 1: append the N_B boundary nodes as targets */
} mhk_targets;

typedef struct {
    double alpha, tol, delta, delta_star;
    int J, prec, batch;
    double kmax;          /* Fourier cut-off of the history part (eq. (kmax_dlp))    */
    double period;        /* period of the history grid (Nyquist rule, eq. (nf))     */
    int64_t n_fine;       /* fine grid points per dimension                          */
    int wspread;          /* window width                                            */
    double band_layer;    /* sqrt(delta*)(12 + 2 alpha sqrt(delta*)), Remark 4.3      */
    double band_volume;   /* sqrt(d)(12 + 2 alpha sqrt(d)), d = delta (delta* with v_levels) */
    double level_radius[8];
    int64_t n_boundary, n_volume, n_targets, n_out;
    int64_t device_bytes; /* device memory owned by the plan                         */
    /* milliseconds of the last timed eval per stage (see mhk_plan_set_timing)   */
    double ms_spread, ms_fft, ms_multiply, ms_interp, ms_levels, ms_local, ms_total;
    int history_truncated; /* 1: smoothly truncated history kernel, tabulated spectrum */
    int64_t n_noconv;      /* targets whose closest-point Newton iteration did not
                              converge where the local part uses the closest point's
                              parameter (layer bands; exterior targets and, with
                              local_order 2, all targets in the volume band) -- the
                              first-order interior volume term needs only the
                              distance, which the safeguarded iteration minimises even
                              where it stalls (past a centre of curvature); read with
                              a wait: plan creation fails with MHK_ENOCONV when it is
                              nonzero, and evaluations with MHK_PART_GEOMETRY add to it */
    double ms_geometry;    /* closest points and local coefficients of the last timed
                              eval with MHK_PART_GEOMETRY (beside the history part)  */
    double ms_plan[6];     /* host-clock milliseconds of plan creation: [0] input checks
                              and bounding box, [1] target sort, [2] dyadic levels
                              (child nodes, cells, candidate lists, tables), [3] history
                              part (source binning, window, multiplier, FFT set-up),
                              [4] local part (panel data, closest points), [5] total  */
} mhk_info;

typedef struct mhk_plan mhk_plan;

/* Resolve the split parameters without creating a plan (host only, no GPU):
 * fills delta (from dx when params->delta <= 0), delta_star, kmax, band_* and
 * level_radius of *info.  Returns MHK_EINVAL for invalid params. */
mhk_status mhk_resolve_params(const mhk_params *params, mhk_info *info);

/* Build a plan: resolve parameters, copy and sort geometry and targets into
 * device buffers, build the level kernel tables and the FFT plans.  The
 * stream (a hipStream_t, NULL for the default stream) is used by every later
 * call on the plan.  *out is set to NULL on error. */
mhk_status mhk_plan_create(const mhk_params *params, const mhk_boundary *boundary,
                           const mhk_volume *volume, const mhk_targets *targets,
                           void *hip_stream, mhk_plan **out);

/* Device bytes a plan with these inputs would own, without allocating. */
mhk_status mhk_plan_footprint(const mhk_params *params, const mhk_boundary *boundary,
                              const mhk_volume *volume, const mhk_targets *targets,
                              int64_t *bytes);

/* S[sigma], D[mu] and V[f] at all targets (Section 2.1 split: history +
 * levels + local).  Any of sigma, mu, f_vol may be NULL: the matching output
 * is then not written.  sigma, mu: [batch][N_B]; f_vol: [batch][N_V] values
 * of f at the volume nodes; f_trg: [batch][n_out] values of f at the targets
 * (needed by the local part of V, Lemma 4.8; required when f_vol is given),
 * or, for a plan with local_order = 2, [batch][6][n_out]: f, f_x, f_y, f_xx,
 * f_xy, f_yy at the targets (the second-order terms of Lemma 4.8 need f's
 * normal and second derivatives; exterior targets keep the first-order
 * complement form); out_S, out_D, out_V: [batch][n_out]. */
mhk_status mhk_eval(mhk_plan *plan, const void *sigma, const void *mu, const void *f_vol,
                    const void *f_trg, void *out_S, void *out_D, void *out_V);

/* Single-potential forms of mhk_eval. */
mhk_status mhk_eval_S(mhk_plan *plan, const void *sigma, void *out_S);
mhk_status mhk_eval_D(mhk_plan *plan, const void *mu, void *out_D);
mhk_status mhk_eval_V(mhk_plan *plan, const void *f_vol, const void *f_trg, void *out_V);

/* As mhk_eval, restricted to the parts in the mask (MHK_PART_*). */
mhk_status mhk_eval_parts(mhk_plan *plan, int parts, const void *sigma, const void *mu,
                          const void *f_vol, const void *f_trg, void *out_S, void *out_D,
                          void *out_V);

/* As mhk_eval_parts for the first nbatch densities only, 1 <= nbatch <=
 * params.batch of the plan: inputs [nbatch][N], outputs [nbatch][n_out],
 * and every stage runs over nbatch densities, so a plan sized for a batch
 * serves smaller ones at their own cost (requests coalesced as they arrive,
 * Section 1's time steps of several simulations).  EINVAL for nbatch out of
 * range. */
mhk_status mhk_eval_batch(mhk_plan *plan, int nbatch, int parts, const void *sigma, const void *mu,
                          const void *f_vol, const void *f_trg, void *out_S, void *out_D, void *out_V);

/* f at the targets as the plan reconstructs it from the volume quadrature
 * when an eval call gets f_trg = NULL (volume.group = 6): f_vol [batch][N_V]
 * in, f_trg [batch][rows][n_out] out (rows 1, or 6 for local_order 2: f,
 * f_x, f_y, f_xx, f_xy, f_yy; zero at exterior off-surface targets, which
 * never need it), caller order, the precision of the eval inputs;
 * asynchronous on the plan's stream.  EINVAL without the grouped volume. */
mhk_status mhk_plan_f_targets(mhk_plan *plan, const void *f_vol, void *f_trg);

/* Record one evaluation (the arguments of mhk_eval_parts) into a HIP graph
 * owned by the plan, bound to these device pointers, without running it; the
 * plan's stream is synchronised first.  mhk_plan_launch_graph then replays
 * the whole evaluation (every stage, all densities of the batch) with one
 * launch on the plan's stream; the caller refreshes the contents of the
 * input buffers between replays and keeps every bound buffer alive.  A new
 * capture replaces the previous graph. */
mhk_status mhk_plan_capture(mhk_plan *plan, int parts, const void *sigma, const void *mu,
                            const void *f_vol, const void *f_trg, void *out_S, void *out_D,
                            void *out_V);
mhk_status mhk_plan_launch_graph(mhk_plan *plan);

/* Enable (1) or disable (0) per-stage timing with HIP events; when enabled,
 * each eval records events on the plan's streams (without waiting), and
 * mhk_plan_info waits for the last timed eval and fills the ms_* fields.
 * The level sums run on a second stream of the plan beside the history
 * part, so ms_levels overlaps ms_spread..ms_interp; ms_fft is the row
 * transforms, ms_multiply the column transforms with the multiplier (or the
 * 2D transforms' multiplier for grids longer than 8192). */
mhk_status mhk_plan_set_timing(mhk_plan *plan, int enable);

mhk_status mhk_plan_info(const mhk_plan *plan, mhk_info *info);
void mhk_plan_destroy(mhk_plan *plan);
const char *mhk_last_error(void);

/* ------------------------------------------------------------------------
 * Boundary integral equations (Section 3.2)
 *
 * The Dirichlet problem (-Lap + alpha^2) u = f in Omega, u = g on the
 * boundary, is solved through u = V[f] + D[mu] (eq. (sol_dirichlet)) and the
 * second-kind equation -mu/2 + D[mu] = g - V[f] on the boundary (eq.
 * (bie_dir)); the Neumann problem (du/dnu = g) through u = V[f] + S[g] -
 * D[u] (eq. (sol_neumann)) and u/2 + D[u] = V[f] + S[g] (eq. (bie_neu)).  On
 * the boundary nodes the double-layer operator is discretised by the
 * Nystrom method with the smooth panel rule (the matrix K of Section 3.2:
 * K_ij = w_j alpha/(2 pi) K_1(alpha r_ij) (x_i - x_j).nu_j / r_ij, i != j;
 * K_ii = -w_i kappa_i/(4 pi), eq. (dlp_diag_limit)), and the discrete
 * systems (eqs. (dirichlet-discrete), (neumann-discrete)) are solved by
 * restarted GMRES on the device.  All vectors of these calls are DEVICE
 * pointers of doubles.
 * ------------------------------------------------------------------------ */
typedef struct mhk_nystrom mhk_nystrom;

typedef struct {
    int64_t n;            /* N_B                                                    */
    double alpha;
    int64_t device_bytes; /* K (8 N_B^2 bytes) plus GMRES and solve workspace      */
    double ms_assemble;   /* time to build K on the device                         */
} mhk_nys_info;

typedef struct {
    int iters;            /* GMRES iterations (matrix-vector products in the Krylov loop) */
    int converged;        /* 1 if |b - A x| <= tol |b| at exit                      */
    double resid;         /* final true relative residual                           */
    double ms_eval, ms_gmres, ms_total;  /* potential evaluations / GMRES / total   */
} mhk_solve_info;

/* Assemble K on the device for the boundary (host arrays as for
 * mhk_plan_create; N_B <= 2^20, K needs 8 N_B^2 bytes of device memory).
 * Later calls run on the given stream (NULL: default stream).  *out is NULL
 * on error (MHK_ENOMEM when K does not fit). */
mhk_status mhk_nystrom_create(double alpha, const mhk_boundary *boundary, void *hip_stream, mhk_nystrom **out);

/* y = shift x + K x, x and y device arrays of N_B doubles (y must not alias x);
 * asynchronous on the object's stream. */
mhk_status mhk_nystrom_apply(mhk_nystrom *nys, double shift, const double *x, double *y);

/* Solve (shift I + K) x = rhs by GMRES(restart), x = 0 initially, until the
 * relative residual is <= tol or maxit iterations were made; synchronises the
 * object's stream (the Arnoldi coefficients are reduced on the host).
 * 0 < tol < 1, 1 <= restart <= 1000, maxit >= 1.  Not converging is not an
 * error: check info->converged. */
mhk_status mhk_nystrom_solve(mhk_nystrom *nys, double shift, const double *rhs, double *x, double tol,
                             int restart, int maxit, mhk_solve_info *info);

/* As mhk_nystrom_solve, for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the GMRES workspace -- the Krylov basis, residual and product vectors,
 * partial sums of the dot products and the small Hessenberg data -- comes
 * from one fixed device array of 32 MiB in the library, not from
 * allocations, and the host side of the least-squares problem from the
 * stack.  The call allocates nothing: no hipMalloc, hipHostMalloc or
 * hipFree.  Limits: restart <= 64, and (restart + 3) N_B + (restart + 1)
 * min(256, N_B/256) + 3 restart doubles (each part rounded up to 256 bytes)
 * within the 32 MiB (N_B = 16384 allows restart 60); larger requests fail
 * with MHK_EINVAL before anything is enqueued.  Every GPU holds its own copy
 * of the array for the life of the process (its address is looked up on the
 * first call made with that device current), and every call on that GPU
 * shares it: calls that overlap on one GPU (other host threads, other
 * objects' streams) race and must be serialised by the caller.  The array
 * keeps the last call's contents; nothing in it is read before it is
 * written.  Otherwise as mhk_nystrom_solve (same results, the object's
 * stream, synchronised at the end); ms_gmres and ms_total are host-clock
 * times. */
mhk_status mhk_nystrom_solve_noalloc(mhk_nystrom *nys, double shift, const double *rhs, double *x, double tol,
                                     int restart, int maxit, mhk_solve_info *info);

/* Dirichlet problem with data g [N_B] and optional source (f_vol [N_V] at
 * the volume nodes and f_trg [n_out] at the outputs, both or neither):
 * mu [N_B] receives the layer density, u [n_out] the solution at every
 * output of the plan (targets, then boundary nodes, where u is the interior
 * limit V + D[mu] - mu/2 of eq. (jumprel)).  The plan must be FP64 with batch
 * 1, on-surface targets, the same boundary and alpha as nys; the work runs on
 * the plan's stream and ends synchronised. */
mhk_status mhk_solve_dirichlet(mhk_plan *plan, mhk_nystrom *nys, const double *g, const double *f_vol,
                               const double *f_trg, double tol, int restart, int maxit, double *mu, double *u,
                               mhk_solve_info *info);

/* Neumann problem with data g = du/dnu [N_B] (outward normal): u_b [N_B]
 * receives the boundary values, u [n_out] the solution at every output (u_b
 * on the boundary nodes).  Same requirements as mhk_solve_dirichlet. */
mhk_status mhk_solve_neumann(mhk_plan *plan, mhk_nystrom *nys, const double *g, const double *f_vol,
                             const double *f_trg, double tol, int restart, int maxit, double *u_b, double *u,
                             mhk_solve_info *info);

/* One step of elliptic marching (Rothe's method, Section 1) for the heat
 * equation u_t = Lap u + F in Omega, u = g on the boundary: the implicit
 * Euler step with time step 1/alpha^2 is the modified Helmholtz problem
 * (-Lap + alpha^2) u^{n+1} = alpha^2 u^n + F^{n+1} (eq. (mod_helm)), solved
 * as the Dirichlet problem above.  The plan's targets must be its volume
 * nodes, in the same order (checked at plan creation), with on-surface
 * targets; u_n, F (may be NULL) and u_next are [n_out] device arrays over
 * the volume nodes then the boundary nodes (u_n there is g^n), g_next [N_B]
 * the boundary data of the new step, mu [N_B] receives the layer density.
 * u_next must not alias u_n.  Same requirements and synchronisation as
 * mhk_solve_dirichlet. */
mhk_status mhk_heat_step(mhk_plan *plan, mhk_nystrom *nys, const double *u_n, const double *F,
                         const double *g_next, double tol, int restart, int maxit, double *u_next, double *mu,
                         mhk_solve_info *info);

mhk_status mhk_nystrom_info(const mhk_nystrom *nys, mhk_nys_info *info);
void mhk_nystrom_destroy(mhk_nystrom *nys);

#ifdef __cplusplus
}
#endif
#endif /* MHK_H */
