/*
 * enufft.h -- C ABI of the MI355X (gfx950) ENUFFT hot path.
 *
 * What it computes (per cell c of a batch, local coordinates on a periodic box
 * of side 2*pi so that wave numbers are integers, Appendix A1 with L = 2*pi):
 *
 *   f_c[k] = scale * sum_{j in c} w_j * W_c(x_j, y_j) * h_j * exp(-i (kx x_j + ky y_j))
 *
 * i.e. the windowed, quadrature-weighted type-1 sum of Section 2.1.1 eq. (quad)
 * and Appendix A2 eq. (discrete_quadrature), evaluated as a type-1 NUFFT
 * (Section 2.1.2: spread, FFT, deconvolve, truncate), followed by Elastic Mode
 * Selection over the resulting power (Section 2.2), and the adjoint (a type-2
 * NUFFT, +i sign of eq. (series)) that gives gradients of a retained-power loss
 * with respect to heights and point coordinates.
 *
 * Conventions shared by every entry point
 *   Layout.    Points are grouped by cell (CSR): cell c owns points
 *              [cell_offsets[c], cell_offsets[c+1]) of the x, y, h, w arrays.
 *              Coefficients are complex interleaved (re, im), per cell a
 *              row-major N2 x N1 block, k_y slow and k_x fast, each ascending
 *              from -floor(N/2) to ceil(N/2) - 1.
 *   Precision. Real arrays are float for ENUFFT_F32 plans and double for
 *              ENUFFT_F64 plans; coefficient arrays are float2 / double2.
 *   Memory.    Pointers documented "device" are caller-owned device memory,
 *              borrowed until the enqueued work completes on the plan's
 *              stream; the library never frees them.  Host arrays passed to
 *              enufft_plan are deep-copied.
 *   Streams.   Every compute call enqueues asynchronously on the plan's stream
 *              and returns; only enufft_plan (which may run timed trial
 *              launches when autotuning) and enufft_get_timing synchronise.
 *   Errors.    Every call returns an enufft_status; no exception crosses the
 *              ABI.  Arguments are validated before any device work, so an
 *              argument error leaves outputs untouched and the plan usable.
 *              enufft_last_error() describes the last failure.
 *   Threads.   A plan is not thread-safe; separate plans may be used
 *              concurrently on separate streams.
 *   Coordinates are any finite reals in box units; they are folded modulo 2*pi
 *   for the transform (the window uses the unfolded values).
 */
#ifndef ENUFFT_H
#define ENUFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct enufft_plan_s *enufft_plan_t;

typedef enum {
    ENUFFT_OK = 0,
    ENUFFT_EINVAL = 1,   /* bad argument (null pointer, bad size, non-monotone offsets, ...) */
    ENUFFT_ENOMEM = 2,   /* device or host allocation failed (or exceeded ENUFFT_ALLOC_CAP_MB) */
    ENUFFT_EDEVICE = 3,  /* HIP runtime error or no usable gfx950 device */
    ENUFFT_EEPS = 4,     /* requested eps is not attainable at the requested precision */
    ENUFFT_ESTATE = 5,   /* plan unusable after an earlier device fault */
    ENUFFT_EUNSUPPORTED = 6 /* valid request outside what the library implements */
} enufft_status;

typedef enum { ENUFFT_F32 = 0, ENUFFT_F64 = 1 } enufft_precision;

/* Per-cell window W_c.  NONE: W = 1.  HANN_RADIAL: W(r) = (1 + cos(pi r / R)) / 2 for
 * r = |(x, y) - (cx, cy)| < R and 0 otherwise (a C^1 taper standing in for the
 * indicator masks of Appendix A1; radius must be > 0). */
typedef enum { ENUFFT_WIN_NONE = 0, ENUFFT_WIN_HANN_RADIAL = 1 } enufft_window_kind;

/* Spreading kernel (Section 2.1.2, Step 1).  ES: the exponential of a semicircle,
 * psi(z) = exp(beta (sqrt(1 - z^2) - 1)), beta = 2.30 W at sigma 2.  KB_MIRT and
 * KB_FESSLER: the Kaiser-Bessel kernel of eq. (kb_compact) with half-width a = W / 2 and
 * the shape of eq. (kaisal_bessel_coeffs) (gamma = pi sqrt((2 a 2.34 / pi)^2 - 0.8)) or
 * of eq. (kb_type_2) (gamma = 2.34); its deconvolution factors come from the closed
 * form of eq. (kb_fourier).  The kernel's constant factor 1 / I0(beta) cancels between
 * spreading and deconvolution, so the KB kernels are used normalised to 1 at 0. */
typedef enum { ENUFFT_KERNEL_ES = 0, ENUFFT_KERNEL_KB_MIRT = 1, ENUFFT_KERNEL_KB_FESSLER = 2 } enufft_kernel_kind;

typedef struct { double cx, cy, radius; } enufft_window;

/* Transform options.
 *   n_modes   N1 (along x) and N2 (along y), each >= 1.  Boxes up to 64 per axis
 *             whose fine grid is at most 128 per axis keep the whole grid in one
 *             workgroup's LDS; larger ones take the large-cell path (grid in HBM,
 *             points sorted by 32 x 32 grid tiles, each axis widened to >= 64).
 *             A fine grid above 4096 per axis or above 2^22 cells in total is
 *             ENUFFT_EUNSUPPORTED.
 *   sigma     oversampling factor (>= 1.25); the fine grid per axis is the
 *             smallest power of two >= max(16, sigma * N) (Section 2.1.2, Step 1).
 *   eps       requested relative accuracy of the spreading approximation; sets the
 *             exponential-of-semicircle kernel width.  F32 needs eps >= 1e-6, F64
 *             eps >= 1e-13 (else ENUFFT_EEPS).
 *   precision enufft_precision.
 *   window_kind enufft_window_kind.
 *   scale     overall factor on f (1 / |D| reproduces eq. (discrete_quadrature)).
 *   autotune  0: default launch shape; 1: timed trials at plan time on synthetic
 *             points with the plan's cell sizes, stored in raster order within
 *             each cell (gridded samples); 2: the same trials on points stored in
 *             no spatial order (scattered samples).  Other values: ENUFFT_EINVAL.
 *             Trials synchronise the stream and allocate trial buffers of up
 *             to 2^27 points (env ENUFFT_TUNE_MAX_POINTS; a prefix of the
 *             cells beyond that).  The choice is cached
 *             in the file ENUFFT_TUNE_CACHE ("off" disables; default
 *             $HOME/.cache/enufft/tune_cache.txt) keyed by device, shape and
 *             the exact cell layout and the trial point order.
 *   kernel_width 0: from eps; otherwise a width >= the eps-derived one (ES), or the
 *             width itself (KB kernels: W = 2 a, even, 4..16).
 *   kernel_kind enufft_kernel_kind. */
typedef struct {
    int32_t n_modes[2];
    double sigma;
    double eps;
    int32_t precision;
    int32_t window_kind;
    double scale;
    int32_t autotune;
    int32_t kernel_width;
    int32_t kernel_kind;
} enufft_opts;

/* Elastic Mode Selection parameters (Section 2.2).
 *   k_min, k_max      the budget K_min <= K* <= K_max of eq. (k_elastic).
 *   alpha_min/max     the target range of eq. (alpha_c), each in [0, 1].
 *   delta             the gap-ratio scale of eq. (s_delta), > 0.
 *   w1, w2            the weights of eq. (c_score), each in [0, 1].
 *   use_pairs         1: units are +-k pairs (energy below eq. (energy)), a mode
 *                     whose partner is outside the box is its own unit; 0: every
 *                     signed mode is a unit.
 *   exclude_dc        1: the k = 0 mode is not a unit (it is never kept). */
typedef struct {
    int32_t k_min, k_max;
    double alpha_min, alpha_max, delta, w1, w2;
    int32_t use_pairs, exclude_dc;
} enufft_ems_params;

typedef struct {
    int32_t n_modes[2];      /* N1, N2 */
    int32_t grid[2];         /* fine grid n1, n2 */
    int32_t kernel_width;    /* spreading kernel width in fine-grid cells */
    double beta;             /* kernel shape: ES beta, or KB gamma */
    int64_t n_cells;
    int64_t n_points;
    int64_t n_items_fwd;     /* work items of the batched forward launch */
    int64_t n_split_cells;   /* cells spread by several workgroups and merged */
    int64_t n_items_adj;     /* work items of the batched adjoint launch */
    int32_t adj_bands;       /* row bands per cell in the adjoint */
    int32_t fwd_threads, fwd_blocks;   /* forward launch shape */
    int32_t adj_threads, adj_blocks;
    int64_t workspace_bytes;
    double kernel_poly_err;  /* max |polynomial - psi| of the kernel fit (FP32 plans, FP64 large-cell plans),
                                0 if the exact kernel is used */
    int32_t tuned;           /* 1 if the autotuner set the launch shape */
    int32_t tune_cache_hit;  /* 1 if that choice came from the on-disk cache */
    int64_t fwd_chunk_min;   /* smallest forward work item (points) */
    int32_t fwd_items_per_slot, adj_items_per_slot;  /* work items per resident workgroup */
    int32_t adj_band_mult;   /* adjoint row bands = this x the fewest that fit LDS */
    int32_t fwd_acc;         /* bytes per forward LDS grid cell: 8 (FP64 sums) or 4 (FP32 sums) */
    double tune_fwd_ms, tune_adj_ms;   /* best trial times of the autotuner */
    int32_t kernel_kind;     /* enufft_kernel_kind of the plan */
    int32_t adj_kernel_width; /* adjoint: width of its own kernel when it gathers value and derivative
                                 taps from one LDS grid per cell (FP32, forward width + 2); 0 when it
                                 gathers from three grids in row bands with the forward's kernel */
} enufft_plan_info;

/* Fill *o with defaults: 64 x 64 modes, sigma 2, eps 1e-5, F32, Hann window,
 * scale 1, no autotuning, ES kernel. */
enufft_status enufft_default_opts(enufft_opts *o);

/* Create a plan for a fixed batch layout.
 *   out          receives the plan (set to NULL on failure).
 *   n_cells      number of cells, >= 0.
 *   cell_offsets host, n_cells + 1 int64, [0] = 0, non-decreasing.
 *   windows      host, n_cells entries (may be NULL for ENUFFT_WIN_NONE).
 *   opts         host, see enufft_opts.
 *   hip_stream   hipStream_t for every later call (NULL = default stream).
 * Builds the deconvolution tables (FP64 quadrature of the kernel's Fourier
 * transform, Section 2.1.2 Step 4), the work schedule and the workspace. */
enufft_status enufft_plan(enufft_plan_t *out, int64_t n_cells, const int64_t *cell_offsets,
                          const enufft_window *windows, const enufft_opts *opts, void *hip_stream);

/* Change the stream later calls enqueue on. */
enufft_status enufft_set_stream(enufft_plan_t p, void *hip_stream);

/* Batched type-1 (Section 2.1.2 Steps 1-4 plus truncation to the mode box).
 *   x, y, h, w  device, n_points each: coordinates, heights, quadrature weights.
 *   f           device, n_cells * N2 * N1 complex: written in full.
 * One persistent launch spreads every cell into an LDS-resident fine grid,
 * runs the FFT in LDS, deconvolves and crops; cells larger than one work
 * item are spread by several workgroups and merged by the last to finish.
 * Large-cell plans instead run, per cell, a device sort of the points by grid
 * tile, tiled spreading into an FP64 grid in HBM, and row and column FFT
 * passes with the deconvolution and crop fused into the column pass. */
enufft_status enufft_type1_batched(enufft_plan_t p, const void *x, const void *y, const void *h,
                                   const void *w, void *f);

/* Allocation-free form of enufft_type1_batched, for callers that cannot allocate device
 * memory while they run (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Arguments and results as enufft_type1_batched.  The forward
 * kernel's scratch -- the persistent loop's work counters, the per-cell merge counters
 * and the partial grids of cells split over several workgroups -- comes from one fixed
 * device array of 64 MiB per GPU (held until the process ends), not from the plan's
 * workspace; the call makes no allocation of any kind (the plan, made beforehand, still
 * owns its tables and work list).  The counters are cleared by a kernel at the start of
 * every call.  Calls that overlap on one GPU share that array and race: serialise them.
 * A plan needing more scratch than the array holds returns ENUFFT_EINVAL (the message
 * gives the size); large-cell plans return ENUFFT_EUNSUPPORTED. */
enufft_status enufft_type1_batched_noalloc(enufft_plan_t p, const void *x, const void *y, const void *h,
                                           const void *w, void *f);

/* Elastic Mode Selection on coefficients f (Section 2.2, eqs. energy ... k_elastic).
 *   f           device, n_cells * N2 * N1 complex (the plan's precision).
 *   prm         host parameters.
 *   mode_weight device, N2 * N1 doubles (the w_mn of eq. (weighted_e)), or NULL for 1.
 *   keep        device, n_cells * N2 * N1 bytes: 1 for kept modes, else 0.
 *   k_star      device, n_cells int32: the elastic count K*.
 *   stats       device, n_cells * 8 doubles: (T, P, N_eff, S_delta, C, alpha_C,
 *               theta(K*), J*) with T the total unit energy and P the kept power
 *               sum |f_k|^2.  Energies, sums and the cumulative threshold are FP64.
 * Units are ordered by descending energy, ties by ascending row-major index of
 * the unit's representative (the member with k_y > 0, or k_y = 0 and k_x > 0).
 * Up to 4096 units per cell are sorted in registers by one workgroup per cell;
 * more take a device bitonic sort per cell. */
enufft_status enufft_ems(enufft_plan_t p, const void *f, const enufft_ems_params *prm,
                         const double *mode_weight, uint8_t *keep, int32_t *k_star, double *stats);

/* Flow-dependent Elastic Mode Selection repeated over timesteps on fixed coefficients
 * (Section 2.2.1 eq. (weighted_e) with the launch weight of Appendix A7; Section 3.3
 * re-selects per timestep as the flow changes).  For step s and cell c the weight of
 * mode k is
 *   w_k = |A_k| / |h_k|^2 = (rho / 2) |k.u| (|k|^2 + m^2) / |k|^2,
 * the wave action of eq. (mw_action) per unit modal power, with the physical wave
 * vector k = kscale (kx, ky), the intrinsic frequency omega = -k.u (eq. mountain_omega)
 * and m^2 from the dispersion relation (eq. mw_dispersion); modes outside the
 * propagating band fc < |omega| < N, and k = 0, weigh 0.  The selection is then
 * enufft_ems's with these weights.
 *   f        device, n_cells * N2 * N1 complex: the coefficients (not recomputed).
 *   prm      host EMS parameters (as enufft_ems).
 *   n_steps  number of timesteps, >= 1 (n_steps * n_cells < 2^31).
 *   flow     device, n_steps * n_cells records of 6 doubles (ux, uy, N, fc, rho,
 *            kscale): background wind (m/s), buoyancy frequency and Coriolis
 *            parameter (1/s), density, and the physical wave number (rad/m) of one
 *            unit of the box's integer wave numbers (2 pi / box side).
 *   keep     device, n_steps * n_cells * N2 * N1 bytes, or NULL to skip the masks.
 *   k_star   device, n_steps * n_cells int32.
 *   stats    device, n_steps * n_cells * 8 doubles (as enufft_ems; T and theta are of
 *            the weighted energies, P is the plain power of the kept modes).
 * Outputs of step s, cell c are at index s * n_cells + c.  One launch covers all steps.
 * Mode boxes above 4096 units per cell return ENUFFT_EUNSUPPORTED. */
enufft_status enufft_ems_flow(enufft_plan_t p, const void *f, const enufft_ems_params *prm, int32_t n_steps,
                              const double *flow, uint8_t *keep, int32_t *k_star, double *stats);

/* Adjoint of the batched type-1 map (a type-2 NUFFT) and the chain rule.
 *   x, y, h, w  device, n_points each, as for enufft_type1_batched (all four required;
 *               NULL gives ENUFFT_EINVAL).
 *   fbar        device, n_cells * N2 * N1 complex cotangent g = dL/dRe f + i dL/dIm f
 *               (for L = sum_c lambda_c P_c this is 2 lambda_c f keep).
 *   grad_h, grad_x, grad_y  device, n_points each, or NULL to skip; written in full:
 *     u_j  = scale Re sum_k g_k exp(+i k.x_j),  (ux_j, uy_j) likewise with (i kx, i ky) g_k,
 *     grad_h = w W u,  grad_x = w h (dW/dx u + W ux),  grad_y = w h (dW/dy u + W uy).
 * The fine grids are recomputed from fbar (never stored by the forward). */
enufft_status enufft_type1_adjoint(enufft_plan_t p, const void *x, const void *y, const void *h,
                                   const void *w, const void *fbar, void *grad_h, void *grad_x,
                                   void *grad_y);

/* Gradients of the retained-power loss L = sum_c lam_c P_c, P_c = sum over kept modes
 * of |f_c[k]|^2 (the quantity EMS preserves, Section 2.2), with the kept set held
 * fixed: enufft_type1_adjoint with the cotangent 2 lam_c f keep formed inside the
 * kernel instead of by the caller.
 *   f     device, n_cells * N2 * N1 complex: the coefficients of the forward pass.
 *   keep  device, n_cells * N2 * N1 bytes from enufft_ems.
 *   lam   device, n_cells doubles, or NULL for lam_c = 1.
 *   other arguments as enufft_type1_adjoint. */
enufft_status enufft_retained_power_adjoint(enufft_plan_t p, const void *x, const void *y, const void *h,
                                            const void *w, const void *f, const uint8_t *keep,
                                            const double *lam, void *grad_h, void *grad_x, void *grad_y);

/* Reconstruction from retained modes and the per-cell diagnostics of Section 3.2.
 * For every sample q of cell c, the truncated series of eq. (series) over the kept modes,
 *   h_rec(x_q) = Re sum_{k kept} coef_c[k] exp(+i (kx x_q + ky y_q)),
 * evaluated as a type-2 NUFFT (the adjoint's pre-corrected inverse transforms and
 * gather, without the plan's scale), and per cell, with the target t_q = W_c(x_q) h_q
 * (the windowed height the coefficients represent; h_q without a window):
 *   diag[8 c + 0]  Q_c
 *   diag[8 c + 1]  sum_q (t_q - h_rec(x_q))^2
 *   diag[8 c + 2]  sum_q t_q^2
 *   diag[8 c + 3]  sigma^2_phys = (1 / |D_c|) sum_q w_q t_q^2     (eq. spectral_variance, left side)
 *   diag[8 c + 4]  sigma^2_spec = sum_{k != 0} |coef_c[k]|^2       (eq. spectral_variance, right side)
 *   diag[8 c + 5]  the same sum over the kept modes only
 *   diag[8 c + 6]  eps_rel = sqrt(diag[1] / diag[2])               (eq. alps_relative_rmse)
 *   diag[8 c + 7]  sigma^2_spec / sigma^2_phys (the Parseval ratio)
 * For the paper's normalisation the coefficients come from a plan with scale = 1 / |D_c|.
 *   x, y, h, w  device, n_points each (as enufft_type1_batched; all required).
 *   coef        device, n_cells * N2 * N1 complex (the plan's precision).
 *   keep        device, n_cells * N2 * N1 bytes (enufft_ems), or NULL for every mode.
 *   area        device, n_cells doubles |D_c|, or NULL for 1.
 *   h_rec       device, n_points reals (the plan's precision), or NULL.
 *   diag        device, n_cells * 8 doubles; sums over samples are FP64, formed per
 *               work item and added per cell in a fixed order.
 * Large-cell plans (mode boxes above 64 per axis) return ENUFFT_EUNSUPPORTED. */
enufft_status enufft_reconstruct(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w,
                                 const void *coef, const uint8_t *keep, const double *area, void *h_rec,
                                 double *diag);

/* Per-cell geometry of a triangular mesh (Appendix A1 local windowing, Appendix A2
 * quadrature weights, Appendix A6 deplaning): turns tangent-plane samples of cell c,
 * which lies on triangle T_c, into the inputs of enufft_type1_batched.
 *   frame    ENUFFT_FRAME_CENTROID: R = I; ENUFFT_FRAME_EDGE: the rotation of eq.
 *            (rotation_matrix) that takes the longest of the edges v2 - v1, v3 - v2,
 *            v1 - v3 onto +x (the first of equally long edges).
 *   local    u = R (x - xbar), xbar the centroid; half-width H = (eta / 2) max(extent
 *            of the rotated vertices along x, along y); square box B = [-H, H]^2.
 *   xb, yb   u * pi / H: B mapped onto the library's 2 pi box (period 2H), centred on
 *            the centroid (the square-domain shift (x', y') = u + H of Appendix A1 only
 *            multiplies every coefficient by (-1)^(kx + ky)).
 *   mask     ENUFFT_MASK_SQUARE (B), ENUFFT_MASK_TRIANGLE (the rotated triangle within
 *            B, edges included), ENUFFT_MASK_CIRCLE (|u| <= H); |D_c| is the mask's area
 *            in B (the triangle clipped to B, exactly).
 *   weights  ENUFFT_WEIGHTS_UNIFORM: w_q = |D| / Q_in over the Q_in samples inside the
 *            mask (eq. uniform_weights).  ENUFFT_WEIGHTS_VORONOI: raster N_g x N_g cell
 *            centres over B (eq. raster_grid); each one inside the mask goes to its
 *            nearest inside sample (eq. nn_assignment; ties to the lowest index), A_q =
 *            n_q |D| / |G| (eq. raster_area); a sample with n_q = 0 gets floor_frac
 *            |D| / |G| and all areas are rescaled to sum to |D| (eq. voronoi_weights).
 *   wb       w_q / |D_c|, 0 outside the mask: the factor eq. (discrete_quadrature) puts on
 *            h_q.  Type-1 with window ENUFFT_WIN_NONE, scale 1 and w = wb gives eq.
 *            (discrete_quadrature) on (xb, yb, hb).
 *   hb       h - hbar with hbar = sum_q wb_q h_q, the weighted mean over the mask (eq.
 *            alps_deplaning), when deplane is set; else h.
 * Arguments:
 *   tri      device, n_cells * 6 doubles (v1x, v1y, v2x, v2y, v3x, v3y) per cell.
 *   x, y, h  device, n_points reals (the plan's precision), grouped by the plan's cells.
 *   opts     host; raster in [1, 4096] for Voronoi weights, eta >= 1, floor_frac >= 0.
 *   xb, yb, hb, wb  device, n_points reals (the plan's precision), all required.
 *   inside   device, n_points bytes (1 inside the mask), or NULL.
 *   info     device, n_cells * 8 doubles (xbar_x, xbar_y, cos, sin, H, |D|, Q_in, hbar;
 *            hbar 0 without deplaning), or NULL.
 *   counts   device, n_points int32 (n_q; 0 for uniform weights), or NULL.
 * Frames, masks and the raster assignment are FP64 with the products and sums rounded
 * one by one (no fused multiply-add), so flags and counts are exact functions of the
 * FP64 inputs; the weight and mean sums are FP64 in the kernel's order.  One launch:
 * resident workgroups take cells largest first; with Voronoi weights each keeps a
 * binned copy of its cell's inside samples in plan workspace (24 bytes per point of
 * the largest cell, per resident workgroup). */
typedef enum { ENUFFT_FRAME_CENTROID = 0, ENUFFT_FRAME_EDGE = 1 } enufft_frame_kind;
typedef enum { ENUFFT_MASK_SQUARE = 0, ENUFFT_MASK_TRIANGLE = 1, ENUFFT_MASK_CIRCLE = 2 } enufft_mask_kind;
typedef enum { ENUFFT_WEIGHTS_UNIFORM = 0, ENUFFT_WEIGHTS_VORONOI = 1 } enufft_weights_kind;
typedef struct {
    int32_t frame;       /* enufft_frame_kind */
    int32_t mask;        /* enufft_mask_kind */
    int32_t weights;     /* enufft_weights_kind */
    int32_t raster;      /* N_g (Voronoi weights) */
    double eta;          /* expansion factor, >= 1 */
    double floor_frac;   /* empty-cell floor, in raster points */
    int32_t deplane;     /* 1: subtract the weighted cell mean */
    int32_t reserved_;
} enufft_geometry_opts;

enufft_status enufft_cell_geometry(enufft_plan_t p, const double *tri, const void *x, const void *y,
                                   const void *h, const enufft_geometry_opts *opts, void *xb, void *yb,
                                   void *hb, void *wb, uint8_t *inside, double *info, int32_t *counts);

/* Sort every cell's samples by the fine-grid cell where their kernel footprint starts
 * (row-major; the footprint of eq. spreading, Section 2.1.2 Step 1): a one-time device
 * counting sort that writes sorted copies.  In that order the batched type-1 spreads
 * consecutive samples as merged runs; samples in no spatial order (shuffled, or grouped
 * by something other than position) otherwise go one point at a time.  The caller then
 * works on the sorted arrays (the coefficients are those of the original order up to
 * rounding; gradients come out in the sorted order, perm maps them back).
 *   x, y, h, w      device, n_points reals each (the plan's precision), grouped by the
 *                   plan's cells; h and w may be NULL when hs, ws are.
 *   xs, ys, hs, ws  device outputs, n_points reals each; hs, ws may be NULL.  Must not
 *                   alias the inputs.
 *   perm            device, n_points int32, or NULL: perm[i] is the input index of the
 *                   sample at sorted position i (a permutation inside each cell).
 * Workspace: on its first call the plan allocates 16 bytes per point (32 in FP64) for
 * interleaved copies of the samples, and with perm NULL 4 bytes per point for its own
 * permutation; both are kept for later calls and freed by enufft_destroy.
 * The order of samples that share a fine cell is not specified.  Large-cell plans sort by
 * the 32 x 32 tile of the footprint origin, the order of their tiled spreading (FP32
 * plans with the kernel polynomial, widths 4, 6 and 8: and by fine cell, row-major,
 * inside each tile).  Their type-1 and adjoint calls sort every call by tile, and skip
 * the sort's scatter when their counting pass finds the input already in tile order; the
 * FP32 ones also find whether it is in cell order, and then sum each run of samples with
 * one footprint origin in registers before it reaches the spreading sub-grid.  Batches
 * of 2^31 points or more return ENUFFT_EUNSUPPORTED. */
enufft_status enufft_sort_points(enufft_plan_t p, const void *x, const void *y, const void *h, const void *w,
                                 void *xs, void *ys, void *hs, void *ws, int32_t *perm);

/* Bind sample coordinates to the plan (large-cell plans; Section 2.1.2 Step 1: the tiled
 * spreading's bins depend on x and y only).  Every type-1 and adjoint call of a large-cell
 * plan otherwise runs the tile sort's counting pass (and its scatter, or its order check)
 * on x and y; once x and y are bound, calls given exactly these two device pointers use
 * the tile ranges, work units and order flags computed here and sort nothing; h and w may
 * change from call to call.
 *   x, y   device, n_points reals each (the plan's precision), in tile order, as
 *          enufft_sort_points leaves them; both NULL unbinds.
 * The contents of x and y must not change while bound: bind again (or unbind) after
 * writing them.  Returns ENUFFT_EINVAL (and leaves the plan unbound) when a cell's samples
 * are not in tile order, or when only one of x, y is NULL.  Binding clears a captured
 * forward graph (the next enufft_forward_graph call captures again).  Plans whose cells fit
 * LDS sort nothing per call: the call checks its arguments and keeps nothing.  Allocates
 * 12 bytes per tile and cell on the first call (freed by enufft_destroy). */
enufft_status enufft_bind_points(enufft_plan_t p, const void *x, const void *y);

/* Plain per-cell form of type-1 + EMS for comparison: the same kernels,
 * launched once per cell from a host loop on the plan's stream (no batching,
 * no graph).  Arguments as enufft_type1_batched and enufft_ems. */
enufft_status enufft_percell_loop(enufft_plan_t p, const void *x, const void *y, const void *h,
                                  const void *w, void *f, const enufft_ems_params *prm,
                                  const double *mode_weight, uint8_t *keep, int32_t *k_star,
                                  double *stats);

/* Type-1 + EMS (enufft_type1_batched then enufft_ems) recorded once as a HIP
 * graph and replayed on the plan's stream: one graph launch per call.  The
 * graph is re-captured when any pointer or EMS parameter differs from the last
 * call.  Arguments as enufft_type1_batched and enufft_ems. */
enufft_status enufft_forward_graph(enufft_plan_t p, const void *x, const void *y, const void *h,
                                   const void *w, void *f, const enufft_ems_params *prm,
                                   const double *mode_weight, uint8_t *keep, int32_t *k_star,
                                   double *stats);

/* Record HIP events around every main-kernel launch (enable = 1), or stop (0). */
enufft_status enufft_set_timing(enufft_plan_t p, int32_t enable);

/* Synchronise on the recorded events and return, per kind, the summed
 * durations in ms and the counts: out[0..3] = ms of type-1, EMS, adjoint and
 * forward-graph launches; out[4..7] = their counts.  Clears the record. */
enufft_status enufft_get_timing(enufft_plan_t p, double *out8);

enufft_status enufft_get_info(enufft_plan_t p, enufft_plan_info *info);

/* Destroy a plan (waits for its stream) and free its workspace.  NULL is a no-op. */
enufft_status enufft_destroy(enufft_plan_t p);

/* Text of the last error of p, or of the calling thread when p is NULL.  The
 * string is owned by the library and valid until the next call. */
const char *enufft_last_error(enufft_plan_t p);

/* Library version string. */
const char *enufft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ENUFFT_H */
