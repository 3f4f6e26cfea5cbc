/*
 * grating.h - C ABI of the MI355X (gfx950) solver for plane-wave scattering from a
 * three-layer periodic grating with many circular inclusions in its middle layer.
 *
 * Method: J. Lai, M. Kobayashi, A. Barnett, "A fast and robust solver for the
 * scattering from a layered periodic structure containing multi-particle
 * inclusions".  Section 2 states the problem (TM Helmholtz, quasi-periodicity,
 * Rayleigh-Bloch radiation conditions); section 3 the empty-structure system
 * A alpha = f (eq. matA, Arhs); section 4 the single-inclusion scattering matrix
 * S and the translation operator T (eqs. scat, trans, scattmatrix); section 5 the
 * coupling blocks B, C (eqs. matB, matC), the pseudo-inverse A^+ (eq. applypA)
 * and the left-preconditioned Schur system solved by GMRES; section 6 the flux
 * identity and Bragg amplitudes.
 *
 * Conventions
 *  - Every call returns grt_status; no C++ exception crosses the ABI.  On error
 *    grt_error_message(ctx) describes the failure (owned by ctx, valid until the
 *    next call on ctx).
 *  - Coefficient vectors (beta, K beta, right-hand side) are complex FP64,
 *    interleaved (re, im), laid out [M][2P+1] with the order n = -P..P at index
 *    n + P; a context with n_rhs >= 2 incidence angles stacks them [n_rhs][M][2P+1].  They live in DEVICE memory owned by the caller, on the context's
 *    device, contiguous; the library never frees caller memory.
 *  - Host arrays passed to grt_set_problem are copied; the caller keeps them.
 *  - Work is enqueued on the context stream.  grt_apply and grt_rhs are
 *    asynchronous; grt_solve and grt_bragg synchronise before returning.
 *  - One context per host thread.  Call order:
 *      create -> set_problem -> build -> {apply | rhs | solve | bragg}* -> destroy;
 *    set_problem invalidates build.
 */
#ifndef GRATING_H
#define GRATING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GRT_OK = 0,
  GRT_EINVAL = -1,  /* bad size or value (P outside [1,40], omega <= 0, |phi| >= pi/2, NaN...) */
  GRT_EGEOM = -2,   /* disks overlap (minimum image) or touch an interface            */
  GRT_ENOMEM = -3,  /* device allocation failed                                       */
  GRT_EHIP = -4,    /* a HIP / rocSOLVER call failed                                  */
  GRT_ENOCONV = -5, /* GMRES did not reach the tolerance; beta and stats still written */
  GRT_ESTATE = -6,  /* call out of order (e.g. apply before build)                     */
  GRT_EUNSUP = -7   /* unsupported option                                             */
} grt_status;

typedef enum { GRT_FP64 = 0, GRT_FP32 = 1, GRT_FP32_RELAXED = 2 } grt_precision;
typedef enum { GRT_TM = 0, GRT_TE = 1 } grt_polarization;

typedef struct grt_ctx grt_ctx;

/* Layered structure and its discretization (paper sec. 3).  Interfaces Gamma_1
 * near y = +h and Gamma_2 near y = -h: flat, or graphs of period d (the curved
 * interfaces of secs. 3 and 6) given by n_fourier > 0 and iface, host
 * [2][2][n_fourier] (copied): for Gamma_1 then Gamma_2, the cosine then the sine
 * coefficients a_m, b_m (m = 1..n_fourier, at most 64) of the graph
 *   y = (+h or -h) + sum_m a_m cos(2 pi m x / d) + b_m sin(2 pi m x / d);
 * the graphs must keep Gamma_1 above Gamma_2 and both strictly between the
 * artificial lines Gamma_u, Gamma_d at +-y0 (GRT_EINVAL).  Period d.
 * Discretization: N nodes per interface, equispaced (cell-centred) in x, the
 * graphs' parameter,
 * Nw[l] Gauss-Legendre nodes on the walls of layer l (0 top, 1 middle, 2 bottom),
 * J expansions of orders -Q[l]..Q[l] about (0, +-(h+y0)/2) and (0, 0), Nu nodes on
 * Gamma_u and on Gamma_d, Rayleigh-Bloch orders n_rb_lo .. n_rb_lo + Nrb - 1,
 * zeta-corrected trapezoid stencils of half-width zeta_K, and the pseudo-inverse
 * singular-value cut pinv_eps (relative to the largest singular value). */
typedef struct {
  double d, h, y0;
  double n_layer[3]; /* refractive indices: top (incidence side), middle, bottom */
  int N;
  int Nw[3];
  int Q[3];
  int Nu;
  int n_rb_lo, Nrb;
  int zeta_K;
  double pinv_eps;
  int n_fourier;        /* 0: flat interfaces                                    */
  const double* iface;  /* [2][2][n_fourier] Fourier coefficients (see above)    */
  /* Absorbing substrate (sec. 7 names complex permittivities as an extension): the
   * bottom layer's index is n_layer[2] + i n3_im, 0 <= n3_im <= 0.1 n_layer[2]
   * (GRT_EINVAL below 0, GRT_EUNSUP above the bound, where the complex-argument
   * Hankel and Bessel routines of the layer matrix are not validated; GRT_EUNSUP
   * also when |k_3| times the reach of the bottom layer's J expansion exceeds 60).
   * The layer matrix then takes H_0, H_1 and J_n at complex arguments and the
   * Rayleigh-Bloch wavenumbers k_3n with positive real and imaginary parts (TE: the
   * substrate's eps_3 = (n_3 + i n3_im)^2 is complex too); the translation, C and
   * B_phys (middle layer only) are unchanged.  TM and TE; no field evaluation
   * (GRT_EUNSUP).  grt_bragg then reports T_n as the power order n carries across
   * Gamma_d and flux_err as NaN: the substrate also absorbs between Gamma_2 and
   * Gamma_d.  0: lossless. */
  double n3_im;
} grt_layers;

/* M inclusions (paper sec. 4, 5): centres (x, y), radius and refractive index.
 * shape NULL: disks of that radius (the Mie diagonal scattering matrix of sec. 4.1).
 * shape non-NULL: non-circular inclusions of the paper's class (eq. par1), host
 * [M][4] = (a1, a2, a3, rot) per inclusion, boundary rho(t) (cos(t + rot),
 * sin(t + rot)), rho = a1 + a2 cos(a3 t), with a1 > 0, |a2| < a1, a3 an integer in
 * [1, 64]; radius[m] must be its enclosing circle a1 + |a2| (it serves the packing
 * checks, the near-pair rule and the normalisation D); shape_nodes (even, 16..512;
 * 0: 64) boundary nodes of each inclusion's integral equation (eqs. intg1, intg2),
 * solved at build time for the dense (2P+1)^2 scattering matrix (formula for s_ln;
 * copies turned by rot need no separate treatment: each inclusion is solved as
 * given).  Shapes need P <= 20 and one angle; the block translation, field
 * evaluation and the warm-start network take disks only (GRT_EUNSUP); single and
 * batched solves, FP64 and mixed, take both. */
typedef struct {
  int64_t M;
  const double *x, *y, *radius, *n_incl;
  const double* shape;
  int shape_nodes;
  /* Absorbing disks: n_incl_im (host [M], copied; NULL: lossless) holds the imaginary
   * parts of the indices, n_incl + i n_incl_im with n_incl_im >= 0 (the field
   * e^{i k x - i omega t} decays for Im k > 0).  The Mie coefficients of sec. 4.1 then
   * take J_n at the complex argument k_p R (Miller's recurrence; GRT_EUNSUP when
   * Im(k_p R) > 2 or |k_p R| > 40, where it is not validated), grt_bragg reports the
   * absorbed fraction, and the rest of the path is unchanged.  Disks only, and no
   * field evaluation or warm-start network (GRT_EUNSUP). */
  const double* n_incl_im;
} grt_inclusions;

/* Plane wave of frequency omega (k_l = omega * n_l), angle phi from the downward
 * normal (horizontal wavenumber k_1 sin phi), TM polarisation; multipole order P
 * (2P+1 coefficients per inclusion).  Several right-hand sides: n_rhs >= 2 angles
 * phis[0 .. n_rhs) (host, copied; phi is then ignored) on the same geometry and
 * frequency, each with its own Bloch phase e^{i k_1 sin(phis[r]) d} (sec. 2) and so
 * its own layer factorisation; every coefficient vector of such a context is
 * angle-major, [n_rhs][M][2P+1].  n_rhs 0 or 1: the single angle phi. */
typedef struct {
  double omega;
  double phi;
  int P;
  int64_t n_rhs;
  const double* phis;
  /* GRT_TM (0, the paper's case: u = E_z, u and du/dn continuous) or GRT_TE (1:
   * u = H_z, u and (1/eps) du/dn continuous, eps = n^2 of each medium; each layer's
   * potentials then carry eps of the layer and the flux rows 1/eps, the Mie
   * coefficients weight the radial derivatives by 1/eps, and the transmitted flux by
   * eps_1/eps_3).  TE takes disks only and no field evaluation (GRT_EUNSUP). */
  int polarization;
} grt_incidence;

typedef struct {
  double tol;      /* stop when ||b - K x|| / ||b|| <= tol (FP64 residual)  */
  int maxit;       /* total Arnoldi steps                                    */
  int restart;     /* Krylov dimension per cycle                             */
  int use_x0;      /* 1: beta_dev holds the initial guess on entry           */
  int precision;   /* GRT_FP64: GMRES on K in FP64.  GRT_FP32: FP64 iterative
                      refinement r = b - K x, x += e, with e from GMRES (FP64
                      orthogonalisation) on K32, whose translation between
                      well-separated inclusions runs in FP32 (FP32 accumulate).
                      GRT_FP32_RELAXED: one FP64 GMRES on K whose Arnoldi
                      applies switch to K32 once the residual estimate is
                      below inner_tol (relaxed inexact Krylov: an apply error
                      of relative size e is harmless once the residual is
                      below tol / e; Bouras and Fraysse 2005, Simoncini and
                      Szyld 2003); every restart and the final check take the
                      FP64 residual b - K x, so a solve that stops has met tol
                      in FP64                                                 */
  double inner_tol;/* GRT_FP32: relative tolerance of each inner solve (0: 1e-5).
                      GRT_FP32_RELAXED: relative residual below which the
                      applies use K32 (0: 1e5 tol, at most 1e-2: tol / (10 e)
                      for the FP32 apply's relative error e of about 1e-7) */
  int max_refine;  /* GRT_FP32: most refinement steps (0: 10)                */
  int use_graph;   /* 1: every apply of K is replayed from a HIP graph captured
                      once per operator (dropped when the table, the launch
                      shape or the problem changes); ignored while kernel
                      timing (grt_profile_enable) is on.  Same results.        */
} grt_solve_opts;

typedef struct {
  int iters;            /* Arnoldi steps taken (all inner solves)            */
  int cycles;           /* restart cycles                                    */
  double rel_resid;     /* true relative residual ||b - K x|| / ||b|| (FP64)  */
  double seconds;       /* wall time of the solve                            */
  int refine_steps;     /* GRT_FP32: FP64 refinement steps taken             */
  int x0_rejected;      /* use_x0 and ||b - K x0|| >= ||b||: the guess was
                           dropped and the solve started from x = 0          */
  int fp32_applies;     /* applies of K32 (GRT_FP32: every inner step;
                           GRT_FP32_RELAXED: the Arnoldi steps past the switch) */
} grt_solve_stats;

typedef struct {
  int64_t M;
  int P;
  int64_t n_beta;   /* M (2P+1): complex entries of a coefficient vector     */
  int64_t n_rows;   /* rows of A                                             */
  int64_t n_alpha;  /* columns of A                                          */
  int64_t rank;     /* singular values kept by the pseudo-inverse            */
  int Nrb;
  int m2l_chunks;   /* source chunks of the translation launch (one partial
                       result of n_beta entries each)                         */
  int m2l_split;    /* variant of the FP64 translation: on the fly, 1 launch or
                       2 (each forming half of the 2P+1 outputs, recomputing
                       the generator); with the resident table, 1 or 2 lanes
                       per target                                             */
  int cx_chunks;    /* source chunks of the C x launch                       */
  int bx_chunks;    /* node chunks of the B_phys w (P2L) launch              */
  int64_t n_rhs;    /* right-hand sides (angles); vectors hold n_rhs * n_beta  */
} grt_sizes;

/* Create a context on HIP device `hip_device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = a stream the context creates and owns). */
grt_status grt_create(grt_ctx** out, int hip_device, void* hip_stream);
grt_status grt_destroy(grt_ctx* ctx);
const char* grt_error_message(const grt_ctx* ctx);

/* Copy and validate the problem (sec. 2).  GRT_EGEOM if two disks overlap under
 * the minimum image in x, a disk crosses an interface or a centre lies outside the
 * cell |x| <= d/2 (the near copies l = -1, 0, 1 of sec. 4.2 assume one cell).  With
 * curved interfaces a disk crosses one when a point of the graph within its x-range,
 * sampled at spacing radius / 256, lies closer than its radius to the centre. */
grt_status grt_set_problem(grt_ctx* ctx, const grt_layers* lay, const grt_inclusions* inc,
                           const grt_incidence* wave);

/* Build everything the apply needs, on the device: the Mie diagonal S (sec. 4.1),
 * the matrix A (sec. 3, eq. matA) with zeta-corrected self blocks, its SVD and the
 * truncated pseudo-inverse factors (eq. applypA), the L2L table and f (eq. Arhs). */
grt_status grt_build(grt_ctx* ctx);

/* Build only what the translation needs (sec. 4.1 Mie diagonal S, the normalisation
 * D = |H_|n|(k2 r)|, the H_0/H_1 table, the translation's workspace), not the layered
 * structure (no A, no SVD).  Afterwards grt_apply_ST_block (any n_rhs), grt_apply_T
 * (n_rhs = 1), grt_set_launch and grt_query work; every call that needs the layers
 * returns GRT_ESTATE until grt_build (which then builds the rest from scratch).  For
 * uses of the translation alone, e.g. timing it at sizes where factorising the layers
 * of every angle would take far longer than the applies. */
grt_status grt_build_translation(grt_ctx* ctx);

grt_status grt_query(const grt_ctx* ctx, grt_sizes* out);

/* Fast translation for large M (the fast-multipole acceleration of T that the
 * paper's complexity remarks in secs. 5 and 7 name), enable = 1: a single-level cell
 * scheme.  The inclusion centres are binned into square cells (about per_cell each; 0:
 * at least 16 and cells at least 13 / (k_2 sqrt 2) wide, below which the default order
 * loses accuracy; at least 3 across the period); a cell and the cells adjacent to it, the
 * neighbours on the copies l = -1, +1 included, are translated pair by pair as in
 * sec. 4.2, every other (cell, copy) pair through cell expansions of order p_cell
 * (0: k_2 times the cell diagonal plus 25, at most 127): outgoing shift to the cell
 * centre, multipole-to-local between cell centres (a generator table over cell
 * offsets built here), local shift to each target (Graf's theorem each).  Same
 * operator as the dense translation up to the expansions' truncation.  Afterwards
 * grt_apply (FP64), grt_apply_T and FP64 grt_solve use it; mixed precision and
 * batches need the dense translation (GRT_EUNSUP), as do several angles, P > 20,
 * and disks wider than half a cell.  info (may be NULL): nx, ny, p.  enable = 0
 * returns to the dense translation.  Allocates O(M + cells (p + offsets p)). */
grt_status grt_set_fmm(grt_ctx* ctx, int enable, int p_cell, int per_cell, int* info);

/* y = K x with K = I - S T + S B_phys A^+ C, the left-preconditioned Schur
 * operator of sec. 5 (B_phys = -B of the paper).  x, y: device [n_rhs][M][2P+1]
 * complex FP64 (each angle's own K), may not alias.  precision GRT_FP64:
 * everything in FP64.  GRT_FP32 with one right-hand side: the translation T between
 * inclusion pairs whose scaled distance k2*rho keeps every H_q, q <= 2P, inside the
 * FP32 range runs in FP32 with FP32 accumulation (the Hankel generator itself is
 * FP64); the remaining near pairs, the layer correction and the preconditioner stay
 * FP64.  GRT_FP32 with n_rhs >= 2: S T of all angles at once as one complex GEMM on
 * the FP32 matrix cores (grt_apply_ST_block), every pair included (in the basis
 * normalised by D = |H_|n|(k2 r)| its entries are at most of order one); the layer
 * correction of each angle in FP64. */
grt_status grt_apply(grt_ctx* ctx, const void* x_dev, void* y_dev, int precision);

/* Resident translation table (FP64 applies).  The Toeplitz generator of every
 * (target, source) pair, tau_q = sum_l alpha^l H_q(k2 rho_l) e^{i q phi_l} (sec. 4.2,
 * eq. repre3_mod), does not depend on beta, so it can be built once per problem
 * (M * Mpad * (4P+1) complex FP64, Mpad = M rounded up to 64: 1.0 GB at M = 1000,
 * P = 15) and streamed by every apply instead of re-evaluating the Hankel functions.
 * mode 1 builds it now (if built) and after every later grt_build, and contracts it
 * with one lane per target; mode 2 is the same table contracted with two lanes per
 * target (each lane half of the 2P+1 outputs, using the reflection symmetry of the
 * Toeplitz product: more waves per SIMD, but twice the load instructions; kept for
 * comparison); 0 frees it and the apply evaluates the generator on the fly again.  Results agree with the on-the-fly apply to rounding.
 * GRT_ENOMEM if it does not fit in free device memory with 1 GiB to spare (the
 * context stays usable, without the table).  The mixed-precision apply has a table
 * of its own (grt_set_table32); batched FP64 solves stream the table of every
 * context that has one when the batch is created (changing the mode afterwards makes
 * grt_batch_solve return GRT_ESTATE). */
grt_status grt_set_table(grt_ctx* ctx, int mode);
/* Resident FP32 table of the mixed-precision apply (GRT_FP32 and GRT_FP32_RELAXED
 * solves and grt_apply with GRT_FP32, one angle).  The same generator as
 * grt_set_table, rounded to FP32, for the well-separated pairs only: a pair with a
 * kept copy at k2 rho below the FP32-safe distance is zero in the table and stays
 * in the FP64 near-pair pass.  M * Mpad * (4P+1) complex FP32 (half the FP64
 * table's bytes), streamed by every mixed apply instead of evaluating the Hankel
 * functions; the contraction and its accumulation are FP32 as on the fly, so the
 * result differs from the on-the-fly mixed apply by FP32 rounding only.  on = 1
 * builds it now (if built) and after every later grt_build; 0 frees it.
 * GRT_ENOMEM as grt_set_table; GRT_EUNSUP for a context with several angles (their
 * FP32 translation is the matrix-core block product).  Batched mixed solves use the
 * tables of the contexts that have one when the batch is created. */
grt_status grt_set_table32(grt_ctx* ctx, int on);

/* The block-diagonal scattering matrix of sec. 4.1 (after grt_build or
 * grt_build_translation): out_dev (device, [M][2P+1][2P+1] complex FP64, caller
 * owned; block m row l = outgoing order l, column n = incoming order n, index + P)
 * receives the dense blocks of non-circular inclusions or the Mie diagonal of
 * disks. */
grt_status grt_scattering_blocks(grt_ctx* ctx, void* out_dev);
/* Launch-shape autotuner: times the translation launch, with the pass that adds
 * its per-chunk partial results, for source chunk counts giving 256 .. 16384
 * wavefronts, in the current mode (on the fly or resident table) and in its two
 * variants (on the fly: one launch, or two each forming half of the outputs with
 * half the accumulators per lane; table: one or two lanes per target, the latter
 * as grt_set_table(ctx, 2)), then the C x and B_phys w launches
 * (each with the pass that adds its per-chunk partial results) for 1 .. 64 sources
 * per wave, and keeps the fastest of each for every later apply of this context
 * (results change only by the order of the chunk sums; grt_query reports the
 * choices).  Up to cap measured (chunk count, split, ms per launch) triples of the
 * translation go to chunks[] / splits[] / ms[] (host; splits may be NULL); *n
 * receives their number.  Without a call every split aims at two work-groups per
 * SIMD, in one launch. */
grt_status grt_autotune(grt_ctx* ctx, int cap, int* n, int* chunks, int* splits, double* ms);

/* Set the translation's launch shape by hand (what grt_autotune would choose):
 * about m2l_chunks source chunks (1 .. the number grt_autotune may try, at most M;
 * the chunk length is rounded up, so grt_query may report fewer) and the variant
 * m2l_split of the current mode, 1 or 2 (on the fly: 2 = two launches, each forming
 * half of the outputs; resident table: 2 = two lanes per target; mixed precision
 * ignores it).  Results change only by the order of the chunk sums.  GRT_EINVAL
 * outside those ranges. */
grt_status grt_set_launch(grt_ctx* ctx, int m2l_chunks, int m2l_split);

/* on = 1: the FP64 apply runs C x, A^+ and B_phys w (bound by FP64 arithmetic) on a
 * second stream of the context, concurrently with the translation T x (bound by HBM
 * in table mode), joining before the combine; every later apply, solve and captured
 * graph of this context does so.  Results are identical (the same kernels with the
 * same inputs).  on = 0: one stream (the default).  GRT_EINVAL for other values. */
grt_status grt_set_overlap(grt_ctx* ctx, int on);

/* Bytes the table of the current problem takes. */
grt_status grt_table_bytes(const grt_ctx* ctx, int64_t* bytes);

/* Diagnostic parts of the apply: y = T x (translation among inclusions and their
 * near copies, sec. 4.2 / eq. repre3_mod) and y = B_phys A^+ C x (the low-rank
 * layer correction, sec. 5).  Same layout as grt_apply. */
grt_status grt_apply_T(grt_ctx* ctx, const void* x_dev, void* y_dev);
grt_status grt_apply_lowrank(grt_ctx* ctx, const void* x_dev, void* y_dev);

/* y_r = S T_r x_r for every right-hand side r (any n_rhs >= 1), the translation of
 * sec. 4.2 with the Bloch phase alpha_r = e^{i kappa_r d} of each angle on the near
 * copies (eq. repre3_mod), computed as one complex GEMM per target on the FP32
 * matrix cores (v_mfma_f32_16x16x4f32): A_j[n, (m, l, nu)] = D_j[n] s_j[n]
 * tau^{(jml)}_{nu - n} / D_m[nu] generated in FP64 from the Hankel recurrence and
 * rounded to FP32, B[(m, l, nu), r] = alpha_r^l (D x_r)_m[nu] in FP32, FP32
 * accumulation.  Same layout as grt_apply; allocates its packed buffers on the
 * first call (M (2P+1) R_64 complex FP32 each, R_64 = n_rhs rounded up to 64). */
grt_status grt_apply_ST_block(grt_ctx* ctx, const void* x_dev, void* y_dev);

/* b = S B_phys A^+ f, the right-hand side of the reduced system (device). */
grt_status grt_rhs(grt_ctx* ctx, void* b_dev);

/* alpha0 = B_phys A^+ f (device, n_beta complex): the incoming coefficients that
 * the layered structure alone sends to each inclusion (sec. 5), so that b = S alpha0. */
grt_status grt_incident(grt_ctx* ctx, void* a_dev);

/* Solve K beta = b by restarted GMRES in FP64 on the device (sec. 5).  beta_dev
 * (device) receives the solution; with opts->use_x0 it holds the initial guess
 * on entry.  GRT_ENOCONV if tol is not reached (beta and stats still written).
 * n_rhs >= 2: every angle's system, [n_rhs][M][2P+1], solved in lockstep as one
 * batch (each angle keeps its own Krylov space: the operators differ by the Bloch
 * phase); stats must then hold n_rhs entries (or be NULL); GRT_FP32 runs the FP64
 * refinement of every angle around inner solves whose translation is the FP32
 * matrix-core block product of all angles. */
grt_status grt_solve(grt_ctx* ctx, const grt_solve_opts* opts, void* beta_dev,
                     grt_solve_stats* stats);

/* Bragg amplitudes (sec. 2 eq. rad1/rad2, sec. 6) of right-hand side rhs (0 ..
 * n_rhs - 1): from beta (device, that angle's [M][2P+1] vector) form
 * alpha = A^+ (f - C beta) and return, for each of the Nrb orders (host arrays of
 * length >= Nrb): orders[i], c[2i..2i+1], d[2i..2i+1] (re, im), the reflected and
 * transmitted energy fractions R[i], T[i] (zero for evanescent orders), the fraction
 * absorbed by the disks (absorbed, may be NULL; 0 without absorbing disks:
 * -4 sum_{m,n} |b_n|^2 (|s_n|^2 + Re s_n) / |s_n|^2 over each disk's outgoing b = beta_m,
 * the flux of sum_n (a_n J_n + b_n H_n) e^{in theta} through a circle with a_n = b_n / s_n,
 * over the incident flux d k_1 cos(phi); TE weights each flux by 1/eps of its medium)
 * and the energy-balance error |sum R + sum T + absorbed - 1| (the flux error of
 * sec. 6 for lossless media).  Over an absorbing substrate (grt_layers.n3_im > 0)
 * T[i] is Re(k_3n) |d_n|^2 over the incident flux for every order (the power order
 * n carries across Gamma_d; TE: eps_1 Re(k_3n / eps_3) |d_n|^2 over k_1 cos(phi)) and
 * flux_err is NaN.  GRT_EINVAL for rhs out of range. */
grt_status grt_bragg(grt_ctx* ctx, int64_t rhs, const void* beta_dev, int64_t cap, int* orders,
                     double* c, double* d, double* R, double* T, double* flux_err,
                     double* absorbed);

/* The total field of right-hand side rhs at n_pts points (host xy[2 i], xy[2 i + 1])
 * for its solution beta (device, that angle's [M][2P+1] vector; ignored when M = 0),
 * written to host u[2 i], u[2 i + 1] (re, im).
 * The representation of sec. 3 (eqs. repre1-repre3) and sec. 5 (eq. repre3_mod): in
 * each truncated layer the three near copies of the interface layer potentials (the
 * trapezoid sums over the nodes the method solves with), the layer's J expansion,
 * and in the middle layer the outgoing multipoles of every disk and of its copies
 * l = -1, 0, 1; above y0 and below -y0 the Rayleigh-Bloch expansions with c_n, d_n
 * (eqs. rad1, rad2); the incident plane wave in the top layer (y > h); inside a disk
 * or one of its near copies the interior expansion sum_n gamma_n J_n(k_p r) e^{in theta}
 * (sec. 4.1) with gamma_n from continuity with the field arriving at the disk.  The
 * representation is evaluated in the unit cell |x| <= d/2 and carried to other x by
 * quasi-periodicity, u(x + l d) = alpha^l u(x) (sec. 2).  A point with |y| = h
 * exactly belongs to the middle layer.  The node sums lose
 * accuracy within a few node spacings (d/N) of an interface and are not the field on
 * it.  Allocates device scratch (O(n_alpha rank + M (2P+1) + n_pts)) and synchronises
 * the context stream.  GRT_EINVAL for null arrays or coordinates that are not finite
 * or exceed 1e6 in size, GRT_EUNSUP for TE, non-circular inclusions and curved
 * interfaces, GRT_ESTATE before grt_build. */
grt_status grt_eval_field(grt_ctx* ctx, int64_t rhs, const void* beta_dev, int64_t n_pts,
                          const double* xy, double* u);

/* Copy the equilibrated matrix A (column-major [n_alpha][n_rows] complex) and its
 * column scales to host buffers (diagnostics / tests; the first angle's). */
grt_status grt_get_A(grt_ctx* ctx, double* A_host, double* colscale_host);

/* Copy the Mie diagonal [M][2P+1] complex to a host buffer (diagnostics / tests; also
 * after grt_build_translation). */
grt_status grt_get_mie(grt_ctx* ctx, double* s_host);

/* Kernel timing for measurement tools.  While enabled, every launch of the
 * translation kernel (the dense part of K, sec. 4.2) is bracketed by HIP events on
 * the context stream.  grt_profile_read synchronises the stream, returns the total
 * milliseconds and the number of launches since the previous read, and resets them. */
grt_status grt_profile_enable(grt_ctx* ctx, int enable);
grt_status grt_profile_read(grt_ctx* ctx, double* m2l_ms_total, int64_t* m2l_launches);

/* ---- Translation without allocation ------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  y = T x, the same
 * translation as grt_apply_T (sec. 4.2, eq. repre3_mod: the three near copies
 * l = -1, 0, 1 of every inclusion, phased by alpha^l, excluding (j, j, 0)), but with
 * no context: the caller passes the geometry as device arrays and the call makes no
 * allocation.  Its per-chunk partial sums go to a fixed scratch array that the
 * library holds on each device for the life of the process
 * (GRT_NOALLOC_SCRATCH_BYTES = 64 MiB); the chunk count is chosen as in grt_apply_T
 * and lowered until the partials fit, so M (2P+1) may be at most 4,194,304 (one
 * partial result); larger problems get GRT_EINVAL.
 *   M: inclusions, centres cx_dev[M], cy_dev[M] (device FP64) inside one cell
 *      |x| <= d/2 (not checked; grt_set_problem checks it on the context path);
 *   P: multipole order (1-6, 8, 10, 12, 15 or 20; others GRT_EUNSUP);
 *   k2: wavenumber of the middle layer (> 0); d: period (> 0);
 *   alpha = alpha_re + i alpha_im: the Bloch phase e^{i kappa d} (|alpha| = 1 to 1e-12);
 *   x_dev, y_dev: device complex FP64 [M][2P+1] (n = -P..P at n + P), not aliased.
 * Work is enqueued on hip_stream (a hipStream_t on the current device; NULL: the null
 * stream) and is asynchronous.  The first call on a device fills that device's
 * H_0 / H_1 table with a synchronous copy, so it must not be made under stream
 * capture (GRT_ESTATE then); later calls may be captured.  Calls that overlap on one
 * device share its scratch array and race: order them (one stream, or events).
 * Results equal grt_apply_T's up to the order of the partial sums. */
#define GRT_NOALLOC_SCRATCH_BYTES (64ll << 20)
grt_status grt_apply_T_noalloc(int64_t M, int P, double k2, double d, double alpha_re,
                               double alpha_im, const double* cx_dev, const double* cy_dev,
                               const void* x_dev, void* y_dev, void* hip_stream);

/* ---- Batched solves --------------------------------------------------------
 * Many problems (different inclusion sets, angles or frequencies; the sweeps of
 * sec. 6) solved together: every GMRES step of the batch is one launch per kernel
 * over all problems, so small problems share the device instead of each leaving
 * it mostly idle.  Each problem converges on its own (its own Hessenberg matrix,
 * rotations and residual) exactly as grt_solve would, in FP64. */
typedef struct grt_batch grt_batch;

/* Make a batch of n built contexts (all with M >= 1, all on one device).  The
 * batch borrows the contexts' device data: they must stay alive until
 * grt_batch_destroy; grt_apply / grt_solve on them share their scratch buffers, so
 * they must not overlap a batch solve; after grt_set_problem, grt_build or a change
 * of table mode on one of them grt_batch_solve returns GRT_ESTATE (make a new
 * batch).  hip_stream: stream to run on, or NULL for a private one.
 * GRT_ESTATE if a context is not built, has no inclusions or is on another
 * device; GRT_EINVAL for n <= 0, NULL arrays, a context with n_rhs >= 2 (grt_solve
 * batches its angles itself) or a context listed twice (every
 * instance writes its own context's scratch buffers during a lockstep step, so the
 * contexts of one batch must be distinct). */
grt_status grt_batch_create(grt_batch** out, int64_t n, grt_ctx* const* ctxs, void* hip_stream);
grt_status grt_batch_destroy(grt_batch* batch);
const char* grt_batch_error_message(const grt_batch* batch);

/* Solve every problem of the batch.  beta[i] is a device vector of the i-th
 * context's n_beta complex entries (its initial guess on entry when
 * opts->use_x0); stats (host, n entries, may be NULL) receives each problem's
 * iterations, restarts and final relative residual (seconds is the batch's).
 * opts->precision GRT_FP64: lockstep GMRES on every problem in FP64.  GRT_FP32:
 * lockstep FP64 iterative refinement (as in grt_solve: the residual b - K x in FP64,
 * then GMRES on the operator with the FP32 translation of well-separated pairs to
 * opts->inner_tol, at most opts->max_refine times); a problem whose FP64 residual
 * meets tol takes no further corrections, and stats report its inner iterations
 * and refinement steps.  opts->maxit bounds the lockstep steps of the whole batch;
 * with opts->use_graph the batch's apply (every kernel launch for all problems; one
 * graph per precision) is captured once as a HIP graph and replayed at every step.
 * GRT_ENOCONV if any problem missed tol; GRT_EINVAL for another precision. */
grt_status grt_batch_solve(grt_batch* batch, const grt_solve_opts* opts, void* const* beta,
                           grt_solve_stats* stats);

/* ---- Learned warm start ------------------------------------------------------
 * A message-passing network over each inclusion's k nearest neighbours (minimum
 * image in x, period d; ties by index) predicts the multiple-scattering part of the
 * incoming coefficients on orders |n| <= p_out; the GMRES initial guess is
 *   beta0_j[n] = s_j[n] (alpha0_j[n] + out_j[n])   (alpha0 from grt_incident, s the
 * Mie diagonal; out = 0 for |n| > p_out),
 * i.e. the exact relation beta = S alpha of sec. 5 with the incoming field alpha
 * predicted.  grt_solve with use_x0 drops a guess no better than zero
 * (stats.x0_rejected), so the plain solve stays the fallback, and GMRES to the
 * requested residual decides the accuracy of the result.
 *
 * Network, width H, L layers, node inputs f_j (32), edge inputs e_jk (8):
 *   h = relu(W_in f + b_in);  per layer: P = A h, Q = B h,
 *   agg_j = mean_k relu(P_j + Q_nbr(j,k) + C e_jk + c),  h <- h + relu(U [h; agg] + u);
 *   out = W_out h + b_out   (out_j: (re, im) for n = -p_out .. p_out).
 * Node inputs: k2 r, n/n2 - 1, y/h, sin phi, omega/40, (D s)_n for n = 0,1,2 and
 * alpha0_n for n = -3..3 as (re, im) pairs (D = |H_|n|(k2 r)|), zero padding.
 * Edge inputs for c_j - c_m = rho e^{i phi}, z = k2 rho:
 *   k2 dx, k2 dy, z, 1/z, H0(z) (re, im), H1(z) e^{i phi} (re, im).
 * Flat FP32 parameter vector, row-major matrices: W_in [H][32], b_in [H]; per layer
 * A [H][H], B [H][H], C [H][8], c [H], U [H][2H], u [H]; W_out [O][H], b_out [O]
 * with O = 2 (2 p_out + 1).  The forward and backward passes use the weights
 * rounded to bfloat16 (nearest, ties to even) with FP32 activations and
 * accumulation; Adam updates the FP32 master copy.
 * Loss of one geometry: sum w (out - t)^2 / wnorm with t the exact correction
 * T beta - B_phys A^+ C beta of a solved geometry, w = (D |s|)^2 and
 * wnorm = sum w |alpha0 + t|^2 over the predicted orders. */
typedef struct grt_nn grt_nn;
typedef struct {
  int width;   /* H: multiple of 64 in [64, 256]                            */
  int layers;  /* L: 1..8                                                   */
  int k;       /* neighbours per inclusion: 1..32                           */
  int p_out;   /* predicted orders |n| <= p_out: 0..20                      */
} grt_nn_config;

/* Create a network (all weights 0 until grt_nn_set_params) on a device and stream
 * (NULL: private stream).  GRT_EINVAL for a configuration outside the ranges. */
grt_status grt_nn_create(grt_nn** out, int hip_device, void* hip_stream, const grt_nn_config* cfg);
grt_status grt_nn_destroy(grt_nn* nn);
const char* grt_nn_error_message(const grt_nn* nn);
grt_status grt_nn_num_params(const grt_nn* nn, int64_t* n);
/* Copy count FP32 weights in (resets the Adam state) or out (host arrays). */
grt_status grt_nn_set_params(grt_nn* nn, const float* host, int64_t count);
grt_status grt_nn_get_params(grt_nn* nn, float* host, int64_t count);

/* Build the graph and inputs of a built context (M >= 1, one angle: GRT_EUNSUP for
 * n_rhs >= 2) and keep them on the
 * device as a sample; with beta_dev (its solution, device) also the training target.
 * The context may be destroyed afterwards.  *id receives the sample's index. */
grt_status grt_nn_add_sample(grt_nn* nn, grt_ctx* ctx, const void* beta_dev, int* id);
grt_status grt_nn_clear_samples(grt_nn* nn);
grt_status grt_nn_sample_size(grt_nn* nn, int id, int64_t* M);
/* Copy a sample's inputs and target to host arrays (any may be NULL):
 * feat [M][32], nbr [M][k] (-1 = none), edge [M][k][8], target and weight [M][O]. */
grt_status grt_nn_get_sample(grt_nn* nn, int id, float* feat, int* nbr, float* edge,
                             float* target, float* weight, double* wnorm);
/* Replace a sample's target, weights (host [M][O]) and normaliser (> 0). */
grt_status grt_nn_set_target(grt_nn* nn, int id, const float* target, const float* weight,
                             double wnorm);

/* Loss of one sample with the current weights; grad_host (num_params floats) and
 * out_host ([M][O]) receive the gradient and the outputs when not NULL. */
grt_status grt_nn_loss_grad(grt_nn* nn, int id, double* loss, float* grad_host, float* out_host);

/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) over the given samples,
 * one step per sample, in an order reshuffled every epoch from seed.
 * last_epoch_loss: mean loss over the last epoch (losses before each step). */
grt_status grt_nn_train(grt_nn* nn, int64_t n_ids, const int* ids, int epochs, float lr,
                        uint64_t seed, double* last_epoch_loss);

/* beta0 (device, n_beta complex) for a built context: graph, inputs and forward
 * pass on the device, then beta0 = s (alpha0 + out).  Pass it to grt_solve with
 * opts.use_x0 = 1. */
grt_status grt_nn_predict(grt_nn* nn, grt_ctx* ctx, void* beta0_dev);

#ifdef __cplusplus
}
#endif
#endif /* GRATING_H */
