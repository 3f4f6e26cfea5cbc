// Internal declarations of the grating library (host + device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include <memory>
#include <string>
#include <vector>

#include "dev_common.h"
#include "../../include/grating.h"

// Row blocks of the empty-structure system, in storage order.
enum RowBlock { RB_G1V = 0, RB_G1N, RB_G2V, RB_G2N, RB_W2V, RB_W2D, RB_W1V, RB_W1D,
                RB_W3V, RB_W3D, RB_UV, RB_UN, RB_DV, RB_DN, RB_COUNT };
// Column blocks (unknowns alpha), in storage order.
enum ColBlock { CB_MU1 = 0, CB_SIG1, CB_MU2, CB_SIG2, CB_A2, CB_A1, CB_A3, CB_C, CB_D, CB_COUNT };

// Everything a device kernel needs to know about one problem (passed by value).
struct DevGeom {
  double d, h, y0, hs;          // period, half thickness, Gamma_u height, d/N
  double k[3];                  // layer wavenumbers (top, middle, bottom): real parts
  double k_im[3];               // their imaginary parts (absorbing substrate: k_im[2] > 0)
  double kappa;                 // k_1 sin(phi)
  cd alpha, alpha_inv;          // Bloch phase e^{i kappa d} and its inverse
  // polarisation factors: the potentials of layer l carry pv[l] and the interface
  // flux rows fl[l] for the field of layer l (TM: all 1; TE: eps_l and 1/eps_l)
  double pv[3], fl[3];
  double pv_im[3], fl_im[3];     // imaginary parts (TE over an absorbing substrate: layer 2)
  int te;
  int N, Nu, n_rb_lo, Nrb, zeta_K, P, M;
  int Nw[3], Q[3];
  double jcy[3];                // J-expansion centres (0, jcy[l])
  int row_off[RB_COUNT + 1];
  int col_off[CB_COUNT + 1];
  int n_rows, n_alpha;
  const double* yw[3];          // wall nodes (device)
  // interface nodes (device) [2][N][NODE_STRIDE]: x, y, unit normal (nx, ny) pointing
  // up, speed |(1, f')| and f'' of the graph y = f(x) (flat: y = +-h, n = (0, 1),
  // speed 1, f'' = 0); the quadrature weight of node j is hs * speed
  const double* node;
  int curved;                   // 1: curved interfaces (graphs of period d)
  // zeta-correction weights per target (device) [2 interfaces][4 kinds: S, D, N, T]
  // [N targets][2K+1 stencil offsets]
  const cd* wcorr;
};
constexpr int NODE_STRIDE = 6;

// q-th x-derivative (q = 0, 1, 2) of interface j's height y = f_j(x): +h (j = 0) or
// -h (j = 1) plus sum_m a_m cos(w_m x) + b_m sin(w_m x), w_m = 2 pi m / d, with
// co[(j * 2 + 0) * F + m - 1] = a_m and co[(j * 2 + 1) * F + m - 1] = b_m (host).
inline double iface_height(const double* co, int F, int j, double h, double d, double x, int q) {
  double v = q == 0 ? (j == 0 ? h : -h) : 0.0;
  for (int m = 1; m <= F; ++m) {
    const double w = 2.0 * M_PI * m / d;
    const double a = co[(j * 2 + 0) * F + m - 1], b = co[(j * 2 + 1) * F + m - 1];
    const double cw = std::cos(w * x), sw = std::sin(w * x);
    if (q == 0) v += a * cw + b * sw;
    else if (q == 1) v += w * (-a * sw + b * cw);
    else v += w * w * (-a * cw - b * sw);
  }
  return v;
}

// Device data of the empty layered structure (wall nodes, quadrature corrections,
// A, its SVD, the pseudo-inverse factor blocks, f) shared by every problem with the
// same layers, discretization, omega and phi.
struct LayerFactors {
  int device = 0;
  double *yw = nullptr, *colscale = nullptr, *sv = nullptr, *htab = nullptr, *node = nullptr;
  cd *wcorr = nullptr, *A = nullptr, *U = nullptr, *VH = nullptr;
  cd *W1 = nullptr, *W2 = nullptr, *W3 = nullptr, *f = nullptr;
  int rank = 0;
  ~LayerFactors();
};

struct grt_batch;

struct grt_ctx {
  std::shared_ptr<LayerFactors> lf;  // owns the layer-side buffers below when set
  // several right-hand sides (incidence angles) on one geometry: this context holds
  // the first angle, rhs[r - 1] the others (contexts of their own, same device and
  // stream); solves of all angles run as one lockstep batch
  int64_t n_rhs = 1;
  std::vector<double> phis;
  std::vector<grt_ctx*> rhs;
  grt_batch* rhs_batch = nullptr;
  // block translation on matrix cores (FP32): packed inputs, outputs, phases
  cf* d_blkX = nullptr;     // [M][NBK][blk_Rp]
  cf* d_blkY = nullptr;     // [M][nb][blk_Rp]
  cf* d_blkph = nullptr;    // [blk_Rp]
  int blk_Rp = 0;
  cd* d_blkw = nullptr;     // [n_rhs][n_beta] low-rank terms of a block apply
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // second stream of the FP64 apply: C x, A^+ and B_phys w concurrently with T x
  bool overlap = false;
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::string err;
  // problem (host copies)
  bool have_problem = false, built = false;
  bool trans_built = false;   // grt_build_translation: translation data only, no layers
  grt_layers lay{};
  grt_incidence inc{};
  int64_t M = 0;
  std::vector<double> hx, hy, hr, hn;
  std::vector<double> hiface;  // [2][2][n_fourier] interface Fourier coefficients
  std::vector<double> hn_im;   // imaginary parts of the disks' indices (absorbing)
  bool lossy = false;
  // derived
  DevGeom g{};
  int P = 0, nb = 0;
  int64_t n_beta = 0;
  int n_g = 0;   // rows of C that are nonzero (prefix): Gamma_1, Gamma_2, wall 2
  int n_b = 0;   // entries of alpha read by B (prefix): mu1, sig1, mu2, sig2, a2
  int rank = 0;
  // device buffers owned by the context
  double *d_cx = nullptr, *d_cy = nullptr, *d_rad = nullptr, *d_kp = nullptr;
  double* d_kp_im = nullptr;  // [M] Im k_p of absorbing disks (null: lossless)
  double* d_yw = nullptr;
  double* d_node = nullptr;  // [2][N][NODE_STRIDE] interface nodes
  cd* d_wcorr = nullptr;
  cd* d_A = nullptr;        // [n_alpha][n_rows] column-major, equilibrated
  double* d_colscale = nullptr;
  double* d_sv = nullptr;
  cd* d_U = nullptr;        // [min][n_rows] column-major
  cd* d_VH = nullptr;       // [n_alpha][n_alpha] column-major (V^H)
  cd* d_W1 = nullptr;       // [rank][n_g]   row-major: Sigma^+ U^H (prefix rows)
  cd* d_W2 = nullptr;       // [n_b][rank]   row-major: E V (prefix entries)
  cd* d_W3 = nullptr;       // [2 Nrb][rank] row-major: E V (c, d entries)
  cd* d_mie = nullptr;      // [M][nb]
  double* d_dnorm = nullptr; // [M][nb] |H_|n|(k2 R_m)|: scaling of the normalised system
  double* d_dinv = nullptr;  // [M][nb] 1 / d_dnorm
  cd* d_xtmp = nullptr;      // [M][nb] scratch of the normalised apply
  cd* d_l2l = nullptr;      // [M][2(Q2+P)+1]  J_m(k rho_j) e^{i m phi_j}
  cd* d_f = nullptr;        // [n_g] right-hand side prefix
  double* d_htab = nullptr; // H_0, H_1 interpolation table (HTAB_SIZE doubles)
  // apply workspace
  int m2l_chunk = 16, m2l_nchunks = 0;
  int m2l_nchunks_cap = 0;  // partial buffers hold this many chunks
  int m2l_split = 1;        // on-the-fly FP64 translation over 1 or 2 launches (halves of n)
  int c_chunk = 64, c_nchunks = 0, c_nchunks_cap = 0;
  int b_chunk = 64, b_nchunks = 0, b_nchunks_cap = 0;
  cd* d_pT = nullptr;       // [m2l_nchunks][M][nb]
  cd* d_pC = nullptr;       // [c_nchunks][n_ctgt][2]
  cd* d_pB = nullptr;       // [b_nchunks][M][nb]
  cd* d_pL = nullptr;       // [M][nb]
  cd* d_gvec = nullptr;     // [n_g]
  cd* d_tvec = nullptr;     // [rank]
  cd* d_wvec = nullptr;     // [n_b]
  // mixed precision: FP32 translation for well-separated pairs, FP64 near-pair lists
  double zsafe = 0.0;
  cf* d_x32 = nullptr;      // [n_beta]
  cf* d_pT32 = nullptr;     // [m2l_nchunks][M][nb]
  cd* d_pN = nullptr;       // [M][nb]
  int* d_noff = nullptr;    // [M+1] CSR offsets
  int* d_nlist = nullptr;   // [n_near] source of each near pair
  int* d_ntgt = nullptr;    // [n_near] target of each near pair
  cd* d_npart = nullptr;    // [n_near][nb] per-pair contributions
  int64_t n_near = 0;
  // resident translation table (FP64 apply only; see table_set)
  uint64_t gen = 0;          // bumped whenever device buffers are freed or replaced (a
                             // batch built on this context checks it before solving)
  bool want_table = false;
  // fast (cell) translation: grid, cell order, binned inclusions, generator table,
  // cell multipoles and locals (fmm.hip)
  bool fmm_on = false;
  int fmm_nx = 0, fmm_ny = 0, fmm_p = 0, fmm_ngroups = 0;
  double fmm_sx = 0, fmm_sy = 0, fmm_x0 = 0, fmm_y0 = 0;
  int* d_fmm_start = nullptr;   // [ncell + 1] CSR offsets into d_fmm_order
  int* d_fmm_order = nullptr;   // [M] inclusions by cell
  int2* d_fmm_groups = nullptr; // [ngroups] (cell, offset) of each 64-target group
  cd* d_fmm_gen = nullptr;      // [(2nx-1)(2ny-1)][4p+1] far generators by cell offset
  cd* d_fmm_M = nullptr;        // [ncell][2p+1]
  cd* d_fmm_L = nullptr;        // [4 source shares][ncell][2p+1] partial locals
  cd* d_table = nullptr;    // [M][4P+1][Mpad]
  int table_mpad = 0;
  int table_lanes = 1;      // lanes per target in the table kernel (1 or 2)
  // non-circular inclusions: host shapes [M][4] = (a1, a2, a3, rot), boundary nodes
  // of each one's integral equation, the resident scattering-matrix blocks
  // [M][2P+1][2P+1] (row = outgoing order) and the apply's S w scratch vector
  std::vector<double> hshape;
  int shape_nodes = 0;
  cd* d_sblk = nullptr;
  cd* d_wS = nullptr;      // [n_beta]
  // resident FP32 table of the well-separated pairs (mixed-precision apply only)
  bool want_table32 = false;
  cf* d_table32 = nullptr;  // [M][4P+1][Mpad], near pairs zero
  int table32_mpad = 0;
  // GMRES workspace
  int krylov_restart = 0;
  cd* d_V = nullptr;        // [restart+1][n_beta]
  cd* d_H = nullptr;        // [restart+1][restart] (column j contiguous: H[j*(restart+1)+i])
  cd* d_y = nullptr;
  double* d_scal = nullptr; // scratch scalars
  cd* d_dotpart = nullptr;  // [restart+1][n_dot_blocks]
  int n_dot_blocks = 0;
  hipEvent_t ev_res[2] = {nullptr, nullptr};
  double* h_pinned = nullptr;
  cd* h_H = nullptr;        // pinned host mirror of H and the least-squares solution
  cd* h_H_dev = nullptr;    // the same memory's device address (kernels write H columns)
  cd* d_wtmp = nullptr;     // output of every apply in the solver (a slot of d_V)
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};  // captured applies: K, mixed K
  // kernel timing (HIP events around every translation-kernel launch)
  bool prof = false;
  std::vector<hipEvent_t> prof_ev;  // pairs: start, stop
  size_t prof_used = 0;             // events in use (even)
  double prof_ms = 0.0;             // accumulated from drained pairs
  int64_t prof_count = 0;
};

// status helpers ---------------------------------------------------------------
grt_status set_err(grt_ctx* c, grt_status s, const std::string& msg);
#define GRT_HIP(ctx, call)                                                           \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return set_err(ctx, GRT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// setup (setup.hip)
grt_status setup_build(grt_ctx* c);
grt_status setup_translation(grt_ctx* c);   // translation-only build (no layers)
void launch_gemv_rows(hipStream_t s, const cd* W, const cd* x, cd* y, int rows, int cols);
// W[i][k] = E[i0 + i] conj(V^H[k][i0 + i]) for i < rows, k < rank: rows of E V
void launch_build_Wv(hipStream_t s, const grt_ctx* c, int i0, int rows, cd* W);

// apply (apply.hip)
bool supported_P(int P);
// y = K x (then y *= oscale elementwise when oscale is given)
grt_status apply_K(grt_ctx* c, const cd* x, cd* y, const double* oscale = nullptr);
grt_status apply_K_mixed(grt_ctx* c, const cd* x, cd* y, const double* oscale = nullptr);
grt_status apply_T_only(grt_ctx* c, const cd* x, cd* y);
// fast cell translation (fmm.hip): set up for the context's inclusions (p_cell 0:
// automatic; per_cell 0: 40), apply into the partials d_pT[0 .. fmm_partials()), release
grt_status fmm_setup(grt_ctx* c, int p_cell, int per_cell);
grt_status fmm_apply(grt_ctx* c, const cd* x, hipStream_t s);
void fmm_release(grt_ctx* c);
int fmm_partials();
grt_status apply_lowrank_only(grt_ctx* c, const cd* x, cd* y);
grt_status rhs_b(grt_ctx* c, cd* b);
grt_status incident_alpha(grt_ctx* c, cd* out);
grt_status bragg_alpha(grt_ctx* c, const cd* beta, cd* out_cd /* device [2 Nrb] */);
// every entry of alpha = A^+ (f - C beta), unscaled (device [n_alpha]); W: device
// scratch of n_alpha * rank entries
grt_status alpha_full(grt_ctx* c, const cd* beta, cd* out, cd* W);
grt_status apply_alloc(grt_ctx* c);
grt_status table_set(grt_ctx* c, bool on);
grt_status table32_set(grt_ctx* c, bool on);
size_t table32_bytes(const grt_ctx* c);
grt_status autotune_m2l(grt_ctx* c, int cap, int* n_out, int* chunks_out, int* splits_out,
                        double* ms_out);
grt_status autotune_coupling(grt_ctx* c);
constexpr int M2L_TUNE_MAX_WAVES = 16384;
size_t table_bytes(const grt_ctx* c);

// non-circular inclusions (inclusion.hip)
bool has_shapes(const grt_ctx* c);
grt_status build_scattering_blocks(grt_ctx* c);
// y = x - S w (mode 0) or y = S w (mode 1), S the resident blocks; then y *= oscale
void launch_sblock_apply(grt_ctx* c, const cd* x, const cd* w, cd* y, int mode,
                         const double* oscale, hipStream_t s);

// block translation of several right-hand sides on FP32 matrix cores (block.hip)
int block_nbk(int P);
grt_status block_prepare(grt_ctx* c, int R, const cd* alphas_host);
grt_status block_product(grt_ctx* c, const cd* x, int64_t ldx, const double* dn, int R,
                         hipStream_t s);
void block_combine(grt_ctx* c, const cd* x, const cd* w, int R, cd* y, hipStream_t s);
void block_unpack(grt_ctx* c, int R, cd* y, hipStream_t s);
// batch.hip: make the batch's mixed apply use the block translation of `owner` (all
// instances: one geometry, the owner's angles in order)
grt_status batch_set_block(grt_batch* b, grt_ctx* owner);
// grt_batch_create without its refusal of contexts that hold several angles
grt_status batch_create_internal(grt_batch** out, int64_t n, grt_ctx* const* ctxs,
                                 void* hip_stream);

// krylov (krylov.hip)
void graph_reset(grt_ctx* c);   // drop captured applies (their configuration changed)
grt_status gmres_solve(grt_ctx* c, const grt_solve_opts* o, cd* x, grt_solve_stats* st);
