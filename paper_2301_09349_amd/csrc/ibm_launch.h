// ibm_launch.h -- device buffers of a context and the host-side launchers of the
// grid and marker kernels (defined in ibm_grid.hip and ibm_markers.hip).
#pragma once

#include "ibm_internal.h"

namespace ibmk {

// The buffers a marker set-up writes: the markers in use at one time and the
// set-up's own work arrays. A context holds two such sets (one in Bufs, the other in
// Bufs::alt), so that a moving body's set-up for a later step can run while a step
// reads the markers of its own.
struct MarkerSet {
  double *cXc, *cUdc;
  int64_t *ckey;
  double *cd2;
  int *ckeep;
  int *mcount, *ids;
  double *X, *Ud, *Tw, *dA, *eps;
  int *sidx;
  double *sw1;
  int64_t *pcell;
  double *pw;
  uint64_t *keys, *keys_in;
  int *seg, *ell_col;
  double *ell_val;
  int *ell_cnt;
  double *ev[4];
};

// Device buffers carved from the caller's workspace.
struct Bufs {
  // conserved state, two copies (ping-pong): rho, mom[3], E, F[3]
  void *rho[2], *mom[2][3], *E[2], *F[2][3];
  // predictor output; mom_s and E_s become mom** and E** after spreading
  void *rho_s, *mom_s[3], *E_s;
  void *E_hist;   // E^{n-2} for the extrapolated CG start (written by the predictor)
  void *E_hist2;  // E^{n-3}, likewise
  // pressure equation: m^ = mom** + dt G p^n, its face flux, psi
  void *mhat[3], *Fhat[3], *psi;
  // pressure CG (FP64, single-reduction form): x and p in place; r, w = A r and
  // s = A p ping-pong between iterations (their neighbour values are read)
  double *b, *x, *pv, *rv[2], *wv[2], *sv[2];
  // FP32 form: second FP64 solution buffer and the FP32 inner-CG vectors (r, w, s
  // ping-pong; p and the correction d in place)
  double *x2;
  float *rv32[2], *wv32[2], *sv32[2], *pv32, *d32;
  double *partials;  // per-block partial sums, 4 per block
  CgScal *cg;
  double *scal;      // [0] mass
  int *flags;        // FLAG_* (ibm_internal.h)
  uint64_t *progress;  // host memory (pinned, coherent): CG progress word

  // candidate markers
  double *cX0, *cUd0, *cTw, *cdA, *ceps;  // ceps: last eps per candidate (warm start)
  double *cXc, *cUdc;                     // candidate positions, velocities at time t
  int64_t *ckey;
  double *cd2;
  int *ckeep;
  // markers in use (indexed 0..n_used-1)
  int *mcount;  // [0] n_used, [1] n_segments, [2] eps CG iterations
  int *ids;
  double *X, *Ud, *Tw, *dA, *eps;
  int *sidx;      // [ns][3][3] cell index per direction and slot
  double *sw1;    // [ns][3][3] 1D kernel weights
  int64_t *pcell; // [ns][27] support cell of each slot
  double *pw;     // [ns][27] support weight of each slot
  uint64_t *keys; // sorted (cell << 20 | pair id), padded to a power of two
  uint64_t *keys_in;  // the same keys before the sort
  int *seg;       // segment starts, [n_segments + 1]
  int *ell_col;   // [ns][kMaxNbr]
  double *ell_val;
  int *ell_cnt;
  double *ev[4];  // eps CG vectors
  double *mk;     // [ns][2 dim + 3]: rho_L, M, E_L, F, Q
  double *mforce; // [ns][3]
  double *mheat;  // [ns]
  double *totals; // [4]

  // tape (IBM_RECORD): per recorded step the state it started from, in the
  // context's storage type (rho, mom[dim], E [N]; F [sum NF]), then its FP64 pressure
  // solution x [N] at a 256-byte aligned offset
  char *tape;
  size_t tape_stride;  // bytes per recorded step
  size_t tape_xoff;    // byte offset of x in a record
  // adjoint work buffers (FP64)
  double *pprim;        // padded primitives [(dim+4)][Npad]: rho, u[dim], theta, mu, p
  double *pbar;         // padded primitive cotangents [(dim+3)][Npad]: rho, u[dim], theta, p
  double *fo;           // per-face reverse outputs [kFaceOut][sum NF]
  double *co;           // per-cell reverse outputs [(dim^2 + dim + 2)][N]
  double *rs_bar, *ms_bar[3], *Es_bar;  // cotangents of rho*, m* (m**), E* (E**)
  double *fbar;         // [sum NF] cotangent of the corrected face flux
  double *tbar;         // [N] cotangent of theta**
  double *lam, *rhs;    // [N] adjoint pressure and its right-hand side
  double *mkbar;        // [nc][2 dim + 3] marker cotangents
  // marker-position gradient: kernel-weight cotangents per pair [nc][27] and
  // quadrature-weight cotangents [nc] accumulated over adjoint steps; predictor
  // fields at the pairs [nc][27][dim + 2]; per-pair cell sums [nc][27][2]; the
  // adjoint quadrature solve [nc]
  double *wbar, *epsbar, *pfld, *gsum, *lam_g;
  // implicit diffusion (FP64): face viscosity per direction [NF[d]]; per variable a
  // ring of three solutions (this step's and the two before, for the start), the
  // CG vectors r, w, s (ping-pong) and p; partial sums and scalars
  double *muf[3];
  double *dring[3][kDiffVars];
  double *dr[2][kDiffVars], *dw[2][kDiffVars], *ds[2][kDiffVars], *dp[kDiffVars];
  double *dpart;
  DiffScal *dsc;
  // density-based step: u**[3], theta** of the intermediate state, state type [N]
  // each
  void *dprim1[5];
  // the second marker set (the first is in the fields above)
  MarkerSet alt;
};

// The marker set held in the fields of B, and B with the fields set to m.
MarkerSet marker_set_of(const Bufs &B);
void put_marker_set(Bufs &B, const MarkerSet &m);

// Kernel view of the diffusion systems' buffers.
struct DiffSys {
  const double *mf[3];
  double *x[kDiffVars];
  const double *y1[kDiffVars], *y2[kDiffVars];
  double *p[kDiffVars];
  double *r[2][kDiffVars], *w[2][kDiffVars], *s[2][kDiffVars];
  double *part;
  DiffScal *sc;
  double kap_th;  // gamma / Pr
};

struct Launch {
  GridK g;
  int prec;      // 0: FP64, 1: FP32
  int pred_lds;  // 1: LDS-tiled predictor, 0: per-cell predictor
  int refine32;  // FP32 form: 1 pressure by iterative refinement with an FP32 inner CG,
                 // 0 the FP64 CG on FP32 psi
  int cg_col;     // 3D: 1 the CG iteration by z-columns (k_cg_col), 0 by tiles (k_cg_iter)
  int nc_cap;     // candidate capacity
  int npairs_pad; // power of two >= nc_cap * nslot
  hipStream_t st;
};

// Up to kCopyParts device byte ranges (each size a multiple of 4 bytes) to copy in one
// launch.
constexpr int kCopyParts = 8;
struct CopyParts {
  const void *src[kCopyParts];
  void *dst[kCopyParts];
  size_t bytes[kCopyParts];
  int n = 0;
  void add(void *d, const void *s, size_t b) {
    dst[n] = d;
    src[n] = s;
    bytes[n] = b;
    ++n;
  }
};

// grid kernels (ibm_grid.hip)
void run_fill(const Launch &L, double *p, int64_t n, double v);
void run_copy_parts(const Launch &L, const CopyParts &cp);
void run_uniform_state(const Launch &L, const Bufs &B, int cur);
void run_init_primitive(const Launch &L, const Bufs &B, int cur, const void *rho, const void *u,
                        const void *theta);
void run_flux_from_momentum(const Launch &L, const Bufs &B, int cur);
// predictor, also writing m^ (= m* + dt G_c p^n), psi and the CG start x for the
// set-up. Fluxes and cell terms from state slot `cur`, the time derivative's old
// values from slot `base` (the same slot except in an outer pass). order -1: x
// is left as it is (an outer pass); 0: x = p^n; 1: the other state slot holds the
// previous state and x = 2 p^n - p^{n-1}; 2: E_hist also holds E^{n-2} and x =
// 3 p^n - 3 p^{n-1} + p^{n-2}; 3: E_hist2 also holds E^{n-3} and x = 4 p^n -
// 6 p^{n-1} + 4 p^{n-2} - p^{n-3}. keep >= 1 (order >= 1): E^{n-1} is copied to
// E_hist for the next step; keep >= 2 (order >= 2): E^{n-2} to E_hist2 as well.
void run_predictor(const Launch &L, const Bufs &B, int base, int cur, int order, int keep);
size_t predictor_lds_bytes(int dim, int prec);
void enable_predictor_lds(int dim, int prec);
// set-up of the pressure equation from the predictor's m^, psi, x (with the spread
// forcing added), ending with the start of its CG (r0, w0 = A r0)
void run_setup(const Launch &L, const Bufs &B, int cur, int tag);
// start of the FP64 CG from r0 = rv[0]: w0 = A r0 and the first dot products
// (nothing in the FP32 form, whose first iteration kernel starts its solve)
void run_cg_start(const Launch &L, const Bufs &B);
// the FP64 CG's start and iteration whatever the context's precision (psi in the
// context's storage type): the forward FP64 solve and every adjoint solve
void run_cg64_start(const Launch &L, const Bufs &B);
void run_cg64_iteration(const Launch &L, const Bufs &B, int it);
void run_cg_iteration(const Launch &L, const Bufs &B, int it);
// kernels of one CG iteration: 1 in FP64, 2 in the FP32 form (part 0: a, 1: b)
int cg_parts(const Launch &L);
void run_cg_half(const Launch &L, const Bufs &B, int it, int part);
void run_correct(const Launch &L, const Bufs &B, int cur, int tag);
// implicit diffusion after the predictor: the face viscosities of state `cur`;
// the start of the dim + 1 solves into solution ring slot `ring` (order 0: from
// the state in slot `cur`; 1: extrapolated from the two previous ring slots; 2:
// from the solution in slot `ring`; progress posted under `tag`), their
// iterations, and the solutions into m*, m^, E*, psi
void run_diff_coef(const Launch &L, const Bufs &B, int cur);
void run_diff_start(const Launch &L, const Bufs &B, int cur, int ring, int order, int tag);
void run_diff_iteration(const Launch &L, const Bufs &B, int ring, int it);
void run_diff_finish(const Launch &L, const Bufs &B, int ring);
void run_mass(const Launch &L, const Bufs &B);
// density-based step (App. B): the central-upwind inviscid part of state `cur` (rho^{n+1} into rho_s, (rho u)** into mhat, u** and theta** into
// dprim1, the mass flux into the other slot's faces), then the explicit viscous
// part into mom_s, E_s; after the marker sources, the finish writes the other
// state slot
void run_density_predictor(const Launch &L, const Bufs &B, int cur);
// lets the inviscid kernel take its LDS beyond 64 KB (once per process and form)
void enable_density_lds(int dim, int prec);
void run_density_finish(const Launch &L, const Bufs &B, int cur, int tag);
int64_t cell_blocks(const GridK &g);

// adjoint kernels (ibm_adjoint.hip); FP64 contexts only. `st` is the state the step
// started from (tape copy loaded into a state slot), `sb_in`/`sb_out` the state
// cotangents after/before the step (ibm_set_state layout).
int64_t padded_cells(const GridK &g);
void run_adj_correction(const Launch &L, const Bufs &B, int slot, const double *sb_in,
                        double *sb_out);
// the adjoint pressure solve then runs run_cg_iteration with x -> lam
void run_adj_cg_init(const Launch &L, const Bufs &B, int tag);
void run_adj_setup(const Launch &L, const Bufs &B, int slot, const double *sb_in, double *sb_out);
// out_bar: host double[4], the cotangents of the step's Fx, Fy, Fz, H; shape: the
// kernel-weight cotangents of the marker-position gradient are accumulated too
void run_adj_markers(const Launch &L, const Bufs &B, const double *out_bar, double *Tw_bar,
                     bool shape);
void run_pair_fields(const Launch &L, const Bufs &B);
bool shape_supported(int nc);
void run_shape_clear(const Launch &L, const Bufs &B, int nc);
void run_shape_gradient(const Launch &L, const Bufs &B, int nc, double *X_bar);
void run_adj_predictor(const Launch &L, const Bufs &B, int slot, double *sb_out);
// copy of the finished pressure solution (either x buffer of the FP32 form)
void run_copy_solution(const Launch &L, const Bufs &B, double *dst);

// marker kernels (ibm_markers.hip)
void run_place_markers(const Launch &L, const Bufs &B, int nc, double off, double vel, int axis,
                       int dedupe);
// supports, sort, segments, Gram rows and the quadrature solve A eps = 1 from eps as
// gathered by run_place_markers (the candidates' saved values); save_eps: the solution
// is saved per candidate as the start of later solves
void run_build_markers(const Launch &L, const Bufs &B, int nc, bool save_eps);
// placement, selection and run_build_markers of the markers at a time: one block and
// a one-wave solve for a small body (up to 256 candidates and 4096 pairs), else
// run_place_markers and run_build_markers
void run_rebuild_markers(const Launch &L, const Bufs &B, int nc, double off, double vel, int axis,
                         int dedupe, bool save_eps);
void run_interp_force(const Launch &L, const Bufs &B, double *hist_row);
void run_spread(const Launch &L, const Bufs &B);
// local heat flux H_k / dA'_k of the markers in use into q [n_used] (device);
// status[0] (device) = 1 when the markers in use carry no surface
void run_heat_flux(const Launch &L, const Bufs &B, int nc, double *q, int *status);
// interpolation, forcing, totals and spread of one step: one single-block kernel
// when the candidate capacity is at most kFusedMarkers, else the kernels above
void run_markers_step(const Launch &L, const Bufs &B, double *hist_row);

}  // namespace ibmk
