// ibm_internal.h -- device-side types and helpers shared by the HIP kernels of the
// IBM-HT library (grid stencils, pressure CG, marker operations) and its host code.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace ibmk {

constexpr int BC_PERIODIC = 0, BC_INFLOW = 1, BC_OUTFLOW = 2, BC_SLIP = 3, BC_SUP_IN = 4,
              BC_SUP_OUT = 5;
constexpr int CONV_VANLEER = 0, CONV_LINEAR = 1;
constexpr int MU_SUTHERLAND = 0, MU_CONSTANT = 1;
// kinds of cell variables, selecting the ghost rule of a boundary side
constexpr int V_RHO = 0, V_U0 = 1, V_TH = 4, V_P = 5, V_PHOM = 7;

constexpr int kTile = 256;         // cells per tile = threads per tile group
#ifndef IBM_BLOCK_THREADS
#define IBM_BLOCK_THREADS 512
#endif
#ifndef IBM_MAX_BLOCKS
#define IBM_MAX_BLOCKS 512
#endif
// Cell kernels: blocks of kBlockThreads threads (kBlockThreads / kTile tile groups),
// at most kMaxBlocks of them (two per CU on 256 CUs). Few large blocks keep the
// per-block partial sums that every block of the next kernel adds up few; of the
// shapes measured on the 1024^2 cylinder (256 to 1024 threads, 256 to 1024 blocks)
// 512 x 512 gave the fastest CG iteration (21.5 against 22.5 us at 1024 x 256).
constexpr int kBlockThreads = IBM_BLOCK_THREADS;
constexpr int kMaxBlocks = IBM_MAX_BLOCKS;
constexpr int kThreads = 256;      // threads per block of the predictor kernels
constexpr int kRedThreads = 1024;  // threads of the single-block marker kernels
constexpr int kPairBits = 20;      // (cell << 20) | pair id in the sorted pair keys
constexpr int kMaxNbr = 192;       // neighbours per marker row of the Gram matrix
constexpr int kFusedMarkers = 1024; // marker capacity up to which one block does a step's marker work
constexpr int kFaceOut = 18;       // per-face values of the reverse predictor (4 dim + 2,
                                   // 5 dim + 3 with van Leer convection)

// Grid, physics and time-step constants, passed by value to every grid kernel.
struct GridK {
  int dim;
  int n[3];
  int fn[3][3];       // dims of the face array of each direction
  int64_t N;
  int64_t NF[3];
  double lo[3], h[3], ih[3];
  int bc[3][2];
  int conv, visc;
  int implicit_diff;  // 1: compact viscous and conductive fluxes by backward Euler
  int no_heat;        // 1: markers without heat exchange (energy source zero)
  double dt, R, cv, inv_cv, cp, gm1, mu_inf, S, Pr, p_inf, dV;
  double cp_Pr;       // c_p / Pr: lambda = cp_Pr mu
  double U_inf[3];
  int tiles[3];       // tiles per direction of the cell kernels
  int64_t ntiles;     // tiles in all
  int64_t nblocks;    // blocks of a cell kernel: a multiple of 8, at most kMaxBlocks
};

template <typename S>
struct StateV {
  S *rho;
  S *mom[3];
  S *E;
  S *F[3];
};

// Scalars of one pressure solve, in device memory. rr[i & 1] holds r.r after
// i CG updates and alpha[i & 1] the step length of update i (two slots, so that
// the kernel of iteration i reads the values of iteration i-1 while writing its
// own).
struct CgScal {
  double bb, tol2, rr[2], res, alpha[2];
  int iters, done, maxit, step_tag;
  // FP32 form (iterative refinement). Values the kernel of iteration `it` reads
  // sit in slot it & 1; block 0 of that kernel writes slot (it + 1) & 1.
  double rr_in0[2];  // r.r at the start of the current inner solve
  int inner_it[2];   // inner iterations since the last refinement
  int outer[2];      // stage of the FP32 form's iteration kernel (MS_*)
  int xpar[2];       // which x buffer holds the current solution
  int xfinal;        // x buffer of the finished solve (read by the correction)
};

// Implicit diffusion: dim + 1 systems (velocity components, temperature) solved
// side by side. Their scalars, in device memory; rr/alpha slot it & 1 as in CgScal.
constexpr int kDiffVars = 4;
struct DiffScal {
  double bb[kDiffVars];
  double rr[2][kDiffVars];
  double alpha[2][kDiffVars];
  double tol2;
  int done[kDiffVars];  // 0 iterating, 1 converged, 2 stopped (limit, error flag, NaN)
  int maxit, iters, step_tag;
};
// per-variable regions of the diffusion partial sums: b.b, r.r (2), w.r (2)
enum { DP_BB = 0, DP_G = 1, DP_D = 3, DP_REGIONS = 5 };

// Progress word the CG posts to host memory after each convergence test:
// bits 32..63 step tag, 8..31 iteration, 4..7 error flags seen, 0..3 done state.
__host__ __device__ inline uint64_t pack_progress(int tag, int it, int err, int done) {
  return ((uint64_t)(uint32_t)tag << 32) | ((uint64_t)(it & 0xFFFFFF) << 8) |
         ((uint64_t)(err & 0xF) << 4) | (uint64_t)(done & 0xF);
}

// Device flags (int): [0] non-finite result, [1] marker support out of the box,
// [2] quadrature solve failed, [3] Gram row overflow, [4] 1 + tag of the first
// step whose correction failed.
enum { FLAG_NONFINITE = 0, FLAG_SUPPORT = 1, FLAG_EPS = 2, FLAG_GRAM = 3, FLAG_BAD_STEP = 4 };

// Per-block partial sums of the cell kernels, each region kMaxBlocks long. The
// single-reduction CG of iteration i reads (r.r, w.r) from regions PART_G + (i & 1),
// PART_D + (i & 1) and writes the other pair.
enum {
  PART_SA = 0,  // adjoint solve's start: rhs.(A lambda) and (A lambda).(A lambda)
  PART_AA = 1,
  PART_BB = 2,
  PART_MASS = 3,
  PART_G = 4,
  PART_D = 6,
  PART_O = 8,  // FP32 form: FP64 r.r of the outer residual (two regions)
  PART_REGIONS = 10
};

__device__ __forceinline__ int64_t cidx(const GridK &g, int i, int j, int k) {
  return i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * k);
}
__device__ __forceinline__ int64_t fidx(const GridK &g, int d, int i, int j, int k) {
  return i + (int64_t)g.fn[d][0] * (j + (int64_t)g.fn[d][1] * k);
}

// Tiles of kTile cells: 64 x 4 (x fastest) in 2D; 64 x 4 x 1 in 3D, ordered z
// fastest, so that a block's range of tiles walks up a column of planes and the
// planes below and above a tile are still in L2 when it needs them. A cell kernel
// runs gridDim.x (a multiple of 8) blocks; block b runs on XCD b % 8 (blocks are
// dealt round-robin to the 8 XCDs), so it is given the logical rank
// (b % 8) * (gridDim / 8) + b / 8 and a contiguous range of tiles: the blocks of
// one XCD sweep neighbouring tiles and share their halos in its L2.
__device__ __forceinline__ void block_tiles(const GridK &g, int64_t &t0, int64_t &t1) {
  const int64_t nb = gridDim.x;
  const int64_t b = blockIdx.x;
  const int64_t rank = (b & 7) * (nb >> 3) + (b >> 3);
  const int64_t per = (g.ntiles + nb - 1) / nb;
  t0 = rank * per;
  t1 = t0 + per < g.ntiles ? t0 + per : g.ntiles;
}

// The tile group of this thread within its block, and the number of groups: a
// block's range of tiles is shared out round-robin over its groups.
__device__ __forceinline__ int64_t tile_group() { return threadIdx.x / kTile; }
__device__ __forceinline__ int64_t tile_groups() { return blockDim.x / kTile; }

// Cell coordinates of this thread in tile t; false outside the grid.
template <int DIM>
__device__ __forceinline__ bool cell_in_tile(const GridK &g, int64_t t, int &i, int &j, int &k) {
  const int lx = threadIdx.x & 63, ly = (threadIdx.x % kTile) >> 6;
  // a grid has at most 2^31 cells (the host checks it), so tile numbers fit 32 bits
  const uint32_t tt = (uint32_t)t;
  const uint32_t n0 = (uint32_t)g.tiles[0], n2 = (uint32_t)g.tiles[2];
  if (DIM == 2) {
    const int tx = (int)(tt % n0);
    const int ty = (int)(tt / n0);
    i = tx * 64 + lx;
    j = ty * 4 + ly;
    k = 0;
  } else {
    k = (int)(tt % n2);
    const auto r = tt / n2;
    const int tx = (int)(r % n0);
    const int ty = (int)(r / n0);
    i = tx * 64 + lx;
    j = ty * 4 + ly;
  }
  return i < g.n[0] && j < g.n[1] && k < g.n[2];
}

// An index up to two layers outside the box, resolved to an interior cell and the
// boundary sides crossed (-1: none, 0: low side, 1: high side) per direction.
struct Resolved {
  int64_t c;
  int side[3];
};

template <int DIM>
__device__ __forceinline__ Resolved resolve(const GridK &g, int i, int j, int k) {
  int ix[3] = {i, j, k};
  Resolved r;
  r.side[0] = r.side[1] = r.side[2] = -1;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    int v = ix[d], n = g.n[d];
    if (v < 0 || v >= n) {
      if (g.bc[d][0] == BC_PERIODIC) {
        v = v < 0 ? v + n : v - n;
      } else {
        r.side[d] = v < 0 ? 0 : 1;
        v = v < 0 ? -v - 1 : 2 * n - 1 - v;
      }
      ix[d] = v;
    }
  }
  r.c = ix[0] + (int64_t)g.n[0] * (ix[1] + (int64_t)g.n[1] * ix[2]);
  return r;
}

// Ghost value of one boundary side: sigma * (mirror value) + c.
template <typename T>
__device__ __forceinline__ T side_rule(const GridK &g, int bc, int var, int d, T v) {
  if (bc == BC_INFLOW) {
    if (var >= V_U0 && var < V_U0 + 3) return T(2.0 * g.U_inf[var - V_U0]) - v;
    if (var == V_TH) return T(2.0) - v;
    return v;
  }
  if (bc == BC_OUTFLOW) {
    if (var == V_P) return T(2.0 * g.p_inf) - v;
    if (var == V_PHOM) return -v;
    return v;
  }
  if (bc == BC_SLIP) {
    if (var == V_U0 + d) return -v;
    return v;
  }
  if (bc == BC_SUP_IN) {  // the free stream on the face
    if (var >= V_U0 && var < V_U0 + 3) return T(2.0 * g.U_inf[var - V_U0]) - v;
    if (var == V_TH || var == V_RHO) return T(2.0) - v;
    if (var == V_P) return T(2.0 * g.p_inf) - v;
    if (var == V_PHOM) return -v;
    return v;
  }
  return v;  // BC_SUP_OUT: every variable extrapolated
}

// Applies the rules of all sides crossed, the last direction first (x outermost).
template <int DIM, typename T>
__device__ __forceinline__ T ghosted(const GridK &g, const Resolved &r, int var, T v) {
#pragma unroll
  for (int d = DIM - 1; d >= 0; --d)
    if (r.side[d] >= 0) v = side_rule(g, g.bc[d][r.side[d]], var, d, v);
  return v;
}

template <int DIM, typename T>
__device__ __forceinline__ bool any_side(const Resolved &r) {
  bool a = false;
#pragma unroll
  for (int d = 0; d < DIM; ++d) a = a || (r.side[d] >= 0);
  return a;
}

// ------------------------------------------- Appendix A, step 3 (operator)
// Homogeneous pressure operator at one cell: psi v - dt^2 div(grad_f v), zero
// normal gradient at inflow and slip faces, v = 0 beyond outflow faces.
// The homogeneous Laplacian of v at (i, j, k), vc = v there.
template <int DIM, typename VF>
__device__ __forceinline__ double helm_lap(const GridK &g, VF v, int i, int j, int k, double vc) {
  double lap = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double ih = g.ih[d];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      int ix[3] = {i, j, k};
      ix[d] += side ? 1 : -1;
      const int n = g.n[d];
      double gf;
      if (ix[d] >= 0 && ix[d] < n) {
        gf = (v(cidx(g, ix[0], ix[1], ix[2])) - vc) * ih;
      } else if (g.bc[d][0] == BC_PERIODIC) {
        ix[d] = ix[d] < 0 ? ix[d] + n : ix[d] - n;
        gf = (v(cidx(g, ix[0], ix[1], ix[2])) - vc) * ih;
      } else {
        gf = (g.bc[d][side] == BC_OUTFLOW) ? (-2.0 * vc) * ih : 0.0;
      }
      lap += gf * ih;
    }
  }
  return lap;
}

template <int DIM, typename S, typename VF>
__device__ __forceinline__ double helm_at(const GridK &g, const S *psi, VF v, int i, int j, int k,
                                          int64_t c, double vc) {
  return double(psi[c]) * vc - g.dt * g.dt * helm_lap<DIM>(g, v, i, j, k, vc);
}

// -------------------------------------------------------------- reductions
// Block sum of a double over a block of blockDim.x threads (multiple of 64);
// fixed shuffle/LDS order, so the result is deterministic. Valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds /* >= 16 */) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    int nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < nw; ++q) s += lds[q];
  }
  return s;
}

// Block sums of NV doubles at once.
template <int NV>
__device__ __forceinline__ void block_sum_n(double *v, double *lds /* >= 16*NV */) {
#pragma unroll
  for (int q = 0; q < NV; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
  }
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) lds[q * 16 + w] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int p = 0; p < nw; ++p) s += lds[q * 16 + p];
      v[q] = s;
    }
  }
}

// Sum of partials[0..n), written by an earlier kernel, in a fixed order; every
// thread of the block gets the result. Blocks of a consumer kernel each form the
// same sum, so no block of a kernel ever waits for another.
__device__ __forceinline__ double sum_partials(const double *partials, int n, double *lds) {
  __shared__ double bcast;
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += partials[i];
  double s = block_sum(v, lds);
  if (threadIdx.x == 0) bcast = s;
  __syncthreads();
  s = bcast;
  __syncthreads();
  return s;
}

// Sums of two partial arrays at once (same order as sum_partials); every thread of
// the block gets both.
__device__ __forceinline__ void sum_partials2(const double *pa, const double *pb, int n,
                                              double *lds, double *out) {
  __shared__ double bc[2];
  double v[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    v[0] += pa[i];
    v[1] += pb[i];
  }
  block_sum_n<2>(v, lds);
  if (threadIdx.x == 0) {
    bc[0] = v[0];
    bc[1] = v[1];
  }
  __syncthreads();
  out[0] = bc[0];
  out[1] = bc[1];
  __syncthreads();
}

}  // namespace ibmk
