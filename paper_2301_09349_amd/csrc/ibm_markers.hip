// ibm_markers.hip -- Lagrangian-marker kernels of the IBM-HT step on gfx950, all in
// FP64: marker placement and the check routine (Sec. 3.1, Sec. 5), supports and
// kernel weights (Sec. 2.2, Eq. (6)), a deterministic sort of the (cell, marker)
// pairs, the Lagrangian quadrature A eps = 1 (Eqs. (8)-(9)) by CG, interpolation
// and forcing (Eqs. (5), (10), (17)) and the spread (Eq. (7)) as a segmented
// reduction in marker order (no floating-point atomics).
//
// Marker counts are read on the device (mcount), so a motion update needs no
// host round trip: the kernels are launched for the candidate capacity and
// threads past the live count return.
#include "ibm_launch.h"

namespace ibmk {

// Pinelli et al. 3-point kernel (Sec. 2.2, Eq. (6)); r in mesh widths.
__device__ __forceinline__ double kernel_phi(double r) {
#pragma clang fp contract(off)
  r = fabs(r);
  if (r <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;
  if (r <= 1.5) return (5.0 - 3.0 * r - sqrt(1.0 - 3.0 * (1.0 - r) * (1.0 - r))) / 6.0;
  return 0.0;
}

// Exclusive block scan of ints (blockDim.x a multiple of 64, <= 1024).
__device__ __forceinline__ int block_scan_excl(int v, int *lds, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  if (w == 0) {
    int t = (lane < nw) ? lds[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int y = __shfl_up(t, o, 64);
      if (lane >= o) t += y;
    }
    if (lane < nw) lds[lane] = t;
  }
  __syncthreads();
  int off = (w > 0 ? lds[w - 1] : 0) + x - v;
  *total = lds[nw - 1];
  __syncthreads();
  return off;
}

// ------------------------------------------------ placement, check routine
// Candidate positions at the current time (Sec. 5, Eq. (19): a common offset
// along `axis`); the containing cell and the squared distance to its centre.
__device__ __forceinline__ void place_one(const GridK &g, int k, const double *X0,
                                          const double *U0, double *X, double *U, double off,
                                          double vel, int axis, int64_t &key, double &d2,
                                          double *xk) {
#pragma clang fp contract(off)
  int64_t b[3] = {0, 0, 0};
  double dd = 0.0;
  for (int a = 0; a < 3; ++a) {
    double x = X0[3 * k + a], u = U0[3 * k + a];
    if (a == axis) {
      x += off;
      u += vel;
    }
    X[3 * k + a] = x;
    U[3 * k + a] = u;
    xk[a] = x;
    if (a < g.dim) {
      double xi = (x - g.lo[a]) / g.h[a];
      int64_t bb = (int64_t)floor(xi);
      double dx = x - (g.lo[a] + (double(bb) + 0.5) * g.h[a]);
      dd += dx * dx;
      if (g.bc[a][0] == BC_PERIODIC) bb = ((bb % g.n[a]) + g.n[a]) % g.n[a];
      b[a] = bb;
    }
  }
  key = b[0] + (int64_t)g.n[0] * (b[1] + (int64_t)g.n[1] * b[2]);
  d2 = dd;
}

__global__ void k_place(GridK g, int nc, const double *X0, const double *U0, double *X, double *U,
                        double off, double vel, int axis, int64_t *key, double *d2) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nc) return;
  double xk[3];
  place_one(g, k, X0, U0, X, U, off, vel, axis, key[k], d2[k], xk);
}

// Sec. 3.1 check routine: a candidate is kept when no other candidate in its
// cell is nearer to the centre (ties: the lower id wins). One wave per candidate:
// its lanes test 64 other candidates at a time.
__global__ void k_dedupe(int nc, const int64_t *key, const double *d2, int *keep) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k >= nc) return;  // the whole wave
  const int64_t kk = key[k];
  const double dk = d2[k];
  int ok = 1;
  for (int j0 = 0; j0 < nc && ok; j0 += 64) {
    const int j = j0 + lane;
    const bool beats = j < nc && key[j] == kk && (d2[j] < dk || (d2[j] == dk && j < k));
    if (__ballot(beats) != 0) ok = 0;
  }
  if (lane == 0) keep[k] = ok;
}

__global__ void k_keep_all(int nc, int *keep) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nc) keep[k] = 1;
}

// Gathers the kept candidates, in increasing id, into the markers in use; eps
// starts from the candidate's last value (warm start of the quadrature solve).
__global__ void k_compact(int nc, const int *keep, const double *cX, const double *cU,
                          const double *cTw, const double *cdA, const double *ceps, int *ids,
                          double *X, double *U, double *Tw, double *dA, double *eps, int *mcount) {
  __shared__ int lds[32];
  int base = 0;
  for (int start = 0; start < nc; start += blockDim.x) {
    int k = start + threadIdx.x;
    int v = (k < nc) ? keep[k] : 0;
    int tot;
    int off = block_scan_excl(v, lds, &tot);
    if (v) {
      int m = base + off;
      ids[m] = k;
      for (int a = 0; a < 3; ++a) {
        X[3 * m + a] = cX[3 * k + a];
        U[3 * m + a] = cU[3 * k + a];
      }
      Tw[m] = cTw[k];
      dA[m] = cdA[k];
      eps[m] = ceps[k];
    }
    base += tot;
  }
  if (threadIdx.x == 0) mcount[0] = base;
}

// ------------------------------------------------------------ supports
// Support of marker k: the 3 cells per direction around the cell containing it,
// weight the product of 1D kernel values at r = (x_c - X)/h; pair keys
// (cell << 20 | k * nslot + slot) for the sort.
__device__ __forceinline__ void support_one(const GridK &g, int k, const double *X, int nslot,
                                            int *sidx, double *sw1, int64_t *pcell, double *pw,
                                            uint64_t *keys, int *flags) {
#pragma clang fp contract(off)
  int idx[3][3];
  double w1[3][3];
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 3; ++s) {
      idx[a][s] = 0;
      w1[a][s] = (s == 0) ? 1.0 : 0.0;
    }
  for (int a = 0; a < g.dim; ++a) {
    double xi = (X[3 * k + a] - g.lo[a]) / g.h[a];
    int64_t b = (int64_t)floor(xi);
    for (int s = 0; s < 3; ++s) {
      int64_t ii = b - 1 + s;
      w1[a][s] = kernel_phi((double(ii) + 0.5) - xi);
      if (g.bc[a][0] == BC_PERIODIC) {
        ii = ((ii % g.n[a]) + g.n[a]) % g.n[a];
      } else if (ii < 0 || ii >= g.n[a]) {
        atomicOr(flags + 1, 1);
        ii = ii < 0 ? 0 : g.n[a] - 1;
      }
      idx[a][s] = (int)ii;
    }
  }
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 3; ++s) {
      sidx[9 * k + 3 * a + s] = idx[a][s];
      sw1[9 * k + 3 * a + s] = w1[a][s];
    }
  const int s2n = (g.dim == 3) ? 3 : 1;
  for (int s2 = 0; s2 < s2n; ++s2)
    for (int s1 = 0; s1 < 3; ++s1)
      for (int s0 = 0; s0 < 3; ++s0) {
        int s = s0 + 3 * (s1 + 3 * s2);
        int64_t cell = idx[0][s0] + (int64_t)g.n[0] * (idx[1][s1] + (int64_t)g.n[1] * idx[2][s2]);
        pcell[27 * k + s] = cell;
        pw[27 * k + s] = w1[0][s0] * w1[1][s1] * w1[2][s2];
        keys[(int64_t)nslot * k + s] = ((uint64_t)cell << kPairBits) | (uint64_t)(nslot * k + s);
      }
}

__global__ void k_support(GridK g, const int *mcount, const double *X, int nslot, int *sidx,
                          double *sw1, int64_t *pcell, double *pw, uint64_t *keys, int *flags) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= mcount[0]) return;
  support_one(g, k, X, nslot, sidx, sw1, pcell, pw, keys, flags);
}

// Bitonic sort of the pair keys in one block (npad a power of two), in place in
// global memory after a copy from keys_in (padded with the largest key); the keys
// are unique, so the order is fully determined. Used above kRankKeys keys.
__global__ void k_sort(const uint64_t *keys_in, uint64_t *keys, int npad, const int *mcount,
                       int nslot) {
  const int np = mcount[0] * nslot;
  for (int i = threadIdx.x; i < npad; i += blockDim.x) keys[i] = (i < np) ? keys_in[i] : ~0ull;
  __syncthreads();
  for (unsigned size = 2; size <= (unsigned)npad; size <<= 1) {
    for (unsigned stride = size >> 1; stride > 0; stride >>= 1) {
      for (unsigned t = threadIdx.x; t < (unsigned)npad / 2; t += blockDim.x) {
        unsigned i = 2 * t - (t & (stride - 1));
        unsigned j = i + stride;
        bool asc = (i & size) == 0;
        uint64_t a = keys[i], b = keys[j];
        if ((a > b) == asc) {
          keys[i] = b;
          keys[j] = a;
        }
      }
      __syncthreads();
    }
  }
}

// The same order by rank, for up to kRankKeys keys: every key's place is the
// number of keys below it (the keys are distinct). Each block ranks 256 keys
// against all of them, held in LDS; the grid covers the live keys.
constexpr int kRankKeys = 4096;
__global__ __launch_bounds__(256) void k_rank_sort(const uint64_t *keys_in, uint64_t *keys,
                                                   const int *mcount, int nslot) {
  extern __shared__ uint64_t sk[];
  const int np = mcount[0] * nslot;
  if ((int)blockIdx.x * 256 >= np) return;  // the whole block
  for (int i = threadIdx.x; i < np; i += blockDim.x) sk[i] = keys_in[i];
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const uint64_t v = sk[i];
  int rank = 0;
  for (int j = 0; j < np; ++j) rank += sk[j] < v ? 1 : 0;
  keys[rank] = v;
}

// Segments of equal cell in the sorted pairs: seg[s] = first pair of segment s.
__global__ void k_segments(const uint64_t *keys, int nslot, int *mcount, int *seg) {
  __shared__ int lds[32];
  const int np = mcount[0] * nslot;
  int base = 0;
  for (int start = 0; start < np; start += blockDim.x) {
    int i = start + threadIdx.x;
    int head = 0;
    if (i < np) head = (i == 0) || ((keys[i] >> kPairBits) != (keys[i - 1] >> kPairBits));
    int tot;
    int off = block_scan_excl(head, lds, &tot);
    if (head) seg[base + off] = i;
    base += tot;
  }
  if (threadIdx.x == 0) {
    seg[base] = np;
    mcount[1] = base;
  }
}

// Rows of the Gram matrix A_kl = sum_c w_ck w_cl (Eq. (9)) in ELL form, from the
// tensor-product structure: A_kl = prod_d sum_{s,t: same cell index} phi_ks phi_lt.
// One block per row k: its threads test the markers l in parallel and a block scan
// keeps the nonzeros in increasing l.
constexpr int kGramThreads = 256;
// A_kl from the supports of k (ks, kw) and l (ls, lw): 3 cell indices and 1D weights
// per direction; returns 0 when the supports do not overlap.
__device__ __forceinline__ int gram_entry(const GridK &g, const int *ks, const double *kw,
                                          const int *ls, const double *lw, double &a) {
  a = 1.0;
  for (int d = 0; d < g.dim; ++d) {
    double s = 0.0;
    bool any = false;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q)
        if (ks[3 * d + p] == ls[3 * d + q]) {
          s += kw[3 * d + p] * lw[3 * d + q];
          any = true;
        }
    if (!any) return 0;
    a *= s;
  }
  return 1;
}
__global__ __launch_bounds__(kGramThreads) void k_gram(GridK g, const int *mcount,
                                                       const int *sidx, const double *sw1,
                                                       int *col, double *val, int *cnt,
                                                       int *flags) {
  __shared__ int lds[32];
  __shared__ int ks[9];
  __shared__ double kw[9];
  const int k = blockIdx.x;
  const int n = mcount[0];
  if (k >= n) return;
  if (threadIdx.x < 9) {
    ks[threadIdx.x] = sidx[9 * k + threadIdx.x];
    kw[threadIdx.x] = sw1[9 * k + threadIdx.x];
  }
  __syncthreads();
  int base = 0;
  for (int start = 0; start < n; start += blockDim.x) {
    const int l = start + threadIdx.x;
    double a = 1.0;
    int nz = 0;
    if (l < n) nz = gram_entry(g, ks, kw, sidx + 9 * l, sw1 + 9 * l, a);
    int tot;
    const int off = block_scan_excl(nz, lds, &tot);
    if (nz && base + off < kMaxNbr) {
      col[(int64_t)kMaxNbr * k + base + off] = l;
      val[(int64_t)kMaxNbr * k + base + off] = a;
    }
    base += tot;
  }
  if (threadIdx.x == 0) {
    if (base > kMaxNbr) atomicOr(flags + 3, 1);
    cnt[k] = base < kMaxNbr ? base : kMaxNbr;
  }
}

__device__ __forceinline__ double block_dot_all(double v, double *lds) {
  double s = block_sum(v, lds);
  __shared__ double bc;
  if (threadIdx.x == 0) bc = s;
  __syncthreads();
  double r = bc;
  __syncthreads();
  return r;
}

__device__ __forceinline__ void ell_matvec(int n, const int *col, const double *val,
                                           const int *cnt, const double *v, double *out) {
  for (int row = threadIdx.x; row < n; row += blockDim.x) {
    double s = 0.0;
    const int m = cnt[row];
    for (int e = 0; e < m; ++e)
      s += val[(int64_t)kMaxNbr * row + e] * v[col[(int64_t)kMaxNbr * row + e]];
    out[row] = s;
  }
}

// A eps = 1 by conjugate gradients in one block, warm started, restarted from the
// true residual until |1 - A eps| <= 1e-13 |1| (a backward-stable FP64 solve).
__global__ void k_eps_cg(int *mcount, const int *col, const double *val, const int *cnt,
                         double *x, double *r, double *p, double *q, int *flags) {
  __shared__ double lds[32];
  const int n = mcount[0];
  if (n == 0) return;
  const double tol_true2 = 1e-26 * n, tol_in2 = 1e-30 * n;
  int total_it = 0;
  bool ok = false;
  for (int restart = 0; restart < 7 && !ok; ++restart) {
    ell_matvec(n, col, val, cnt, x, q);
    __syncthreads();
    double rr = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double ri = 1.0 - q[i];
      r[i] = ri;
      p[i] = ri;
      rr += ri * ri;
    }
    rr = block_dot_all(rr, lds);
    if (rr <= tol_true2) {
      ok = true;
      break;
    }
    if (restart == 6) break;
    const int maxit = 4 * n + 50;
    for (int it = 0; it < maxit; ++it) {
      ell_matvec(n, col, val, cnt, p, q);
      __syncthreads();
      double pq = 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) pq += p[i] * q[i];
      pq = block_dot_all(pq, lds);
      const double alpha = rr / pq;
      double rn = 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        x[i] += alpha * p[i];
        double ri = r[i] - alpha * q[i];
        r[i] = ri;
        rn += ri * ri;
      }
      rn = block_dot_all(rn, lds);
      ++total_it;
      if (rn <= tol_in2) break;
      const double beta = rn / rr;
      for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = r[i] + beta * p[i];
      rr = rn;
      __syncthreads();
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mcount[2] = total_it;
    if (!ok) atomicOr(flags + 2, 1);
  }
}

// Sums of NV doubles over the block, returned to every thread: a butterfly within
// each wave (every lane ends with the same value: the additions pair the same
// operands in every lane), one barrier, then every wave sums the per-wave partials
// itself. The two halves of `lds` ([2][NV][16]) alternate between calls, so that
// a call needs no second barrier: a wave writes a half again only after the next
// call's barrier, which every wave reaches after reading it.
template <int NV>
__device__ __forceinline__ void block_allsum(double *v, double *lds, int &half) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  double *bf = lds + half * NV * 16;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) bf[q * 16 + w] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = lane < nw ? bf[q * 16 + lane] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    v[q] = t;
  }
  half ^= 1;
}

// The same solve with the vectors held by the block, as the single-reduction CG
// of Chronopoulos and Gear (s = A p carried as s = w + beta s, one reduction of
// r.r and w.r per iteration): each thread keeps x, r, p, w, s of its rows (i =
// threadIdx.x + j blockDim.x, j < R) in registers; r is shared through LDS for
// the product w = A r; the first NR entries of each row of the ELL arrays are held
// in registers too (the rest, if any, read each time). Same restarts from the true
// residual and tolerances as k_eps_cg (relative to |rhs|); for n <= R * blockDim.x.
// rhs NULL: the right-hand side 1 (the quadrature weights); otherwise A x = rhs
// (the adjoint of that solve). The iteration count goes to *it_out.
constexpr int kEpsRegNnz = 16;  // Gram entries per row held in registers (n <= 1024)
template <int R, int NR>
__global__ __launch_bounds__(kRedThreads) void k_eps_cg_regs(const int *mcount, const int *col,
                                                             const double *val, const int *cnt,
                                                             const double *rhs, double *xg,
                                                             int *it_out, int *flags) {
  extern __shared__ double ps[];  // n values of the vector multiplied by A
  __shared__ double lds[2 * 2 * 16];
  int half = 0;
  const int n = mcount[0];
  if (n == 0) return;
  const int nt = blockDim.x;
  double x[R], r[R], w[R], p[R], sv[R], bv[R];
  double bb[1] = {0.0};
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int i = threadIdx.x + j * nt;
    x[j] = i < n ? xg[i] : 0.0;
    bv[j] = i < n ? (rhs ? rhs[i] : 1.0) : 0.0;
    bb[0] += bv[j] * bv[j];
    r[j] = w[j] = p[j] = sv[j] = 0.0;
  }
  block_allsum<1>(bb, lds, half);
  if (!(bb[0] > 0.0)) {  // zero right-hand side: x = 0
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int i = threadIdx.x + j * nt;
      if (i < n) xg[i] = 0.0;
    }
    if (threadIdx.x == 0) *it_out = 0;
    return;
  }
  const double tol_true2 = 1e-26 * bb[0], tol_in2 = 1e-30 * bb[0];
  int mrow[R], creg[R][NR > 0 ? NR : 1];
  double vreg[R][NR > 0 ? NR : 1];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int i = threadIdx.x + j * nt;
    mrow[j] = i < n ? cnt[i] : 0;
#pragma unroll
    for (int e = 0; e < NR; ++e) {
      const bool in = e < mrow[j];
      creg[j][e] = in ? col[(int64_t)kMaxNbr * i + e] : 0;
      vreg[j][e] = in ? val[(int64_t)kMaxNbr * i + e] : 0.0;
    }
  }
  // out = A v for this thread's rows, in the ELL order (v is put in LDS first; the
  // barrier after the writes also ends every read of the previous product, whose
  // reduction barrier comes before)
  auto product = [&](const double *v, double *out) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int i = threadIdx.x + j * nt;
      if (i < n) ps[i] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int i = threadIdx.x + j * nt;
      double sacc = 0.0;
#pragma unroll
      for (int e = 0; e < NR; ++e)
        if (e < mrow[j]) sacc += vreg[j][e] * ps[creg[j][e]];
      for (int e = NR; e < mrow[j]; ++e)
        sacc += val[(int64_t)kMaxNbr * i + e] * ps[col[(int64_t)kMaxNbr * i + e]];
      out[j] = sacc;
    }
  };
  int total_it = 0;
  bool ok = false;
  for (int restart = 0; restart < 7 && !ok; ++restart) {
    product(x, w);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int i = threadIdx.x + j * nt;
      r[j] = i < n ? bv[j] - w[j] : 0.0;
    }
    __syncthreads();  // every read of x in LDS is done before r replaces it
    product(r, w);
    double gd[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < R; ++j) {
      gd[0] += r[j] * r[j];
      gd[1] += w[j] * r[j];
    }
    block_allsum<2>(gd, lds, half);
    double gam = gd[0];
    if (gam <= tol_true2) {
      ok = true;
      break;
    }
    if (restart == 6) break;
    double alpha = gam / gd[1];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      p[j] = r[j];
      sv[j] = w[j];
    }
    const int maxit = 4 * n + 50;
    for (int it = 0; it < maxit; ++it) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        x[j] += alpha * p[j];
        r[j] -= alpha * sv[j];
      }
      product(r, w);
      double g2[2] = {0.0, 0.0};
#pragma unroll
      for (int j = 0; j < R; ++j) {
        g2[0] += r[j] * r[j];
        g2[1] += w[j] * r[j];
      }
      block_allsum<2>(g2, lds, half);
      ++total_it;
      if (g2[0] <= tol_in2) break;
      const double beta = g2[0] / gam;
      alpha = g2[0] / (g2[1] - beta * g2[0] / alpha);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        p[j] = r[j] + beta * p[j];
        sv[j] = w[j] + beta * sv[j];
      }
      gam = g2[0];
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int i = threadIdx.x + j * nt;
    if (i < n) xg[i] = x[j];
  }
  if (threadIdx.x == 0) {
    *it_out = total_it;
    if (!ok) atomicOr(flags + 2, 1);
  }
}

// A 64-bit lane value moved within rows of 16 lanes by the DPP control CTRL (every
// lane of the wave active).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_value(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
// Sum over the 64 lanes of a wave, the same in every lane: each lane adds the value
// of lane^1 and of lane^2 (quad permutes), then of its mirror in the half row of 8
// and in the row of 16 (both lanes of a pair add the same two operands), and the four
// row sums, read from lanes 0, 16, 32 and 48, are added in that order.
__device__ __forceinline__ double wave_allsum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}
// Two such sums, their steps interleaved.
__device__ __forceinline__ void wave_allsum2(double &a, double &b) {
  a += dpp_move<0xB1>(a);
  b += dpp_move<0xB1>(b);
  a += dpp_move<0x4E>(a);
  b += dpp_move<0x4E>(b);
  a += dpp_move<0x141>(a);
  b += dpp_move<0x141>(b);
  a += dpp_move<0x140>(a);
  b += dpp_move<0x140>(b);
  a = (lane_value(a, 0) + lane_value(a, 16)) + (lane_value(a, 32) + lane_value(a, 48));
  b = (lane_value(b, 0) + lane_value(b, 16)) + (lane_value(b, 32) + lane_value(b, 48));
}

// The solve of k_eps_cg_regs (the same single-reduction iteration, restarts and
// tolerances) in one wave, for n <= 64 R rows: lane l holds rows l + 64 j (j < R)
// with their first NR Gram entries in registers, entries past a row's count being
// zero weights on the row itself so that the product has no branch (a longer row
// reads the rest each time); groups of 64 rows past n are skipped. The two sums of
// an iteration are wave sums, with no barrier between the waves of a block and no
// trip through LDS; the step lengths take one division on the iteration's critical
// path: with q = 1/alpha and g = 1/gamma kept, beta = rho g, the new denominator is
// d = (w.r) - beta rho q, alpha = rho / d, and q = d / rho, g = 1 / rho follow off it.
template <int R, int NR>
__global__ __launch_bounds__(64) void k_eps_cg_wave(const int *mcount, const int *col,
                                                    const double *val, const int *cnt,
                                                    const double *rhs, double *xg, int *it_out,
                                                    int *flags, const int *save_ids,
                                                    double *save_to) {
  __shared__ double ps[64 * R];  // the vector multiplied by A
  const int n = mcount[0];
  if (n == 0) return;
  const int lane = threadIdx.x;
  double x[R], r[R], w[R], p[R], sv[R], bv[R];
  double bb = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int i = lane + 64 * j;
    x[j] = i < n ? xg[i] : 0.0;
    bv[j] = i < n ? (rhs ? rhs[i] : 1.0) : 0.0;
    bb += bv[j] * bv[j];
    r[j] = w[j] = p[j] = sv[j] = 0.0;
  }
  bb = wave_allsum(bb);
  if (!(bb > 0.0)) {  // zero right-hand side: x = 0
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int i = lane + 64 * j;
      if (i < n) xg[i] = 0.0;
    }
    if (lane == 0) *it_out = 0;
    return;
  }
  const double tol_true2 = 1e-26 * bb, tol_in2 = 1e-30 * bb;
  int mrow[R], creg[R][NR];
  double vreg[R][NR];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int i = lane + 64 * j;
    mrow[j] = i < n ? cnt[i] : 0;
#pragma unroll
    for (int e = 0; e < NR; ++e) {
      const bool in = e < mrow[j];
      creg[j][e] = in ? col[(int64_t)kMaxNbr * i + e] : i;
      vreg[j][e] = in ? val[(int64_t)kMaxNbr * i + e] : 0.0;
    }
  }
  // out = A v for this lane's rows, in the ELL order
  auto product = [&](const double *v, double *out) {
    __syncthreads();  // the previous product's reads of ps come first
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (64 * j < n) ps[lane + 64 * j] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (64 * j >= n) {
        out[j] = 0.0;
        continue;
      }
      const int i = lane + 64 * j;
      double sacc = 0.0;
#pragma unroll
      for (int e = 0; e < NR; ++e) sacc += vreg[j][e] * ps[creg[j][e]];
      for (int e = NR; e < mrow[j]; ++e)
        sacc += val[(int64_t)kMaxNbr * i + e] * ps[col[(int64_t)kMaxNbr * i + e]];
      out[j] = sacc;
    }
  };
  // the two sums r.r and w.r of this lane's rows
  auto dots = [&](double &rr, double &wr) {
    rr = 0.0;
    wr = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      rr += r[j] * r[j];
      wr += w[j] * r[j];
    }
    wave_allsum2(rr, wr);
  };
  int total_it = 0;
  bool ok = false;
  for (int restart = 0; restart < 7 && !ok; ++restart) {
    product(x, w);
#pragma unroll
    for (int j = 0; j < R; ++j) r[j] = bv[j] - w[j];
    product(r, w);
    double gam, wr;
    dots(gam, wr);
    if (gam <= tol_true2) {
      ok = true;
      break;
    }
    if (restart == 6) break;
    double alpha = gam / wr, q = wr / gam, g = 1.0 / gam;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      p[j] = r[j];
      sv[j] = w[j];
    }
    const int maxit = 4 * n + 50;
    for (int it = 0; it < maxit; ++it) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        x[j] += alpha * p[j];
        r[j] -= alpha * sv[j];
      }
      product(r, w);
      double rho, wr1;
      dots(rho, wr1);
      ++total_it;
      if (rho <= tol_in2) break;
      const double beta = rho * g;
      const double d = wr1 - beta * rho * q;
      alpha = rho / d;
      g = 1.0 / rho;
      q = d * g;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        p[j] = r[j] + beta * p[j];
        sv[j] = w[j] + beta * sv[j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int i = lane + 64 * j;
    if (i < n) {
      xg[i] = x[j];
      if (save_to) save_to[save_ids[i]] = x[j];
    }
  }
  if (lane == 0) {
    *it_out = total_it;
    if (!ok) atomicOr(flags + 2, 1);
  }
}

__global__ void k_eps_save(const int *mcount, const int *ids, const double *eps, double *ceps) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < mcount[0]) ceps[ids[k]] = eps[k];
}

// ------------------------------------------------ interpolation and forcing
// Eq. (5) at each marker from the predictor fields, then Eq. (10) with a_s = 1/dt
// and Eq. (17) with a_e = 1/dt: F = (rho_L U^d - M)/dt, Q = (c_v rho_L Theta^d - E_L)/dt.
// Per-marker force on the body -dV eps F and heat given to the fluid dV eps Q.
template <int DIM, typename S>
__device__ __forceinline__ void interp_force_one(const GridK &g, int k, const int64_t *pcell,
                                                 const double *pw, const S *rho_s,
                                                 const S *const *ms, const S *E_s,
                                                 const double *Ud, const double *Tw,
                                                 const double *eps, double *mk, double *mforce,
                                                 double *mheat) {
  constexpr int dim = DIM, W = 2 * DIM + 3, nslot = (DIM == 3) ? 27 : 9;
  double rl = 0.0, el = 0.0, M[3] = {0.0, 0.0, 0.0};
  // slots in groups of 9: the loads of a group are issued together (the sums keep
  // the slot order)
#pragma unroll
  for (int s0 = 0; s0 < nslot; s0 += 9) {
    int64_t cc[9];
    double ww[9], vr[9], ve[9], vm[DIM][9];
#pragma unroll
    for (int u = 0; u < 9; ++u) {
      cc[u] = pcell[27 * k + s0 + u];
      ww[u] = pw[27 * k + s0 + u];
    }
#pragma unroll
    for (int u = 0; u < 9; ++u) {
      vr[u] = double(rho_s[cc[u]]);
      ve[u] = double(E_s[cc[u]]);
#pragma unroll
      for (int q = 0; q < DIM; ++q) vm[q][u] = double(ms[q][cc[u]]);
    }
#pragma unroll
    for (int u = 0; u < 9; ++u) {
      rl += ww[u] * vr[u];
#pragma unroll
      for (int q = 0; q < DIM; ++q) M[q] += ww[u] * vm[q][u];
      el += ww[u] * ve[u];
    }
  }
  double *o = mk + (int64_t)W * k;
  o[0] = rl;
#pragma unroll
  for (int q = 0; q < dim; ++q) o[1 + q] = M[q];
  o[1 + dim] = el;
  const double e = eps[k];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double F = 0.0;
    if (q < dim) {
      F = (rl * Ud[3 * k + q] - M[q]) / g.dt;
      o[2 + dim + q] = F;
    }
    mforce[3 * k + q] = -(g.dV * (e * F));
  }
  const double Q = g.no_heat ? 0.0 : (g.cv * rl * Tw[k] - el) / g.dt;
  o[2 + 2 * dim] = Q;
  mheat[k] = g.dV * (e * Q);
}

template <int DIM, typename S>
__global__ void k_interp_force(GridK g, const int *mcount, const int64_t *pcell, const double *pw,
                               const S *rho_s, const S *ms0, const S *ms1, const S *ms2,
                               const S *E_s, const double *Ud, const double *Tw,
                               const double *eps, double *mk, double *mforce, double *mheat) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= mcount[0]) return;
  const S *ms[3] = {ms0, ms1, ms2};
  interp_force_one<DIM>(g, k, pcell, pw, rho_s, ms, E_s, Ud, Tw, eps, mk, mforce, mheat);
}

// Totals over the markers in use (fixed order); one history row if given.
__device__ __forceinline__ void totals_block(const int *mcount, const double *mforce,
                                             const double *mheat, double *totals,
                                             double *hist_row, double *lds) {
  const int n = mcount[0];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    v[0] += mforce[3 * k];
    v[1] += mforce[3 * k + 1];
    v[2] += mforce[3 * k + 2];
    v[3] += mheat[k];
  }
  block_sum_n<4>(v, lds);
  if (threadIdx.x == 0) {
    for (int q = 0; q < 4; ++q) totals[q] = v[q];
    if (hist_row)
      for (int q = 0; q < 4; ++q) hist_row[q] = v[q];
  }
}

__global__ void k_totals(const int *mcount, const double *mforce, const double *mheat,
                         double *totals, double *hist_row) {
  __shared__ double lds[64];
  totals_block(mcount, mforce, mheat, totals, hist_row, lds);
}

// Local heat flux of each marker in use (Sec. 3.1, the wall heat flux behind a
// local Nusselt number): q_k = H_k / dA'_k, H_k = dV eps_k Q_k the marker's heat,
// dA'_k = dA_k (sum of the candidates' dA) / (sum of the used markers' dA), the
// surface elements of the markers in use scaled to the whole given surface (the
// check routine drops candidates, whose surface the kept markers then represent).
// One block; fixed-order sums. status[0] = 1 when the markers in use carry no
// surface (nothing written).
__global__ void k_heat_flux(int nc, const int *mcount, const double *cdA, const double *dA,
                            const double *mheat, double *q, int *status) {
  __shared__ double lds[64];
  __shared__ double sc[2];
  const int nu = mcount[0];
  double v[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < nc; k += blockDim.x) v[0] += cdA[k];
  for (int k = threadIdx.x; k < nu; k += blockDim.x) v[1] += dA[k];
  block_sum_n<2>(v, lds);
  if (threadIdx.x == 0) {
    sc[0] = v[0];
    sc[1] = v[1];
    status[0] = (v[1] > 0.0) ? 0 : 1;
  }
  __syncthreads();
  if (!(sc[1] > 0.0)) return;
  const double scale = sc[0] / sc[1];
  for (int k = threadIdx.x; k < nu; k += blockDim.x) q[k] = mheat[k] / (dA[k] * scale);
}

// Fields the spread updates: mom** = mom* + dt f, E** = E* + dt q, the set-up's
// m^ (+ dt f) and psi = 1/(R theta**), theta** = E**/(rho* c_v).
template <typename S>
struct SpreadSet {
  S *ms[3];
  S *E_s;
  S *mh[3];
  S *psi;
  const S *rho_s;
};

// The updates of SpreadSet at one cell from its sums of w eps F and w eps Q.
template <int DIM, typename S>
__device__ __forceinline__ void spread_apply(const GridK &g, int64_t cell, const double *acc,
                                             double aq, const SpreadSet<S> &sp) {
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    sp.ms[q][cell] = S(double(sp.ms[q][cell]) + g.dt * acc[q]);
    sp.mh[q][cell] = S(double(sp.mh[q][cell]) + g.dt * acc[q]);
  }
  const S es = S(double(sp.E_s[cell]) + g.dt * aq);
  sp.E_s[cell] = es;
  const S theta = es / (sp.rho_s[cell] * S(g.cv));
  sp.psi[cell] = S(1) / (S(g.R) * theta);
}

// Eq. (7) as a segmented reduction: one thread per cell touched by a support,
// summing w eps F and w eps Q over its pairs in increasing marker id, then the
// updates of SpreadSet in place.
template <int DIM, typename S>
__device__ __forceinline__ void spread_one(const GridK &g, int s, const int *seg,
                                           const uint64_t *keys, const double *pw,
                                           const double *eps, const double *mk,
                                           const SpreadSet<S> &sp) {
  constexpr int dim = DIM, W = 2 * DIM + 3, nslot = (DIM == 3) ? 27 : 9;
  const int a = seg[s], b = seg[s + 1];
  const int64_t cell = (int64_t)(keys[a] >> kPairBits);
  const uint64_t mask = (1ull << kPairBits) - 1;
  double acc[3] = {0.0, 0.0, 0.0}, aq = 0.0;
  // pairs in groups of 4, the loads of a group issued together (sums in pair order)
  for (int i0 = a; i0 < b; i0 += 4) {
    double coef[4], f[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      coef[u] = 0.0;
      f[u][0] = f[u][1] = f[u][2] = f[u][3] = 0.0;
      if (i0 + u < b) {
        const int pid = (int)(keys[i0 + u] & mask);
        const int k = pid / nslot, slot = pid - k * nslot;
        coef[u] = pw[27 * k + slot] * eps[k];
        const double *o = mk + (int64_t)W * k;
#pragma unroll
        for (int q = 0; q < dim; ++q) f[u][q] = o[2 + dim + q];
        f[u][3] = o[2 + 2 * dim];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + u < b) {
#pragma unroll
        for (int q = 0; q < dim; ++q) acc[q] += coef[u] * f[u][q];
        aq += coef[u] * f[u][3];
      }
    }
  }
  spread_apply<DIM>(g, cell, acc, aq, sp);
}

template <int DIM, typename S>
__global__ void k_spread(GridK g, const int *mcount, const int *seg, const uint64_t *keys,
                         const double *pw, const double *eps, const double *mk,
                         SpreadSet<S> sp) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= mcount[1]) return;
  spread_one<DIM>(g, s, seg, keys, pw, eps, mk, sp);
}

// The three steps above in one block (for small marker sets, where launch latency
// dominates): interpolation and forcing per marker, the totals, then the spread.
// The block barrier between the phases also makes the marker values written in one
// phase visible to the threads of the next.
template <int DIM, typename S>
__global__ __launch_bounds__(kRedThreads) void k_markers_fused(
    GridK g, const int *mcount, const int64_t *pcell, const double *pw, const int *seg,
    const uint64_t *keys, SpreadSet<S> sp, const double *Ud, const double *Tw, const double *eps,
    double *mk, double *mforce, double *mheat, double *totals, double *hist_row) {
  __shared__ double lds[64];
  const S *msc[3] = {sp.ms[0], sp.ms[1], sp.ms[2]};
  const int n = mcount[0];
  for (int k = threadIdx.x; k < n; k += blockDim.x)
    interp_force_one<DIM>(g, k, pcell, pw, sp.rho_s, msc, (const S *)sp.E_s, Ud, Tw, eps, mk,
                          mforce, mheat);
  __syncthreads();
  totals_block(mcount, mforce, mheat, totals, hist_row, lds);
  const int nseg = mcount[1];
  if constexpr (DIM == 2) {
    // two segments per thread at a time: the loads of both are issued before either
    // sum is formed (the sums keep each segment's pair order, as spread_one); 1.0 us
    // less per step for 212 markers. (In 3D the registers would spill.)
    constexpr int dim = DIM, W = 2 * DIM + 3, nslot = 9;
    const uint64_t mask = (1ull << kPairBits) - 1;
    const int bd = blockDim.x;
    for (int s0 = threadIdx.x; s0 < nseg; s0 += 2 * bd) {
      int a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int s = s0 + u * bd;
        a[u] = b[u] = 0;
        if (s < nseg) {
          a[u] = seg[s];
          b[u] = seg[s + 1];
        }
      }
      uint64_t key[2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) key[u][q] = (a[u] + q < b[u]) ? keys[a[u] + q] : 0;
      double coef[2][4], f[2][4][4];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          coef[u][q] = 0.0;
          f[u][q][0] = f[u][q][1] = f[u][q][2] = f[u][q][3] = 0.0;
          if (a[u] + q < b[u]) {
            const int pid = (int)(key[u][q] & mask);
            const int k = pid / nslot, slot = pid - k * nslot;
            coef[u][q] = pw[27 * k + slot] * eps[k];
            const double *o = mk + (int64_t)W * k;
#pragma unroll
            for (int c = 0; c < dim; ++c) f[u][q][c] = o[2 + dim + c];
            f[u][q][3] = o[2 + 2 * dim];
          }
        }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (a[u] >= b[u]) continue;
        double acc[3] = {0.0, 0.0, 0.0}, aq = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (a[u] + q < b[u]) {
#pragma unroll
            for (int c = 0; c < dim; ++c) acc[c] += coef[u][q] * f[u][q][c];
            aq += coef[u][q] * f[u][q][3];
          }
        }
        // pairs past the first four (rare), in order
        for (int p = a[u] + 4; p < b[u]; ++p) {
          const int pid = (int)(keys[p] & mask);
          const int k = pid / nslot, slot = pid - k * nslot;
          const double cf = pw[27 * k + slot] * eps[k];
          const double *o = mk + (int64_t)W * k;
#pragma unroll
          for (int c = 0; c < dim; ++c) acc[c] += cf * o[2 + dim + c];
          aq += cf * o[2 + 2 * dim];
        }
        spread_apply<DIM>(g, (int64_t)(key[u][0] >> kPairBits), acc, aq, sp);
      }
    }
  } else {
    for (int s = threadIdx.x; s < nseg; s += blockDim.x)
      spread_one<DIM>(g, s, seg, keys, pw, eps, mk, sp);
  }
}

// ------------------------------------------------- marker-position gradient
// (not in the paper: the adjoint's derivative with respect to the candidate
// positions X_k, for markers at rest). The adjoint steps accumulate the cotangent
// of every kernel weight w_ck (wbar, per pair) and of every quadrature weight eps_k
// (epsbar). A = W^T W with A eps = 1 gives, with A lambda = epsbar,
//   wbar_ck -= lambda_k (W eps)_c + eps_k (W lambda)_c,
// and w_ck = prod_d phi(r_d), r_d = (i_d + 1/2) - (X_d - lo_d)/h_d gives
//   Xbar_kd = sum_c wbar_ck * (-phi'(r_d)/h_d) prod_{e != d} phi(r_e).

// d phi / d r of the 3-point kernel.
__device__ __forceinline__ double kernel_dphi(double r) {
#pragma clang fp contract(off)
  const double a = fabs(r), sg = r < 0.0 ? -1.0 : 1.0;
  if (a <= 0.5) return sg * (-a / sqrt(1.0 - 3.0 * a * a));
  if (a <= 1.5) {
    const double b = 1.0 - a;
    return sg * (-3.0 - 3.0 * b / sqrt(1.0 - 3.0 * b * b)) / 6.0;
  }
  return 0.0;
}

// Per cell of the sorted pairs: (W eps)_c and (W lambda)_c, written to each of
// the cell's pairs.
__global__ void k_shape_cellsums(const int *mcount, const int *seg, const uint64_t *keys,
                                 const double *pw, int nslot, const double *eps,
                                 const double *lam, double *gsum) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= mcount[1]) return;
  const int a = seg[s], b = seg[s + 1];
  const uint64_t mask = (1ull << kPairBits) - 1;
  double se = 0.0, sl = 0.0;
  for (int p = a; p < b; ++p) {
    const int pid = (int)(keys[p] & mask);
    const int k = pid / nslot, slot = pid - k * nslot;
    const double w = pw[27 * k + slot];
    se += w * eps[k];
    sl += w * lam[k];
  }
  for (int p = a; p < b; ++p) {
    const int pid = (int)(keys[p] & mask);
    const int k = pid / nslot, slot = pid - k * nslot;
    gsum[2 * (27 * k + slot)] = se;
    gsum[2 * (27 * k + slot) + 1] = sl;
  }
}

// Per marker in use: Xbar_k from its pairs, added to X_bar of its candidate id;
// its accumulators are cleared.
__global__ void k_shape_grad(GridK g, const int *mcount, const double *X, const int *ids,
                             const double *eps, const double *lam, const double *gsum,
                             double *wbar, double *epsbar, double *X_bar) {
#pragma clang fp contract(off)
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= mcount[0]) return;
  double ph[3][3], dph[3][3];
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 3; ++s) {
      ph[a][s] = (s == 0) ? 1.0 : 0.0;
      dph[a][s] = 0.0;
    }
  for (int a = 0; a < g.dim; ++a) {
    const double xi = (X[3 * k + a] - g.lo[a]) / g.h[a];
    const int64_t b = (int64_t)floor(xi);
    for (int s = 0; s < 3; ++s) {
      const double r = (double(b - 1 + s) + 0.5) - xi;
      ph[a][s] = kernel_phi(r);
      dph[a][s] = -kernel_dphi(r) / g.h[a];
    }
  }
  double xb[3] = {0.0, 0.0, 0.0};
  const int s2n = (g.dim == 3) ? 3 : 1;
  for (int s2 = 0; s2 < s2n; ++s2)
    for (int s1 = 0; s1 < 3; ++s1)
      for (int s0 = 0; s0 < 3; ++s0) {
        const int s = s0 + 3 * (s1 + 3 * s2);
        const int64_t pq = 27 * k + s;
        const double wb = wbar[pq] - lam[k] * gsum[2 * pq] - eps[k] * gsum[2 * pq + 1];
        wbar[pq] = 0.0;
        xb[0] += wb * dph[0][s0] * ph[1][s1] * ph[2][s2];
        xb[1] += wb * ph[0][s0] * dph[1][s1] * ph[2][s2];
        if (g.dim == 3) xb[2] += wb * ph[0][s0] * ph[1][s1] * dph[2][s2];
      }
  epsbar[k] = 0.0;
  for (int a = 0; a < g.dim; ++a) X_bar[(int64_t)ids[k] * g.dim + a] += xb[a];
}

__global__ void k_shape_clear(int n, double *wbar, double *epsbar) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 27 * n) wbar[i] = 0.0;
  if (i < n) epsbar[i] = 0.0;
}

// ------------------------------------------------------------------ launchers
static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename S>
static SpreadSet<S> spread_set(const Bufs &B) {
  SpreadSet<S> sp;
  for (int q = 0; q < 3; ++q) {
    sp.ms[q] = (S *)B.mom_s[q];
    sp.mh[q] = (S *)B.mhat[q];
  }
  sp.E_s = (S *)B.E_s;
  sp.psi = (S *)B.psi;
  sp.rho_s = (const S *)B.rho_s;
  return sp;
}

void run_place_markers(const Launch &L, const Bufs &B, int nc, double off, double vel, int axis,
                       int dedupe) {
  hipLaunchKernelGGL(k_place, dim3(nblk(nc, 256)), dim3(256), 0, L.st, L.g, nc,
                     (const double *)B.cX0, (const double *)B.cUd0, B.cXc, B.cUdc, off, vel, axis,
                     B.ckey, B.cd2);
  if (dedupe)
    hipLaunchKernelGGL(k_dedupe, dim3(nblk((int64_t)nc * 64, 256)), dim3(256), 0, L.st, nc,
                       (const int64_t *)B.ckey, (const double *)B.cd2, B.ckeep);
  else
    hipLaunchKernelGGL(k_keep_all, dim3(nblk(nc, 256)), dim3(256), 0, L.st, nc, B.ckeep);
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(kRedThreads), 0, L.st, nc, (const int *)B.ckeep,
                     (const double *)B.cXc, (const double *)B.cUdc, (const double *)B.cTw,
                     (const double *)B.cdA, (const double *)B.ceps, B.ids, B.X, B.Ud, B.Tw, B.dA,
                     B.eps, B.mcount);
}

// ------------------------------------------ marker set-up of a small body
// For up to kSmallCand candidates and kSmallKeys (cell, pair) keys: placement and the
// check routine, compaction, supports, the key sort, segments and the Gram rows in one
// block of 4 kSmallCand threads (the arithmetic of k_place, k_dedupe, k_compact,
// k_support, k_sort, k_segments and k_gram, phase after phase, with the candidates,
// supports and keys in LDS), so that a moving body's markers are set up again with two
// launches (this and the quadrature solve).
constexpr int kSmallCand = 256;
constexpr int kSmallKeys = 4096;
static_assert(kRedThreads == 4 * kSmallCand, "one block of four threads per candidate");

// Number of entries of the ascending list L[0, n) below v (n <= 256).
__device__ __forceinline__ int count_below(const uint64_t *L, int n, uint64_t v) {
  int pos = 0;
#pragma unroll
  for (int step = 256; step > 0; step >>= 1)
    if (pos + step <= n && L[pos + step - 1] < v) pos += step;
  return pos;
}

// A_kl (Eq. (9)) of two markers whose supports are known to overlap in every
// direction, from the offset of their centre cells: the 1D sum over the cell indices
// the two windows share pairs slot p of k with slot p + (c_k - c_l) of l, p
// ascending (the terms and order of gram_entry when no periodic direction has fewer
// than six cells).
__device__ __forceinline__ double gram_entry_offset(int dim, const int *dl, const double *kw,
                                                    const double *lw) {
  double a = 1.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d >= dim) break;
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int q = p + dl[d];
      if (q >= 0 && q < 3) s += kw[3 * d + p] * lw[3 * d + q];
    }
    a *= s;
  }
  return a;
}

__global__ __launch_bounds__(kRedThreads) void k_rebuild_small(
    GridK g, int nc, int nslot, const double *X0, const double *U0, double off, double vel,
    int axis, int dedupe, const double *cTw, const double *cdA, const double *ceps, double *cXc,
    double *cUdc, int *ids, double *X, double *U, double *Tw, double *dA, double *eps,
    int *mcount, int64_t *pcell, double *pw, uint64_t *keys, int *seg, int *ell_col,
    double *ell_val, int *ell_cnt, int *flags) {
  __shared__ int64_t skey[kSmallCand];
  __shared__ double sd2[kSmallCand];
  __shared__ double sX[3 * kSmallCand];
  __shared__ int sbeat[4][kSmallCand];
  __shared__ int ssi[9 * kSmallCand];     // support cell indices per direction and slot
  __shared__ double ssw[9 * kSmallCand];  // their 1D kernel weights
  __shared__ uint64_t sk[kSmallKeys];     // pair keys by pair, then in increasing order
  __shared__ uint64_t sl[kSmallKeys];     // the same keys as one ascending list per slot
  __shared__ uint64_t sm[kSmallCand];     // marker keys (centre cell << kPairBits | marker)
  __shared__ int sord[kSmallCand];        // markers by increasing marker key
  __shared__ int lds[32];
  __shared__ int nsh;
  const int t = threadIdx.x;
  // placement (Sec. 5, Eq. (19)) of candidate t
  double xk[3] = {0.0, 0.0, 0.0};
  if (t < nc) place_one(g, t, X0, U0, cXc, cUdc, off, vel, axis, skey[t], sd2[t], xk);
  __syncthreads();
  // the check routine (Sec. 3.1): kept when no candidate of its cell is nearer its
  // centre (ties: the lower id); four threads per candidate, each testing a quarter
  // of the others
  {
    const int c = t % kSmallCand, part = t / kSmallCand, len = (nc + 3) / 4;
    int beat = 0;
    if (c < nc && dedupe) {
      const int64_t kk = skey[c];
      const double dk = sd2[c];
      const int j1 = min(nc, (part + 1) * len);
#pragma unroll 8
      for (int j = part * len; j < j1; ++j)
        beat |= (skey[j] == kk && (sd2[j] < dk || (sd2[j] == dk && j < c))) ? 1 : 0;
    }
    sbeat[part][c] = beat;
  }
  __syncthreads();
  const int keep = t < nc ? !(sbeat[0][t] | sbeat[1][t] | sbeat[2][t] | sbeat[3][t]) : 0;
  // compaction in increasing id
  int tot;
  const int m = block_scan_excl(keep, lds, &tot);
  if (keep) {
    ids[m] = t;
    for (int a = 0; a < 3; ++a) {
      X[3 * m + a] = xk[a];
      U[3 * m + a] = cUdc[3 * t + a];
      sX[3 * m + a] = xk[a];
    }
    Tw[m] = cTw[t];
    dA[m] = cdA[t];
    eps[m] = ceps[t];
  }
  if (t == 0) {
    mcount[0] = tot;
    nsh = tot;
  }
  __syncthreads();
  const int n = nsh;
  const int np = n * nslot;
  // supports and pair keys of marker t; its key by centre cell
  if (t < n) {
    support_one(g, t, sX, nslot, ssi, ssw, pcell, pw, sk, flags);
    sm[t] = (sk[nslot * t + nslot / 2] >> kPairBits << kPairBits) | (uint64_t)t;
  }
  __syncthreads();
  // the markers by centre cell: the place of each is the number of keys below it
  {
    const int c = t % kSmallCand, part = t / kSmallCand, len = (n + 3) / 4;
    int below = 0;
    if (c < n) {
      const uint64_t v = sm[c];
      const int j1 = min(n, (part + 1) * len);
#pragma unroll 8
      for (int j = part * len; j < j1; ++j) below += sm[j] < v ? 1 : 0;
    }
    sbeat[part][c] = below;
  }
  __syncthreads();
  if (t < n) sord[sbeat[0][t] + sbeat[1][t] + sbeat[2][t] + sbeat[3][t]] = t;
  __syncthreads();
  // the keys of slot s in that marker order: ascending unless a support wraps round a
  // periodic direction
  bool unsorted = false;
  for (int i = t; i < np; i += blockDim.x) {
    const int sl_s = i / n, mm = i - sl_s * n;
    sl[i] = sk[nslot * sord[mm] + sl_s];
  }
  __syncthreads();
  for (int i = t; i < np; i += blockDim.x) {
    const int mm = i % n;
    if (mm + 1 < n && sl[i] > sl[i + 1]) unsorted = true;
  }
  if (__syncthreads_or(unsorted)) {
    // bitonic sort in LDS, padded with the largest key to a power of two (the keys are
    // distinct, so the order is fully determined)
    int npad = 1;
    while (npad < np) npad <<= 1;
    for (int i = np + t; i < npad; i += blockDim.x) sk[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= npad; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int q = t; q < npad / 2; q += blockDim.x) {
          const int i = 2 * q - (q & (stride - 1)), j = i + stride;
          const bool asc = (i & size) == 0;
          const uint64_t u = sk[i], v = sk[j];
          if ((u > v) == asc) {
            sk[i] = v;
            sk[j] = u;
          }
        }
        __syncthreads();
      }
  } else {
    // merge of the slot lists: a key's place is its place in its own list plus the
    // number of keys below it in each other list
    for (int i = t; i < np; i += blockDim.x) {
      const int s0 = i / n;
      const uint64_t v = sl[i];
      int rank = i - s0 * n;
      for (int s1 = 0; s1 < nslot; ++s1)
        if (s1 != s0) rank += count_below(sl + s1 * n, n, v);
      sk[rank] = v;
    }
    __syncthreads();
  }
  for (int i = t; i < np; i += blockDim.x) keys[i] = sk[i];
  // segments of equal cell
  int base = 0;
  for (int start = 0; start < np; start += blockDim.x) {
    const int i = start + t;
    int head = 0;
    if (i < np) head = (i == 0) || ((sk[i] >> kPairBits) != (sk[i - 1] >> kPairBits));
    int cnt;
    const int o = block_scan_excl(head, lds, &cnt);
    if (head) seg[base + o] = i;
    base += cnt;
  }
  if (t == 0) {
    seg[base] = np;
    mcount[1] = base;
  }
  // Gram rows (Eq. (9)), one wave per row: its lanes test 64 markers at a time (first
  // the offsets of the centre cells, then the weights where every direction's windows
  // share a cell) and a ballot keeps the nonzeros in increasing column
  bool by_offset = true;  // every periodic direction has at least six cells
  for (int d = 0; d < g.dim; ++d)
    if (g.bc[d][0] == BC_PERIODIC && g.n[d] < 6) by_offset = false;
  const int lane = t & 63, nw = blockDim.x >> 6;
  for (int k = t >> 6; k < n; k += nw) {
    int c = 0;
    for (int l0 = 0; l0 < n; l0 += 64) {
      const int l = l0 + lane;
      double a = 0.0;
      int nz = 0;
      if (l < n) {
        if (by_offset) {
          int dl[3] = {0, 0, 0};
          nz = 1;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            if (d >= g.dim) break;
            int e = ssi[9 * k + 3 * d + 1] - ssi[9 * l + 3 * d + 1];
            if (g.bc[d][0] == BC_PERIODIC) {
              if (e > g.n[d] / 2) e -= g.n[d];
              if (e < -(g.n[d] / 2)) e += g.n[d];
            }
            dl[d] = e;
            if (e < -2 || e > 2) nz = 0;
          }
          if (nz) a = gram_entry_offset(g.dim, dl, ssw + 9 * k, ssw + 9 * l);
        } else {
          nz = gram_entry(g, ssi + 9 * k, ssw + 9 * k, ssi + 9 * l, ssw + 9 * l, a);
        }
      }
      const uint64_t bal = __ballot(nz);
      const int o = c + __popcll(bal & ((1ull << lane) - 1ull));
      if (nz && o < kMaxNbr) {
        ell_col[(int64_t)kMaxNbr * k + o] = l;
        ell_val[(int64_t)kMaxNbr * k + o] = a;
      }
      c += __popcll(bal);
    }
    if (lane == 0) {
      if (c > kMaxNbr) atomicOr(flags + 3, 1);
      ell_cnt[k] = c < kMaxNbr ? c : kMaxNbr;
    }
  }
}

// Whether the one-block set-up applies to nc candidates.
static bool small_body(const Launch &L, int nc) {
  const int nslot = (L.g.dim == 3) ? 27 : 9;
  return nc <= kSmallCand && nc * nslot <= kSmallKeys;
}

// A x = rhs (rhs NULL: the quadrature weights, rhs 1) for at most nc <= 256 rows, from
// x, in one wave; the solution also goes to save_to[save_ids[i]] when save_to is given.
// Gram entries held in registers per row: 10 in 2D (a curve's rows have about 7), 24
// or 12 in 3D.
template <int R, int NR>
static void launch_eps_wave(const Launch &L, const Bufs &B, const double *rhs, double *x,
                            int *it_out, const int *save_ids, double *save_to) {
  hipLaunchKernelGGL((k_eps_cg_wave<R, NR>), dim3(1), dim3(64), 0, L.st, (const int *)B.mcount,
                     (const int *)B.ell_col, (const double *)B.ell_val, (const int *)B.ell_cnt,
                     rhs, x, it_out, B.flags, save_ids, save_to);
}
static void launch_eps_solve(const Launch &L, const Bufs &B, int nc, const double *rhs,
                             double *x, int *it_out, const int *save_ids, double *save_to) {
  if (L.g.dim == 2) {
    if (nc <= 128)
      launch_eps_wave<2, 10>(L, B, rhs, x, it_out, save_ids, save_to);
    else
      launch_eps_wave<4, 10>(L, B, rhs, x, it_out, save_ids, save_to);
  } else {
    if (nc <= 128)
      launch_eps_wave<2, 24>(L, B, rhs, x, it_out, save_ids, save_to);
    else
      launch_eps_wave<4, 12>(L, B, rhs, x, it_out, save_ids, save_to);
  }
}

MarkerSet marker_set_of(const Bufs &B) {
  MarkerSet m;
  m.cXc = B.cXc;
  m.cUdc = B.cUdc;
  m.ckey = B.ckey;
  m.cd2 = B.cd2;
  m.ckeep = B.ckeep;
  m.mcount = B.mcount;
  m.ids = B.ids;
  m.X = B.X;
  m.Ud = B.Ud;
  m.Tw = B.Tw;
  m.dA = B.dA;
  m.eps = B.eps;
  m.sidx = B.sidx;
  m.sw1 = B.sw1;
  m.pcell = B.pcell;
  m.pw = B.pw;
  m.keys = B.keys;
  m.keys_in = B.keys_in;
  m.seg = B.seg;
  m.ell_col = B.ell_col;
  m.ell_val = B.ell_val;
  m.ell_cnt = B.ell_cnt;
  for (int v = 0; v < 4; ++v) m.ev[v] = B.ev[v];
  return m;
}

void put_marker_set(Bufs &B, const MarkerSet &m) {
  B.cXc = m.cXc;
  B.cUdc = m.cUdc;
  B.ckey = m.ckey;
  B.cd2 = m.cd2;
  B.ckeep = m.ckeep;
  B.mcount = m.mcount;
  B.ids = m.ids;
  B.X = m.X;
  B.Ud = m.Ud;
  B.Tw = m.Tw;
  B.dA = m.dA;
  B.eps = m.eps;
  B.sidx = m.sidx;
  B.sw1 = m.sw1;
  B.pcell = m.pcell;
  B.pw = m.pw;
  B.keys = m.keys;
  B.keys_in = m.keys_in;
  B.seg = m.seg;
  B.ell_col = m.ell_col;
  B.ell_val = m.ell_val;
  B.ell_cnt = m.ell_cnt;
  for (int v = 0; v < 4; ++v) B.ev[v] = m.ev[v];
}

void run_rebuild_markers(const Launch &L, const Bufs &B, int nc, double off, double vel, int axis,
                         int dedupe, bool save_eps) {
  if (!small_body(L, nc)) {
    run_place_markers(L, B, nc, off, vel, axis, dedupe);
    run_build_markers(L, B, nc, save_eps);
    return;
  }
  const int nslot = (L.g.dim == 3) ? 27 : 9;
  hipLaunchKernelGGL(k_rebuild_small, dim3(1), dim3(kRedThreads), 0, L.st, L.g, nc, nslot,
                     (const double *)B.cX0, (const double *)B.cUd0, off, vel, axis, dedupe,
                     (const double *)B.cTw, (const double *)B.cdA, (const double *)B.ceps, B.cXc,
                     B.cUdc, B.ids, B.X, B.Ud, B.Tw, B.dA, B.eps, B.mcount, B.pcell, B.pw, B.keys,
                     B.seg, B.ell_col, B.ell_val, B.ell_cnt, B.flags);
  launch_eps_solve(L, B, nc, nullptr, B.eps, B.mcount + 2, save_eps ? B.ids : nullptr,
                   save_eps ? B.ceps : nullptr);
}

// Threads of the one-row-per-thread quadrature solve for nc candidates.
static unsigned eps_threads(int nc) {
  const int t = (nc + 63) / 64 * 64;
  return (unsigned)(t < 64 ? 64 : t > kRedThreads ? kRedThreads : t);
}

void run_build_markers(const Launch &L, const Bufs &B, int nc, bool save_eps) {
  const int nslot = (L.g.dim == 3) ? 27 : 9;
  hipLaunchKernelGGL(k_support, dim3(nblk(nc, 256)), dim3(256), 0, L.st, L.g,
                     (const int *)B.mcount, (const double *)B.X, nslot, B.sidx, B.sw1, B.pcell,
                     B.pw, B.keys_in, B.flags);
  if (L.npairs_pad <= kRankKeys) {
    const size_t shm = (size_t)L.npairs_pad * sizeof(uint64_t);
    hipLaunchKernelGGL(k_rank_sort, dim3(nblk(L.npairs_pad, 256)), dim3(256), shm, L.st,
                       (const uint64_t *)B.keys_in, B.keys, (const int *)B.mcount, nslot);
  } else {
    hipLaunchKernelGGL(k_sort, dim3(1), dim3(kRedThreads), 0, L.st,
                       (const uint64_t *)B.keys_in, B.keys, L.npairs_pad, (const int *)B.mcount,
                       nslot);
  }
  hipLaunchKernelGGL(k_segments, dim3(1), dim3(kRedThreads), 0, L.st, (const uint64_t *)B.keys,
                     nslot, B.mcount, B.seg);
  hipLaunchKernelGGL(k_gram, dim3((unsigned)nc), dim3(kGramThreads), 0, L.st, L.g,
                     (const int *)B.mcount, (const int *)B.sidx, (const double *)B.sw1,
                     B.ell_col, B.ell_val, B.ell_cnt, B.flags);
  // the live count is on the device; the candidate count bounds it
  const size_t psb = (size_t)nc * sizeof(double);
  if (nc <= 256) {  // one wave: no barrier
    launch_eps_solve(L, B, nc, nullptr, B.eps, B.mcount + 2, save_eps ? B.ids : nullptr,
                     save_eps ? B.ceps : nullptr);
    return;
  }
  if (nc <= kRedThreads)  // one row per thread: as few waves as rows need
    hipLaunchKernelGGL((k_eps_cg_regs<1, kEpsRegNnz>), dim3(1), dim3(eps_threads(nc)), psb,
                       L.st, (const int *)B.mcount, (const int *)B.ell_col,
                       (const double *)B.ell_val, (const int *)B.ell_cnt, (const double *)nullptr,
                       B.eps, B.mcount + 2, B.flags);
  else if (nc <= 4 * kRedThreads)
    hipLaunchKernelGGL((k_eps_cg_regs<4, 0>), dim3(1), dim3(kRedThreads), psb, L.st,
                       (const int *)B.mcount, (const int *)B.ell_col, (const double *)B.ell_val,
                       (const int *)B.ell_cnt, (const double *)nullptr, B.eps, B.mcount + 2,
                       B.flags);
  else
    hipLaunchKernelGGL(k_eps_cg, dim3(1), dim3(kRedThreads), 0, L.st, B.mcount,
                       (const int *)B.ell_col, (const double *)B.ell_val, (const int *)B.ell_cnt,
                       B.eps, B.ev[0], B.ev[1], B.ev[2], B.flags);
  if (save_eps)
    hipLaunchKernelGGL(k_eps_save, dim3(nblk(nc, 256)), dim3(256), 0, L.st,
                       (const int *)B.mcount, (const int *)B.ids, (const double *)B.eps, B.ceps);
}

bool shape_supported(int nc) { return nc <= 4 * kRedThreads; }


void run_shape_clear(const Launch &L, const Bufs &B, int nc) {
  hipLaunchKernelGGL(k_shape_clear, dim3(nblk(27 * (int64_t)nc, 256)), dim3(256), 0, L.st, nc,
                     B.wbar, B.epsbar);
}

void run_shape_gradient(const Launch &L, const Bufs &B, int nc, double *X_bar) {
  const int nslot = (L.g.dim == 3) ? 27 : 9;
  // lambda = A^{-1} epsbar, from zero
  run_fill(L, B.lam_g, nc, 0.0);
  const size_t psb = (size_t)nc * sizeof(double);
  if (nc <= 256)
    launch_eps_solve(L, B, nc, B.epsbar, B.lam_g, B.mcount + 3, nullptr, nullptr);
  else if (nc <= kRedThreads)
    hipLaunchKernelGGL((k_eps_cg_regs<1, kEpsRegNnz>), dim3(1), dim3(eps_threads(nc)), psb,
                       L.st, (const int *)B.mcount, (const int *)B.ell_col,
                       (const double *)B.ell_val, (const int *)B.ell_cnt,
                       (const double *)B.epsbar, B.lam_g, B.mcount + 3, B.flags);
  else
    hipLaunchKernelGGL((k_eps_cg_regs<4, 0>), dim3(1), dim3(kRedThreads), psb, L.st,
                       (const int *)B.mcount, (const int *)B.ell_col, (const double *)B.ell_val,
                       (const int *)B.ell_cnt, (const double *)B.epsbar, B.lam_g, B.mcount + 3,
                       B.flags);
  hipLaunchKernelGGL(k_shape_cellsums, dim3(nblk((int64_t)nc * nslot, 256)), dim3(256), 0, L.st,
                     (const int *)B.mcount, (const int *)B.seg, (const uint64_t *)B.keys,
                     (const double *)B.pw, nslot, (const double *)B.eps,
                     (const double *)B.lam_g, B.gsum);
  hipLaunchKernelGGL(k_shape_grad, dim3(nblk(nc, 128)), dim3(128), 0, L.st, L.g,
                     (const int *)B.mcount, (const double *)B.X, (const int *)B.ids,
                     (const double *)B.eps, (const double *)B.lam_g, (const double *)B.gsum,
                     B.wbar, B.epsbar, X_bar);
}

// Launches kernel template K<DIM, S> for the context's dimension and precision.
#define MK_DISPATCH(L, ...)                      \
  do {                                           \
    if ((L).g.dim == 2 && (L).prec == 0) {       \
      constexpr int DIM = 2;                     \
      using S = double;                          \
      __VA_ARGS__;                               \
    } else if ((L).g.dim == 2) {                 \
      constexpr int DIM = 2;                     \
      using S = float;                           \
      __VA_ARGS__;                               \
    } else if ((L).prec == 0) {                  \
      constexpr int DIM = 3;                     \
      using S = double;                          \
      __VA_ARGS__;                               \
    } else {                                     \
      constexpr int DIM = 3;                     \
      using S = float;                           \
      __VA_ARGS__;                               \
    }                                            \
  } while (0)

void run_interp_force(const Launch &L, const Bufs &B, double *hist_row) {
  MK_DISPATCH(L, {
    hipLaunchKernelGGL((k_interp_force<DIM, S>), dim3(nblk(L.nc_cap, 128)), dim3(128), 0, L.st,
                       L.g, (const int *)B.mcount, (const int64_t *)B.pcell, (const double *)B.pw,
                       (const S *)B.rho_s, (const S *)B.mom_s[0], (const S *)B.mom_s[1],
                       (const S *)B.mom_s[2], (const S *)B.E_s, (const double *)B.Ud,
                       (const double *)B.Tw, (const double *)B.eps, B.mk, B.mforce, B.mheat);
  });
  hipLaunchKernelGGL(k_totals, dim3(1), dim3(kRedThreads), 0, L.st, (const int *)B.mcount,
                     (const double *)B.mforce, (const double *)B.mheat, B.totals, hist_row);
}

void run_markers_step(const Launch &L, const Bufs &B, double *hist_row) {
  if (L.nc_cap > kFusedMarkers) {
    run_interp_force(L, B, hist_row);
    run_spread(L, B);
    return;
  }
  MK_DISPATCH(L, {
    hipLaunchKernelGGL((k_markers_fused<DIM, S>), dim3(1), dim3(kRedThreads), 0, L.st, L.g,
                       (const int *)B.mcount, (const int64_t *)B.pcell, (const double *)B.pw,
                       (const int *)B.seg, (const uint64_t *)B.keys, spread_set<S>(B),
                       (const double *)B.Ud, (const double *)B.Tw, (const double *)B.eps, B.mk,
                       B.mforce, B.mheat, B.totals, hist_row);
  });
}

void run_heat_flux(const Launch &L, const Bufs &B, int nc, double *q, int *status) {
  hipLaunchKernelGGL(k_heat_flux, dim3(1), dim3(256), 0, L.st, nc, B.mcount, B.cdA, B.dA,
                     B.mheat, q, status);
}

void run_spread(const Launch &L, const Bufs &B) {
  const int nslot = (L.g.dim == 3) ? 27 : 9;
  const int64_t cap = (int64_t)L.nc_cap * nslot;
  MK_DISPATCH(L, {
    hipLaunchKernelGGL((k_spread<DIM, S>), dim3(nblk(cap, 256)), dim3(256), 0, L.st, L.g,
                       (const int *)B.mcount, (const int *)B.seg, (const uint64_t *)B.keys,
                       (const double *)B.pw, (const double *)B.eps, (const double *)B.mk,
                       spread_set<S>(B));
  });
}

}  // namespace ibmk
