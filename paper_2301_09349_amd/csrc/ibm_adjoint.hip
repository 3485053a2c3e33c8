// ibm_adjoint.hip -- hand-written discrete adjoint of one IBM-HT step (FP64,
// linear convection, markers at rest). The step's forward pieces are recomputed
// from the tape (the state the step started from and its pressure solution);
// these kernels then run the transposed operations in reverse order:
//   correction -> pressure CG (symmetric operator: one more CG solve) -> set-up
//   -> forcing and spreading (spreading transposes to an interpolation and the
//   interpolation to an unweighted spread) -> predictor.
// Every transpose is written as a gather: a kernel owns the outputs it writes and
// reads the cotangents that reach them in a fixed order, so there are no atomics
// and results are bitwise repeatable. The predictor's transpose works on a padded
// grid with one ghost layer as real entries, then folds the ghost entries back
// onto the cells they mirror.
#include <algorithm>

#include "ibm_launch.h"

namespace ibmk {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ double mu_law_d(const GridK &g, double th) {
  if (g.visc == MU_CONSTANT) return g.mu_inf;
  return g.mu_inf * th * sqrt(th) * (1.0 + g.S) / (th + g.S);
}
// d mu / d theta of Sutherland's law: mu (3 / (2 theta) - 1 / (theta + S))
__device__ __forceinline__ double dmu_law_d(const GridK &g, double th) {
  if (g.visc == MU_CONSTANT) return 0.0;
  return mu_law_d(g, th) * (1.5 / th - 1.0 / (th + g.S));
}

// Factor of the mirror value in the ghost rule of one side (the affine constant
// carries no cotangent).
__device__ __forceinline__ double side_sigma(const GridK &g, int bc, int var, int d) {
  if (bc == BC_INFLOW) return ((var >= V_U0 && var < V_U0 + 3) || var == V_TH) ? -1.0 : 1.0;
  if (bc == BC_OUTFLOW) return (var == V_P) ? -1.0 : 1.0;
  if (bc == BC_SLIP) return (var == V_U0 + d) ? -1.0 : 1.0;
  return 1.0;
}

// Padded grid: kPad ghost layers per active direction (the van Leer face value
// reads the far-upwind cell, two layers out at a boundary face), index
// (i + kPad) + (n0 + 2 kPad) * (...).
constexpr int kPad = 2;
__host__ __device__ __forceinline__ int64_t padded_count(const GridK &g) {
  return (int64_t)(g.n[0] + 2 * kPad) * (g.n[1] + 2 * kPad) *
         (g.dim == 3 ? g.n[2] + 2 * kPad : 1);
}
__device__ __forceinline__ int64_t pidx(const GridK &g, int i, int j, int k) {
  return (i + kPad) + (int64_t)(g.n[0] + 2 * kPad) *
                          ((j + kPad) + (int64_t)(g.n[1] + 2 * kPad) * (g.dim == 3 ? k + kPad : 0));
}
// Padded linear index t back to (i, j, k).
template <int DIM>
__device__ __forceinline__ void padded_cell(const GridK &g, int64_t t, int *X) {
  const int pn0 = g.n[0] + 2 * kPad, pn1 = g.n[1] + 2 * kPad;
  X[0] = (int)(t % pn0) - kPad;
  X[1] = (int)((t / pn0) % pn1) - kPad;
  X[2] = (DIM == 3) ? (int)(t / ((int64_t)pn0 * pn1)) - kPad : 0;
}

// van Leer face value from the upwind (C), downwind (D) and far-upwind (U)
// values, as the predictor forms it, with its partial derivatives. Where the
// limiter is off (a b <= 0) the value is phi_C: the almost-everywhere derivative
// is 1 in C and 0 elsewhere.
__device__ __forceinline__ double vanleer_d(double C, double D, double U, double &dC, double &dD,
                                            double &dU) {
  const double a = C - U, b = D - C, ab = a * b;
  if (ab > 0.0) {
    const double s = a + b, is2 = 1.0 / (s * s);
    const double a2 = a * a * is2, b2 = b * b * is2;
    dC = 1.0 + b2 - a2;
    dD = a2;
    dU = -b2;
    return C + ab / s;
  }
  dC = 1.0;
  dD = 0.0;
  dU = 0.0;
  return C;
}

__device__ __forceinline__ bool face_entry_valid(const GridK &g, int d, const int *f) {
  for (int e = 0; e < g.dim; ++e) {
    if (e == d) {
      if (f[e] < 0 || f[e] > g.n[e]) return false;
    } else if (f[e] < 0 || f[e] >= g.n[e]) {
      return false;
    }
  }
  return true;
}

// Transpose of the centred difference G_q (with the ghost rule of `var`) at cell c:
// sum over the cells Y whose G_q reads a value resolving to c.
template <int DIM>
__device__ __forceinline__ double gct(const GridK &g, const double *v, int var, int q, const int *c) {
  const int n = g.n[q];
  const bool per = g.bc[q][0] == BC_PERIODIC;
  const double hh = 0.5 * g.ih[q];
  double acc = 0.0;
  for (int s = 1; s >= -1; s -= 2) {
    int Y[3] = {c[0], c[1], c[2]};
    Y[q] -= s;  // Y + s e_q = c
    if (per) Y[q] = (Y[q] + n) % n;
    if (per || (Y[q] >= 0 && Y[q] < n)) acc += s * hh * v[cidx(g, Y[0], Y[1], Y[2])];
    if (!per) {
      const int z = c[q] + s;  // c reads its own ghost at c + s e_q
      if (z < 0 || z >= n) {
        const int side = z < 0 ? 0 : 1;
        acc += s * hh * side_sigma(g, g.bc[q][side], var, q) * v[cidx(g, c[0], c[1], c[2])];
      }
    }
  }
  return acc;
}

// Transpose of the face gradient delta_f (pressure ghost rule) at cell c for the
// face entries of direction d: entries whose P or Q resolves to c.
template <int DIM>
__device__ __forceinline__ double dft(const GridK &g, const double *fb, int d, const int *c) {
  const int n = g.n[d];
  const bool per = g.bc[d][0] == BC_PERIODIC;
  const double ih = g.ih[d];
  int e[3] = {c[0], c[1], c[2]};
  double acc = 0.0;
  // lower entry (Q = c)
  acc += fb[fidx(g, d, e[0], e[1], e[2])] * ih;
  if (!per && c[d] == 0) acc -= side_sigma(g, g.bc[d][0], V_P, d) * fb[fidx(g, d, e[0], e[1], e[2])] * ih;
  // upper entry (P = c)
  e[d] = c[d] + 1;
  acc -= fb[fidx(g, d, e[0], e[1], e[2])] * ih;
  if (!per && c[d] == n - 1) acc += side_sigma(g, g.bc[d][1], V_P, d) * fb[fidx(g, d, e[0], e[1], e[2])] * ih;
  if (per) {
    if (c[d] == 0) {  // entry n has Q = n, which wraps to c
      e[d] = n;
      acc += fb[fidx(g, d, e[0], e[1], e[2])] * ih;
    }
    if (c[d] == n - 1) {  // entry 0 has P = -1, which wraps to c
      e[d] = 0;
      acc -= fb[fidx(g, d, e[0], e[1], e[2])] * ih;
    }
  }
  return acc;
}

template <int DIM>
__device__ __forceinline__ bool cell_of_linear(const GridK &g, int64_t t, int &i, int &j, int &k) {
  if (t >= g.N) return false;
  i = (int)(t % g.n[0]);
  int64_t r = t / g.n[0];
  j = (int)(r % g.n[1]);
  k = (int)(r / g.n[1]);
  return true;
}

struct SBar {  // a state cotangent in the ibm_set_state layout
  const double *rho, *mom[3], *E, *F[3];
};
struct SBarW {
  double *rho, *mom[3], *E, *F[3];
};

// ------------------------------------------------ R1: correction transpose
// Cotangent of the corrected face flux, per face entry: F^{n+1} feeds the state
// directly and rho^{n+1} = rho^n - dt D(F^{n+1}), whose cotangent is
// rhoT = rho_bar' + E_bar' c_v theta** (E^{n+1} = rho^{n+1} c_v theta**).
template <int DIM, typename S>
__global__ void k_adj_corr_face(GridK g, int d, SBar sb, const S *rho_s, const S *E_s,
                                double *fbar) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= g.NF[d]) return;
  int fc[3] = {(int)(f % g.fn[d][0]), (int)((f / g.fn[d][0]) % g.fn[d][1]),
               (int)(f / ((int64_t)g.fn[d][0] * g.fn[d][1]))};
  const int fd = fc[d], n = g.n[d];
  auto rT = [&](int64_t c) {
    const double th = E_s[c] / (rho_s[c] * g.cv);
    return sb.rho[c] + sb.E[c] * g.cv * th;
  };
  double acc = 0.0;
  if (fd >= 1) {
    int P[3] = {fc[0], fc[1], fc[2]};
    P[d] -= 1;
    acc += rT(cidx(g, P[0], P[1], P[2]));
  }
  if (fd <= n - 1) acc -= rT(cidx(g, fc[0], fc[1], fc[2]));
  fbar[f] = sb.F[d][f] - g.dt * g.ih[d] * acc;
}

// Per cell: rho_bar (init), theta**_bar, and the right-hand side of the adjoint
// pressure equation: p_bar = -dt sum_q G_q^T(m_bar') - dt sum_d delta_f^T(F_bar).
template <int DIM, typename S>
__global__ void k_adj_corr_cell(GridK g, StateV<S> st, SBar sb, SBarW so, const S *rho_s,
                                const S *E_s, const S *Fh0, const S *Fh1, const S *Fh2,
                                const double *x, const double *fb0,
                                const double *fb1, const double *fb2, double *tbar, double *rhs) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_of_linear<DIM>(g, t, i, j, k)) return;
  const int c3[3] = {i, j, k};
  const int64_t c = cidx(g, i, j, k);
  const S *Fh[3] = {Fh0, Fh1, Fh2};
  const double *fb[3] = {fb0, fb1, fb2};
  const double dt = g.dt;
  const double th = E_s[c] / (rho_s[c] * g.cv);
  const double rT = sb.rho[c] + sb.E[c] * g.cv * th;
  so.rho[c] = rT;
#pragma unroll
  for (int q = 0; q < DIM; ++q) so.mom[q][c] = 0.0;
  so.E[c] = 0.0;
  // rho^{n+1}, recomputed as in the correction
  auto pres = [&](int a, int b2, int c2) {
    Resolved r = resolve<DIM>(g, a, b2, c2);
    return ghosted<DIM>(g, r, V_P, x[r.c]);
  };
  const double xc = pres(i, j, k);
  double div = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
    lo[d] -= 1;
    hi[d] += 1;
    const double xl = pres(lo[0], lo[1], lo[2]), xh = pres(hi[0], hi[1], hi[2]);
    const double Fl = Fh[d][fidx(g, d, i, j, k)] - dt * ((xc - xl) * g.ih[d]);
    const double Fu = Fh[d][fidx(g, d, hi[0], hi[1], hi[2])] - dt * ((xh - xc) * g.ih[d]);
    div += (Fu - Fl) * g.ih[d];
  }
  const double rn = st.rho[c] - dt * div;
  tbar[c] = sb.E[c] * g.cv * rn;
  double pb = 0.0;
#pragma unroll
  for (int q = 0; q < DIM; ++q) pb -= dt * gct<DIM>(g, sb.mom[q], V_P, q, c3);
#pragma unroll
  for (int d = 0; d < DIM; ++d) pb -= dt * dft<DIM>(g, fb[d], d, c3);
  rhs[c] = pb;
}

// ------------------------------------------------------ R2: adjoint pressure
// Start of the solve A lambda = rhs from the lambda of the previous adjoint step
// (the next step in time, whose solution is close), scaled by the c that minimises
// |rhs - c A lambda| so that the start is never worse than lambda = 0 (a start of
// another objective's scale would otherwise limit the attainable accuracy).
// First pass: a = A lambda into r, partials of rhs.a and a.a.
template <int DIM, typename S>
__global__ __launch_bounds__(kBlockThreads) void k_adj_cg_guess(GridK g, const S *psi,
                                                           const double *rhs, const double *lam,
                                                           double *r, double *partials) {
  __shared__ double lds[32];
  double sums[2] = {0.0, 0.0};
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    const double a = helm_at<DIM>(g, psi, [&](int64_t q) { return lam[q]; }, i, j, k, c, lam[c]);
    r[c] = a;
    sums[0] += rhs[c] * a;
    sums[1] += a * a;
  }
  block_sum_n<2>(sums, lds);
  if (threadIdx.x == 0) {
    partials[PART_SA * kMaxBlocks + blockIdx.x] = sums[0];
    partials[PART_AA * kMaxBlocks + blockIdx.x] = sums[1];
  }
}

// Second pass: lambda = c lambda, r0 = rhs - c a; partial b.b (the CG's own start,
// w0 = A r0, follows).
template <int DIM>
__global__ __launch_bounds__(kBlockThreads) void k_adj_cg_init(GridK g, const double *rhs, double *r,
                                                          double *lam, double *partials,
                                                          CgScal *cs, int tag) {
  __shared__ double lds[32];
  double sa[2];
  sum_partials2(partials + PART_SA * kMaxBlocks, partials + PART_AA * kMaxBlocks, gridDim.x, lds,
                sa);
  const double cf = sa[1] > 0.0 ? sa[0] / sa[1] : 0.0;
  double s = 0.0;
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    const double v = rhs[c];
    r[c] = v - cf * r[c];
    lam[c] *= cf;
    s += v * v;
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) {
    partials[PART_BB * kMaxBlocks + blockIdx.x] = s;
    if (blockIdx.x == 0) {
      cs->done = 0;
      cs->iters = 0;
      cs->step_tag = tag;
      cs->xfinal = 0;
    }
  }
}

// ------------------------------------------------------ R3: set-up transpose
// Per cell: total m^_bar (m_bar' plus the transpose of F^ = lin_f(m^) against
// F^_bar = F_bar - dt D^T(lambda)), rho_bar += lambda and the inflow terms; the
// transposes of psi = 1/(R theta**) and theta** = E**/(rho* c_v).
template <int DIM, typename S>
__global__ void k_adj_setup_a(GridK g, SBar sb, SBarW so, const S *rho_s, const S *E_s,
                              const double *x, const double *lam, const double *fb0,
                              const double *fb1, const double *fb2, const double *tbar,
                              double *ms0, double *ms1, double *ms2, double *Es_bar,
                              double *rs_bar) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_of_linear<DIM>(g, t, i, j, k)) return;
  const int64_t c = cidx(g, i, j, k);
  const double *fb[3] = {fb0, fb1, fb2};
  double *msb[3] = {ms0, ms1, ms2};
  const double dt = g.dt;
  double rb = lam[c];
  // F^_bar at entry e of direction d: F_bar - dt ih (lambda_P [e_d >= 1] - lambda_Q [e_d <= n-1])
  auto Fht = [&](int d, int ed) {
    int e[3] = {i, j, k};
    e[d] = ed;
    double a = 0.0;
    if (ed >= 1) {
      int P[3] = {e[0], e[1], e[2]};
      P[d] -= 1;
      a += lam[cidx(g, P[0], P[1], P[2])];
    }
    if (ed <= g.n[d] - 1) a -= lam[cidx(g, e[0], e[1], e[2])];
    return fb[d][fidx(g, d, e[0], e[1], e[2])] - dt * g.ih[d] * a;
  };
  const int c3[3] = {i, j, k};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int n = g.n[d], cd = c3[d];
    double mhb = sb.mom[d][c];
    if (g.bc[d][0] == BC_PERIODIC) {
      mhb += 0.5 * Fht(d, cd) + 0.5 * Fht(d, cd + 1);
      if (cd == 0) mhb += 0.5 * Fht(d, n);
      if (cd == n - 1) mhb += 0.5 * Fht(d, 0);
    } else {
      if (cd >= 1) {
        mhb += 0.5 * Fht(d, cd);
      } else {
        const int b = g.bc[d][0];
        if (b == BC_INFLOW) rb += Fht(d, 0) * g.U_inf[d];
        else if (b == BC_OUTFLOW) mhb += Fht(d, 0);
      }
      if (cd + 1 <= n - 1) {
        mhb += 0.5 * Fht(d, cd + 1);
      } else {
        const int b = g.bc[d][1];
        if (b == BC_INFLOW) rb += Fht(d, n) * g.U_inf[d];
        else if (b == BC_OUTFLOW) mhb += Fht(d, n);
      }
    }
    msb[d][c] = mhb;
  }
  so.rho[c] += rb;
  const double th = E_s[c] / (rho_s[c] * g.cv);
  const double psib = -lam[c] * x[c];
  const double tb = tbar[c] + psib * (-1.0 / (g.R * th * th));
  Es_bar[c] = tb / (rho_s[c] * g.cv);
  rs_bar[c] = -tb * th / rho_s[c];
}

// E_bar += (gamma-1) dt sum_q G_q^T(m^_bar): p^n = (gamma-1) E^n enters m^.
template <int DIM>
__global__ void k_adj_setup_b(GridK g, const double *ms0, const double *ms1, const double *ms2,
                              SBarW so) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_of_linear<DIM>(g, t, i, j, k)) return;
  const int c3[3] = {i, j, k};
  const double *msb[3] = {ms0, ms1, ms2};
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < DIM; ++q) acc += gct<DIM>(g, msb[q], V_P, q, c3);
  so.E[cidx(g, i, j, k)] += g.gm1 * g.dt * acc;
}

// ---------------------------------------- R4: forcing and spreading transpose
// Per marker: Q_bar and F_bar from the interpolated E**_bar and m**_bar (spreading
// transposed, weighted by eps) and the output seeds; then the forcing formulas
// transposed; T_w_bar of the marker's candidate.
__global__ void k_adj_markers(GridK g, const int *mcount, const int64_t *pcell, const double *pw,
                              int nslot, const double *ms0, const double *ms1, const double *ms2,
                              const double *Es_bar, const double *eps, const double *Ud,
                              const double *Tw, const double *mk, const int *ids, double sFx,
                              double sFy, double sFz, double sH, double *mkbar, double *Tw_bar,
                              double *epsbar) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= mcount[0]) return;
  const int dim = g.dim, W = 2 * dim + 3;
  const double *msb[3] = {ms0, ms1, ms2};
  double eint = 0.0, mint[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < nslot; ++s) {
    const int64_t c = pcell[27 * k + s];
    const double w = pw[27 * k + s];
    eint += w * Es_bar[c];
    for (int q = 0; q < dim; ++q) mint[q] += w * msb[q][c];
  }
  const double e = eps[k], dt = g.dt;
  const double seeds[3] = {sFx, sFy, sFz};
  const double Qb = dt * e * eint + g.dV * e * sH;
  double Fb[3], rLb = 0.0;
  for (int q = 0; q < dim; ++q) {
    Fb[q] = dt * e * mint[q] - g.dV * e * seeds[q];
    rLb += Ud[3 * k + q] * Fb[q] / dt;
  }
  rLb += g.cv * Tw[k] * Qb / dt;
  const double rhoL = mk[(int64_t)W * k];
  Tw_bar[ids[k]] += g.cv * rhoL * Qb / dt;
  if (epsbar) {
    // eps_k enters the spread (f = sum w eps F) and the body totals
    const double *mf = mk + (int64_t)W * k;
    double eb = dt * mf[2 + 2 * dim] * eint + g.dV * sH * mf[2 + 2 * dim];
    for (int q = 0; q < dim; ++q)
      eb += dt * mf[2 + dim + q] * mint[q] - g.dV * seeds[q] * mf[2 + dim + q];
    epsbar[k] += eb;
  }
  double *o = mkbar + (int64_t)W * k;
  o[0] = rLb;
  for (int q = 0; q < dim; ++q) o[1 + q] = -Fb[q] / dt;
  o[1 + dim] = -Qb / dt;
}

// Cotangent of every kernel weight w_ck of the step (added to wbar): through the
// spread f_c = sum_k w_ck eps_k F_k (and the heat), and through the interpolation
// rho_L = sum_c w_ck rho*_c (and M, E_L) of the predictor fields pf at the pair.
__global__ void k_adj_shape_pairs(GridK g, const int *mcount, const int64_t *pcell, int nslot,
                                  const double *ms0, const double *ms1, const double *ms2,
                                  const double *Es_bar, const double *eps, const double *mk,
                                  const double *mkbar, const double *pf, double *wbar) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = (int)(p / nslot), slot = (int)(p - (int64_t)k * nslot);
  if (k >= mcount[0]) return;
  const int dim = g.dim, W = 2 * dim + 3;
  const double *msb[3] = {ms0, ms1, ms2};
  const int64_t c = pcell[27 * k + slot];
  const double *mf = mk + (int64_t)W * k, *mb = mkbar + (int64_t)W * k;
  const double *f = pf + (int64_t)(27 * k + slot) * (dim + 2);
  double sp = mf[2 + 2 * dim] * Es_bar[c];
  double ip = mb[0] * f[0] + mb[1 + dim] * f[1 + dim];
  for (int q = 0; q < dim; ++q) {
    sp += mf[2 + dim + q] * msb[q][c];
    ip += mb[1 + q] * f[1 + q];
  }
  wbar[27 * k + slot] += g.dt * eps[k] * sp + ip;
}

// The predictor fields (before the spread) at every pair, for k_adj_shape_pairs.
template <typename S>
__global__ void k_pair_fields(GridK g, const int *mcount, const int64_t *pcell, int nslot,
                              const S *rho_s, const S *m0, const S *m1, const S *m2, const S *E_s,
                              double *pf) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = (int)(p / nslot), slot = (int)(p - (int64_t)k * nslot);
  if (k >= mcount[0]) return;
  const int dim = g.dim;
  const S *ms[3] = {m0, m1, m2};
  const int64_t c = pcell[27 * k + slot];
  double *f = pf + (int64_t)(27 * k + slot) * (dim + 2);
  f[0] = double(rho_s[c]);
  for (int q = 0; q < dim; ++q) f[1 + q] = double(ms[q][c]);
  f[1 + dim] = double(E_s[c]);
}

// Interpolation transposed: an unweighted spread of the marker cotangents, by
// the same sorted segments as the forward spread.
__global__ void k_adj_spread_t(GridK g, const int *mcount, const int *seg, const uint64_t *keys,
                               const double *pw, int nslot, const double *mkbar, double *rs_bar,
                               double *ms0, double *ms1, double *ms2, double *Es_bar) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= mcount[1]) return;
  const int dim = g.dim, W = 2 * dim + 3;
  const int a = seg[s], b = seg[s + 1];
  const int64_t cell = (int64_t)(keys[a] >> kPairBits);
  const uint64_t mask = (1ull << kPairBits) - 1;
  double ar = 0.0, am[3] = {0.0, 0.0, 0.0}, ae = 0.0;
  for (int p = a; p < b; ++p) {
    const int pid = (int)(keys[p] & mask);
    const int k = pid / nslot, slot = pid - k * nslot;
    const double w = pw[27 * k + slot];
    const double *o = mkbar + (int64_t)W * k;
    ar += w * o[0];
    for (int q = 0; q < dim; ++q) am[q] += w * o[1 + q];
    ae += w * o[1 + dim];
  }
  double *msb[3] = {ms0, ms1, ms2};
  rs_bar[cell] += ar;
  for (int q = 0; q < dim; ++q) msb[q][cell] += am[q];
  Es_bar[cell] += ae;
}

// ------------------------------------------------- R5: predictor transpose
// Primitives on the padded grid (ghost rules applied), as the predictor sees them.
template <int DIM, typename S>
__global__ void k_adj_prims(GridK g, StateV<S> st, double *pp) {
  const int64_t Np = padded_count(g);
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Np) return;
  int X[3];
  padded_cell<DIM>(g, t, X);
  Resolved r = resolve<DIM>(g, X[0], X[1], X[2]);
  const double rho = st.rho[r.c];
  const double inv = 1.0 / rho;
  double u[3];
#pragma unroll
  for (int q = 0; q < DIM; ++q) u[q] = st.mom[q][r.c] * inv;
  const double E = st.E[r.c];
  double th = E * inv * g.inv_cv, p = g.gm1 * E, rr = rho;
  if (any_side<DIM, double>(r)) {
    rr = ghosted<DIM>(g, r, V_RHO, rr);
#pragma unroll
    for (int q = 0; q < DIM; ++q) u[q] = ghosted<DIM>(g, r, V_U0 + q, u[q]);
    th = ghosted<DIM>(g, r, V_TH, th);
    p = ghosted<DIM>(g, r, V_P, p);
  }
  pp[t] = rr;
#pragma unroll
  for (int q = 0; q < DIM; ++q) pp[(1 + q) * Np + t] = u[q];
  pp[(DIM + 1) * Np + t] = th;
  pp[(DIM + 2) * Np + t] = mu_law_d(g, th);
  pp[(DIM + 3) * Np + t] = p;
}

// Per face entry of direction d: the face fluxes recomputed, their cotangents
// from the cells that read the entry, and the local reverse. Stored per face:
// u_bar at P [dim], u_bar at Q [dim], theta_bar at P, Q, half mu_bar, half
// rho_bar, and per tangential direction t the cotangents A_t (of the face average
// of d u_d/d x_t) and B_t (of d u_t / d x_t in the face divergence), each shared by
// the centred differences at P and Q; with van Leer convection also u_bar [dim]
// and theta_bar at the far-upwind cell. The state face-flux cotangent is written.
template <int DIM, typename S>
__global__ void k_adj_faces(GridK g, int d, StateV<S> st, const double *pp,
                            const double *rs_bar, const double *ms0, const double *ms1,
                            const double *ms2, const double *Es_bar, double *fo, int64_t NFtot,
                            int64_t foff, double *Fbar_out) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= g.NF[d]) return;
  const int64_t Np = padded_count(g);
  const double *msb[3] = {ms0, ms1, ms2};
  int Q[3] = {(int)(f % g.fn[d][0]), (int)((f / g.fn[d][0]) % g.fn[d][1]),
              (int)(f / ((int64_t)g.fn[d][0] * g.fn[d][1]))};
  int P[3] = {Q[0], Q[1], Q[2]};
  P[d] -= 1;
  const int64_t iP = pidx(g, P[0], P[1], P[2]), iQ = pidx(g, Q[0], Q[1], Q[2]);
  const double rP = pp[iP], rQ = pp[iQ];
  double uP[3], uQ[3];
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    uP[q] = pp[(1 + q) * Np + iP];
    uQ[q] = pp[(1 + q) * Np + iQ];
  }
  const double thP = pp[(DIM + 1) * Np + iP], thQ = pp[(DIM + 1) * Np + iQ];
  const double muP = pp[(DIM + 2) * Np + iP], muQ = pp[(DIM + 2) * Np + iQ];
  const double F = st.F[d][f];
  const double dt = g.dt, ih = g.ih[d], cv = g.cv;
  const double lr = 0.5 * (rP + rQ);
  const double U = F / lr;
  const double muf = 0.5 * (muP + muQ);
  const double lamf = g.cp_Pr * muf;
  double dn[3], tg[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < DIM; ++q) dn[q] = (uQ[q] - uP[q]) * ih;
  double divf = dn[d];
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    if (t == d) continue;
    const double hh = 0.5 * g.ih[t];
    int a1[3] = {P[0], P[1], P[2]}, a0[3] = {P[0], P[1], P[2]};
    int b1[3] = {Q[0], Q[1], Q[2]}, b0[3] = {Q[0], Q[1], Q[2]};
    a1[t] += 1;
    a0[t] -= 1;
    b1[t] += 1;
    b0[t] -= 1;
    const int64_t ia1 = pidx(g, a1[0], a1[1], a1[2]), ia0 = pidx(g, a0[0], a0[1], a0[2]);
    const int64_t ib1 = pidx(g, b1[0], b1[1], b1[2]), ib0 = pidx(g, b0[0], b0[1], b0[2]);
    const double gdP = (pp[(1 + d) * Np + ia1] - pp[(1 + d) * Np + ia0]) * hh;
    const double gdQ = (pp[(1 + d) * Np + ib1] - pp[(1 + d) * Np + ib0]) * hh;
    const double gtP = (pp[(1 + t) * Np + ia1] - pp[(1 + t) * Np + ia0]) * hh;
    const double gtQ = (pp[(1 + t) * Np + ib1] - pp[(1 + t) * Np + ib0]) * hh;
    tg[t] = 0.5 * (gdP + gdQ);
    divf += 0.5 * (gtP + gtQ);
  }
  // convected face values (u and c_v theta) and their weights on P, Q and the
  // far-upwind cell (van Leer: P - e_d when F >= 0, else Q + e_d)
  double cu[3], wPu[3], wQu[3], wUu[3], ce, wPe, wQe, wUe;
  const bool vl = g.conv == CONV_VANLEER;
  if (!vl) {
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      cu[q] = 0.5 * (uP[q] + uQ[q]);
      wPu[q] = wQu[q] = 0.5;
      wUu[q] = 0.0;
    }
    ce = 0.5 * (cv * thP + cv * thQ);
    wPe = wQe = 0.5;
    wUe = 0.0;
  } else {
    const bool pos = F >= 0.0;
    int Uc[3] = {pos ? P[0] : Q[0], pos ? P[1] : Q[1], pos ? P[2] : Q[2]};
    Uc[d] += pos ? -1 : 1;
    const int64_t iU = pidx(g, Uc[0], Uc[1], Uc[2]);
    double dC, dD;
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      const double uU = pp[(1 + q) * Np + iU];
      // upwind and downwind operands chosen first: one limiter per value
      cu[q] = vanleer_d(pos ? uP[q] : uQ[q], pos ? uQ[q] : uP[q], uU, dC, dD, wUu[q]);
      wPu[q] = pos ? dC : dD;
      wQu[q] = pos ? dD : dC;
    }
    const double thU = pp[(DIM + 1) * Np + iU];
    ce = vanleer_d(cv * (pos ? thP : thQ), cv * (pos ? thQ : thP), cv * thU, dC, dD, wUe);
    wPe = pos ? dC : dD;
    wQe = pos ? dD : dC;
  }
  // cotangents of the entry's fluxes: the predictor's divergence at P (entry is
  // its upper face, when f_d >= 1) and at Q (its lower face, when f_d <= n-1)
  const bool wP = Q[d] >= 1, wQ = Q[d] <= g.n[d] - 1;
  const int64_t cP = wP ? cidx(g, P[0], P[1], P[2]) : 0, cQ = wQ ? cidx(g, Q[0], Q[1], Q[2]) : 0;
  const double a = -dt * ih;
  double FMb[3];
#pragma unroll
  for (int q = 0; q < DIM; ++q) FMb[q] = a * ((wP ? msb[q][cP] : 0.0) - (wQ ? msb[q][cQ] : 0.0));
  const double FEb = a * ((wP ? Es_bar[cP] : 0.0) - (wQ ? Es_bar[cQ] : 0.0));
  const double Fdir = a * ((wP ? rs_bar[cP] : 0.0) - (wQ ? rs_bar[cQ] : 0.0));
  const double Ub = a * ((wP ? g.gm1 * st.E[cP] * Es_bar[cP] : 0.0) -
                         (wQ ? g.gm1 * st.E[cQ] * Es_bar[cQ] : 0.0));
  // local reverse of the face fluxes
  double Fb = Fdir + FEb * ce + Ub / lr;
  double uPb[3], uQb[3];
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    Fb += FMb[q] * cu[q];
    uPb[q] = wPu[q] * FMb[q] * F;
    uQb[q] = wQu[q] * FMb[q] * F;
  }
  const double ceb = FEb * F;
  double thPb = wPe * cv * ceb, thQb = wQe * cv * ceb;
  const double lamfb = -FEb * (thQ - thP) * ih;
  thQb += -FEb * lamf * ih;
  thPb += FEb * lamf * ih;
  double mufb = 0.0, dnb[3] = {0.0, 0.0, 0.0}, tgb[3] = {0.0, 0.0, 0.0}, divfb = 0.0;
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    const double taub = -FMb[q];
    if (q != d) {
      mufb += taub * (dn[q] + tg[q]);
      dnb[q] += muf * taub;
      tgb[q] += muf * taub;
    } else {
      mufb += taub * (2.0 * dn[d] - (2.0 / 3.0) * divf);
      dnb[d] += 2.0 * muf * taub;
      divfb += -(2.0 / 3.0) * muf * taub;
    }
  }
  dnb[d] += divfb;
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    uQb[q] += dnb[q] * ih;
    uPb[q] -= dnb[q] * ih;
  }
  const double muh = 0.5 * (mufb + g.cp_Pr * lamfb);
  const double rhoh = 0.5 * (-Ub * U / lr);
  double *o = fo + foff + f;
  int v = 0;
#pragma unroll
  for (int q = 0; q < DIM; ++q) o[(int64_t)(v++) * NFtot] = uPb[q];
#pragma unroll
  for (int q = 0; q < DIM; ++q) o[(int64_t)(v++) * NFtot] = uQb[q];
  o[(int64_t)(v++) * NFtot] = thPb;
  o[(int64_t)(v++) * NFtot] = thQb;
  o[(int64_t)(v++) * NFtot] = muh;
  o[(int64_t)(v++) * NFtot] = rhoh;
#pragma unroll
  for (int t = 0; t < DIM; ++t)
    if (t != d) o[(int64_t)(v++) * NFtot] = 0.5 * tgb[t];  // A_t
#pragma unroll
  for (int t = 0; t < DIM; ++t)
    if (t != d) o[(int64_t)(v++) * NFtot] = 0.5 * divfb;  // B_t
  if (vl) {  // far-upwind u_bar [dim], theta_bar
#pragma unroll
    for (int q = 0; q < DIM; ++q) o[(int64_t)(v++) * NFtot] = wUu[q] * FMb[q] * F;
    o[(int64_t)(v++) * NFtot] = wUe * cv * ceb;
  }
  Fbar_out[f] = Fb;
}

// Per cell: reverse of the cell-centred terms. Viscous dissipation
// Phi = mu (sum_ab (g_ab + g_ba) g_ab - 2/3 (div u)^2) enters E* with dt;
// -dt G_b(p) enters m*_b; -dt p div(u_f) enters E*. Stored: g_bar [dim][dim],
// G_b(p)_bar [dim], the direct p_bar and mu_bar.
template <int DIM, typename S>
__global__ void k_adj_cells(GridK g, StateV<S> st, const double *pp, const double *ms0,
                            const double *ms1, const double *ms2, const double *Es_bar,
                            double *co) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_of_linear<DIM>(g, t, i, j, k)) return;
  const int64_t c = cidx(g, i, j, k), Np = padded_count(g), N = g.N;
  const double *msb[3] = {ms0, ms1, ms2};
  double gr[3][3];
#pragma unroll
  for (int b = 0; b < DIM; ++b) {
    int a1[3] = {i, j, k}, a0[3] = {i, j, k};
    a1[b] += 1;
    a0[b] -= 1;
    const int64_t i1 = pidx(g, a1[0], a1[1], a1[2]), i0 = pidx(g, a0[0], a0[1], a0[2]);
    const double hh = 0.5 * g.ih[b];
#pragma unroll
    for (int a = 0; a < DIM; ++a) gr[a][b] = (pp[(1 + a) * Np + i1] - pp[(1 + a) * Np + i0]) * hh;
  }
  double divu = 0.0, sgg = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) divu += gr[a][a];
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int b = 0; b < DIM; ++b) sgg += (gr[a][b] + gr[b][a]) * gr[a][b];
  const int64_t ic = pidx(g, i, j, k);
  const double muc = pp[(DIM + 2) * Np + ic];
  const double Phib = g.dt * Es_bar[c];
  int v = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int b = 0; b < DIM; ++b)
      co[(v++) * N + c] =
          Phib * muc * (2.0 * gr[a][b] + 2.0 * gr[b][a] - (a == b ? (4.0 / 3.0) * divu : 0.0));
#pragma unroll
  for (int b = 0; b < DIM; ++b) co[(v++) * N + c] = -g.dt * msb[b][c];
  // div(u_f) at the cell from the stored face fluxes
  double divU = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    int hi[3] = {i, j, k}, lo[3] = {i, j, k};
    hi[d] += 1;
    lo[d] -= 1;
    const double rc = pp[ic];
    const double rl = pp[pidx(g, lo[0], lo[1], lo[2])], rh = pp[pidx(g, hi[0], hi[1], hi[2])];
    const double Ul = st.F[d][fidx(g, d, i, j, k)] / (0.5 * (rl + rc));
    const double Uh = st.F[d][fidx(g, d, hi[0], hi[1], hi[2])] / (0.5 * (rc + rh));
    divU += (Uh - Ul) * g.ih[d];
  }
  co[(v++) * N + c] = -g.dt * divU * Es_bar[c];
  co[(v++) * N + c] = Phib * (sgg - (2.0 / 3.0) * divu * divu);
}

// Per padded cell X: every cotangent that reaches the primitives at X from the face
// reverses (own faces and faces that take centred differences through X) and the
// cell reverses of its neighbours; mu_bar is turned into theta_bar at X's theta.
template <int DIM, typename S>
__global__ void k_adj_gather(GridK g, StateV<S> st, const double *pp, const double *fo,
                             int64_t NFtot, int64_t foff0, int64_t foff1, int64_t foff2,
                             const double *co, double *pb) {
  const int64_t Np = padded_count(g);
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Np) return;
  int X[3];
  padded_cell<DIM>(g, t, X);
  const int64_t foff[3] = {foff0, foff1, foff2};
  const int64_t N = g.N;
  double rb = 0.0, ub[3] = {0.0, 0.0, 0.0}, thb = 0.0, mub = 0.0, ppb = 0.0;
  auto fv = [&](int d, const int *e, int v) {
    return fo[(int64_t)v * NFtot + foff[d] + fidx(g, d, e[0], e[1], e[2])];
  };
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    // own faces: lower entry (X is its Q), upper entry (X is its P)
    {
      int e[3] = {X[0], X[1], X[2]};
      if (face_entry_valid(g, d, e)) {
#pragma unroll
        for (int q = 0; q < DIM; ++q) ub[q] += fv(d, e, DIM + q);
        thb += fv(d, e, 2 * DIM + 1);
        mub += fv(d, e, 2 * DIM + 2);
        rb += fv(d, e, 2 * DIM + 3);
      }
      e[d] += 1;
      if (face_entry_valid(g, d, e)) {
#pragma unroll
        for (int q = 0; q < DIM; ++q) ub[q] += fv(d, e, q);
        thb += fv(d, e, 2 * DIM);
        mub += fv(d, e, 2 * DIM + 2);
        rb += fv(d, e, 2 * DIM + 3);
      }
    }
    // van Leer: X is the far-upwind cell of the entry X + 2 e_d when its flux is
    // >= 0 and of the entry X - e_d when its flux is < 0
    if (g.conv == CONV_VANLEER) {
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        int e[3] = {X[0], X[1], X[2]};
        e[d] += sd == 0 ? 2 : -1;
        if (!face_entry_valid(g, d, e)) continue;
        const bool pos = (double)st.F[d][fidx(g, d, e[0], e[1], e[2])] >= 0.0;
        if (pos != (sd == 0)) continue;
#pragma unroll
        for (int q = 0; q < DIM; ++q) ub[q] += fv(d, e, 4 * DIM + 2 + q);
        thb += fv(d, e, 5 * DIM + 2);
      }
    }
    // faces of direction d whose P or Q is X -/+ e_t
    int jt = 0;
#pragma unroll
    for (int tt = 0; tt < DIM; ++tt) {
      if (tt == d) continue;
      const double hh = 0.5 * g.ih[tt];
#pragma unroll
      for (int s = 1; s >= -1; s -= 2) {
        int Y[3] = {X[0], X[1], X[2]};
        Y[tt] -= s;
#pragma unroll
        for (int up = 0; up < 2; ++up) {  // entry with Q = Y, then entry with P = Y
          int e[3] = {Y[0], Y[1], Y[2]};
          e[d] += up;
          if (!face_entry_valid(g, d, e)) continue;
          ub[d] += s * hh * fv(d, e, 2 * DIM + 4 + jt);
          ub[tt] += s * hh * fv(d, e, 2 * DIM + 4 + (DIM - 1) + jt);
        }
      }
      ++jt;
    }
  }
  // cell-centred differences of interior neighbours Y = X - s e_b
#pragma unroll
  for (int b = 0; b < DIM; ++b) {
    const double hh = 0.5 * g.ih[b];
#pragma unroll
    for (int s = 1; s >= -1; s -= 2) {
      int Y[3] = {X[0], X[1], X[2]};
      Y[b] -= s;
      bool in = true;
#pragma unroll
      for (int e = 0; e < DIM; ++e) in = in && Y[e] >= 0 && Y[e] < g.n[e];
      if (!in) continue;
      const int64_t cy = cidx(g, Y[0], Y[1], Y[2]);
#pragma unroll
      for (int a = 0; a < DIM; ++a) ub[a] += s * hh * co[(a * DIM + b) * N + cy];
      ppb += s * hh * co[(DIM * DIM + b) * N + cy];
    }
  }
  bool xin = true;
#pragma unroll
  for (int e = 0; e < DIM; ++e) xin = xin && X[e] >= 0 && X[e] < g.n[e];
  if (xin) {
    const int64_t cx = cidx(g, X[0], X[1], X[2]);
    ppb += co[(DIM * DIM + DIM) * N + cx];
    mub += co[(DIM * DIM + DIM + 1) * N + cx];
  }
  thb += mub * dmu_law_d(g, pp[(DIM + 1) * Np + t]);
  pb[t] = rb;
#pragma unroll
  for (int q = 0; q < DIM; ++q) pb[(1 + q) * Np + t] = ub[q];
  pb[(DIM + 1) * Np + t] = thb;
  pb[(DIM + 2) * Np + t] = ppb;
}

// Per cell: the padded cotangents of the cell and of its ghost images (factor of
// each crossed side's rule), then the primitive-to-conserved transpose; the direct
// dependence of rho*, m*, E* on rho, m, E is added.
template <int DIM, typename S>
__global__ void k_adj_fold(GridK g, StateV<S> st, const double *pb, const double *rs_bar,
                           const double *ms0, const double *ms1, const double *ms2,
                           const double *Es_bar, SBarW so) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_of_linear<DIM>(g, t, i, j, k)) return;
  const int64_t c = cidx(g, i, j, k), Np = padded_count(g);
  const double *msb[3] = {ms0, ms1, ms2};
  const int c3[3] = {i, j, k};
  // per direction: own coordinate and the ghost positions (within kPad layers)
  // that resolve to it, each with the side it crosses (-1: none or periodic)
  int pos[3][1 + 2 * kPad], side[3][1 + 2 * kPad], cnt[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    pos[d][0] = c3[d];
    side[d][0] = -1;
    cnt[d] = 1;
    if (d >= DIM) continue;
    const int n = g.n[d];
    const bool per = g.bc[d][0] == BC_PERIODIC;
    for (int l = 1; l <= kPad; ++l) {
      // low ghost -l and high ghost n - 1 + l
      const int lo = per ? n - l : l - 1, hi = per ? l - 1 : n - l;
      if (lo == c3[d]) { pos[d][cnt[d]] = -l; side[d][cnt[d]] = per ? -1 : 0; ++cnt[d]; }
      if (hi == c3[d]) { pos[d][cnt[d]] = n - 1 + l; side[d][cnt[d]] = per ? -1 : 1; ++cnt[d]; }
    }
  }
  double rb = 0.0, ub[3] = {0.0, 0.0, 0.0}, thb = 0.0, ppb = 0.0;
  for (int a0 = 0; a0 < cnt[0]; ++a0)
    for (int a1 = 0; a1 < cnt[1]; ++a1)
      for (int a2 = 0; a2 < cnt[2]; ++a2) {
        const int sel[3] = {a0, a1, a2};
        double sr = 1.0, su[3] = {1.0, 1.0, 1.0}, sth = 1.0, sp = 1.0;
        int P[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          P[d] = pos[d][sel[d]];
          const int sd = side[d][sel[d]];
          if (sd >= 0) {
            const int b = g.bc[d][sd];
            sr *= side_sigma(g, b, V_RHO, d);
#pragma unroll
            for (int q = 0; q < DIM; ++q) su[q] *= side_sigma(g, b, V_U0 + q, d);
            sth *= side_sigma(g, b, V_TH, d);
            sp *= side_sigma(g, b, V_P, d);
          }
        }
        const int64_t ip = pidx(g, P[0], P[1], P[2]);
        rb += sr * pb[ip];
#pragma unroll
        for (int q = 0; q < DIM; ++q) ub[q] += su[q] * pb[(1 + q) * Np + ip];
        thb += sth * pb[(DIM + 1) * Np + ip];
        ppb += sp * pb[(DIM + 2) * Np + ip];
      }
  const double rho = st.rho[c], inv = 1.0 / rho;
  const double E = st.E[c];
  const double th = E * inv * g.inv_cv;
  double rtot = rb - thb * th * inv + rs_bar[c];
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    const double u = st.mom[q][c] * inv;
    rtot -= ub[q] * u * inv;
    so.mom[q][c] += ub[q] * inv + msb[q][c];
  }
  so.rho[c] += rtot;
  so.E[c] += thb * inv * g.inv_cv + g.gm1 * ppb + Es_bar[c];
}

// ------------------------------------------------------------------ launchers
static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename S>
static StateV<S> state_slot(const Bufs &B, int slot) {
  StateV<S> s;
  s.rho = (S *)B.rho[slot];
  s.E = (S *)B.E[slot];
  for (int q = 0; q < 3; ++q) {
    s.mom[q] = (S *)B.mom[slot][q];
    s.F[q] = (S *)B.F[slot][q];
  }
  return s;
}

static SBar sbar_of(const GridK &g, const double *p) {
  SBar s;
  s.rho = p;
  for (int q = 0; q < 3; ++q) s.mom[q] = q < g.dim ? p + (1 + q) * g.N : nullptr;
  s.E = p + (1 + g.dim) * g.N;
  int64_t off = (2 + g.dim) * g.N;
  for (int q = 0; q < 3; ++q) {
    s.F[q] = q < g.dim ? p + off : nullptr;
    if (q < g.dim) off += g.NF[q];
  }
  return s;
}
static SBarW sbarw_of(const GridK &g, double *p) {
  SBar r = sbar_of(g, p);
  SBarW s;
  s.rho = const_cast<double *>(r.rho);
  s.E = const_cast<double *>(r.E);
  for (int q = 0; q < 3; ++q) {
    s.mom[q] = const_cast<double *>(r.mom[q]);
    s.F[q] = const_cast<double *>(r.F[q]);
  }
  return s;
}

int64_t padded_cells(const GridK &g) { return padded_count(g); }

static int64_t face_total(const GridK &g) { return g.NF[0] + g.NF[1] + g.NF[2]; }
static int64_t face_off(const GridK &g, int d) {
  int64_t o = 0;
  for (int q = 0; q < d; ++q) o += g.NF[q];
  return o;
}

// Runs the body with DIM and the state's storage type S of the context.
#define ADJ_DISPATCH(L, ...)                \
  do {                                      \
    if ((L).g.dim == 2 && (L).prec == 0) {  \
      constexpr int DIM = 2;                \
      using S = double;                     \
      __VA_ARGS__;                          \
    } else if ((L).g.dim == 2) {            \
      constexpr int DIM = 2;                \
      using S = float;                      \
      __VA_ARGS__;                          \
    } else if ((L).prec == 0) {             \
      constexpr int DIM = 3;                \
      using S = double;                     \
      __VA_ARGS__;                          \
    } else {                                \
      constexpr int DIM = 3;                \
      using S = float;                      \
      __VA_ARGS__;                          \
    }                                       \
  } while (0)

void run_adj_correction(const Launch &L, const Bufs &B, int slot, const double *sb_in,
                        double *sb_out) {
  const GridK &g = L.g;
  SBar sb = sbar_of(g, sb_in);
  SBarW so = sbarw_of(g, sb_out);
  double *fb[3] = {B.fbar, B.fbar + g.NF[0], B.fbar + g.NF[0] + g.NF[1]};
  ADJ_DISPATCH(L, {
    for (int d = 0; d < DIM; ++d)
      hipLaunchKernelGGL((k_adj_corr_face<DIM, S>), dim3(nb256(g.NF[d])), dim3(256), 0, L.st, g,
                         d, sb, (const S *)B.rho_s, (const S *)B.E_s, fb[d]);
    hipLaunchKernelGGL((k_adj_corr_cell<DIM, S>), dim3(nb256(g.N)), dim3(256), 0, L.st, g,
                       state_slot<S>(B, slot), sb, so, (const S *)B.rho_s, (const S *)B.E_s,
                       (const S *)B.Fhat[0], (const S *)B.Fhat[1], (const S *)B.Fhat[2],
                       (const double *)B.x, (const double *)fb[0], (const double *)fb[1],
                       (const double *)fb[2], B.tbar, B.rhs);
  });
}

void run_adj_cg_init(const Launch &L, const Bufs &B, int tag) {
  ADJ_DISPATCH(L, {
    hipLaunchKernelGGL((k_adj_cg_guess<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads),
                       0, L.st, L.g, (const S *)B.psi, (const double *)B.rhs,
                       (const double *)B.lam, B.rv[0], B.partials);
    hipLaunchKernelGGL((k_adj_cg_init<DIM>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0,
                       L.st, L.g, (const double *)B.rhs, B.rv[0], B.lam, B.partials, B.cg, tag);
  });
  run_cg64_start(L, B);
}

void run_adj_setup(const Launch &L, const Bufs &B, int slot, const double *sb_in, double *sb_out) {
  (void)slot;
  const GridK &g = L.g;
  SBar sb = sbar_of(g, sb_in);
  SBarW so = sbarw_of(g, sb_out);
  const double *fb[3] = {B.fbar, B.fbar + g.NF[0], B.fbar + g.NF[0] + g.NF[1]};
  ADJ_DISPATCH(L, {
    hipLaunchKernelGGL((k_adj_setup_a<DIM, S>), dim3(nb256(g.N)), dim3(256), 0, L.st, g, sb, so,
                       (const S *)B.rho_s, (const S *)B.E_s, (const double *)B.x,
                       (const double *)B.lam, fb[0], fb[1], fb[2], (const double *)B.tbar,
                       B.ms_bar[0], B.ms_bar[1], B.ms_bar[2], B.Es_bar, B.rs_bar);
    hipLaunchKernelGGL((k_adj_setup_b<DIM>), dim3(nb256(g.N)), dim3(256), 0, L.st, g,
                       (const double *)B.ms_bar[0], (const double *)B.ms_bar[1],
                       (const double *)B.ms_bar[2], so);
  });
}

void run_adj_markers(const Launch &L, const Bufs &B, const double *out_bar, double *Tw_bar,
                     bool shape) {
  const int nslot = (L.g.dim == 3) ? 27 : 9;
  hipLaunchKernelGGL(k_adj_markers, dim3((unsigned)((L.nc_cap + 127) / 128)), dim3(128), 0, L.st,
                     L.g, (const int *)B.mcount, (const int64_t *)B.pcell, (const double *)B.pw,
                     nslot, (const double *)B.ms_bar[0], (const double *)B.ms_bar[1],
                     (const double *)B.ms_bar[2], (const double *)B.Es_bar, (const double *)B.eps,
                     (const double *)B.Ud, (const double *)B.Tw, (const double *)B.mk,
                     (const int *)B.ids, out_bar[0], out_bar[1], out_bar[2], out_bar[3], B.mkbar,
                     Tw_bar, B.epsbar);
  const int64_t cap = (int64_t)L.nc_cap * nslot;
  if (B.wbar && shape)
    hipLaunchKernelGGL(k_adj_shape_pairs, dim3(nb256(cap)), dim3(256), 0, L.st, L.g,
                       (const int *)B.mcount, (const int64_t *)B.pcell, nslot,
                       (const double *)B.ms_bar[0], (const double *)B.ms_bar[1],
                       (const double *)B.ms_bar[2], (const double *)B.Es_bar,
                       (const double *)B.eps, (const double *)B.mk, (const double *)B.mkbar,
                       (const double *)B.pfld, B.wbar);
  hipLaunchKernelGGL(k_adj_spread_t, dim3(nb256(cap)), dim3(256), 0, L.st, L.g,
                     (const int *)B.mcount, (const int *)B.seg, (const uint64_t *)B.keys,
                     (const double *)B.pw, nslot, (const double *)B.mkbar, B.rs_bar, B.ms_bar[0],
                     B.ms_bar[1], B.ms_bar[2], B.Es_bar);
}

void run_pair_fields(const Launch &L, const Bufs &B) {
  if (!B.pfld) return;
  const int nslot = (L.g.dim == 3) ? 27 : 9;
  const int64_t cap = (int64_t)L.nc_cap * nslot;
  if (L.prec == 0)
    hipLaunchKernelGGL((k_pair_fields<double>), dim3(nb256(cap)), dim3(256), 0, L.st, L.g,
                       (const int *)B.mcount, (const int64_t *)B.pcell, nslot,
                       (const double *)B.rho_s, (const double *)B.mom_s[0],
                       (const double *)B.mom_s[1], (const double *)B.mom_s[2],
                       (const double *)B.E_s, B.pfld);
  else
    hipLaunchKernelGGL((k_pair_fields<float>), dim3(nb256(cap)), dim3(256), 0, L.st, L.g,
                       (const int *)B.mcount, (const int64_t *)B.pcell, nslot,
                       (const float *)B.rho_s, (const float *)B.mom_s[0],
                       (const float *)B.mom_s[1], (const float *)B.mom_s[2],
                       (const float *)B.E_s, B.pfld);
}

void run_adj_predictor(const Launch &L, const Bufs &B, int slot, double *sb_out) {
  const GridK &g = L.g;
  const int64_t Np = padded_count(g), NFt = face_total(g);
  SBarW so = sbarw_of(g, sb_out);
  ADJ_DISPATCH(L, {
    StateV<S> st = state_slot<S>(B, slot);
    hipLaunchKernelGGL((k_adj_prims<DIM, S>), dim3(nb256(Np)), dim3(256), 0, L.st, g, st,
                       B.pprim);
    for (int d = 0; d < DIM; ++d)
      hipLaunchKernelGGL((k_adj_faces<DIM, S>), dim3(nb256(g.NF[d])), dim3(256), 0, L.st, g, d,
                         st, (const double *)B.pprim, (const double *)B.rs_bar,
                         (const double *)B.ms_bar[0], (const double *)B.ms_bar[1],
                         (const double *)B.ms_bar[2], (const double *)B.Es_bar, B.fo, NFt,
                         face_off(g, d), so.F[d]);
    hipLaunchKernelGGL((k_adj_cells<DIM, S>), dim3(nb256(g.N)), dim3(256), 0, L.st, g, st,
                       (const double *)B.pprim, (const double *)B.ms_bar[0],
                       (const double *)B.ms_bar[1], (const double *)B.ms_bar[2],
                       (const double *)B.Es_bar, B.co);
    hipLaunchKernelGGL((k_adj_gather<DIM, S>), dim3(nb256(Np)), dim3(256), 0, L.st, g, st,
                       (const double *)B.pprim, (const double *)B.fo, NFt, face_off(g, 0),
                       face_off(g, 1), face_off(g, 2), (const double *)B.co, B.pbar);
    hipLaunchKernelGGL((k_adj_fold<DIM, S>), dim3(nb256(g.N)), dim3(256), 0, L.st, g, st,
                       (const double *)B.pbar, (const double *)B.rs_bar,
                       (const double *)B.ms_bar[0], (const double *)B.ms_bar[1],
                       (const double *)B.ms_bar[2], (const double *)B.Es_bar, so);
  });
}

// The finished pressure solution (FP32 form: the x buffer of the refinement that
// ended the solve) copied to `dst`.
__global__ void k_copy_solution(const CgScal *cs, const double *xa, const double *xb, double *dst,
                                int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dst[i] = (cs->xfinal && xb) ? xb[i] : xa[i];
}

void run_copy_solution(const Launch &L, const Bufs &B, double *dst) {
  hipLaunchKernelGGL(k_copy_solution, dim3(nb256(L.g.N)), dim3(256), 0, L.st,
                     (const CgScal *)B.cg, (const double *)B.x, (const double *)B.x2, dst, L.g.N);
}

}  // namespace ibmk
