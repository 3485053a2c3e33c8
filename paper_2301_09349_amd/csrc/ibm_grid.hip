// ibm_grid.hip -- grid kernels of one IBM-HT time step on gfx950: the predictor
// flux stencil, the pressure-equation set-up, the matrix-free CG and the
// correction (Appendix A of Riahi, Goncalves da Silva, Meldi), plus state
// initialisation. Templated on the dimension and on the storage/stencil type
// (double, or float for the reduced-precision form).
#include <algorithm>
#include <type_traits>

#include "ibm_launch.h"

namespace ibmk {

// ------------------------------------------------------------------ physics
// a / b with FAST (b nonzero and of moderate size: densities, temperatures and
// limiter denominators, so the correctly rounded division's operand scaling and
// special-case fix-up are not needed). FP64: the hardware reciprocal of b refined by
// two Newton steps, the quotient corrected by its residual, within about an ulp of
// the rounded quotient in 8 operations instead of 11. FP32: the hardware reciprocal
// and one residual correction (4 operations instead of about 10). Otherwise a / b.
template <bool FAST, typename S>
__device__ __forceinline__ S qdiv(S a, S b) {
  if constexpr (FAST && std::is_same<S, double>::value) {
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    const double q = a * r;
    return fma(fma(-b, q, a), r, q);
  } else if constexpr (FAST) {
    // FP32: the hardware reciprocal (about an ulp) and one residual correction
    const float r = __builtin_amdgcn_rcpf(b);
    const float q = a * r;
    return fmaf(fmaf(-b, q, a), r, q);
  } else {
    return a / b;
  }
}
// sqrt(x) for FAST FP32: the hardware square root (about an ulp) instead of the
// correctly rounded sequence; otherwise sqrt(x).
template <bool FAST, typename S>
__device__ __forceinline__ S qsqrt(S x) {
  if constexpr (FAST && std::is_same<S, float>::value)
    return __builtin_amdgcn_sqrtf(x);
  else
    return sqrt(x);
}
// Sutherland's law (Sec. 2.1), theta^{3/2} as theta*sqrt(theta).
template <typename S, bool FAST = false>
__device__ __forceinline__ S mu_of(const GridK &g, S th) {
  if (g.visc == MU_CONSTANT) return S(g.mu_inf);
  S sut = S(g.S);
  return qdiv<FAST>(S(g.mu_inf) * th * qsqrt<FAST>(th) * (S(1) + sut), th + sut);
}
// van Leer limited face value from the upwind (C), downwind (D) and far-upwind
// (U) cell values: phi_C + (1/2) psi(r) (phi_D - phi_C), written without r.
template <typename S, bool FAST = false>
__device__ __forceinline__ S vanleer(S phC, S phD, S phU) {
  S a = phC - phU, b = phD - phC;
  S ab = a * b;
  return (ab > S(0)) ? phC + qdiv<FAST>(ab, a + b) : phC;
}

// Primitive variables at a (possibly ghost) cell from the conserved values of the
// cell r resolves to: cons = rho, m[DIM], E.
template <int DIM, typename S, bool FAST = false>
__device__ __forceinline__ void prim_from(const GridK &g, const Resolved &r, const S *cons, S &rho,
                                          S *u, S &th, S &p) {
  rho = cons[0];
  S inv = qdiv<FAST>(S(1), rho);
#pragma unroll
  for (int q = 0; q < DIM; ++q) u[q] = cons[1 + q] * inv;
  S E = cons[DIM + 1];
  th = E * inv * S(g.inv_cv);
  p = S(g.gm1) * E;
  if (any_side<DIM, S>(r)) {
    rho = ghosted<DIM>(g, r, V_RHO, rho);
#pragma unroll
    for (int q = 0; q < DIM; ++q) u[q] = ghosted<DIM>(g, r, V_U0 + q, u[q]);
    th = ghosted<DIM>(g, r, V_TH, th);
    p = ghosted<DIM>(g, r, V_P, p);
  }
}

// Primitive variables at a (possibly ghost) cell.
template <int DIM, typename S, bool FAST = false>
__device__ __forceinline__ void load_prim(const GridK &g, const StateV<S> &st, int i, int j, int k,
                                          S &rho, S *u, S &th, S &p) {
  Resolved r = resolve<DIM>(g, i, j, k);
  S cons[DIM + 2];
  cons[0] = st.rho[r.c];
#pragma unroll
  for (int q = 0; q < DIM; ++q) cons[1 + q] = st.mom[q][r.c];
  cons[DIM + 1] = st.E[r.c];
  prim_from<DIM, S, FAST>(g, r, cons, rho, u, th, p);
}

template <int DIM, typename S>
__device__ __forceinline__ void load_u(const GridK &g, const StateV<S> &st, int i, int j, int k,
                                       S *u) {
  Resolved r = resolve<DIM>(g, i, j, k);
  S inv = S(1) / st.rho[r.c];
#pragma unroll
  for (int q = 0; q < DIM; ++q) u[q] = st.mom[q][r.c] * inv;
  if (any_side<DIM, S>(r)) {
#pragma unroll
    for (int q = 0; q < DIM; ++q) u[q] = ghosted<DIM>(g, r, V_U0 + q, u[q]);
  }
}

template <int DIM, typename S>
__device__ __forceinline__ void load_u_th(const GridK &g, const StateV<S> &st, int i, int j, int k,
                                          S *u, S &th) {
  Resolved r = resolve<DIM>(g, i, j, k);
  S inv = S(1) / st.rho[r.c];
#pragma unroll
  for (int q = 0; q < DIM; ++q) u[q] = st.mom[q][r.c] * inv;
  th = st.E[r.c] * inv * S(g.inv_cv);
  if (any_side<DIM, S>(r)) {
#pragma unroll
    for (int q = 0; q < DIM; ++q) u[q] = ghosted<DIM>(g, r, V_U0 + q, u[q]);
    th = ghosted<DIM>(g, r, V_TH, th);
  }
}

// Fluxes through the face of direction d with face index (fi, fj, fk), between
// cells P = (.., f_d - 1, ..) and Q = (.., f_d, ..), in the +e_d direction:
// face-normal velocity uf = F / lin_f(rho), momentum fluxes F u_f - tau_{d,q},
// energy flux F e_f - lambda_f d theta / d n. Normal velocity derivatives are
// compact, tangential ones the face average of the two centred cell gradients.
template <int DIM, typename S>
__device__ __forceinline__ void face_flux(const GridK &g, const StateV<S> &st, int d, int fi,
                                          int fj, int fk, S &uf, S *fm, S &fe) {
  int P[3] = {fi, fj, fk}, Q[3] = {fi, fj, fk};
  P[d] -= 1;
  const S F = st.F[d][fidx(g, d, fi, fj, fk)];
  S rP, uP[3], thP, pP, rQ, uQ[3], thQ, pQ;
  load_prim<DIM>(g, st, P[0], P[1], P[2], rP, uP, thP, pP);
  load_prim<DIM>(g, st, Q[0], Q[1], Q[2], rQ, uQ, thQ, pQ);
  uf = F / (S(0.5) * (rP + rQ));
  const S muf = S(0.5) * (mu_of(g, thP) + mu_of(g, thQ));
  const S lamf = S(g.cp_Pr) * muf;
  const S ih = S(g.ih[d]);
  S dn[3], tg[3] = {S(0), S(0), S(0)};
#pragma unroll
  for (int q = 0; q < DIM; ++q) dn[q] = (uQ[q] - uP[q]) * ih;
  S divf = dn[d];
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    if (t == d) continue;
    const S hh = S(0.5 * g.ih[t]);
    S up[3], um[3];
    int a[3] = {P[0], P[1], P[2]}, b[3] = {P[0], P[1], P[2]};
    a[t] += 1;
    b[t] -= 1;
    load_u<DIM>(g, st, a[0], a[1], a[2], up);
    load_u<DIM>(g, st, b[0], b[1], b[2], um);
    S gdP = (up[d] - um[d]) * hh, gtP = (up[t] - um[t]) * hh;
    int c2[3] = {Q[0], Q[1], Q[2]}, e2[3] = {Q[0], Q[1], Q[2]};
    c2[t] += 1;
    e2[t] -= 1;
    load_u<DIM>(g, st, c2[0], c2[1], c2[2], up);
    load_u<DIM>(g, st, e2[0], e2[1], e2[2], um);
    S gdQ = (up[d] - um[d]) * hh, gtQ = (up[t] - um[t]) * hh;
    tg[t] = S(0.5) * (gdP + gdQ);
    divf += S(0.5) * (gtP + gtQ);
  }
  S cu[3], ce;
  const S cv = S(g.cv);
  if (g.conv == CONV_LINEAR) {
#pragma unroll
    for (int q = 0; q < DIM; ++q) cu[q] = S(0.5) * (uP[q] + uQ[q]);
    ce = S(0.5) * (cv * thP + cv * thQ);
  } else {
    const bool pos = F >= S(0);
    int U[3] = {pos ? P[0] : Q[0], pos ? P[1] : Q[1], pos ? P[2] : Q[2]};
    U[d] += pos ? -1 : 1;
    S uU[3], thU;
    load_u_th<DIM>(g, st, U[0], U[1], U[2], uU, thU);
    // the upwind (C) and downwind (D) cells are P and Q for F >= 0, else Q and P:
    // the operands are chosen first, so that one limiter is evaluated per value
#pragma unroll
    for (int q = 0; q < DIM; ++q)
      cu[q] = vanleer(pos ? uP[q] : uQ[q], pos ? uQ[q] : uP[q], uU[q]);
    ce = vanleer(cv * (pos ? thP : thQ), cv * (pos ? thQ : thP), cv * thU);
  }
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    S tau = (q == d) ? muf * (S(2) * dn[d] - S(2.0 / 3.0) * divf) : muf * (dn[q] + tg[q]);
    // implicit diffusion: the compact part mu_f dn[q] is taken at the new time
    if (g.implicit_diff) tau = tau - muf * dn[q];
    fm[q] = F * cu[q] - tau;
  }
  fe = g.implicit_diff ? F * ce : F * ce - lamf * (thQ - thP) * ih;
}


// ----------------------------------------------------- Appendix A, step 1
// What the predictor also writes for the pressure set-up (App. A step 3), so that
// no separate pass reads its outputs back: m^ = m* + dt G_c p^n, i.e. the momentum
// update without the pressure gradient; psi = 1/(R theta*) with theta* = E*/(rho* c_v);
// the CG start: p^n extrapolated in time from the pressures of the last states
// (p = (gamma - 1) E) -- p^n alone, 2 p^n - p^{n-1} when E_prev (the previous
// state's energy) is given, 3 p^n - 3 p^{n-1} + p^{n-2} when E_prev2 is given too,
// 4 p^n - 6 p^{n-1} + 4 p^{n-2} - p^{n-3} when E_prev3 is given as well.
// E_keep, when given, receives E^{n-1} for the next step's E_prev2 (it may be the
// E_prev2 array), E_keep2 receives E^{n-2} for the next step's E_prev3 (it may be
// the E_prev3 array): each cell is read before it is written. The spread of the
// forcing then adds its increment to m^ and recomputes psi on the cells it touches.
// In an outer pass of a step (App. A step 3 repeated), the fluxes and cell terms
// are those of the latest iterate (the kernels' state) while the time
// derivative's old values rho_b, mom_b, E_b stay those of the step's start; x is
// then NULL (the previous pass's solution is the start).
template <typename S>
struct PredOut {
  S *mh[3];
  S *psi;
  double *x;
  const S *E_prev;
  const S *E_prev2;
  const S *E_prev3;
  S *E_keep;
  S *E_keep2;
  const S *rho_b;
  const S *mom_b[3];
  const S *E_b;
};

// The same from the previous energies Ep, E2, E3 of cell c already read (each read
// only where po gives its array).
template <typename S, bool FAST = false>
__device__ __forceinline__ void pred_setup_out_vals(const GridK &g, const PredOut<S> &po,
                                                    int64_t c, S rho_s, S E_s, S E, S Ep, S E2,
                                                    S E3) {
  const S theta = qdiv<FAST>(E_s, rho_s * S(g.cv));
  po.psi[c] = qdiv<FAST>(S(1), S(g.R) * theta);
  if (!po.x) return;
  const double pn = double(S(g.gm1) * E);
  double x0 = pn;
  if (po.E_prev) {
    const double pp = double(S(g.gm1) * Ep);
    if (po.E_prev2) {
      const double p2 = double(S(g.gm1) * E2);
      if (po.E_prev3)
        x0 = 4.0 * (pn + p2) - 6.0 * pp - double(S(g.gm1) * E3);
      else
        x0 = 3.0 * (pn - pp) + p2;
      if (po.E_keep2) po.E_keep2[c] = E2;
    } else {
      x0 = 2.0 * pn - pp;
    }
    if (po.E_keep) po.E_keep[c] = Ep;
  }
  po.x[c] = x0;
}

template <typename S, bool FAST = false>
__device__ __forceinline__ void pred_setup_out(const GridK &g, const PredOut<S> &po, int64_t c,
                                               S rho_s, S E_s, S E) {
  const S Ep = (po.x && po.E_prev) ? po.E_prev[c] : S(0);
  const S E2 = (po.x && po.E_prev && po.E_prev2) ? po.E_prev2[c] : S(0);
  const S E3 = (po.x && po.E_prev && po.E_prev2 && po.E_prev3) ? po.E_prev3[c] : S(0);
  pred_setup_out_vals<S, FAST>(g, po, c, rho_s, E_s, E, Ep, E2, E3);
}

// Predictor (f = q = 0): explicit update of mass, momentum and internal energy.
template <int DIM, typename S>
__device__ __forceinline__ void predictor_cell(const GridK &g, const StateV<S> &st, int i, int j,
                                               int k, S *rho_s, S *const *ms, S *E_s,
                                               const PredOut<S> &po) {
  const int64_t c = cidx(g, i, j, k);
  S divF = S(0), divU = S(0), divE = S(0), divM[3] = {S(0), S(0), S(0)};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
    hi[d] += 1;
    S ufL, fmL[3], feL, ufH, fmH[3], feH;
    face_flux<DIM>(g, st, d, lo[0], lo[1], lo[2], ufL, fmL, feL);
    face_flux<DIM>(g, st, d, hi[0], hi[1], hi[2], ufH, fmH, feH);
    const S FL = st.F[d][fidx(g, d, lo[0], lo[1], lo[2])];
    const S FH = st.F[d][fidx(g, d, hi[0], hi[1], hi[2])];
    const S ih = S(g.ih[d]);
    divF += (FH - FL) * ih;
    divU += (ufH - ufL) * ih;
    divE += (feH - feL) * ih;
#pragma unroll
    for (int q = 0; q < DIM; ++q) divM[q] += (fmH[q] - fmL[q]) * ih;
  }
  // cell-centred velocity gradients gr[a][b] = d u_a / d x_b and pressure gradient
  S gr[3][3], gp[3];
#pragma unroll
  for (int b = 0; b < DIM; ++b) {
    int a1[3] = {i, j, k}, a0[3] = {i, j, k};
    a1[b] += 1;
    a0[b] -= 1;
    S r1, u1[3], t1, p1, r0, u0[3], t0, p0;
    load_prim<DIM>(g, st, a1[0], a1[1], a1[2], r1, u1, t1, p1);
    load_prim<DIM>(g, st, a0[0], a0[1], a0[2], r0, u0, t0, p0);
    const S hh = S(0.5 * g.ih[b]);
#pragma unroll
    for (int a = 0; a < DIM; ++a) gr[a][b] = (u1[a] - u0[a]) * hh;
    gp[b] = (p1 - p0) * hh;
  }
  S divu = S(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) divu += gr[a][a];
  S phi = S(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int b = 0; b < DIM; ++b) phi += (gr[a][b] + gr[b][a]) * gr[a][b];
  const S rho = st.rho[c], E = st.E[c];
  const S th = E * (S(1) / rho) * S(g.inv_cv);
  phi = mu_of(g, th) * (phi - S(2.0 / 3.0) * divu * divu);
  const S dt = S(g.dt);
  const S pc = S(g.gm1) * E;
  const S rs = po.rho_b[c] - dt * divF;
  rho_s[c] = rs;
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    const S mhq = po.mom_b[q][c] - dt * divM[q];
    ms[q][c] = mhq - dt * gp[q];
    po.mh[q][c] = mhq;
  }
  const S es = po.E_b[c] - dt * divE - dt * pc * divU + dt * phi;
  E_s[c] = es;
  pred_setup_out(g, po, c, rs, es, E);
}

template <int DIM, typename S>
__global__ __launch_bounds__(kThreads) void k_predictor(GridK g, StateV<S> st, S *rho_s, S *ms0,
                                                        S *ms1, S *ms2, S *E_s, PredOut<S> po) {
  S *ms[3] = {ms0, ms1, ms2};
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0; t < t1; ++t) {
    int i, j, k;
    if (cell_in_tile<DIM>(g, t, i, j, k))
      predictor_cell<DIM>(g, st, i, j, k, rho_s, ms, E_s, po);
  }
}

// ------------------------------------------------------ LDS-tiled predictor
// The same update with its work shared through LDS: a block owns a tile of
// TX x TY (x TZ) cells; the primitive variables (rho, u, theta, mu) of the tile
// and a two-cell halo are computed once into LDS with the ghost rules applied;
// the fluxes of each face direction are then computed once per face into an LDS
// buffer, from which every cell sums its divergence.
template <int DIM, typename S>
struct PTile;
// Tile shapes (measured on gfx950): FP64 tiles are smaller so that more blocks fit
// the LDS of a CU.
#ifndef IBM_PRED_TX2D
#define IBM_PRED_TX2D 32
#define IBM_PRED_TY2D 8
#endif
#ifndef IBM_PRED_TX2F
#define IBM_PRED_TX2F 64
#define IBM_PRED_TY2F 8
#endif
#ifndef IBM_PRED_TX3D
#define IBM_PRED_TX3D 8
#define IBM_PRED_TY3D 8
#define IBM_PRED_TZ3D 4
#endif
#ifndef IBM_PRED_TX3F
#define IBM_PRED_TX3F 16
#define IBM_PRED_TY3F 4
#define IBM_PRED_TZ3F 4
#endif
#ifndef IBM_PRED_MAXB
#define IBM_PRED_MAXB 1024
#endif
template <>
struct PTile<2, double> {
  static constexpr int TX = IBM_PRED_TX2D, TY = IBM_PRED_TY2D, TZ = 1;
};
template <>
struct PTile<2, float> {
  static constexpr int TX = IBM_PRED_TX2F, TY = IBM_PRED_TY2F, TZ = 1;
};
template <>
struct PTile<3, double> {
  static constexpr int TX = IBM_PRED_TX3D, TY = IBM_PRED_TY3D, TZ = IBM_PRED_TZ3D;
};
template <>
struct PTile<3, float> {
  static constexpr int TX = IBM_PRED_TX3F, TY = IBM_PRED_TY3F, TZ = IBM_PRED_TZ3F;
};

template <int DIM, typename S>
struct PredLds {
  static constexpr int TX = PTile<DIM, S>::TX, TY = PTile<DIM, S>::TY, TZ = PTile<DIM, S>::TZ;
  static constexpr int SX = TX + 4, SY = TY + 4, SZ = (DIM == 3) ? TZ + 4 : 1;
  static constexpr int NP = SX * SY * SZ;
  // the pressure p = (gamma - 1) E of every point is kept too where the LDS allows it
  // (3D FP64: two blocks per CU either way), so that -grad p reads no global memory
  static constexpr bool PL = DIM == 3 && sizeof(S) == 8;
  static constexpr int NV = DIM + 3 + (PL ? 1 : 0);  // rho, u[DIM], theta, mu (, p)
  static constexpr int F0 = (TX + 1) * TY * TZ, F1 = TX * (TY + 1) * TZ,
                       F2 = (DIM == 3) ? TX * TY * (TZ + 1) : 0;
  static constexpr int NFMAX = F0 > F1 ? (F0 > F2 ? F0 : F2) : (F1 > F2 ? F1 : F2);
  static constexpr int NFV = DIM + 3;  // F, uf, fm[DIM], fe
  static constexpr int CPT = TX * TY * TZ / kThreads;  // cells per thread
  static constexpr size_t bytes = sizeof(S) * (size_t)(NP * NV + NFMAX * NFV);
  // 3D: the z planes are a ring (SZ a power of two): local plane c of a tile whose
  // first plane has ring offset zoff sits in slot (c + 2 + zoff) mod SZ, so that the
  // next tile up a column finds the planes it shares with this one in place
  static constexpr bool RING = DIM == 3 && (SZ & (SZ - 1)) == 0;
  // Where the global reads of a tile are issued. PFO (3D): the face fluxes and the
  // outputs' inputs are read into registers at the tile's start, so that their loads
  // overlap those of the halo, instead of where they are used. PFH (3D FP64, whose
  // occupancy the LDS bounds at two blocks per CU whatever the registers): the halo
  // points are loaded in rounds of PCH per thread, each round's loads issued
  // together.
  static constexpr bool PFO = DIM == 3;
  static constexpr bool PFH = PL;
  // MAP (3D): one cell per thread, and the faces a thread forms are those of face_of
  // (no divisions by the face counts)
  static constexpr bool MAP = DIM == 3;
  // RP: the row order of cell_of below (3D FP64)
  static constexpr bool RP = PFH;
  // FQ (3D): quotients and square roots through qdiv / qsqrt with FAST
  static constexpr bool FQ = DIM == 3;
  static_assert(!(PFO || MAP) || TX * TY * TZ == kThreads, "one cell per thread");
  static_assert(!RP || TY % 4 == 0, "rows in groups of four");
  static_assert(!PFO || MAP, "the prefetched faces are those of face_of");
  // halo points a thread loads per round (their loads issued together): the new
  // planes of a tile up a column (3D), the tile with its halo (2D); faces per thread
  // and direction
  static constexpr int NEWP = SX * SY * (DIM == 3 ? (RING ? TZ : SZ) : 1);
  static constexpr int PCH = (NEWP + kThreads - 1) / kThreads;
  static constexpr int FPT = (NFMAX + kThreads - 1) / kThreads;
  // Local cell lc of the tile: x fastest. With RP (TX 8, row pitch SX 12 values) the
  // rows of each group of four are taken in the order 0 2 1 3, so that the two 8-lane
  // rows of a 16-lane group of a wave are 24 doubles apart in LDS and fall on disjoint
  // banks (rows 12 doubles apart share a quarter of theirs).
  __device__ static int row_perm(int r) {
    return RP ? (r & ~3) | ((r & 1) << 1) | ((r >> 1) & 1) : r;
  }
  __device__ static void cell_of(int lc, int &ci, int &cj, int &ck) {
    ci = lc % TX;
    cj = row_perm((lc / TX) % TY);
    ck = lc / (TX * TY);
  }
  // Slot in the face buffer of face (fi, fj, fk) of a direction with FX x FY faces per
  // plane: rows stored in the cells' row order, so that a wave's faces are contiguous
  // (row_perm is its own inverse, and leaves row TY in place).
  __device__ static int fslot(int fi, int fj, int fk, int FX, int FY) {
    return fi + FX * (row_perm(fj) + FY * fk);
  }
  // With MAP, the face of direction d that thread t forms for part m: m = 0 the low face
  // of its own cell (the cells' order above), m = 1 a face of the tile's far plane (the
  // threads below that plane's count); false when there is none.
  __device__ static bool face_of(int d, int m, int t, int &fi, int &fj, int &fk) {
    if (m == 0) {
      cell_of(t, fi, fj, fk);
      return t < TX * TY * TZ;
    }
    if (d == 0) {
      fi = TX;
      fj = t % TY;
      fk = t / TY;
      return t < TY * TZ;
    }
    if (d == 1) {
      fi = t % TX;
      fj = TY;
      fk = t / TX;
      return t < TX * TZ;
    }
    fi = t % TX;
    fj = t / TX;
    fk = TZ;
    return t < TX * TY;
  }
  __device__ static constexpr int pt(int a, int b, int c, int zoff) {
    return (a + 2) +
           SX * ((b + 2) + SY * (DIM == 3 ? (RING ? ((c + 2 + zoff) & (SZ - 1)) : c + 2) : 0));
  }
};

// Face fluxes from the LDS primitives; Q is the cell at local (qa, qb, qc), P the
// cell below it along d. Same arithmetic as face_flux.
// CONV: the convection scheme fixed at compile time (-1: read from g); FAST: qdiv's
// quotients.
template <int DIM, typename S, int CONV = -1, bool FAST = false>
__device__ __forceinline__ void face_flux_lds(const GridK &g, const S *lv, int zoff, int d, int qa,
                                              int qb, int qc, S F, S &uf, S *fm, S &fe) {
  using T = PredLds<DIM, S>;
  constexpr int NP = T::NP;
  int Q[3] = {qa, qb, qc}, P[3] = {qa, qb, qc};
  P[d] -= 1;
  const int iP = T::pt(P[0], P[1], P[2], zoff), iQ = T::pt(Q[0], Q[1], Q[2], zoff);
  const S rP = lv[iP], rQ = lv[iQ];
  S uP[3], uQ[3];
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    uP[q] = lv[(1 + q) * NP + iP];
    uQ[q] = lv[(1 + q) * NP + iQ];
  }
  const S thP = lv[(DIM + 1) * NP + iP], thQ = lv[(DIM + 1) * NP + iQ];
  const S muP = lv[(DIM + 2) * NP + iP], muQ = lv[(DIM + 2) * NP + iQ];
  uf = qdiv<FAST>(F, S(0.5) * (rP + rQ));
  const S muf = S(0.5) * (muP + muQ);
  const S lamf = S(g.cp_Pr) * muf;
  const S ih = S(g.ih[d]);
  S dn[3], tg[3] = {S(0), S(0), S(0)};
#pragma unroll
  for (int q = 0; q < DIM; ++q) dn[q] = (uQ[q] - uP[q]) * ih;
  S divf = dn[d];
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    if (t == d) continue;
    const S hh = S(0.5 * g.ih[t]);
    int a[3] = {P[0], P[1], P[2]}, b[3] = {P[0], P[1], P[2]};
    a[t] += 1;
    b[t] -= 1;
    const int ia = T::pt(a[0], a[1], a[2], zoff), ib = T::pt(b[0], b[1], b[2], zoff);
    S gdP = (lv[(1 + d) * NP + ia] - lv[(1 + d) * NP + ib]) * hh;
    S gtP = (lv[(1 + t) * NP + ia] - lv[(1 + t) * NP + ib]) * hh;
    int c2[3] = {Q[0], Q[1], Q[2]}, e2[3] = {Q[0], Q[1], Q[2]};
    c2[t] += 1;
    e2[t] -= 1;
    const int ic = T::pt(c2[0], c2[1], c2[2], zoff), ie = T::pt(e2[0], e2[1], e2[2], zoff);
    S gdQ = (lv[(1 + d) * NP + ic] - lv[(1 + d) * NP + ie]) * hh;
    S gtQ = (lv[(1 + t) * NP + ic] - lv[(1 + t) * NP + ie]) * hh;
    tg[t] = S(0.5) * (gdP + gdQ);
    divf += S(0.5) * (gtP + gtQ);
  }
  S cu[3], ce;
  const S cv = S(g.cv);
  if (CONV >= 0 ? CONV == CONV_LINEAR : g.conv == CONV_LINEAR) {
#pragma unroll
    for (int q = 0; q < DIM; ++q) cu[q] = S(0.5) * (uP[q] + uQ[q]);
    ce = S(0.5) * (cv * thP + cv * thQ);
  } else {
    const bool pos = F >= S(0);
    int U[3] = {pos ? P[0] : Q[0], pos ? P[1] : Q[1], pos ? P[2] : Q[2]};
    U[d] += pos ? -1 : 1;
    const int iU = T::pt(U[0], U[1], U[2], zoff);
    const S thU = lv[(DIM + 1) * NP + iU];
    // upwind and downwind operands chosen first: one limiter per value
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      const S uU = lv[(1 + q) * NP + iU];
      cu[q] = vanleer<S, FAST>(pos ? uP[q] : uQ[q], pos ? uQ[q] : uP[q], uU);
    }
    ce = vanleer<S, FAST>(cv * (pos ? thP : thQ), cv * (pos ? thQ : thP), cv * thU);
  }
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    S tau = (q == d) ? muf * (S(2) * dn[d] - S(2.0 / 3.0) * divf) : muf * (dn[q] + tg[q]);
    // implicit diffusion: the compact part mu_f dn[q] is taken at the new time
    if (g.implicit_diff) tau = tau - muf * dn[q];
    fm[q] = F * cu[q] - tau;
  }
  fe = g.implicit_diff ? F * ce : F * ce - lamf * (thQ - thP) * ih;
}

template <int DIM, typename S, int CONV = -1>
__global__ __launch_bounds__(kThreads) void k_predictor_lds(GridK g, StateV<S> st, S *rho_s,
                                                            S *ms0, S *ms1, S *ms2, S *E_s,
                                                            PredOut<S> po) {
  using T = PredLds<DIM, S>;
  constexpr int NP = T::NP, NFM = T::NFMAX, CPT = T::CPT;
  extern __shared__ __align__(16) unsigned char smem[];
  S *lv = reinterpret_cast<S *>(smem);  // [NV][NP]
  S *lf = lv + T::NV * NP;              // [NFV][NFMAX]
  S *ms[3] = {ms0, ms1, ms2};
  const int ptx = (g.n[0] + T::TX - 1) / T::TX, pty = (g.n[1] + T::TY - 1) / T::TY;
  const int ptz = (DIM == 3) ? (g.n[2] + T::TZ - 1) / T::TZ : 1;
  const int64_t ntile = (int64_t)ptx * pty * ptz;
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t rank = (b & 7) * (nb >> 3) + (b >> 3);
  const int64_t per = (ntile + nb - 1) / nb;
  const int64_t t0 = rank * per, t1 = (t0 + per < ntile) ? t0 + per : ntile;
  const S dt = S(g.dt), gm1 = S(g.gm1);
  for (int64_t t = t0; t < t1; ++t) {
    // 2D: x fastest; 3D: z fastest (a block walks up a column of tiles, so the halo
    // planes below a tile were loaded by its previous tile)
    int x0, y0, z0;
    if (DIM == 2) {
      x0 = (int)(t % ptx) * T::TX;
      y0 = (int)(t / ptx) * T::TY;
      z0 = 0;
    } else {
      z0 = (int)(t % ptz) * T::TZ;
      x0 = (int)((t / ptz) % ptx) * T::TX;
      y0 = (int)(t / ((int64_t)ptz * ptx)) * T::TY;
    }
    // the tile's face fluxes and the values its outputs need, read into registers
    // first so that their loads overlap those of the halo below
    S fpre[DIM][T::FPT];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (!T::PFO) break;
#pragma unroll
      for (int m = 0; m < T::FPT; ++m) {
        fpre[d][m] = S(0);
        int fi, fj, fk;
        if (!T::face_of(d, m, threadIdx.x, fi, fj, fk)) continue;
        const int gc[3] = {x0 + fi, y0 + fj, z0 + fk};
        bool ok = true;
#pragma unroll
        for (int e = 0; e < DIM; ++e) ok = ok && (gc[e] < g.n[e] + (e == d ? 1 : 0));
        if (ok) fpre[d][m] = st.F[d][fidx(g, d, gc[0], gc[1], gc[2])];
      }
    }
    // per cell: E, rho_b, mom_b[DIM], E_b, and the previous energies the CG start uses
    S opre[CPT][DIM + 6];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
      if (!T::PFO) break;
      int ci, cj, ck;
      T::cell_of(threadIdx.x + kThreads * m, ci, cj, ck);
      const int i = x0 + ci, j = y0 + cj, k = z0 + ck;
#pragma unroll
      for (int v = 0; v < DIM + 6; ++v) opre[m][v] = S(0);
      if (!(i < g.n[0] && j < g.n[1] && (DIM == 2 || k < g.n[2]))) continue;
      const int64_t c = cidx(g, i, j, k);
      opre[m][0] = st.E[c];
      opre[m][1] = po.rho_b[c];
#pragma unroll
      for (int q = 0; q < DIM; ++q) opre[m][2 + q] = po.mom_b[q][c];
      opre[m][DIM + 2] = po.E_b[c];
      if (po.x && po.E_prev) {
        opre[m][DIM + 3] = po.E_prev[c];
        if (po.E_prev2) {
          opre[m][DIM + 4] = po.E_prev2[c];
          if (po.E_prev3) opre[m][DIM + 5] = po.E_prev3[c];
        }
      }
    }
    __syncthreads();  // the previous tile is done with LDS
    // phase 1: primitives of the tile and its halo (points beyond two ghost
    // layers are not needed and not loaded). Up a column (3D), the planes shared
    // with the previous tile (local -2..1) are already in the ring: only the TZ
    // new planes (local 2..TZ+1) are loaded. Each round issues the loads of its
    // points before converting any of them.
    const int zoff = T::RING ? (z0 & (T::SZ - 1)) : 0;
    const bool cont = T::RING && t > t0 && z0 != 0;
    const int cfirst = cont ? 2 : -2, nplanes = cont ? T::TZ : T::SZ;
    const int npts = T::SX * T::SY * nplanes;
    for (int p = threadIdx.x; !T::PFH && p < npts; p += kThreads) {
      const int li = p % T::SX, lj = (p / T::SX) % T::SY, lc = cfirst + p / (T::SX * T::SY);
      const int gi = x0 - 2 + li, gj = y0 - 2 + lj, gk = (DIM == 3) ? z0 + lc : 0;
      bool ok = gi >= -2 && gi <= g.n[0] + 1 && gj >= -2 && gj <= g.n[1] + 1;
      if (DIM == 3) ok = ok && gk >= -2 && gk <= g.n[2] + 1;
      if (!ok) continue;
      const int lp = T::pt(li - 2, lj - 2, lc, zoff);
      S r, u[3], th, pp;
      load_prim<DIM, S, T::FQ>(g, st, gi, gj, gk, r, u, th, pp);
      lv[lp] = r;
#pragma unroll
      for (int q = 0; q < DIM; ++q) lv[(1 + q) * NP + lp] = u[q];
      lv[(DIM + 1) * NP + lp] = th;
      lv[(DIM + 2) * NP + lp] = mu_of<S, T::FQ>(g, th);
      if (T::PL) lv[(DIM + 3) * NP + lp] = pp;
    }
    for (int base = 0; T::PFH && base < npts; base += T::PCH * kThreads) {
      Resolved rr[T::PCH];
      S cons[T::PCH][DIM + 2];
      int lp[T::PCH];
      bool okp[T::PCH];
#pragma unroll
      for (int m = 0; m < T::PCH; ++m) {
        const int p = base + threadIdx.x + kThreads * m;
        okp[m] = false;
        lp[m] = 0;
        if (p >= npts) continue;
        const int li = p % T::SX, lj = (p / T::SX) % T::SY, lc = cfirst + p / (T::SX * T::SY);
        const int gi = x0 - 2 + li, gj = y0 - 2 + lj, gk = (DIM == 3) ? z0 + lc : 0;
        bool ok = gi >= -2 && gi <= g.n[0] + 1 && gj >= -2 && gj <= g.n[1] + 1;
        if (DIM == 3) ok = ok && gk >= -2 && gk <= g.n[2] + 1;
        if (!ok) continue;
        okp[m] = true;
        lp[m] = T::pt(li - 2, lj - 2, lc, zoff);
        rr[m] = resolve<DIM>(g, gi, gj, gk);
        cons[m][0] = st.rho[rr[m].c];
#pragma unroll
        for (int q = 0; q < DIM; ++q) cons[m][1 + q] = st.mom[q][rr[m].c];
        cons[m][DIM + 1] = st.E[rr[m].c];
      }
#pragma unroll
      for (int m = 0; m < T::PCH; ++m) {
        if (!okp[m]) continue;
        S r, u[3], th, pp;
        prim_from<DIM, S, T::FQ>(g, rr[m], cons[m], r, u, th, pp);
        const int q0 = lp[m];
        lv[q0] = r;
#pragma unroll
        for (int q = 0; q < DIM; ++q) lv[(1 + q) * NP + q0] = u[q];
        lv[(DIM + 1) * NP + q0] = th;
        lv[(DIM + 2) * NP + q0] = mu_of<S, T::FQ>(g, th);
        if (T::PL) lv[(DIM + 3) * NP + q0] = pp;
      }
    }
    __syncthreads();
    // phase 2: cell-centred terms (-grad p, viscous dissipation) into registers
    S acc[CPT][DIM + 3];  // rho, mom[DIM] (without -grad p), E, div(uf)
    S gpr[CPT][DIM];      // -dt grad p
    int cl[CPT][3];
    bool cv_ok[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
      int ci, cj, ck;
      T::cell_of(threadIdx.x + kThreads * m, ci, cj, ck);
      cl[m][0] = ci;
      cl[m][1] = cj;
      cl[m][2] = ck;
      const int i = x0 + ci, j = y0 + cj, k = z0 + ck;
      cv_ok[m] = i < g.n[0] && j < g.n[1] && (DIM == 2 || k < g.n[2]);
#pragma unroll
      for (int v = 0; v < DIM + 3; ++v) acc[m][v] = S(0);
#pragma unroll
      for (int q = 0; q < DIM; ++q) gpr[m][q] = S(0);
      if (!cv_ok[m]) continue;
      S gr[3][3], gp[3];
#pragma unroll
      for (int bd = 0; bd < DIM; ++bd) {
        int a1[3] = {ci, cj, ck}, a0[3] = {ci, cj, ck};
        a1[bd] += 1;
        a0[bd] -= 1;
        const int i1 = T::pt(a1[0], a1[1], a1[2], zoff), i0 = T::pt(a0[0], a0[1], a0[2], zoff);
        const S hh = S(0.5 * g.ih[bd]);
#pragma unroll
        for (int a = 0; a < DIM; ++a) gr[a][bd] = (lv[(1 + a) * NP + i1] - lv[(1 + a) * NP + i0]) * hh;
        if (T::PL) {
          gp[bd] = (lv[(DIM + 3) * NP + i1] - lv[(DIM + 3) * NP + i0]) * hh;
        } else {
          int g1[3] = {i, j, k}, g0[3] = {i, j, k};
          g1[bd] += 1;
          g0[bd] -= 1;
          Resolved r1 = resolve<DIM>(g, g1[0], g1[1], g1[2]);
          Resolved r0 = resolve<DIM>(g, g0[0], g0[1], g0[2]);
          S p1 = ghosted<DIM>(g, r1, V_P, gm1 * st.E[r1.c]);
          S p0 = ghosted<DIM>(g, r0, V_P, gm1 * st.E[r0.c]);
          gp[bd] = (p1 - p0) * hh;
        }
      }
      S divu = S(0);
#pragma unroll
      for (int a = 0; a < DIM; ++a) divu += gr[a][a];
      S phi = S(0);
#pragma unroll
      for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int bd = 0; bd < DIM; ++bd) phi += (gr[a][bd] + gr[bd][a]) * gr[a][bd];
      phi = lv[(DIM + 2) * NP + T::pt(ci, cj, ck, zoff)] * (phi - S(2.0 / 3.0) * divu * divu);
#pragma unroll
      for (int q = 0; q < DIM; ++q) gpr[m][q] = -dt * gp[q];
      acc[m][DIM + 1] = dt * phi;
    }
    // phase 3: faces, one direction at a time
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int FX = T::TX + (d == 0), FY = T::TY + (d == 1), FZ = T::TZ + (d == 2 ? 1 : 0);
      const int nfd = FX * FY * FZ;
#pragma unroll
      for (int m = 0; m < T::FPT; ++m) {
        int f, fi, fj, fk;
        if (T::MAP) {
          if (!T::face_of(d, m, threadIdx.x, fi, fj, fk)) continue;
          f = T::fslot(fi, fj, fk, FX, FY);
        } else {
          f = threadIdx.x + kThreads * m;
          if (f >= nfd) continue;
          fi = f % FX;
          fj = (f / FX) % FY;
          fk = f / (FX * FY);
        }
        const int gi = x0 + fi, gj = y0 + fj, gk = z0 + fk;
        const int gc[3] = {gi, gj, gk};
        bool ok = true;
#pragma unroll
        for (int e = 0; e < DIM; ++e) ok = ok && (gc[e] < g.n[e] + (e == d ? 1 : 0));
        if (!ok) continue;
        const S F = T::PFO ? fpre[d][m] : st.F[d][fidx(g, d, gi, gj, gk)];
        S uf, fm[3], fe;
        face_flux_lds<DIM, S, CONV, T::FQ>(g, lv, zoff, d, fi, fj, fk, F, uf, fm, fe);
        lf[f] = F;
        lf[NFM + f] = uf;
#pragma unroll
        for (int q = 0; q < DIM; ++q) lf[(2 + q) * NFM + f] = fm[q];
        lf[(2 + DIM) * NFM + f] = fe;
      }
      __syncthreads();
      const S ih = S(g.ih[d]);
#pragma unroll
      for (int m = 0; m < CPT; ++m) {
        if (!cv_ok[m]) continue;
        const int fl = T::fslot(cl[m][0], cl[m][1], cl[m][2], FX, FY);
        const int fh = T::fslot(cl[m][0] + (d == 0), cl[m][1] + (d == 1), cl[m][2] + (d == 2),
                                FX, FY);
        acc[m][0] += (lf[fh] - lf[fl]) * ih;
        acc[m][DIM + 2] += (lf[NFM + fh] - lf[NFM + fl]) * ih;
#pragma unroll
        for (int q = 0; q < DIM; ++q)
          acc[m][1 + q] -= dt * ((lf[(2 + q) * NFM + fh] - lf[(2 + q) * NFM + fl]) * ih);
        acc[m][DIM + 1] -= dt * ((lf[(2 + DIM) * NFM + fh] - lf[(2 + DIM) * NFM + fl]) * ih);
      }
      __syncthreads();
    }
    // phase 4: outputs
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
      if (!cv_ok[m]) continue;
      const int64_t c = cidx(g, x0 + cl[m][0], y0 + cl[m][1], z0 + cl[m][2]);
      const S E = T::PFO ? opre[m][0] : st.E[c];
      const S rs = (T::PFO ? opre[m][1] : po.rho_b[c]) - dt * acc[m][0];
      rho_s[c] = rs;
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        const S mhq = (T::PFO ? opre[m][2 + q] : po.mom_b[q][c]) + acc[m][1 + q];
        ms[q][c] = mhq + gpr[m][q];
        po.mh[q][c] = mhq;
      }
      const S es = (T::PFO ? opre[m][DIM + 2] : po.E_b[c]) + acc[m][DIM + 1] -
                   dt * (gm1 * E) * acc[m][DIM + 2];
      E_s[c] = es;
      if (T::PFO)
        pred_setup_out_vals<S, T::FQ>(g, po, c, rs, es, E, opre[m][DIM + 3], opre[m][DIM + 4],
                                      opre[m][DIM + 5]);
      else
        pred_setup_out<S, T::FQ>(g, po, c, rs, es, E);
    }
  }
}

// ------------------------------------------------------- initialisation
// Byte ranges copied in one launch: part p moves units[p] elements of type T (4 or
// 16 bytes) from src[p] to dst[p]; the grid strides over each part in turn.
template <typename T>
__global__ void k_copy_parts(CopyParts cp) {
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int p = 0; p < cp.n; ++p) {
    const T *src = static_cast<const T *>(cp.src[p]);
    T *dst = static_cast<T *>(cp.dst[p]);
    const int64_t n = (int64_t)(cp.bytes[p] / sizeof(T));
    for (int64_t k = i0; k < n; k += stride) dst[k] = src[k];
  }
}

void run_copy_parts(const Launch &L, const CopyParts &cp) {
  if (cp.n == 0) return;
  bool wide = true;
  size_t most = 0;
  for (int p = 0; p < cp.n; ++p) {
    wide = wide && (reinterpret_cast<uintptr_t>(cp.src[p]) % 16 == 0) &&
           (reinterpret_cast<uintptr_t>(cp.dst[p]) % 16 == 0) && cp.bytes[p] % 16 == 0;
    most = std::max(most, cp.bytes[p]);
  }
  const size_t unit = wide ? 16 : 4;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((most / unit + 255) / 256, 2048));
  if (wide)
    hipLaunchKernelGGL(k_copy_parts<uint4>, dim3((unsigned)blocks), dim3(256), 0, L.st, cp);
  else
    hipLaunchKernelGGL(k_copy_parts<unsigned>, dim3((unsigned)blocks), dim3(256), 0, L.st, cp);
}

__global__ void k_fill(double *p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// uniform stream rho = 1, u = U_inf, theta = 1
template <int DIM, typename S>
__global__ void k_uniform(GridK g, StateV<S> st) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  st.rho[c] = S(1);
#pragma unroll
  for (int q = 0; q < DIM; ++q) st.mom[q][c] = S(g.U_inf[q]);
  st.E[c] = S(g.cv);
}

template <int DIM, typename S>
__global__ void k_init_primitive(GridK g, StateV<S> st, const S *rho, const S *u, const S *th) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  S r = rho[c];
  st.rho[c] = r;
#pragma unroll
  for (int q = 0; q < DIM; ++q) st.mom[q][c] = r * u[(int64_t)q * g.N + c];
  st.E[c] = r * S(g.cv) * th[c];
}

// Face mass flux from cell momentum: linear interpolation inside; boundary faces
// by their rule (inflow rho_P U_inf, slip 0, outflow m_P).
template <int DIM, typename S, typename M>
__device__ __forceinline__ S face_from_cells(const GridK &g, M *const *m, const S *rho0, int d,
                                             int fi, int fj, int fk) {
  int ix[3] = {fi, fj, fk};
  int id = ix[d], n = g.n[d];
  if (g.bc[d][0] == BC_PERIODIC || (id > 0 && id < n)) {
    int P[3] = {fi, fj, fk}, Q[3] = {fi, fj, fk};
    P[d] = id > 0 ? id - 1 : n - 1;  // id is in [0, n]
    Q[d] = id < n ? id : 0;
    return S(0.5) * (S(m[d][cidx(g, P[0], P[1], P[2])]) + S(m[d][cidx(g, Q[0], Q[1], Q[2])]));
  }
  int side = (id == 0) ? 0 : 1;
  int A[3] = {fi, fj, fk};
  A[d] = side == 0 ? 0 : n - 1;
  int64_t ca = cidx(g, A[0], A[1], A[2]);
  int b = g.bc[d][side];
  if (b == BC_INFLOW) return rho0[ca] * S(g.U_inf[d]);
  if (b == BC_SLIP) return S(0);
  return S(m[d][ca]);
}

template <int DIM, typename S>
__global__ void k_flux_from_mom(GridK g, StateV<S> st, int d) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= g.NF[d]) return;
  int fi = (int)(f % g.fn[d][0]);
  int64_t r = f / g.fn[d][0];
  int fj = (int)(r % g.fn[d][1]);
  int fk = (int)(r / g.fn[d][1]);
  st.F[d][f] = face_from_cells<DIM, S>(g, st.mom, st.rho, d, fi, fj, fk);
}

// --------------------------------------------------- Appendix A, step 3
// (m^, psi and the CG start come from the predictor and the spread.)
// Pressure set-up from the predictor's m^, psi, x: predicted face flux
// F^ = lin_f(m^) (boundary rules), b = rho^n - dt D(F^) + outflow terms,
// r0 = b - A x; per-block FP64 partial sums of b.b.
template <int DIM, typename S>
__global__ __launch_bounds__(kBlockThreads) void k_setup2(GridK g, const S *rho_n, const S *mh0,
                                                     const S *mh1, const S *mh2, S *Fh0, S *Fh1,
                                                     S *Fh2, const S *psi, const double *x,
                                                     double *b, double *r0, double *partials,
                                                     CgScal *cs, int tag) {
  __shared__ double lds[32];
  const S *mh[3] = {mh0, mh1, mh2};
  S *Fh[3] = {Fh0, Fh1, Fh2};
  double bb = 0.0;
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    const int ix[3] = {i, j, k};
    double div = 0.0, aff = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int hi[3] = {i, j, k};
      hi[d] += 1;
      S fl = face_from_cells<DIM, S>(g, mh, rho_n, d, i, j, k);
      S fh = face_from_cells<DIM, S>(g, mh, rho_n, d, hi[0], hi[1], hi[2]);
      Fh[d][fidx(g, d, i, j, k)] = fl;
      if (ix[d] == g.n[d] - 1) Fh[d][fidx(g, d, hi[0], hi[1], hi[2])] = fh;
      div += (double(fh) - double(fl)) * g.ih[d];
      if (g.bc[d][0] != BC_PERIODIC) {
        if (ix[d] == 0 && g.bc[d][0] == BC_OUTFLOW) aff += 2.0 * g.p_inf * g.ih[d] * g.ih[d];
        if (ix[d] == g.n[d] - 1 && g.bc[d][1] == BC_OUTFLOW)
          aff += 2.0 * g.p_inf * g.ih[d] * g.ih[d];
      }
    }
    const double bc_ = double(rho_n[c]) - g.dt * div + g.dt * g.dt * aff;
    const double xc = x[c];
    const double ax = helm_at<DIM>(g, psi, [&](int64_t q) { return x[q]; }, i, j, k, c, xc);
    b[c] = bc_;
    r0[c] = bc_ - ax;
    bb += bc_ * bc_;
  }
  bb = block_sum(bb, lds);
  if (threadIdx.x == 0) {
    partials[PART_BB * kMaxBlocks + blockIdx.x] = bb;
    if (blockIdx.x == 0) {
      cs->done = 0;
      cs->iters = 0;
      cs->step_tag = tag;
      cs->xfinal = 0;
    }
  }
}

// Start of the single-reduction CG (Chronopoulos and Gear's variant): w0 = A r0
// and the per-block partials of gamma_0 = r0.r0 and delta_0 = w0.r0.
template <int DIM, typename S>
__global__ __launch_bounds__(kBlockThreads) void k_cg_start(GridK g, const S *psi, const double *r0,
                                                       double *w0, double *partials) {
  __shared__ double lds[32];
  double sums[2] = {0.0, 0.0};
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    const double rc = r0[c];
    const double wc = helm_at<DIM>(g, psi, [&](int64_t m) { return r0[m]; }, i, j, k, c, rc);
    w0[c] = wc;
    sums[0] += rc * rc;
    sums[1] += wc * rc;
  }
  block_sum_n<2>(sums, lds);
  if (threadIdx.x == 0) {
    partials[PART_G * kMaxBlocks + blockIdx.x] = sums[0];
    partials[PART_D * kMaxBlocks + blockIdx.x] = sums[1];
  }
}

// Update of one cell in a CG iteration (see k_cg_iter): rc, wc, sc0, pc0, xc, psc
// are r, w, s_old, p_old, x, psi at the cell. FIRST: p = r, s = w (the old p, s are
// not read).
template <int DIM, bool FIRST, typename S>
__device__ __forceinline__ void cg_cell(const GridK &g, double alpha, double beta, int i, int j,
                                        int k, double rc, double wc, double sc0, double pc0,
                                        double xc, S psc, const double *__restrict__ r,
                                        const double *__restrict__ w,
                                        const double *__restrict__ sold, double *__restrict__ rn,
                                        double *__restrict__ wn, double *__restrict__ snew,
                                        double *__restrict__ p, double *__restrict__ x,
                                        double *sums) {
  const int64_t c = cidx(g, i, j, k);
  const double pc = FIRST ? rc : rc + beta * pc0;
  const double sc = FIRST ? wc : wc + beta * sc0;
  x[c] = xc + alpha * pc;
  const double rnc = rc - alpha * sc;
  auto rv = [&](int64_t m) {
    return FIRST ? r[m] - alpha * w[m] : r[m] - alpha * (w[m] + beta * sold[m]);
  };
  const double wnc = double(psc) * rnc - g.dt * g.dt * helm_lap<DIM>(g, rv, i, j, k, rnc);
  p[c] = pc;
  snew[c] = sc;
  rn[c] = rnc;
  wn[c] = wnc;
  sums[0] += rnc * rnc;
  sums[1] += wnc * rnc;
}

// All tiles of this thread's tile group.
template <int DIM, bool FIRST, typename S>
__device__ __forceinline__ void cg_sweep(const GridK &g, double alpha, double beta, int64_t t0,
                                         int64_t t1, const S *__restrict__ psi,
                                         const double *__restrict__ r,
                                         const double *__restrict__ w,
                                         const double *__restrict__ sold, double *__restrict__ rn,
                                         double *__restrict__ wn, double *__restrict__ snew,
                                         double *__restrict__ p, double *__restrict__ x,
                                         double *sums) {
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    cg_cell<DIM, FIRST>(g, alpha, beta, i, j, k, r[c], w[c], FIRST ? 0.0 : sold[c],
                        FIRST ? 0.0 : p[c], x[c], psi[c], r, w, sold, rn, wn, snew, p, x, sums);
  }
}

// The common start of a single-reduction CG iteration: every block forms gamma_it
// = r.r and delta_it = w.r from the partials of the previous kernel and tests
// convergence (|r| <= rtol |b|) or the end (iteration limit, an error flag, NaN);
// block 0 records the scalars and posts (step tag, it, error flags, done) to
// `progress`. Returns false when the solve has ended (nothing to update);
// otherwise alpha and beta of the update. Every load of the head (the solve's
// scalars, the flags, the partials) is issued before its first barrier, so that
// they wait out one memory latency together.
__device__ __forceinline__ bool cg_head(int it, const double *partials, CgScal *cs,
                                        const int *flags, uint64_t *progress, double *lds,
                                        int &done0, double &alpha, double &beta) {
  __shared__ double bc[3];
  const int nb = gridDim.x;
  const int par = it & 1, prv = par ^ 1;
  // block 0 of this kernel may set `done` while other blocks start: one read per
  // block, published to the block by the barriers of the sums below
  if (threadIdx.x == 0) done0 = cs->done;
  const double bb_prev = cs->bb, tol2 = cs->tol2;
  const double rr_prev = cs->rr[prv], alpha_prev = cs->alpha[prv];
  const int maxit = cs->maxit;
  const int err = (flags[FLAG_NONFINITE] ? 1 : 0) | (flags[FLAG_SUPPORT] ? 2 : 0) |
                  (flags[FLAG_EPS] ? 4 : 0) | (flags[FLAG_GRAM] ? 8 : 0);
  // the sums in the order of sum_partials: strided over the threads, then the block
  const double *pg = partials + (PART_G + par) * kMaxBlocks;
  const double *pd = partials + (PART_D + par) * kMaxBlocks;
  const double *pb = partials + PART_BB * kMaxBlocks;
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    v[0] += pg[i];
    v[1] += pd[i];
    if (it == 0) v[2] += pb[i];
  }
  block_sum_n<3>(v, lds);
  if (threadIdx.x == 0) {
    bc[0] = v[0];
    bc[1] = v[1];
    bc[2] = v[2];
  }
  __syncthreads();
  if (done0) return false;
  const double gam = bc[0], del = bc[1];
  const double bb = (it == 0) ? bc[2] : bb_prev;
  const bool conv = gam <= tol2 * bb;
  const bool out = !conv && (it >= maxit || err != 0 || !(gam == gam));
  beta = 0.0;
  alpha = gam / del;
  if (it > 0) {
    beta = gam / rr_prev;
    alpha = gam / (del - beta * gam / alpha_prev);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (it == 0) cs->bb = bb;
    cs->rr[par] = gam;
    cs->alpha[par] = alpha;
    cs->res = bb > 0.0 ? sqrt(gam / bb) : 0.0;
    cs->iters = it;
    if (conv || out) cs->done = conv ? 1 : 2;
    if (progress)
      __hip_atomic_store(progress, pack_progress(cs->step_tag, it, err, conv ? 1 : out ? 2 : 0),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  return !(conv || out);
}

// The common end: per-block partials of r'.r' and w'.r' for the next iteration.
__device__ __forceinline__ void cg_tail(int it, double *sums, double *partials, double *lds) {
  const int par = it & 1;
  block_sum_n<2>(sums, lds);
  if (threadIdx.x == 0) {
    partials[(PART_G + (par ^ 1)) * kMaxBlocks + blockIdx.x] = sums[0];
    partials[(PART_D + (par ^ 1)) * kMaxBlocks + blockIdx.x] = sums[1];
  }
}

// CG iteration `it` with one global reduction (the recurrences of Chronopoulos and
// Gear: s = A p is carried as s = w + beta s_old, so r.r and w.r of the new
// residual are reduced together). Every block forms gamma_it = r.r and delta_it =
// w.r from the partials of the previous kernel; converged (|r| <= rtol |b|) or out
// of iterations -> all blocks stop and block 0 records it. Otherwise
//   beta = gamma_it / gamma_{it-1} (0 at it = 0),
//   alpha = gamma_it / (delta_it - beta gamma_it / alpha_{it-1}) (gamma/delta at 0),
//   p = r + beta p, s = w + beta s, x += alpha p, r' = r - alpha s, w' = A r',
// with r' of the neighbours formed on the fly from r, w, s; partials of r'.r' and
// w'.r'. r, w, s are read from slot it & 1 and written to the other slot.
// Block 0 posts (step tag, it, error flags, done) to `progress` (host memory, may
// be NULL) so that the host can follow the solve without synchronising; a step
// whose flags show an error stops its solve.
template <int DIM, typename S>
__global__ __launch_bounds__(kBlockThreads) void k_cg_iter(
    GridK g, int it, const S *__restrict__ psi, const double *__restrict__ r,
    const double *__restrict__ w, const double *__restrict__ sold, double *__restrict__ rn,
    double *__restrict__ wn, double *__restrict__ snew, double *__restrict__ p,
    double *__restrict__ x, double *partials, CgScal *cs, const int *flags, uint64_t *progress) {
  __shared__ double lds[48];
  __shared__ int done0;
  double alpha, beta;
  if (!cg_head(it, partials, cs, flags, progress, lds, done0, alpha, beta)) return;
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  double sums[2] = {0.0, 0.0};
  if (it == 0)
    cg_sweep<DIM, true>(g, alpha, beta, t0, t1, psi, r, w, sold, rn, wn, snew, p, x, sums);
  else
    cg_sweep<DIM, false>(g, alpha, beta, t0, t1, psi, r, w, sold, rn, wn, snew, p, x, sums);
  cg_tail(it, sums, partials, lds);
}

// ------------------------------------------- 3D CG iteration by z-columns
// The same iteration as k_cg_iter in 3D, with the neighbour values of the new
// residual r' = r - alpha (w + beta s_old) formed once per cell instead of once per
// stencil use: a block owns an x-y tile of kColTX x kColTY cells (a wave per x row)
// and walks a chunk of z planes. r' of planes k-1, k, k+1 of a thread's own column
// stay in registers; the x-y neighbours come from a plane of r' in LDS (double
// buffered by plane parity, one barrier per plane) with a one-cell halo that halo
// threads form from r, w, s of the neighbouring tiles. The loads of plane k+2 are
// issued while plane k is finished. Outside the box a slot holds the ghost value
// of the homogeneous pressure operator, sigma r'(mirror) with sigma = -1 beyond an
// outflow side (zero on the face) and +1 elsewhere (zero normal gradient), which
// gives helm_lap's face terms; periodic directions wrap.
constexpr int kColTX = 64;
#ifndef IBM_CG_COL_TY
#define IBM_CG_COL_TY 8
#endif
constexpr int kColTY = IBM_CG_COL_TY;
constexpr int kColThreads = kColTX * kColTY;
constexpr int kColPitch = kColTX + 2;
constexpr int kColSlots = (kColTY + 2) * kColPitch;
constexpr int kColHalo = 2 * kColTX + 2 * kColTY;
static_assert(kColHalo <= kColThreads, "halo slots exceed the block's threads");
// The CG iteration's tiles are twice as tall (64 x 16, 1024 threads): less of the
// y halo of r, w, s is read again per cell (304 against 313 us per iteration on
// 256^3); the other column kernels keep 64 x 8, where the taller tile was slower.
#ifndef IBM_CG_ITER_TY
#define IBM_CG_ITER_TY 16
#endif
constexpr int kCgTY = IBM_CG_ITER_TY;
static_assert(2 * kColTX + 2 * kCgTY <= kColTX * kCgTY, "halo slots exceed the block's threads");

// Index v along direction d resolved to a cell of the box and the sign of the
// homogeneous ghost rule: wrap (periodic), else the mirror cell with sigma -1 beyond
// an outflow side and +1 beyond the others. Far outside (ragged tiles) the index is
// clamped so that loads stay inside the arrays (those slots are never used).
__device__ __forceinline__ int col_resolve(const GridK &g, int d, int v, double &sig) {
  const int n = g.n[d];
  sig = 1.0;
  if (v >= 0 && v < n) return v;
  if (g.bc[d][0] == BC_PERIODIC) {
    v %= n;
    return v < 0 ? v + n : v;
  }
  const int side = v < 0 ? 0 : 1;
  if (g.bc[d][side] == BC_OUTFLOW) sig = -1.0;
  v = v < 0 ? -v - 1 : 2 * n - 1 - v;
  return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// The halo slot of this thread in a tile (tx, ty) of the column kernels: threads
// 0..kColHalo-1 take rows y = -1 and kColTY, then columns x = -1 and kColTX; their
// cell (resolved into the box, in plane 0) and the sign of its ghost rule.
__device__ __forceinline__ void col_halo_slot(const GridK &g, int tx, int ty, int &hslot,
                                              int64_t &hcol, double &hsig) {
  if (threadIdx.x >= kColHalo) return;
  const int t = threadIdx.x;
  int hx, hy;
  if (t < kColTX) {
    hx = t;
    hy = -1;
  } else if (t < 2 * kColTX) {
    hx = t - kColTX;
    hy = kColTY;
  } else if (t < 2 * kColTX + kColTY) {
    hx = -1;
    hy = t - 2 * kColTX;
  } else {
    hx = kColTX;
    hy = t - 2 * kColTX - kColTY;
  }
  double s1, s2;
  hcol = col_resolve(g, 0, tx * kColTX + hx, s1) +
         (int64_t)g.n[0] * col_resolve(g, 1, ty * kColTY + hy, s2);
  hsig = s1 * s2;
  hslot = (hy + 1) * kColPitch + (hx + 1);
}

// FP32 form's solve by refinement (see k_mcg_iter): an inner solve stops at 1e-5 of
// its start residual (or kInnerMax iterations); the stages of its kernels. (At 1e-4
// the 256^3 sphere took 9.9 inner launches per step, at 1e-5 9.0, at 1e-6 9.0.)
constexpr double kInnerTol2 = 1e-10;
constexpr int kInnerMax = 60;
enum { MS_INNER = 0, MS_START = 1, MS_FIRST = 2 };

// Loads of one plane of a thread's own column.
struct ColLoad {
  double r, w, s, p, x, ps, sg;
};

// Modes of the column CG kernel: the start of a solve (w0 = A r0 and the partials of
// r0.r0 and w0.r0, no convergence test), its first iteration (p = r, s = w) and the
// later iterations.
enum { COL_START = 0, COL_FIRST = 1, COL_ITER = 2 };

template <int MODE>
__device__ __forceinline__ double col_rprime(double alpha, double beta, double r, double w,
                                             double s) {
  return MODE == COL_START ? r : MODE == COL_FIRST ? r - alpha * w : r - alpha * (w + beta * s);
}

template <int MODE, typename S, int TY = kCgTY>
__global__ __launch_bounds__(kColTX * TY) void k_cg_col(
    GridK g, int it, int tiles_x, int tiles_y, int zc, int64_t items, const S *__restrict__ psi,
    const double *__restrict__ r, const double *__restrict__ w, const double *__restrict__ sold,
    double *__restrict__ rn, double *__restrict__ wn, double *__restrict__ snew,
    double *__restrict__ p, double *__restrict__ x, double *partials, CgScal *cs,
    const int *flags, uint64_t *progress) {
  constexpr bool START = MODE == COL_START, FIRST = MODE == COL_FIRST;
  __shared__ double lds[48];
  __shared__ int done0;
  constexpr int kSlots = (TY + 2) * kColPitch, kHalo = 2 * kColTX + 2 * TY;
  __shared__ double plane_lds[2][kSlots];
  double alpha = 0.0, beta = 0.0;
  if (!START && !cg_head(it, partials, cs, flags, progress, lds, done0, alpha, beta)) return;
  const int lx = threadIdx.x % kColTX, ly = threadIdx.x / kColTX;
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t rank = (b & 7) * (nb >> 3) + (b >> 3);
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const int64_t pl = (int64_t)n0 * n1;
  const double dt2 = g.dt * g.dt;
  const double ih0 = g.ih[0], ih1 = g.ih[1], ih2 = g.ih[2];
  const int myslot = (ly + 1) * kColPitch + (lx + 1);
  double sums[2] = {0.0, 0.0};
  for (int64_t item = rank; item < items; item += nb) {
    const int tx = (int)(item % tiles_x);
    const int64_t rest = item / tiles_x;
    const int ty = (int)(rest % tiles_y);
    const int ch = (int)(rest / tiles_y);
    const int i = tx * kColTX + lx, j = ty * TY + ly;
    const int k0 = ch * zc, k1 = min(k0 + zc, n2);
    const bool inside = i < n0 && j < n1;
    double sx, sy;
    const int64_t col = col_resolve(g, 0, i, sx) + (int64_t)n0 * col_resolve(g, 1, j, sy);
    const double sxy = sx * sy;
    // halo slot of this thread: rows y = -1 and TY, then columns x = -1 and kColTX
    int hslot = -1;
    int64_t hcol = 0;
    double hsig = 1.0;
    if (threadIdx.x < kHalo) {
      const int t = threadIdx.x;
      int hx, hy;
      if (t < kColTX) {
        hx = t;
        hy = -1;
      } else if (t < 2 * kColTX) {
        hx = t - kColTX;
        hy = TY;
      } else if (t < 2 * kColTX + TY) {
        hx = -1;
        hy = t - 2 * kColTX;
      } else {
        hx = kColTX;
        hy = t - 2 * kColTX - TY;
      }
      double s1, s2;
      hcol = col_resolve(g, 0, tx * kColTX + hx, s1) +
             (int64_t)n0 * col_resolve(g, 1, ty * TY + hy, s2);
      hsig = s1 * s2;
      hslot = (hy + 1) * kColPitch + (hx + 1);
    }
    auto load = [&](int k, ColLoad &L) {
      double sz;
      const int64_t c = col + pl * col_resolve(g, 2, k, sz);
      L.r = r[c];
      L.w = START ? 0.0 : w[c];
      L.s = (START || FIRST) ? 0.0 : sold[c];
      if (inside && k >= k0 && k < k1) {
        L.p = (START || FIRST) ? 0.0 : p[c];
        L.x = START ? 0.0 : x[c];
        L.ps = double(psi[c]);
      }
      L.sg = sxy * sz;
    };
    auto load_halo = [&](int k, double &hr, double &hw, double &hs, double &hg) {
      if (hslot < 0) return;
      double sz;
      const int64_t c = hcol + pl * col_resolve(g, 2, k, sz);
      hr = r[c];
      hw = START ? 0.0 : w[c];
      hs = (START || FIRST) ? 0.0 : sold[c];
      hg = hsig * sz;
    };
    ColLoad A, B, C;
    double rqm, rqc, rqp;
    {
      ColLoad M;
      load(k0 - 1, M);
      rqm = M.sg * col_rprime<MODE>(alpha, beta, M.r, M.w, M.s);
    }
    load(k0, A);
    load(k0 + 1, B);
    double hr = 0.0, hw = 0.0, hs = 0.0, hg = 1.0;
    load_halo(k0, hr, hw, hs, hg);
    rqc = A.sg * col_rprime<MODE>(alpha, beta, A.r, A.w, A.s);
    for (int k = k0; k < k1; ++k) {
      double hr2 = 0.0, hw2 = 0.0, hs2 = 0.0, hg2 = 1.0;
      if (k + 2 <= k1) load(k + 2, C);
      if (k + 1 < k1) load_halo(k + 1, hr2, hw2, hs2, hg2);
      rqp = B.sg * col_rprime<MODE>(alpha, beta, B.r, B.w, B.s);
      double *lp = plane_lds[(k - k0) & 1];
      lp[myslot] = rqc;
      if (hslot >= 0) lp[hslot] = hg * col_rprime<MODE>(alpha, beta, hr, hw, hs);
      __syncthreads();
      if (inside) {
        // the face terms in helm_lap's order: -x, +x, -y, +y, -z, +z
        const double vc = rqc;
        double lap = 0.0, gf;
        gf = (lp[myslot - 1] - vc) * ih0;
        lap += gf * ih0;
        gf = (lp[myslot + 1] - vc) * ih0;
        lap += gf * ih0;
        gf = (lp[myslot - kColPitch] - vc) * ih1;
        lap += gf * ih1;
        gf = (lp[myslot + kColPitch] - vc) * ih1;
        lap += gf * ih1;
        gf = (rqm - vc) * ih2;
        lap += gf * ih2;
        gf = (rqp - vc) * ih2;
        lap += gf * ih2;
        const double wnc = A.ps * vc - dt2 * lap;
        const int64_t c = col + pl * k;
        if (!START) {
          const double pc = FIRST ? A.r : A.r + beta * A.p;
          const double sc = FIRST ? A.w : A.w + beta * A.s;
          x[c] = A.x + alpha * pc;
          p[c] = pc;
          snew[c] = sc;
          rn[c] = vc;
        }
        wn[c] = wnc;
        sums[0] += vc * vc;
        sums[1] += wnc * vc;
      }
      A = B;
      B = C;
      hr = hr2;
      hw = hw2;
      hs = hs2;
      hg = hg2;
      rqm = rqc;
      rqc = rqp;
    }
    __syncthreads();  // the next item's first plane reuses the LDS buffers
  }
  if (START) {
    block_sum_n<2>(sums, lds);
    if (threadIdx.x == 0) {
      partials[PART_G * kMaxBlocks + blockIdx.x] = sums[0];
      partials[PART_D * kMaxBlocks + blockIdx.x] = sums[1];
    }
  } else {
    cg_tail(it, sums, partials, lds);
  }
}

// 3D pressure set-up by z-columns (the arithmetic of k_setup2 with its face values,
// divergence, outflow terms and operator in the same order): a block owns a
// kColTX x kColTY tile and walks a chunk of planes; m^_x, m^_y and x of a plane
// with a one-cell halo are shared through LDS, m^_z and x of planes k-1, k, k+1 of
// a thread's own column stay in registers. Boundary faces take face_from_cells'
// rules; x beyond a side holds the homogeneous ghost of the pressure operator.
// REF32 (the FP32 form's solve by refinement, S = float): the start residual goes to
// the inner solve as FP32 (r32) with its FP64 r.r as the outer partial, and the
// solve's first kernel is a refinement-start stage.
template <typename S, bool REF32 = false>
__global__ __launch_bounds__(kColThreads) void k_setup_col(
    GridK g, int tiles_x, int tiles_y, int zc, int64_t items, const S *__restrict__ rho_n,
    const S *__restrict__ mh0, const S *__restrict__ mh1, const S *__restrict__ mh2,
    S *__restrict__ Fh0, S *__restrict__ Fh1, S *__restrict__ Fh2, const S *__restrict__ psi,
    const double *__restrict__ x, double *__restrict__ b, double *__restrict__ r0,
    float *__restrict__ r32, double *partials, CgScal *cs, int tag) {
  __shared__ double lds[32];
  __shared__ S mx_lds[2][kColSlots];
  __shared__ S my_lds[2][kColSlots];
  __shared__ double x_lds[2][kColSlots];
  const int lx = threadIdx.x % kColTX, ly = threadIdx.x / kColTX;
  const int64_t nb = gridDim.x, bk = blockIdx.x;
  const int64_t rank = (bk & 7) * (nb >> 3) + (bk >> 3);
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const int64_t pl = (int64_t)n0 * n1;
  const int fx0 = g.fn[0][0];                  // x faces per row
  const int64_t fpl1 = (int64_t)n0 * g.fn[1][1];  // y faces per plane
  const double dt = g.dt, dt2 = g.dt * g.dt;
  const double ih0 = g.ih[0], ih1 = g.ih[1], ih2 = g.ih[2];
  const bool per0 = g.bc[0][0] == BC_PERIODIC, per1 = g.bc[1][0] == BC_PERIODIC,
             per2 = g.bc[2][0] == BC_PERIODIC;
  const int myslot = (ly + 1) * kColPitch + (lx + 1);
  // the rule of a boundary face (face_from_cells): inflow rho_P U_inf, slip 0, else m_P
  auto rule = [&](int bc, int d, S rho_c, S m_c) -> S {
    if (bc == BC_INFLOW) return rho_c * S(g.U_inf[d]);
    if (bc == BC_SLIP) return S(0);
    return m_c;
  };
  double bb = 0.0, rr = 0.0;
  for (int64_t item = rank; item < items; item += nb) {
    const int tx = (int)(item % tiles_x);
    const int64_t rest = item / tiles_x;
    const int ty = (int)(rest % tiles_y);
    const int ch = (int)(rest / tiles_y);
    const int i = tx * kColTX + lx, j = ty * kColTY + ly;
    const int k0 = ch * zc, k1 = min(k0 + zc, n2);
    const bool inside = i < n0 && j < n1;
    double sx, sy;
    const int64_t col = col_resolve(g, 0, i, sx) + (int64_t)n0 * col_resolve(g, 1, j, sy);
    const double sxy = sx * sy;
    int hslot = -1;
    int64_t hcol = 0;
    double hsig = 1.0;
    col_halo_slot(g, tx, ty, hslot, hcol, hsig);
    // own column: m^_z and x of a plane (any plane, resolved), and the rest of a
    // plane inside the chunk
    struct Own {
      S mz, mx, my, rho, ps;
      double x, sg;
    };
    auto load = [&](int k, Own &o) {
      double sz;
      const int64_t c = col + pl * col_resolve(g, 2, k, sz);
      o.mz = mh2[c];
      o.x = x[c];
      o.sg = sxy * sz;
      if (k >= k0 && k < k1) {
        o.mx = mh0[c];
        o.my = mh1[c];
        if (inside) {
          o.rho = rho_n[c];
          o.ps = psi[c];
        }
      }
    };
    Own A, B, C, M;
    load(k0 - 1, M);
    load(k0, A);
    load(k0 + 1, B);
    S hmx = S(0), hmy = S(0);
    double hx_ = 0.0;
    auto load_halo = [&](int k, S &a, S &bq, double &xv) {
      if (hslot < 0) return;
      double sz;
      const int64_t c = hcol + pl * col_resolve(g, 2, k, sz);
      a = mh0[c];
      bq = mh1[c];
      xv = hsig * sz * x[c];
    };
    load_halo(k0, hmx, hmy, hx_);
    S mz_m = M.mz;
    double x_m = M.sg * M.x;
    for (int k = k0; k < k1; ++k) {
      S hmx2 = S(0), hmy2 = S(0);
      double hx2 = 0.0;
      if (k + 2 <= k1) load(k + 2, C);
      if (k + 1 < k1) load_halo(k + 1, hmx2, hmy2, hx2);
      const int buf = (k - k0) & 1;
      mx_lds[buf][myslot] = A.mx;
      my_lds[buf][myslot] = A.my;
      x_lds[buf][myslot] = A.sg * A.x;
      if (hslot >= 0) {
        mx_lds[buf][hslot] = hmx;
        my_lds[buf][hslot] = hmy;
        x_lds[buf][hslot] = hx_;
      }
      __syncthreads();
      if (inside) {
        const S *mxl = mx_lds[buf];
        const S *myl = my_lds[buf];
        const double *xl = x_lds[buf];
        const int64_t c = col + pl * k;
        const S rc = A.rho;
        double div = 0.0, aff = 0.0;
        // x faces
        {
          const S fl = (i > 0 || per0) ? S(0.5) * (mxl[myslot - 1] + mxl[myslot])
                                       : rule(g.bc[0][0], 0, rc, A.mx);
          const S fh = (i < n0 - 1 || per0) ? S(0.5) * (mxl[myslot] + mxl[myslot + 1])
                                            : rule(g.bc[0][1], 0, rc, A.mx);
          const int64_t f = i + (int64_t)fx0 * (j + (int64_t)n1 * k);
          Fh0[f] = fl;
          if (i == n0 - 1) Fh0[f + 1] = fh;
          div += (double(fh) - double(fl)) * ih0;
          if (!per0) {
            if (i == 0 && g.bc[0][0] == BC_OUTFLOW) aff += 2.0 * g.p_inf * ih0 * ih0;
            if (i == n0 - 1 && g.bc[0][1] == BC_OUTFLOW) aff += 2.0 * g.p_inf * ih0 * ih0;
          }
        }
        // y faces
        {
          const S fl = (j > 0 || per1) ? S(0.5) * (myl[myslot - kColPitch] + myl[myslot])
                                       : rule(g.bc[1][0], 1, rc, A.my);
          const S fh = (j < n1 - 1 || per1) ? S(0.5) * (myl[myslot] + myl[myslot + kColPitch])
                                            : rule(g.bc[1][1], 1, rc, A.my);
          const int64_t f = i + (int64_t)n0 * j + fpl1 * k;
          Fh1[f] = fl;
          if (j == n1 - 1) Fh1[f + n0] = fh;
          div += (double(fh) - double(fl)) * ih1;
          if (!per1) {
            if (j == 0 && g.bc[1][0] == BC_OUTFLOW) aff += 2.0 * g.p_inf * ih1 * ih1;
            if (j == n1 - 1 && g.bc[1][1] == BC_OUTFLOW) aff += 2.0 * g.p_inf * ih1 * ih1;
          }
        }
        // z faces
        {
          const S fl = (k > 0 || per2) ? S(0.5) * (mz_m + A.mz) : rule(g.bc[2][0], 2, rc, A.mz);
          const S fh = (k < n2 - 1 || per2) ? S(0.5) * (A.mz + B.mz)
                                            : rule(g.bc[2][1], 2, rc, A.mz);
          const int64_t f = c;  // z faces: i + n0 (j + n1 k)
          Fh2[f] = fl;
          if (k == n2 - 1) Fh2[f + pl] = fh;
          div += (double(fh) - double(fl)) * ih2;
          if (!per2) {
            if (k == 0 && g.bc[2][0] == BC_OUTFLOW) aff += 2.0 * g.p_inf * ih2 * ih2;
            if (k == n2 - 1 && g.bc[2][1] == BC_OUTFLOW) aff += 2.0 * g.p_inf * ih2 * ih2;
          }
        }
        const double bc_ = double(rc) - dt * div + dt2 * aff;
        // the operator on x in helm_lap's order: -x, +x, -y, +y, -z, +z
        const double xc = A.x;
        double lap = 0.0, gf;
        gf = (xl[myslot - 1] - xc) * ih0;
        lap += gf * ih0;
        gf = (xl[myslot + 1] - xc) * ih0;
        lap += gf * ih0;
        gf = (xl[myslot - kColPitch] - xc) * ih1;
        lap += gf * ih1;
        gf = (xl[myslot + kColPitch] - xc) * ih1;
        lap += gf * ih1;
        gf = (x_m - xc) * ih2;
        lap += gf * ih2;
        gf = (B.sg * B.x - xc) * ih2;
        lap += gf * ih2;
        const double ax = double(A.ps) * xc - dt2 * lap;
        b[c] = bc_;
        const double res = bc_ - ax;
        if (REF32) {
          r32[c] = float(res);
          rr += res * res;
        } else {
          r0[c] = res;
        }
        bb += bc_ * bc_;
      }
      mz_m = A.mz;
      x_m = A.sg * A.x;
      A = B;
      B = C;
      hmx = hmx2;
      hmy = hmy2;
      hx_ = hx2;
    }
    __syncthreads();
  }
  double v2[2] = {bb, rr};
  block_sum_n<2>(v2, lds);
  if (threadIdx.x == 0) {
    partials[PART_BB * kMaxBlocks + blockIdx.x] = v2[0];
    if (REF32) partials[PART_O * kMaxBlocks + blockIdx.x] = v2[1];
    if (blockIdx.x == 0) {
      cs->done = 0;
      cs->iters = 0;
      cs->step_tag = tag;
      cs->xfinal = 0;
      if (REF32) {
        cs->outer[0] = MS_START;
        cs->xpar[0] = 0;
        cs->inner_it[0] = 0;
        cs->rr_in0[0] = 0.0;
      }
    }
  }
}

// ------------------------- implicit diffusion (backward Euler), after the predictor
// For each velocity component (variable v < dim) and the temperature (v = dim),
// with the predictor's explicit part as right-hand side:
//   rho* y - dt kap div(mu_f grad_n y) = rhs,  kap = 1 (velocity), gamma/Pr
//   (temperature, the equation divided by c_v), mu_f the face viscosity of the
//   state at step n.
// The dim + 1 systems share rho* and mu_f and are solved together: one kernel per
// iteration runs the single-reduction CG step of every variable still iterating
// (each with its own step lengths and its own test |r_v| <= rtol |b_v|), so that
// the shared coefficients are loaded once and the partial sums of all variables
// are formed in one pass.
// Ghost value of y beyond a boundary face: sigma y + cst (the variable's rule);
// the constant goes to the right-hand side, the operator keeps sigma y.
__device__ __forceinline__ void diff_rule(const GridK &g, int bc, int q, int d, double &sg,
                                          double &cst) {
  sg = 1.0;
  cst = 0.0;
  if (bc == BC_INFLOW) {
    sg = -1.0;
    cst = (q < 3) ? 2.0 * g.U_inf[q] : 2.0;
  } else if (bc == BC_SLIP && q == d) {
    sg = -1.0;
  }
}

// The 2 dim faces of a cell: dt ih^2 mu_f, and the neighbour across (its index,
// or -1 beyond a non-periodic boundary, with that side's boundary type). Face e
// is direction e / 2, low side for even e.
template <int DIM>
struct DiffNbr {
  int64_t m[2 * DIM];
  double cf[2 * DIM];
  int bc[2 * DIM];
};

template <int DIM>
__device__ __forceinline__ void diff_nbr(const GridK &g, const double *const *mf, int i, int j,
                                         int k, DiffNbr<DIM> &nb) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double w = g.dt * g.ih[d] * g.ih[d];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int e = 2 * d + side;
      int ix[3] = {i, j, k};
      int fx[3] = {i, j, k};
      fx[d] += side;
      ix[d] += side ? 1 : -1;
      nb.cf[e] = w * mf[d][fidx(g, d, fx[0], fx[1], fx[2])];
      nb.bc[e] = g.bc[d][side];
      const int n = g.n[d];
      if (ix[d] >= 0 && ix[d] < n) {
        nb.m[e] = cidx(g, ix[0], ix[1], ix[2]);
      } else if (g.bc[d][0] == BC_PERIODIC) {
        ix[d] = ix[d] < 0 ? ix[d] + n : ix[d] - n;
        nb.m[e] = cidx(g, ix[0], ix[1], ix[2]);
      } else {
        nb.m[e] = -1;
      }
    }
  }
}

// rho* yc + kap sum_e cf_e (yc - y_nb), with Y(m) the value at cell m and the
// homogeneous ghost sigma yc beyond a boundary face.
template <int DIM, typename YF>
__device__ __forceinline__ double diff_apply(const GridK &g, const DiffNbr<DIM> &nb, int q,
                                             double kap, double rs, double yc, YF Y) {
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < 2 * DIM; ++e) {
    double yn;
    if (nb.m[e] >= 0) {
      yn = Y(nb.m[e]);
    } else {
      double sg, cst;
      diff_rule(g, nb.bc[e], q, e >> 1, sg, cst);
      yn = sg * yc;
    }
    acc += nb.cf[e] * (yc - yn);
  }
  return rs * yc + kap * acc;
}

// kap sum over boundary faces of cf cst: the ghost rules' constant part.
template <int DIM>
__device__ __forceinline__ double diff_bnd(const GridK &g, const DiffNbr<DIM> &nb, int q,
                                           double kap) {
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < 2 * DIM; ++e) {
    if (nb.m[e] >= 0) continue;
    double sg, cst;
    diff_rule(g, nb.bc[e], q, e >> 1, sg, cst);
    acc += nb.cf[e] * cst;
  }
  return kap * acc;
}

// Face viscosity of direction d from the state at step n (the predictor's mu_f).
template <int DIM, typename S>
__global__ void k_diff_coef(GridK g, int d, StateV<S> st, double *mf) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= g.NF[d]) return;
  int Q[3] = {(int)(f % g.fn[d][0]), (int)((f / g.fn[d][0]) % g.fn[d][1]),
              (int)(f / ((int64_t)g.fn[d][0] * g.fn[d][1]))};
  int P[3] = {Q[0], Q[1], Q[2]};
  P[d] -= 1;
  S uP[3], uQ[3], thP, thQ;
  load_u_th<DIM>(g, st, P[0], P[1], P[2], uP, thP);
  load_u_th<DIM>(g, st, Q[0], Q[1], Q[2], uQ, thQ);
  mf[f] = double(S(0.5) * (mu_of(g, thP) + mu_of(g, thQ)));
}

// The variable's value in the state at step n (velocity component, or 3: theta).
template <typename S>
__device__ __forceinline__ double diff_state_value(const GridK &g, const StateV<S> &st, int q,
                                                   int64_t c) {
  const S inv = S(1) / st.rho[c];
  return q < 3 ? double(st.mom[q][c] * inv) : double(st.E[c] * inv * S(g.inv_cv));
}

__device__ __forceinline__ int diff_q(int v, int dim) { return v < dim ? v : 3; }

// Start of the solves: x0 (order 0: the state's values; 1: 2 y1 - y2, the linear
// extrapolation of the last two steps' solutions; 2: x as it is, the previous
// outer pass's solution), rhs = explicit part + boundary constants, r0 = rhs -
// A x0; partial sums of b.b; the scalars reset.
template <int DIM, typename S>
__global__ __launch_bounds__(kBlockThreads) void k_dsys_init(GridK g, DiffSys D, StateV<S> st,
                                                        const S *rho_s, const S *ms0,
                                                        const S *ms1, const S *ms2,
                                                        const S *E_s, int order, int tag) {
  constexpr int NV = DIM + 1;
  __shared__ double lds[16 * NV];
  const S *src[3] = {ms0, ms1, ms2};
  double bb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) bb[v] = 0.0;
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    DiffNbr<DIM> nb;
    diff_nbr<DIM>(g, D.mf, i, j, k, nb);
    const double rs = double(rho_s[c]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int q = diff_q(v, DIM);
      const double kap = v < DIM ? 1.0 : D.kap_th;
      const double *y1 = D.y1[v], *y2 = D.y2[v], *xv = D.x[v];
      auto X0 = [&](int64_t m) {
        return order == 0 ? diff_state_value(g, st, q, m)
                          : order == 1 ? 2.0 * y1[m] - y2[m] : xv[m];
      };
      const double xc = X0(c);
      const double rhs =
          (v < DIM ? double(src[v][c]) : double(E_s[c]) * g.inv_cv) + diff_bnd<DIM>(g, nb, q, kap);
      if (order != 2) D.x[v][c] = xc;
      D.r[0][v][c] = rhs - diff_apply<DIM>(g, nb, q, kap, rs, xc, X0);
      bb[v] += rhs * rhs;
    }
  }
  block_sum_n<NV>(bb, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) D.part[(v * DP_REGIONS + DP_BB) * kMaxBlocks + blockIdx.x] = bb[v];
    if (blockIdx.x == 0) {
#pragma unroll
      for (int v = 0; v < kDiffVars; ++v) D.sc->done[v] = v < NV ? 0 : 1;
      D.sc->iters = 0;
      D.sc->step_tag = tag;
    }
  }
}

// w0 = A r0 and the partials of gamma_0 = r0.r0, delta_0 = w0.r0, per variable.
template <int DIM, typename S>
__global__ __launch_bounds__(kBlockThreads) void k_dsys_start(GridK g, DiffSys D, const S *rho_s) {
  constexpr int NV = DIM + 1;
  __shared__ double lds[16 * 2 * NV];
  double sums[2 * NV];
#pragma unroll
  for (int v = 0; v < 2 * NV; ++v) sums[v] = 0.0;
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    DiffNbr<DIM> nb;
    diff_nbr<DIM>(g, D.mf, i, j, k, nb);
    const double rs = double(rho_s[c]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double *r0 = D.r[0][v];
      const double rc = r0[c];
      const double wc = diff_apply<DIM>(g, nb, diff_q(v, DIM), v < DIM ? 1.0 : D.kap_th, rs, rc,
                                        [&](int64_t m) { return r0[m]; });
      D.w[0][v][c] = wc;
      sums[2 * v] += rc * rc;
      sums[2 * v + 1] += wc * rc;
    }
  }
  block_sum_n<2 * NV>(sums, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      D.part[(v * DP_REGIONS + DP_G) * kMaxBlocks + blockIdx.x] = sums[2 * v];
      D.part[(v * DP_REGIONS + DP_D) * kMaxBlocks + blockIdx.x] = sums[2 * v + 1];
    }
  }
}

// Iteration `it` of all solves still running: the recurrences of k_cg_iter per
// variable. Every block forms gamma, delta (and b.b at it = 0) of each running
// variable from the previous kernel's partials, tests it (converged, or out of
// iterations, an error flag or NaN: that variable stops) and updates the running
// ones; block 0 records the scalars and posts (tag, it, error flags, state) to
// `progress`, the state 0 while any variable runs, then 1 (all converged) or 2.
template <int DIM, typename S>
__global__ __launch_bounds__(kBlockThreads) void k_dsys_iter(GridK g, int it, DiffSys D,
                                                        const S *__restrict__ rho_s,
                                                        const int *flags, uint64_t *progress) {
  constexpr int NV = DIM + 1;
  __shared__ double lds[16 * 3 * NV];
  __shared__ double red[3 * NV];
  __shared__ int run0[NV];
  DiffScal *sc = D.sc;
  // Every load of the head (which solves still run, the scalars, the error flags,
  // the partials of every variable) is issued before its first barrier, so that
  // they wait out one memory latency together. Block 0 of this kernel may end a
  // solve while other blocks start: one read of the `done` words per block,
  // published to the block by the barriers of the sums below.
  if (threadIdx.x < NV) run0[threadIdx.x] = sc->done[threadIdx.x] == 0;
  const int par = it & 1, prv = par ^ 1;
  const double tol2 = sc->tol2;
  const int maxit = sc->maxit;
  double bb_prev[NV], rr_prev[NV], alpha_prev[NV];
  int done_prev[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    bb_prev[v] = sc->bb[v];
    rr_prev[v] = sc->rr[prv][v];
    alpha_prev[v] = sc->alpha[prv][v];
    done_prev[v] = sc->done[v];
  }
  const int err = (flags[FLAG_NONFINITE] ? 1 : 0) | (flags[FLAG_SUPPORT] ? 2 : 0) |
                  (flags[FLAG_EPS] ? 4 : 0) | (flags[FLAG_GRAM] ? 8 : 0);
  {
    // the partials of finished variables are summed too (and not used)
    double acc[3 * NV];
#pragma unroll
    for (int v = 0; v < 3 * NV; ++v) acc[v] = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        acc[v] += D.part[(v * DP_REGIONS + DP_G + par) * kMaxBlocks + b];
        acc[NV + v] += D.part[(v * DP_REGIONS + DP_D + par) * kMaxBlocks + b];
        if (it == 0) acc[2 * NV + v] += D.part[(v * DP_REGIONS + DP_BB) * kMaxBlocks + b];
      }
    }
    block_sum_n<3 * NV>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int v = 0; v < 3 * NV; ++v) red[v] = acc[v];
    }
    __syncthreads();
  }
  bool any = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) any = any || run0[v];
  if (!any) return;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  double alpha[NV], beta[NV];
  bool run[NV];
  bool all_end = true;
  int state = 1;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    alpha[v] = beta[v] = 0.0;
    run[v] = false;
    if (!run0[v]) {
      // ended before this kernel: its word was set then and is not changed since
      if (done_prev[v] == 2) state = 2;
      continue;
    }
    const double gam = red[v], del = red[NV + v];
    const double bb = (it == 0) ? red[2 * NV + v] : bb_prev[v];
    const bool conv = gam <= tol2 * bb;
    const bool out = !conv && (it >= maxit || err != 0 || !(gam == gam));
    alpha[v] = gam / del;
    if (it > 0) {
      beta[v] = gam / rr_prev[v];
      alpha[v] = gam / (del - beta[v] * gam / alpha_prev[v]);
    }
    run[v] = !(conv || out);
    if (run[v]) all_end = false;
    if (out) state = 2;
    if (lead) {
      if (it == 0) sc->bb[v] = bb;
      sc->rr[par][v] = gam;
      sc->alpha[par][v] = alpha[v];
      if (!run[v]) sc->done[v] = conv ? 1 : 2;
    }
  }
  if (lead) {
    sc->iters = it;
    if (progress)
      __hip_atomic_store(progress, pack_progress(sc->step_tag, it, err, all_end ? state : 0),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (all_end) return;
  const bool first = it == 0;
  double sums[2 * NV];
#pragma unroll
  for (int v = 0; v < 2 * NV; ++v) sums[v] = 0.0;
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    DiffNbr<DIM> nb;
    diff_nbr<DIM>(g, D.mf, i, j, k, nb);
    const double rs = double(rho_s[c]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (!run[v]) continue;
      const double *__restrict__ r = D.r[par][v];
      const double *__restrict__ w = D.w[par][v];
      const double *__restrict__ so = D.s[par][v];
      const double a = alpha[v], be = beta[v];
      const double rc = r[c], wc = w[c];
      const double pc = first ? rc : rc + be * D.p[v][c];
      const double scc = first ? wc : wc + be * so[c];
      D.x[v][c] = D.x[v][c] + a * pc;
      const double rnc = rc - a * scc;
      auto RV = [&](int64_t m) {
        return first ? r[m] - a * w[m] : r[m] - a * (w[m] + be * so[m]);
      };
      const double wnc =
          diff_apply<DIM>(g, nb, diff_q(v, DIM), v < DIM ? 1.0 : D.kap_th, rs, rnc, RV);
      D.p[v][c] = pc;
      D.s[par ^ 1][v][c] = scc;
      D.r[par ^ 1][v][c] = rnc;
      D.w[par ^ 1][v][c] = wnc;
      sums[2 * v] += rnc * rnc;
      sums[2 * v + 1] += wnc * rnc;
    }
  }
  block_sum_n<2 * NV>(sums, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (!run[v]) continue;
      D.part[(v * DP_REGIONS + DP_G + (par ^ 1)) * kMaxBlocks + blockIdx.x] = sums[2 * v];
      D.part[(v * DP_REGIONS + DP_D + (par ^ 1)) * kMaxBlocks + blockIdx.x] = sums[2 * v + 1];
    }
  }
}

// The solutions into the predictor's outputs: m*_q = rho* u*_q (m^ moves by the
// same amount), E* = c_v rho* theta* and psi = 1/(R theta*).
template <int DIM, typename S>
__global__ void k_dsys_finish(GridK g, DiffSys D, const S *rho_s, S *ms0, S *ms1, S *ms2,
                              S *mh0, S *mh1, S *mh2, S *E_s, S *psi) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  S *ms[3] = {ms0, ms1, ms2};
  S *mh[3] = {mh0, mh1, mh2};
  const double rs = double(rho_s[c]);
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    const S mnew = S(rs * D.x[q][c]);
    mh[q][c] = mh[q][c] + (mnew - ms[q][c]);
    ms[q][c] = mnew;
  }
  const S Es = S(g.cv * rs * D.x[DIM][c]);
  E_s[c] = Es;
  const S theta = Es / (rho_s[c] * S(g.cv));
  psi[c] = S(1) / (S(g.R) * theta);
}

// ------------------------------------------ App. B (density-based variant)
// u**, theta** of the density-based step's intermediate state, formed once per cell
// so that the viscous stencils only load them.
template <typename S>
struct DensPrim {
  S *v[5];  // u0, u1, u2, theta (the last unused)
};

// Central-upwind flux (Kurganov, Noelle, Petrova; the scheme of rhoCentralFoam)
// of rho, rho u and rho e_t through a face of direction d, from rho, u, theta at
// the four cells along d around it (index 0: far low, 1: P, 2: Q, 3: far high):
// the values reconstructed on both sides (van Leer limited, or the linear
// average with linear convection), p = rho R theta, c^2 = gamma R theta; local
// speeds a+ = max(uL + cL, uR + cR, 0), a- = min(uL - cL, uR - cR, 0) of the
// normal velocities; alpha = a+/(a+ - a-), omega = -a+ a-/(a+ - a-);
// flux = alpha f(L) + (1 - alpha) f(R) - omega (W_R - W_L), with the pressure
// alpha pL + (1 - alpha) pR in the normal momentum flux.
template <int DIM, typename S, bool FAST = false>
__device__ __forceinline__ void knp_flux(const GridK &g, int d, const S *r, const S (*u)[3],
                                         const S *th, S &fr, S *fm, S &fe) {
  S rL, rR, thL, thR, uL[3], uR[3];
  if (g.conv == CONV_LINEAR) {
    rL = rR = S(0.5) * (r[1] + r[2]);
    thL = thR = S(0.5) * (th[1] + th[2]);
#pragma unroll
    for (int q = 0; q < DIM; ++q) uL[q] = uR[q] = S(0.5) * (u[1][q] + u[2][q]);
  } else {
    rL = vanleer<S, FAST>(r[1], r[2], r[0]);
    rR = vanleer<S, FAST>(r[2], r[1], r[3]);
    thL = vanleer<S, FAST>(th[1], th[2], th[0]);
    thR = vanleer<S, FAST>(th[2], th[1], th[3]);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      uL[q] = vanleer<S, FAST>(u[1][q], u[2][q], u[0][q]);
      uR[q] = vanleer<S, FAST>(u[2][q], u[1][q], u[3][q]);
    }
  }
  S kL = S(0), kR = S(0);
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    kL += uL[q] * uL[q];
    kR += uR[q] * uR[q];
  }
  const S Rg = S(g.R), gam = S(g.gm1 + 1.0), cv = S(g.cv);
  const S pL = rL * Rg * thL, pR = rR * Rg * thR;
  const S cL = qsqrt<FAST>(gam * Rg * thL), cR = qsqrt<FAST>(gam * Rg * thR);
  const S vL = uL[d], vR = uR[d];
  S ap = vL + cL, am = vL - cL;
  if (vR + cR > ap) ap = vR + cR;
  if (ap < S(0)) ap = S(0);
  if (vR - cR < am) am = vR - cR;
  if (am > S(0)) am = S(0);
  const S span = ap - am;
  const S al = qdiv<FAST>(ap, span), om = -qdiv<FAST>(ap * am, span), bl = S(1) - al;
  const S eL = rL * (cv * thL + S(0.5) * kL), eR = rR * (cv * thR + S(0.5) * kR);
  fr = al * vL * rL + bl * vR * rR - om * (rR - rL);
#pragma unroll
  for (int q = 0; q < DIM; ++q)
    fm[q] = al * vL * (rL * uL[q]) + bl * vR * (rR * uR[q]) - om * (rR * uR[q] - rL * uL[q]);
  fm[d] += al * pL + bl * pR;
  fe = al * vL * (eL + pL) + bl * vR * (eR + pR) - om * (eR - eL);
}

// True while an earlier step of the call has failed (its input must survive).
__device__ __forceinline__ bool dens_skip(const int *flags) {
  __shared__ int skip;
  if (threadIdx.x == 0)
    skip = flags[FLAG_NONFINITE] || flags[FLAG_SUPPORT] || flags[FLAG_EPS] || flags[FLAG_GRAM];
  __syncthreads();
  return skip != 0;
}

// Tiles of the density-based kernels: one cell per thread (32 x 8 in 2D, 8 x 8 x TZ3
// in 3D) and a halo of H cells on every side, corners included, in LDS; each face of
// the tile is formed once.
template <int DIM, int H, int TZ3 = 4>
struct DTile {
  static constexpr int TX = DIM == 2 ? 32 : 8, TY = 8, TZ = DIM == 2 ? 1 : TZ3;
  static constexpr int HZ = DIM == 2 ? 0 : H;
  static constexpr int SX = TX + 2 * H, SY = TY + 2 * H, SZ = TZ + 2 * HZ;
  static constexpr int NP = SX * SY * SZ;
  // most faces of one direction in a tile
  static constexpr int NFD = (TX + 1) * TY * TZ > TX * (TY + 1) * TZ
                                 ? ((TX + 1) * TY * TZ > TX * TY * (TZ + 1) ? (TX + 1) * TY * TZ
                                                                             : TX * TY * (TZ + 1))
                                 : (TX * (TY + 1) * TZ > TX * TY * (TZ + 1) ? TX * (TY + 1) * TZ
                                                                             : TX * TY * (TZ + 1));
  __device__ static int pt(int i, int j, int k) { return ((k + HZ) * SY + (j + H)) * SX + (i + H); }
  // tile origin of block b (x fastest)
  __device__ static void origin(const GridK &g, int64_t b, int &x0, int &y0, int &z0) {
    const int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY;
    x0 = (int)(b % ntx) * TX;
    y0 = (int)((b / ntx) % nty) * TY;
    z0 = (int)(b / ((int64_t)ntx * nty)) * TZ;
  }
  __host__ static int64_t tiles(const GridK &g) {
    return (int64_t)((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY) *
           (DIM == 3 ? (g.n[2] + TZ - 1) / TZ : 1);
  }
};

// The points of a DTile<DIM, 2> that the inviscid faces read -- the tile and its
// two-deep halo, but only where at most one coordinate lies outside the tile (the
// faces reconstruct along their normal) -- stored in three slabs: A the tile's rows
// with their x halo ((TX + 4) x TY x TZ), B the y halo of the tile's columns
// (TX x 4 x TZ), C the z halo (TX x TY x 4, 3D): 1280 points for an 8 x 8 x 8 tile
// instead of the box's 1728.
// the inviscid kernel's 3D tiles are 8 x 8 x 8 (512 threads): fewer halo points per
// cell than 8 x 8 x 4, and two blocks of eight waves per CU in FP64 (LDS 74 KB)
#ifndef IBM_DENS_TZ
#define IBM_DENS_TZ 8
#endif
template <int DIM>
struct DCross {
  using T = DTile<DIM, 2, IBM_DENS_TZ>;
  static constexpr int TX = T::TX, TY = T::TY, TZ = T::TZ;
  static constexpr int NT = TX * TY * TZ;  // threads: one per cell
  static constexpr int AX = TX + 4;
  static constexpr int NA = AX * TY * TZ, NB = TX * 4 * TZ, NC = DIM == 3 ? TX * TY * 4 : 0;
  static constexpr int NP = NA + NB + NC;
  // the halo layer (-2, -1, n, n + 1 -> 0..3) of a coordinate outside [0, n)
  __device__ static int layer(int v, int n) { return v < 0 ? v + 2 : v - n + 2; }
  __device__ static int a(int i, int j, int k) { return (k * TY + j) * AX + (i + 2); }
  __device__ static int b(int i, int j, int k) { return NA + (k * 4 + layer(j, TY)) * TX + i; }
  __device__ static int c(int i, int j, int k) { return NA + NB + (layer(k, TZ) * TY + j) * TX + i; }
  // local point of slot p (the inverse of a, b and c)
  __device__ static void point(int p, int &i, int &j, int &k) {
    if (p < NA) {
      i = p % AX - 2;
      j = (p / AX) % TY;
      k = p / (AX * TY);
    } else if (p < NA + NB) {
      const int q = p - NA, l = (q / TX) % 4;
      i = q % TX;
      j = l < 2 ? l - 2 : TY + l - 2;
      k = q / (TX * 4);
    } else {
      const int q = p - NA - NB, l = q / (TX * TY);
      i = q % TX;
      j = (q / TX) % TY;
      k = l < 2 ? l - 2 : TZ + l - 2;
    }
  }
};

// Inviscid part: rho^{n+1} = rho^n - dt D(F_rho), (rho u)** = (rho u)^n - dt D(F_m),
// (rho e_t)** = (rho e_t)^n - dt D(F_e) from the central-upwind fluxes of the
// state at step n; u** = (rho u)**/rho^{n+1} and theta** = ((rho e_t)**/rho^{n+1}
// - |u**|^2/2)/c_v into p1; the mass flux into the next state's face arrays.
template <int DIM, typename S>
__global__ __launch_bounds__(DCross<DIM>::NT) void k_dens_inviscid(GridK g, StateV<S> st, StateV<S> nxt,
                                                           S *rho1, S *m0,
                                                           S *m1, S *m2, DensPrim<S> p1,
                                                           const int *flags) {
  using X = DCross<DIM>;
  using T = typename X::T;
  constexpr int NV = DIM + 2;  // rho, u[DIM], theta
  extern __shared__ __align__(16) unsigned char smem[];
  S *lv = reinterpret_cast<S *>(smem);  // [NV][NP]
  S *lf = lv + NV * X::NP;              // [NV][NFD]
  if (dens_skip(flags)) return;
  int x0, y0, z0;
  T::origin(g, blockIdx.x, x0, y0, z0);
  // phase 1: primitives of the points the faces read (up to two layers outside the
  // box), from the state
  for (int p = threadIdx.x; p < X::NP; p += X::NT) {
    int li, lj, lk;
    X::point(p, li, lj, lk);
    const int gi = x0 + li, gj = y0 + lj, gk = z0 + lk;
    bool ok = gi >= -2 && gi <= g.n[0] + 1 && gj >= -2 && gj <= g.n[1] + 1;
    if (DIM == 3) ok = ok && gk >= -2 && gk <= g.n[2] + 1;
    if (!ok) continue;
    S r, u[3], th, pp;
    load_prim<DIM>(g, st, gi, gj, gk, r, u, th, pp);
    lv[p] = r;
#pragma unroll
    for (int q = 0; q < DIM; ++q) lv[(1 + q) * X::NP + p] = u[q];
    lv[(1 + DIM) * X::NP + p] = th;
  }
  __syncthreads();
  const int ci = threadIdx.x % T::TX, cj = (threadIdx.x / T::TX) % T::TY;
  const int ck = DIM == 3 ? threadIdx.x / (T::TX * T::TY) : 0;
  const int ix[3] = {x0 + ci, y0 + cj, z0 + ck};
  const bool valid = ix[0] < g.n[0] && ix[1] < g.n[1] && (DIM == 2 || ix[2] < g.n[2]);
  S acc[NV + 1];  // rho, m[DIM], e_t (the last unused)
#pragma unroll
  for (int v = 0; v < NV + 1; ++v) acc[v] = S(0);
  const S dt = S(g.dt);
  // phase 2: faces of one direction at a time
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int FX = T::TX + (d == 0), FY = T::TY + (d == 1), FZ = T::TZ + (d == 2);
    for (int f = threadIdx.x; f < FX * FY * FZ; f += X::NT) {
      const int fi = f % FX, fj = (f / FX) % FY, fk = f / (FX * FY);
      const int gf[3] = {x0 + fi, y0 + fj, z0 + fk};
      bool ok = true;
#pragma unroll
      for (int e = 0; e < DIM; ++e) ok = ok && gf[e] < g.n[e] + (e == d ? 1 : 0);
      if (!ok) continue;
      S r[4], u[4][3], th[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        // the point m - 2 cells from the face's high cell along d: in slab A, or in
        // the halo slab of direction d
        int lp;
        if (d == 0) {
          lp = X::a(fi + m - 2, fj, fk);
        } else if (d == 1) {
          const int j = fj + m - 2;
          lp = (j >= 0 && j < T::TY) ? X::a(fi, j, fk) : X::b(fi, j, fk);
        } else {
          const int k = fk + m - 2;
          lp = (k >= 0 && k < T::TZ) ? X::a(fi, fj, k) : X::c(fi, fj, k);
        }
        r[m] = lv[lp];
#pragma unroll
        for (int q = 0; q < DIM; ++q) u[m][q] = lv[(1 + q) * X::NP + lp];
        th[m] = lv[(1 + DIM) * X::NP + lp];
      }
      S fr, fm[3], fe;
      knp_flux<DIM, S, DIM == 3>(g, d, r, u, th, fr, fm, fe);
      lf[f] = fr;
#pragma unroll
      for (int q = 0; q < DIM; ++q) lf[(1 + q) * T::NFD + f] = fm[q];
      lf[(1 + DIM) * T::NFD + f] = fe;
      // the face belongs to this tile unless it is the next tile's first face
      if ((d == 0 ? fi : d == 1 ? fj : fk) < (d == 0 ? T::TX : d == 1 ? T::TY : T::TZ) ||
          gf[d] == g.n[d])
        nxt.F[d][fidx(g, d, gf[0], gf[1], gf[2])] = fr;
    }
    __syncthreads();
    if (valid) {
      const int step = d == 0 ? 1 : d == 1 ? FX : FX * FY;
      const int lo = ci + FX * (cj + FY * ck), hi = lo + step;
      const S ih = S(g.ih[d]);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += (lf[v * T::NFD + hi] - lf[v * T::NFD + lo]) * ih;
    }
    __syncthreads();
  }
  if (!valid) return;
  // phase 3: the update of the cell
  const int64_t c = cidx(g, ix[0], ix[1], ix[2]);
  S *mo[3] = {m0, m1, m2};
  const S r = st.rho[c];
  S kn = S(0);
#pragma unroll
  for (int q = 0; q < DIM; ++q) kn += st.mom[q][c] * st.mom[q][c];
  const S et = st.E[c] + S(0.5) * kn / r;
  const S r1 = r - dt * acc[0];
  rho1[c] = r1;
  S k2 = S(0);
#pragma unroll
  for (int q = 0; q < DIM; ++q) {
    const S mq = st.mom[q][c] - dt * acc[1 + q];
    mo[q][c] = mq;
    const S uq = mq / r1;  // u**
    p1.v[q][c] = uq;
    k2 += uq * uq;
  }
  p1.v[3][c] = ((et - dt * acc[1 + DIM]) / r1 - S(0.5) * k2) / S(g.cv);  // theta**
}

// u** and theta** at a (possibly ghost) cell of the intermediate state, from p1.
template <int DIM, typename S>
__device__ __forceinline__ void load_star(const GridK &g, const DensPrim<S> &p1, int i, int j,
                                          int k, S *u, S &th) {
  Resolved rs = resolve<DIM>(g, i, j, k);
#pragma unroll
  for (int q = 0; q < DIM; ++q) u[q] = p1.v[q][rs.c];
  th = p1.v[3][rs.c];
  if (any_side<DIM, S>(rs)) {
#pragma unroll
    for (int q = 0; q < DIM; ++q) u[q] = ghosted<DIM>(g, rs, V_U0 + q, u[q]);
    th = ghosted<DIM>(g, rs, V_TH, th);
  }
}

// Viscous and conductive part at (u**, theta**): (rho u)* = (rho u)** + dt div tau,
// (rho e)* = rho^{n+1} c_v theta** + dt (div(lambda grad_n theta**) + Phi). Face
// stress tau_{d,q} with the normal derivatives compact and the tangential ones the
// average of the two centred cell gradients, mu_f the face average; heat flux
// lambda_f d theta / d n; Phi = tau:grad u at the cell from centred gradients.
// Into ms, E_s (the body's sources are then added by the marker kernels).
// 3D tiles of the viscous kernel: 8 x 8 x 8 (512 threads; fewer halo points per cell)
#ifndef IBM_DENSV_TZ
#define IBM_DENSV_TZ 8
#endif
template <int DIM>
using DVTile = DTile<DIM, 1, IBM_DENSV_TZ>;
template <int DIM, typename S>
__global__ __launch_bounds__(DVTile<DIM>::TX * DVTile<DIM>::TY * DVTile<DIM>::TZ) void k_dens_viscous(GridK g, const S *rho1, const S *m0,
                                                          const S *m1, const S *m2,
                                                          DensPrim<S> p1, S *ms0, S *ms1,
                                                          S *ms2, S *E_s, const int *flags) {
  using T = DVTile<DIM>;
  constexpr int NT = T::TX * T::TY * T::TZ;
  constexpr int NV = DIM + 2;  // u[DIM], theta, mu
  __shared__ S lv[NV * T::NP];
  __shared__ S lf[(DIM + 1) * T::NFD];
  if (dens_skip(flags)) return;
  int x0, y0, z0;
  T::origin(g, blockIdx.x, x0, y0, z0);
  for (int p = threadIdx.x; p < T::NP; p += NT) {
    const int li = p % T::SX - 1, lj = (p / T::SX) % T::SY - 1;
    const int lk = DIM == 3 ? p / (T::SX * T::SY) - 1 : 0;
    const int gi = x0 + li, gj = y0 + lj, gk = z0 + lk;
    bool ok = gi >= -1 && gi <= g.n[0] && gj >= -1 && gj <= g.n[1];
    if (DIM == 3) ok = ok && gk >= -1 && gk <= g.n[2];
    if (!ok) continue;
    S u[3], th;
    load_star<DIM>(g, p1, gi, gj, gk, u, th);
#pragma unroll
    for (int q = 0; q < DIM; ++q) lv[q * T::NP + p] = u[q];
    lv[DIM * T::NP + p] = th;
    lv[(DIM + 1) * T::NP + p] = mu_of(g, th);
  }
  __syncthreads();
  const int ci = threadIdx.x % T::TX, cj = (threadIdx.x / T::TX) % T::TY;
  const int ck = DIM == 3 ? threadIdx.x / (T::TX * T::TY) : 0;
  const int ix[3] = {x0 + ci, y0 + cj, z0 + ck};
  const bool valid = ix[0] < g.n[0] && ix[1] < g.n[1] && (DIM == 2 || ix[2] < g.n[2]);
  auto U = [&](int q, int i, int j, int k) { return lv[q * T::NP + T::pt(i, j, k)]; };
  S dT[3] = {S(0), S(0), S(0)}, dQ = S(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int FX = T::TX + (d == 0), FY = T::TY + (d == 1), FZ = T::TZ + (d == 2);
    for (int f = threadIdx.x; f < FX * FY * FZ; f += NT) {
      const int fi = f % FX, fj = (f / FX) % FY, fk = f / (FX * FY);
      const int gf[3] = {x0 + fi, y0 + fj, z0 + fk};
      bool ok = true;
#pragma unroll
      for (int e = 0; e < DIM; ++e) ok = ok && gf[e] < g.n[e] + (e == d ? 1 : 0);
      if (!ok) continue;
      int P[3] = {fi, fj, fk};
      const int Q[3] = {fi, fj, fk};
      P[d] -= 1;
      const S thP = U(DIM, P[0], P[1], P[2]), thQ = U(DIM, Q[0], Q[1], Q[2]);
      const S muf = S(0.5) * (U(DIM + 1, P[0], P[1], P[2]) + U(DIM + 1, Q[0], Q[1], Q[2]));
      const S ih = S(g.ih[d]);
      S dn[3], tg[3] = {S(0), S(0), S(0)};
#pragma unroll
      for (int q = 0; q < DIM; ++q) dn[q] = (U(q, Q[0], Q[1], Q[2]) - U(q, P[0], P[1], P[2])) * ih;
      S divf = dn[d];
#pragma unroll
      for (int t = 0; t < DIM; ++t) {
        if (t == d) continue;
        const S hh = S(0.5 * g.ih[t]);
        int a1[3] = {P[0], P[1], P[2]}, a0[3] = {P[0], P[1], P[2]};
        int b1[3] = {Q[0], Q[1], Q[2]}, b0[3] = {Q[0], Q[1], Q[2]};
        a1[t] += 1;
        a0[t] -= 1;
        b1[t] += 1;
        b0[t] -= 1;
        const S gdP = (U(d, a1[0], a1[1], a1[2]) - U(d, a0[0], a0[1], a0[2])) * hh;
        const S gtP = (U(t, a1[0], a1[1], a1[2]) - U(t, a0[0], a0[1], a0[2])) * hh;
        const S gdQ = (U(d, b1[0], b1[1], b1[2]) - U(d, b0[0], b0[1], b0[2])) * hh;
        const S gtQ = (U(t, b1[0], b1[1], b1[2]) - U(t, b0[0], b0[1], b0[2])) * hh;
        tg[t] = S(0.5) * (gdP + gdQ);
        divf += S(0.5) * (gtP + gtQ);
      }
#pragma unroll
      for (int q = 0; q < DIM; ++q)
        lf[q * T::NFD + f] =
            (q == d) ? muf * (S(2) * dn[d] - S(2.0 / 3.0) * divf) : muf * (dn[q] + tg[q]);
      lf[DIM * T::NFD + f] = S(g.cp_Pr) * muf * (thQ - thP) * ih;
    }
    __syncthreads();
    if (valid) {
      const int step = d == 0 ? 1 : d == 1 ? FX : FX * FY;
      const int lo = ci + FX * (cj + FY * ck), hi = lo + step;
      const S ih = S(g.ih[d]);
      dQ += (lf[DIM * T::NFD + hi] - lf[DIM * T::NFD + lo]) * ih;
#pragma unroll
      for (int q = 0; q < DIM; ++q) dT[q] += (lf[q * T::NFD + hi] - lf[q * T::NFD + lo]) * ih;
    }
    __syncthreads();
  }
  if (!valid) return;
  S gr[3][3];
#pragma unroll
  for (int b2 = 0; b2 < DIM; ++b2) {
    int a1[3] = {ci, cj, ck}, a0[3] = {ci, cj, ck};
    a1[b2] += 1;
    a0[b2] -= 1;
    const S hh = S(0.5 * g.ih[b2]);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      gr[a][b2] = (U(a, a1[0], a1[1], a1[2]) - U(a, a0[0], a0[1], a0[2])) * hh;
  }
  S divu = S(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) divu += gr[a][a];
  S phi = S(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int b2 = 0; b2 < DIM; ++b2) phi += (gr[a][b2] + gr[b2][a]) * gr[a][b2];
  const S thc = U(DIM, ci, cj, ck);
  phi = U(DIM + 1, ci, cj, ck) * (phi - S(2.0 / 3.0) * divu * divu);
  const int64_t c = cidx(g, ix[0], ix[1], ix[2]);
  const S *m[3] = {m0, m1, m2};
  S *ms[3] = {ms0, ms1, ms2};
  const S dt = S(g.dt);
#pragma unroll
  for (int q = 0; q < DIM; ++q) ms[q][c] = m[q][c] + dt * dT[q];
  E_s[c] = rho1[c] * S(g.cv) * thc + dt * (dQ + phi);
}

// The new state from the sourced results (rho*, m**, E**): checked (positive,
// finite; a failure sets the flags and the step number), written unless an
// earlier step of the call failed; partial sums of the mass.
template <int DIM, typename S>
__global__ __launch_bounds__(kBlockThreads) void k_dens_finish(GridK g, const S *rho_s,
                                                          const S *ms0, const S *ms1,
                                                          const S *ms2, const S *E_s,
                                                          StateV<S> nxt, double *partials,
                                                          int *flags, int tag) {
  __shared__ double lds[32];
  if (dens_skip(flags)) return;
  const S *ms[3] = {ms0, ms1, ms2};
  double mass = 0.0;
  bool bad = false;
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    const S r = rho_s[c], e = E_s[c];
    nxt.rho[c] = r;
    nxt.E[c] = e;
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      nxt.mom[q][c] = ms[q][c];
      bad = bad || !isfinite(double(ms[q][c]));
    }
    bad = bad || !(r > S(0)) || !(e > S(0)) || !isfinite(double(r)) || !isfinite(double(e));
    mass += double(r) * g.dV;
  }
  if (bad) {
    atomicOr(flags + FLAG_NONFINITE, 1);
    atomicCAS(flags + FLAG_BAD_STEP, 0, tag + 1);
  }
  double s = block_sum(mass, lds);
  if (threadIdx.x == 0) partials[PART_MASS * kMaxBlocks + blockIdx.x] = s;
}

// ------------------------------------- FP32 form: pressure by iterative refinement
// x and the outer residual r = b - A x are FP64; each inner solve A d = r runs the
// single-reduction CG on FP32 vectors with FP64 dot products to a relative 1e-5 (or
// kInnerMax iterations), then x += d and the FP64 residual is formed again. The
// solve ends when the FP64 residual meets |r| <= rtol |b|. One kernel per
// iteration: an inner CG iteration, or a refinement that also starts the next
// inner solve (w = A r of the new FP32 residual).

// Set-up of the FP32 form: as k_setup2, with the FP64 start residual
// handed to the inner solve as FP32 (r32) and its FP64 r.r as the outer partial.
template <int DIM>
__global__ __launch_bounds__(kBlockThreads) void k_setup2m(GridK g, const float *rho_n, const float *mh0,
                                                      const float *mh1, const float *mh2,
                                                      float *Fh0, float *Fh1, float *Fh2,
                                                      const float *psi, const double *x,
                                                      double *b, float *r32, double *partials,
                                                      CgScal *cs, int tag) {
  using S = float;
  __shared__ double lds[32];
  const S *mh[3] = {mh0, mh1, mh2};
  S *Fh[3] = {Fh0, Fh1, Fh2};
  double sums[2] = {0.0, 0.0};
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    const int ix[3] = {i, j, k};
    double div = 0.0, aff = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int hi[3] = {i, j, k};
      hi[d] += 1;
      S fl = face_from_cells<DIM, S>(g, mh, rho_n, d, i, j, k);
      S fh = face_from_cells<DIM, S>(g, mh, rho_n, d, hi[0], hi[1], hi[2]);
      Fh[d][fidx(g, d, i, j, k)] = fl;
      if (ix[d] == g.n[d] - 1) Fh[d][fidx(g, d, hi[0], hi[1], hi[2])] = fh;
      div += (double(fh) - double(fl)) * g.ih[d];
      if (g.bc[d][0] != BC_PERIODIC) {
        if (ix[d] == 0 && g.bc[d][0] == BC_OUTFLOW) aff += 2.0 * g.p_inf * g.ih[d] * g.ih[d];
        if (ix[d] == g.n[d] - 1 && g.bc[d][1] == BC_OUTFLOW)
          aff += 2.0 * g.p_inf * g.ih[d] * g.ih[d];
      }
    }
    const double bc_ = double(rho_n[c]) - g.dt * div + g.dt * g.dt * aff;
    const double xc = x[c];
    const double ax = helm_at<DIM>(g, psi, [&](int64_t q) { return x[q]; }, i, j, k, c, xc);
    const double rc = bc_ - ax;
    b[c] = bc_;
    r32[c] = float(rc);
    sums[0] += bc_ * bc_;
    sums[1] += rc * rc;
  }
  block_sum_n<2>(sums, lds);
  if (threadIdx.x == 0) {
    partials[PART_BB * kMaxBlocks + blockIdx.x] = sums[0];
    partials[PART_O * kMaxBlocks + blockIdx.x] = sums[1];
    if (blockIdx.x == 0) {
      cs->done = 0;
      cs->iters = 0;
      cs->step_tag = tag;
      cs->xfinal = 0;
      cs->outer[0] = MS_START;
      cs->xpar[0] = 0;
      cs->inner_it[0] = 0;
      cs->rr_in0[0] = 0.0;
    }
  }
}

// FP32 pressure operator at one cell (single precision arithmetic); v(i, j, k, m)
// gives the value of cell m at (i, j, k).
template <int DIM, typename VF>
__device__ __forceinline__ float helm32_at(const GridK &g, const float *psi, VF v, int i, int j,
                                           int k, int64_t c, float vc) {
  float lap = 0.0f;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const float ih = float(g.ih[d]);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      int ix[3] = {i, j, k};
      ix[d] += side ? 1 : -1;
      const int n = g.n[d];
      float gf;
      if (ix[d] >= 0 && ix[d] < n) {
        gf = (v(ix[0], ix[1], ix[2], cidx(g, ix[0], ix[1], ix[2])) - vc) * ih;
      } else if (g.bc[d][0] == BC_PERIODIC) {
        ix[d] = ix[d] < 0 ? ix[d] + n : ix[d] - n;
        gf = (v(ix[0], ix[1], ix[2], cidx(g, ix[0], ix[1], ix[2])) - vc) * ih;
      } else {
        gf = (g.bc[d][side] == BC_OUTFLOW) ? (-2.0f * vc) * ih : 0.0f;
      }
      lap += gf * ih;
    }
  }
  return psi[c] * vc - float(g.dt * g.dt) * lap;
}

// Stages of the FP32 form's solve, one kernel each (the stage a kernel runs is in
// CgScal::outer of its slot):
//  MS_START: the partials hold the FP64 r.r of the outer residual r (set-up or a
//            refinement): |r| <= rtol |b| -> done; otherwise w = A r32 and the
//            partials of r32.r32, w.r32 (r32 is copied to the next slot);
//  MS_FIRST: first iteration of an inner solve: p = r, s = w, d = alpha p;
//  MS_INNER: inner single-reduction iteration, or, once the inner residual is 1e-4
//            of its start or meets the outer tolerance, a refinement: x' = x + d,
//            r = b - A x' in FP64, r32 = r, partial of r.r (-> MS_START).
// The step of a kernel of the refinement solve: its stage, whether an inner solve
// ends in a refinement, the inner CG's step lengths, the x buffer in use.
struct McgStep {
  int stage;
  bool refine;
  double alpha, beta;
  int xp;
};

// The common start of the refinement solve's kernels: the sums of the previous
// kernel's partials, the stage's tests, and block 0's record of the scalars (the
// progress word posted to the host). False once the solve has ended.
__device__ __forceinline__ bool mcg_head(int it, const double *partials, CgScal *cs,
                                         const int *flags, uint64_t *progress, double *lds,
                                         int &done0, McgStep &ms) {
  if (threadIdx.x == 0) done0 = cs->done;
  __syncthreads();
  if (done0) return false;
  const int nb = gridDim.x, sl = it & 1, sn = sl ^ 1;
  const int stage = cs->outer[sl];
  double gd[2] = {0.0, 0.0}, rro = 0.0;
  if (stage == MS_START)
    rro = sum_partials(partials + (PART_O + sl) * kMaxBlocks, nb, lds);
  else
    sum_partials2(partials + (PART_G + sl) * kMaxBlocks, partials + (PART_D + sl) * kMaxBlocks,
                  nb, lds, gd);
  const double gam = gd[0], del = gd[1];
  const double bb = (it == 0) ? sum_partials(partials + PART_BB * kMaxBlocks, nb, lds) : cs->bb;
  const double tol2 = cs->tol2;
  const int err = (flags[FLAG_NONFINITE] ? 1 : 0) | (flags[FLAG_SUPPORT] ? 2 : 0) |
                  (flags[FLAG_EPS] ? 4 : 0) | (flags[FLAG_GRAM] ? 8 : 0);
  const int xp = cs->xpar[sl];
  const bool bad = err != 0;
  bool conv = false, out = false, refine = false;
  double alpha = 0.0, beta = 0.0;
  int ni = 0;
  if (stage == MS_START) {
    conv = rro <= tol2 * bb;
    out = !conv && (it >= cs->maxit || bad || !(rro == rro));
  } else if (stage == MS_FIRST) {
    alpha = gam / del;
  } else {
    ni = cs->inner_it[sl];
    // an inner solve ends at 1e-4 of its start, or once its residual already meets
    // the outer tolerance (the refinement then checks that in FP64)
    refine = gam <= kInnerTol2 * cs->rr_in0[sl] || gam <= tol2 * bb || ni >= kInnerMax ||
             it >= cs->maxit || bad || !(gam == gam);
    if (!refine) {
      beta = gam / cs->rr[(it - 1) & 1];
      alpha = gam / (del - beta * gam / cs->alpha[(it - 1) & 1]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (it == 0) cs->bb = bb;
    cs->iters = it;
    if (stage == MS_START) {
      cs->res = bb > 0.0 ? sqrt(rro / bb) : 0.0;
      if (conv || out) {
        cs->done = conv ? 1 : 2;
        cs->xfinal = xp;
      } else {
        cs->outer[sn] = MS_FIRST;
        cs->xpar[sn] = xp;
      }
    } else if (stage == MS_FIRST) {
      cs->rr[sl] = gam;
      cs->alpha[sl] = alpha;
      cs->rr_in0[sn] = gam;
      cs->inner_it[sn] = 1;
      cs->outer[sn] = MS_INNER;
      cs->xpar[sn] = xp;
    } else if (refine) {
      cs->outer[sn] = MS_START;
      cs->xpar[sn] = xp ^ 1;
    } else {
      cs->rr[sl] = gam;
      cs->alpha[sl] = alpha;
      cs->rr_in0[sn] = cs->rr_in0[sl];
      cs->inner_it[sn] = ni + 1;
      cs->outer[sn] = MS_INNER;
      cs->xpar[sn] = xp;
    }
    if (progress)
      __hip_atomic_store(progress, pack_progress(cs->step_tag, it, err, conv ? 1 : out ? 2 : 0),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  ms.stage = stage;
  ms.refine = refine;
  ms.alpha = alpha;
  ms.beta = beta;
  ms.xp = xp;
  return !(conv || out);
}

// The common end: the partials for the next kernel (the FP64 r.r of a refinement, or
// the inner CG's r.r and w.r).
__device__ __forceinline__ void mcg_tail(int it, const McgStep &ms, double *sums,
                                         double *partials, double *lds) {
  const int sn = (it & 1) ^ 1;
  block_sum_n<2>(sums, lds);
  if (threadIdx.x == 0) {
    if (ms.refine) {
      partials[(PART_O + sn) * kMaxBlocks + blockIdx.x] = sums[0];
    } else {
      partials[(PART_G + sn) * kMaxBlocks + blockIdx.x] = sums[0];
      partials[(PART_D + sn) * kMaxBlocks + blockIdx.x] = sums[1];
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(kBlockThreads) void k_mcg_iter(
    GridK g, int it, const float *__restrict__ psi, const double *__restrict__ b, double *x0,
    double *x1, const float *__restrict__ r, const float *__restrict__ w,
    const float *__restrict__ sold, float *__restrict__ rn, float *__restrict__ wn,
    float *__restrict__ snew, float *__restrict__ p, float *__restrict__ d, double *partials,
    CgScal *cs, const int *flags, uint64_t *progress) {
  __shared__ double lds[32];
  __shared__ int done0;
  McgStep ms;
  if (!mcg_head(it, partials, cs, flags, progress, lds, done0, ms)) return;
  const int stage = ms.stage, xp = ms.xp;
  const bool refine = ms.refine;
  const double alpha = ms.alpha, beta = ms.beta;
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  double sums[2] = {0.0, 0.0};
  if (stage == MS_START) {
    for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
      int i, j, k;
      if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
      const int64_t c = cidx(g, i, j, k);
      const float rc = r[c];
      const float wc = helm32_at<DIM>(g, psi, [&](int, int, int, int64_t m) { return r[m]; }, i,
                                      j, k, c, rc);
      rn[c] = rc;
      wn[c] = wc;
      sums[0] += double(rc) * double(rc);
      sums[1] += double(wc) * double(rc);
    }
  } else if (refine) {
    const double *xo = xp ? x1 : x0;
    double *xnew = xp ? x0 : x1;
    auto xv = [&](int64_t m) { return xo[m] + double(d[m]); };
    for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
      int i, j, k;
      if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
      const int64_t c = cidx(g, i, j, k);
      const double xc = xv(c);
      const double rc = b[c] - helm_at<DIM>(g, psi, xv, i, j, k, c, xc);
      xnew[c] = xc;
      rn[c] = float(rc);
      sums[0] += rc * rc;
    }
  } else {
    const bool first = stage == MS_FIRST;
    const float af = float(alpha), bf = float(beta);
    for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
      int i, j, k;
      if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
      const int64_t c = cidx(g, i, j, k);
      float pc, sc, rnc, wnc;
      if (first) {  // the old p, s, d are not read
        pc = r[c];
        sc = w[c];
        d[c] = af * pc;
        rnc = pc - af * sc;
        auto rv = [&](int, int, int, int64_t m) { return r[m] - af * w[m]; };
        wnc = helm32_at<DIM>(g, psi, rv, i, j, k, c, rnc);
      } else {
        pc = r[c] + bf * p[c];
        sc = w[c] + bf * sold[c];
        d[c] += af * pc;
        rnc = r[c] - af * sc;
        auto rv = [&](int, int, int, int64_t m) { return r[m] - af * (w[m] + bf * sold[m]); };
        wnc = helm32_at<DIM>(g, psi, rv, i, j, k, c, rnc);
      }
      p[c] = pc;
      snew[c] = sc;
      rn[c] = rnc;
      wn[c] = wnc;
      sums[0] += double(rnc) * double(rnc);
      sums[1] += double(wnc) * double(rnc);
    }
  }
  mcg_tail(it, ms, sums, partials, lds);
}

// ------------------------------ FP32 form's refinement solve by z-columns (3D)
// The stages of k_mcg_iter (same head, same arithmetic) with the sweeps of the
// column kernels: a block owns a kColTX x kColTY tile and walks a chunk of planes,
// the stencil variable of planes k-1, k, k+1 of a thread's column in registers and
// its x-y neighbours through an LDS plane with a one-cell halo.
enum { MC_START = 0, MC_FIRST = 1, MC_INNER = 2, MC_REFINE = 3 };

template <int KIND>
__device__ __forceinline__ void mcg_col_sweep(const GridK &g, int tiles_x, int tiles_y, int zc,
                                              int64_t items, float af, float bf,
                                              const float *__restrict__ psi,
                                              const double *__restrict__ b,
                                              const double *__restrict__ xo,
                                              double *__restrict__ xnew,
                                              const float *__restrict__ r,
                                              const float *__restrict__ w,
                                              const float *__restrict__ sold,
                                              float *__restrict__ rn, float *__restrict__ wn,
                                              float *__restrict__ snew, float *__restrict__ p,
                                              float *__restrict__ d, double *plane_mem,
                                              double *sums) {
  using V = typename std::conditional<KIND == MC_REFINE, double, float>::type;
  V(*plane_lds)[kColSlots] = reinterpret_cast<V(*)[kColSlots]>(plane_mem);
  const int lx = threadIdx.x % kColTX, ly = threadIdx.x / kColTX;
  const int64_t nb = gridDim.x, bk = blockIdx.x;
  const int64_t rank = (bk & 7) * (nb >> 3) + (bk >> 3);
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const int64_t pl = (int64_t)n0 * n1;
  const V ih0 = V(g.ih[0]), ih1 = V(g.ih[1]), ih2 = V(g.ih[2]);
  const int myslot = (ly + 1) * kColPitch + (lx + 1);
  // one plane of a thread's own column: the stencil variable and what the cell's
  // update needs
  struct Own {
    V v;
    float r, w, s, pp, dd, ps;
    double x, bv;
  };
  auto value = [&](int64_t c) -> V {
    if (KIND == MC_START) return V(r[c]);
    if (KIND == MC_FIRST) return V(r[c] - af * w[c]);
    if (KIND == MC_INNER) return V(r[c] - af * (w[c] + bf * sold[c]));
    return V(xo[c] + double(d[c]));
  };
  for (int64_t item = rank; item < items; item += nb) {
    const int tx = (int)(item % tiles_x);
    const int64_t rest = item / tiles_x;
    const int ty = (int)(rest % tiles_y);
    const int ch = (int)(rest / tiles_y);
    const int i = tx * kColTX + lx, j = ty * kColTY + ly;
    const int k0 = ch * zc, k1 = min(k0 + zc, n2);
    const bool inside = i < n0 && j < n1;
    double sx, sy;
    const int64_t col = col_resolve(g, 0, i, sx) + (int64_t)n0 * col_resolve(g, 1, j, sy);
    const double sxy = sx * sy;
    int hslot = -1;
    int64_t hcol = 0;
    double hsig = 1.0;
    col_halo_slot(g, tx, ty, hslot, hcol, hsig);
    auto load = [&](int k, Own &o) {
      double sz;
      const int64_t c = col + pl * col_resolve(g, 2, k, sz);
      o.v = V(sxy * sz) * value(c);
      if (inside && k >= k0 && k < k1) {
        o.ps = psi[c];
        if (KIND == MC_REFINE) {
          o.x = xo[c] + double(d[c]);
          o.bv = b[c];
        } else {
          o.r = r[c];
          if (KIND != MC_START) o.w = w[c];
          if (KIND == MC_INNER) {
            o.s = sold[c];
            o.pp = p[c];
            o.dd = d[c];
          }
        }
      }
    };
    auto load_halo = [&](int k, V &hv) {
      if (hslot < 0) return;
      double sz;
      const int64_t c = hcol + pl * col_resolve(g, 2, k, sz);
      hv = V(hsig * sz) * value(c);
    };
    Own A, B, C, M;
    load(k0 - 1, M);
    load(k0, A);
    load(k0 + 1, B);
    V hv = V(0);
    load_halo(k0, hv);
    V vm = M.v;
    for (int k = k0; k < k1; ++k) {
      V hv2 = V(0);
      if (k + 2 <= k1) load(k + 2, C);
      if (k + 1 < k1) load_halo(k + 1, hv2);
      V *lp = plane_lds[(k - k0) & 1];
      lp[myslot] = A.v;
      if (hslot >= 0) lp[hslot] = hv;
      __syncthreads();
      if (inside) {
        const V vc = A.v;
        V lap = V(0), gf;
        gf = (lp[myslot - 1] - vc) * ih0;
        lap += gf * ih0;
        gf = (lp[myslot + 1] - vc) * ih0;
        lap += gf * ih0;
        gf = (lp[myslot - kColPitch] - vc) * ih1;
        lap += gf * ih1;
        gf = (lp[myslot + kColPitch] - vc) * ih1;
        lap += gf * ih1;
        gf = (vm - vc) * ih2;
        lap += gf * ih2;
        gf = (B.v - vc) * ih2;
        lap += gf * ih2;
        const int64_t c = col + pl * k;
        if (KIND == MC_REFINE) {
          const double ax = double(A.ps) * double(vc) - g.dt * g.dt * double(lap);
          const double rc = A.bv - ax;
          xnew[c] = A.x;
          rn[c] = float(rc);
          sums[0] += rc * rc;
        } else {
          const float wc = A.ps * float(vc) - float(g.dt * g.dt) * float(lap);
          if (KIND == MC_START) {
            rn[c] = A.r;
          } else {
            const float pc = KIND == MC_FIRST ? A.r : A.r + bf * A.pp;
            const float sc = KIND == MC_FIRST ? A.w : A.w + bf * A.s;
            if (KIND == MC_FIRST)
              d[c] = af * pc;
            else
              d[c] = A.dd + af * pc;
            p[c] = pc;
            snew[c] = sc;
            rn[c] = float(vc);
          }
          wn[c] = wc;
          sums[0] += double(float(vc)) * double(float(vc));
          sums[1] += double(wc) * double(float(vc));
        }
      }
      vm = A.v;
      A = B;
      B = C;
      hv = hv2;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kColThreads) void k_mcg_col(
    GridK g, int it, int tiles_x, int tiles_y, int zc, int64_t items,
    const float *__restrict__ psi, const double *__restrict__ b, double *x0, double *x1,
    const float *__restrict__ r, const float *__restrict__ w, const float *__restrict__ sold,
    float *__restrict__ rn, float *__restrict__ wn, float *__restrict__ snew,
    float *__restrict__ p, float *__restrict__ d, double *partials, CgScal *cs,
    const int *flags, uint64_t *progress) {
  __shared__ double lds[32];
  __shared__ int done0;
  __shared__ double plane_mem[2 * kColSlots];
  McgStep m;
  if (!mcg_head(it, partials, cs, flags, progress, lds, done0, m)) return;
  double sums[2] = {0.0, 0.0};
  const float af = float(m.alpha), bf = float(m.beta);
  const double *xo = m.xp ? x1 : x0;
  double *xn = m.xp ? x0 : x1;
  if (m.stage == MS_START)
    mcg_col_sweep<MC_START>(g, tiles_x, tiles_y, zc, items, af, bf, psi, b, xo, xn, r, w, sold,
                            rn, wn, snew, p, d, plane_mem, sums);
  else if (m.refine)
    mcg_col_sweep<MC_REFINE>(g, tiles_x, tiles_y, zc, items, af, bf, psi, b, xo, xn, r, w, sold,
                             rn, wn, snew, p, d, plane_mem, sums);
  else if (m.stage == MS_FIRST)
    mcg_col_sweep<MC_FIRST>(g, tiles_x, tiles_y, zc, items, af, bf, psi, b, xo, xn, r, w, sold,
                            rn, wn, snew, p, d, plane_mem, sums);
  else
    mcg_col_sweep<MC_INNER>(g, tiles_x, tiles_y, zc, items, af, bf, psi, b, xo, xn, r, w, sold,
                            rn, wn, snew, p, d, plane_mem, sums);
  mcg_tail(it, m, sums, partials, lds);
}

// Pressure with its ghost rule (zero gradient at inflow and slip, p_inf on
// outflow faces).
template <int DIM>
__device__ __forceinline__ double pres_at(const GridK &g, const double *x, int i, int j, int k) {
  Resolved r = resolve<DIM>(g, i, j, k);
  return ghosted<DIM>(g, r, V_P, x[r.c]);
}

// Correction: F^{n+1} = F^ - dt grad_f p; rho^{n+1} = rho^n - dt D(F^{n+1});
// m^{n+1} = m^ - dt G_c p; E^{n+1} = rho^{n+1} c_v theta**. Writes the other
// state copy; flags non-finite results; per-block partial sums of the mass.
template <int DIM, typename S>
__global__ __launch_bounds__(kBlockThreads) void k_correct(GridK g, StateV<S> cur, StateV<S> nxt,
                                                      const S *rho_s, const S *E_s, const S *mh0,
                                                      const S *mh1, const S *mh2, const S *Fh0,
                                                      const S *Fh1, const S *Fh2,
                                                      const double *xa, const double *xb,
                                                      double *partials, int *flags,
                                                      const CgScal *cs, int tag) {
  __shared__ double lds[32];
  // Runs only after a finished solve of this step and while no earlier step has
  // failed: a failed step leaves the state it started from untouched. (Decided by
  // one thread: other blocks may raise a flag while this one starts.)
  __shared__ int skip;
  // the solution buffer of the FP32 form's solve (final once the solve has ended);
  // loaded with the test, before the barrier
  const int xfinal = cs->xfinal;
  if (threadIdx.x == 0)
    skip = cs->step_tag != tag || cs->done == 0 || flags[FLAG_NONFINITE] ||
           flags[FLAG_SUPPORT] || flags[FLAG_EPS] || flags[FLAG_GRAM];
  __syncthreads();
  if (skip) return;
  const double *x = xfinal ? xb : xa;
  const S *mh[3] = {mh0, mh1, mh2};
  const S *Fh[3] = {Fh0, Fh1, Fh2};
  const double dt = g.dt;
  double m = 0.0;
  bool bad = false;
  int64_t t0, t1;
  block_tiles(g, t0, t1);
  for (int64_t t = t0 + tile_group(); t < t1; t += tile_groups()) {
    int i, j, k;
    if (!cell_in_tile<DIM>(g, t, i, j, k)) continue;
    const int64_t c = cidx(g, i, j, k);
    const int ix[3] = {i, j, k};
    const double xc = pres_at<DIM>(g, x, i, j, k);
    double div = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int lo[3] = {i, j, k}, hi[3] = {i, j, k};
      lo[d] -= 1;
      hi[d] += 1;
      const double xl = pres_at<DIM>(g, x, lo[0], lo[1], lo[2]);
      const double xh = pres_at<DIM>(g, x, hi[0], hi[1], hi[2]);
      const int64_t fl = fidx(g, d, i, j, k), fh = fidx(g, d, hi[0], hi[1], hi[2]);
      const double Fl = double(Fh[d][fl]) - dt * ((xc - xl) * g.ih[d]);
      const double Fu = double(Fh[d][fh]) - dt * ((xh - xc) * g.ih[d]);
      nxt.F[d][fl] = S(Fl);
      if (ix[d] == g.n[d] - 1) nxt.F[d][fh] = S(Fu);
      div += (Fu - Fl) * g.ih[d];
      const double mn = double(mh[d][c]) - dt * ((xh - xl) * (0.5 * g.ih[d]));
      nxt.mom[d][c] = S(mn);
      bad = bad || !isfinite(mn);
    }
    const double rn = double(cur.rho[c]) - dt * div;
    const double theta = double(E_s[c] / (rho_s[c] * S(g.cv)));
    const double En = rn * g.cv * theta;
    nxt.rho[c] = S(rn);
    nxt.E[c] = S(En);
    bad = bad || !(rn > 0.0) || !(theta > 0.0) || !isfinite(rn) || !isfinite(En);
    m += rn * g.dV;
  }
  if (bad) {
    atomicOr(flags + FLAG_NONFINITE, 1);
    atomicCAS(flags + FLAG_BAD_STEP, 0, tag + 1);
  }
  double s = block_sum(m, lds);
  if (threadIdx.x == 0) partials[PART_MASS * kMaxBlocks + blockIdx.x] = s;
}

// 3D correction by z-columns (k_correct's arithmetic, in the same order): a block
// owns a kColTX x kColTY tile and walks a chunk of planes; the pressure of a plane
// with a one-cell halo is shared through LDS, that of planes k-1 and k+1 of a
// thread's own column stays in registers. Beyond a side the pressure takes its ghost
// rule (zero gradient at inflow and slip, p_inf on the face at outflow); periodic
// directions wrap.
template <typename S>
__global__ __launch_bounds__(kColThreads) void k_correct_col(
    GridK g, int tiles_x, int tiles_y, int zc, int64_t items, StateV<S> cur, StateV<S> nxt,
    const S *__restrict__ rho_s, const S *__restrict__ E_s, const S *__restrict__ mh0,
    const S *__restrict__ mh1, const S *__restrict__ mh2, const S *__restrict__ Fh0,
    const S *__restrict__ Fh1, const S *__restrict__ Fh2, const double *xa, const double *xb,
    double *partials, int *flags, const CgScal *cs, int tag) {
  __shared__ double lds[32];
  __shared__ int skip;
  __shared__ double x_lds[2][kColSlots];
  // as k_correct: only after a finished solve of this step and while no earlier step
  // has failed
  const int xfinal = cs->xfinal;
  if (threadIdx.x == 0)
    skip = cs->step_tag != tag || cs->done == 0 || flags[FLAG_NONFINITE] ||
           flags[FLAG_SUPPORT] || flags[FLAG_EPS] || flags[FLAG_GRAM];
  __syncthreads();
  if (skip) return;
  const double *x = xfinal ? xb : xa;
  const int lx = threadIdx.x % kColTX, ly = threadIdx.x / kColTX;
  const int64_t nb = gridDim.x, bk = blockIdx.x;
  const int64_t rank = (bk & 7) * (nb >> 3) + (bk >> 3);
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const int64_t pl = (int64_t)n0 * n1;
  const int fx0 = g.fn[0][0];
  const int64_t fpl1 = (int64_t)n0 * g.fn[1][1];
  const double dt = g.dt, p2 = 2.0 * g.p_inf;
  const double ih0 = g.ih[0], ih1 = g.ih[1], ih2 = g.ih[2];
  const int myslot = (ly + 1) * kColPitch + (lx + 1);
  // ghost of the pressure from the mirror value and the side's sign (-1: outflow)
  auto ghost = [&](double v, double sg) { return sg < 0.0 ? p2 - v : v; };
  double mass = 0.0;
  bool bad = false;
  for (int64_t item = rank; item < items; item += nb) {
    const int tx = (int)(item % tiles_x);
    const int64_t rest = item / tiles_x;
    const int ty = (int)(rest % tiles_y);
    const int ch = (int)(rest / tiles_y);
    const int i = tx * kColTX + lx, j = ty * kColTY + ly;
    const int k0 = ch * zc, k1 = min(k0 + zc, n2);
    const bool inside = i < n0 && j < n1;
    double sx, sy;
    const int64_t col = col_resolve(g, 0, i, sx) + (int64_t)n0 * col_resolve(g, 1, j, sy);
    const double sxy = sx * sy;
    int hslot = -1;
    int64_t hcol = 0;
    double hsig = 1.0;
    col_halo_slot(g, tx, ty, hslot, hcol, hsig);
    struct Own {
      double x;
      S fxl, fxh, fyl, fyh, fzl, fzh, m0, m1, m2, rs, es, rn;
    };
    auto load = [&](int k, Own &o) {
      double sz;
      const int64_t c = col + pl * col_resolve(g, 2, k, sz);
      o.x = ghost(x[c], sxy * sz);
      if (inside && k >= k0 && k < k1) {
        const int64_t fx = i + (int64_t)fx0 * (j + (int64_t)n1 * k);
        const int64_t fy = i + (int64_t)n0 * j + fpl1 * k;
        o.fxl = Fh0[fx];
        o.fxh = Fh0[fx + 1];
        o.fyl = Fh1[fy];
        o.fyh = Fh1[fy + n0];
        o.fzl = Fh2[c];
        o.fzh = Fh2[c + pl];
        o.m0 = mh0[c];
        o.m1 = mh1[c];
        o.m2 = mh2[c];
        o.rs = rho_s[c];
        o.es = E_s[c];
        o.rn = cur.rho[c];
      }
    };
    auto load_halo = [&](int k, double &hv) {
      if (hslot < 0) return;
      double sz;
      const int64_t c = hcol + pl * col_resolve(g, 2, k, sz);
      hv = ghost(x[c], hsig * sz);
    };
    Own A, B, C, M;
    load(k0 - 1, M);
    load(k0, A);
    load(k0 + 1, B);
    double hv = 0.0;
    load_halo(k0, hv);
    double xm = M.x;
    for (int k = k0; k < k1; ++k) {
      double hv2 = 0.0;
      if (k + 2 <= k1) load(k + 2, C);
      if (k + 1 < k1) load_halo(k + 1, hv2);
      double *lp = x_lds[(k - k0) & 1];
      lp[myslot] = A.x;
      if (hslot >= 0) lp[hslot] = hv;
      __syncthreads();
      if (inside) {
        const int64_t c = col + pl * k;
        const double xc = A.x;
        double div = 0.0;
        // x
        {
          const double xl = lp[myslot - 1], xh = lp[myslot + 1];
          const double Fl = double(A.fxl) - dt * ((xc - xl) * ih0);
          const double Fu = double(A.fxh) - dt * ((xh - xc) * ih0);
          const int64_t f = i + (int64_t)fx0 * (j + (int64_t)n1 * k);
          nxt.F[0][f] = S(Fl);
          if (i == n0 - 1) nxt.F[0][f + 1] = S(Fu);
          div += (Fu - Fl) * ih0;
          const double mn = double(A.m0) - dt * ((xh - xl) * (0.5 * ih0));
          nxt.mom[0][c] = S(mn);
          bad = bad || !isfinite(mn);
        }
        // y
        {
          const double xl = lp[myslot - kColPitch], xh = lp[myslot + kColPitch];
          const double Fl = double(A.fyl) - dt * ((xc - xl) * ih1);
          const double Fu = double(A.fyh) - dt * ((xh - xc) * ih1);
          const int64_t f = i + (int64_t)n0 * j + fpl1 * k;
          nxt.F[1][f] = S(Fl);
          if (j == n1 - 1) nxt.F[1][f + n0] = S(Fu);
          div += (Fu - Fl) * ih1;
          const double mn = double(A.m1) - dt * ((xh - xl) * (0.5 * ih1));
          nxt.mom[1][c] = S(mn);
          bad = bad || !isfinite(mn);
        }
        // z
        {
          const double xl = xm, xh = B.x;
          const double Fl = double(A.fzl) - dt * ((xc - xl) * ih2);
          const double Fu = double(A.fzh) - dt * ((xh - xc) * ih2);
          nxt.F[2][c] = S(Fl);
          if (k == n2 - 1) nxt.F[2][c + pl] = S(Fu);
          div += (Fu - Fl) * ih2;
          const double mn = double(A.m2) - dt * ((xh - xl) * (0.5 * ih2));
          nxt.mom[2][c] = S(mn);
          bad = bad || !isfinite(mn);
        }
        const double rn = double(A.rn) - dt * div;
        const double theta = double(A.es / (A.rs * S(g.cv)));
        const double En = rn * g.cv * theta;
        nxt.rho[c] = S(rn);
        nxt.E[c] = S(En);
        bad = bad || !(rn > 0.0) || !(theta > 0.0) || !isfinite(rn) || !isfinite(En);
        mass += rn * g.dV;
      }
      xm = A.x;
      A = B;
      B = C;
      hv = hv2;
    }
    __syncthreads();
  }
  if (bad) {
    atomicOr(flags + FLAG_NONFINITE, 1);
    atomicCAS(flags + FLAG_BAD_STEP, 0, tag + 1);
  }
  double sm = block_sum(mass, lds);
  if (threadIdx.x == 0) partials[PART_MASS * kMaxBlocks + blockIdx.x] = sm;
}

// One block: the sum of per-block partials into a scalar.
__global__ void k_reduce(const double *partials, int n, double *out) {
  __shared__ double lds[32];
  double s = sum_partials(partials, n, lds);
  if (threadIdx.x == 0) *out = s;
}

// ------------------------------------------------------------------ launchers
int64_t cell_blocks(const GridK &g) { return g.nblocks; }

template <typename S>
static StateV<S> state_of(const Bufs &B, int cur) {
  StateV<S> s;
  s.rho = (S *)B.rho[cur];
  s.E = (S *)B.E[cur];
  for (int q = 0; q < 3; ++q) {
    s.mom[q] = (S *)B.mom[cur][q];
    s.F[q] = (S *)B.F[cur][q];
  }
  return s;
}

#define IBM_DISPATCH(L, ...)                         \
  do {                                               \
    if ((L).g.dim == 2 && (L).prec == 0) {           \
      constexpr int DIM = 2;                         \
      using S = double;                              \
      __VA_ARGS__;                                   \
    } else if ((L).g.dim == 2) {                     \
      constexpr int DIM = 2;                         \
      using S = float;                               \
      __VA_ARGS__;                                   \
    } else if ((L).prec == 0) {                      \
      constexpr int DIM = 3;                         \
      using S = double;                              \
      __VA_ARGS__;                                   \
    } else {                                         \
      constexpr int DIM = 3;                         \
      using S = float;                               \
      __VA_ARGS__;                                   \
    }                                                \
  } while (0)

void run_fill(const Launch &L, double *p, int64_t n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.st, p, n, v);
}

void run_uniform_state(const Launch &L, const Bufs &B, int cur) {
  IBM_DISPATCH(L, {
    int64_t nb = (L.g.N + 255) / 256;
    hipLaunchKernelGGL((k_uniform<DIM, S>), dim3((unsigned)nb), dim3(256), 0, L.st, L.g,
                       state_of<S>(B, cur));
  });
  run_flux_from_momentum(L, B, cur);
}

void run_init_primitive(const Launch &L, const Bufs &B, int cur, const void *rho, const void *u,
                        const void *theta) {
  IBM_DISPATCH(L, {
    int64_t nb = (L.g.N + 255) / 256;
    hipLaunchKernelGGL((k_init_primitive<DIM, S>), dim3((unsigned)nb), dim3(256), 0, L.st, L.g,
                       state_of<S>(B, cur), (const S *)rho, (const S *)u, (const S *)theta);
  });
  run_flux_from_momentum(L, B, cur);
}

void run_flux_from_momentum(const Launch &L, const Bufs &B, int cur) {
  IBM_DISPATCH(L, {
    for (int d = 0; d < DIM; ++d) {
      int64_t nb = (L.g.NF[d] + 255) / 256;
      hipLaunchKernelGGL((k_flux_from_mom<DIM, S>), dim3((unsigned)nb), dim3(256), 0, L.st, L.g,
                         state_of<S>(B, cur), d);
    }
  });
}

size_t predictor_lds_bytes(int dim, int prec) {
  if (dim == 2) return prec ? PredLds<2, float>::bytes : PredLds<2, double>::bytes;
  return prec ? PredLds<3, float>::bytes : PredLds<3, double>::bytes;
}

template <int DIM, typename S>
static void enable_lds_kernels(int bytes) {
  (void)hipFuncSetAttribute((const void *)k_predictor_lds<DIM, S, CONV_LINEAR>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute((const void *)k_predictor_lds<DIM, S, CONV_VANLEER>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

void enable_predictor_lds(int dim, int prec) {
  const int bytes = (int)predictor_lds_bytes(dim, prec);
  if (dim == 2 && prec == 0)
    enable_lds_kernels<2, double>(bytes);
  else if (dim == 2)
    enable_lds_kernels<2, float>(bytes);
  else if (prec == 0)
    enable_lds_kernels<3, double>(bytes);
  else
    enable_lds_kernels<3, float>(bytes);
}

void run_predictor(const Launch &L, const Bufs &B, int base, int cur, int order, int keep) {
  IBM_DISPATCH(L, {
    PredOut<S> po;
    for (int q = 0; q < 3; ++q) po.mh[q] = (S *)B.mhat[q];
    po.psi = (S *)B.psi;
    po.x = order >= 0 ? B.x : nullptr;
    po.E_prev = order >= 1 ? (const S *)B.E[cur ^ 1] : nullptr;
    po.E_prev2 = order >= 2 ? (const S *)B.E_hist : nullptr;
    po.E_prev3 = order >= 3 ? (const S *)B.E_hist2 : nullptr;
    po.E_keep = (order >= 1 && keep >= 1) ? (S *)B.E_hist : nullptr;
    po.E_keep2 = (order >= 2 && keep >= 2) ? (S *)B.E_hist2 : nullptr;
    po.rho_b = (const S *)B.rho[base];
    for (int q = 0; q < 3; ++q) po.mom_b[q] = (const S *)B.mom[base][q];
    po.E_b = (const S *)B.E[base];
    if (L.pred_lds) {
      using T = PredLds<DIM, S>;
      const int64_t nt = (int64_t)((L.g.n[0] + T::TX - 1) / T::TX) *
                         ((L.g.n[1] + T::TY - 1) / T::TY) *
                         (DIM == 3 ? (L.g.n[2] + T::TZ - 1) / T::TZ : 1);
      const int64_t nb = std::min<int64_t>(((nt + 7) / 8) * 8, IBM_PRED_MAXB);
      // the convection scheme compiled in (straight-line face code, fewer registers)
      if (L.g.conv == CONV_LINEAR)
        hipLaunchKernelGGL((k_predictor_lds<DIM, S, CONV_LINEAR>), dim3((unsigned)nb),
                           dim3(kThreads), T::bytes, L.st, L.g, state_of<S>(B, cur),
                           (S *)B.rho_s, (S *)B.mom_s[0], (S *)B.mom_s[1], (S *)B.mom_s[2],
                           (S *)B.E_s, po);
      else
        hipLaunchKernelGGL((k_predictor_lds<DIM, S, CONV_VANLEER>), dim3((unsigned)nb),
                           dim3(kThreads), T::bytes, L.st, L.g, state_of<S>(B, cur),
                           (S *)B.rho_s, (S *)B.mom_s[0], (S *)B.mom_s[1], (S *)B.mom_s[2],
                           (S *)B.E_s, po);
    } else {
      hipLaunchKernelGGL((k_predictor<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kThreads), 0,
                         L.st, L.g, state_of<S>(B, cur), (S *)B.rho_s, (S *)B.mom_s[0],
                         (S *)B.mom_s[1], (S *)B.mom_s[2], (S *)B.E_s, po);
    }
  });
}

// Work items of the column kernels: x-y tiles times chunks of z planes, about one
// item per block. The kernels run g.nblocks blocks, as every kernel whose per-block
// partial sums the CG's head adds up (the head sums gridDim.x of them).
void col_plan(const GridK &g, int &tiles_x, int &tiles_y, int &zc, int64_t &items, int &blocks,
              int tile_y) {
  tiles_x = (g.n[0] + kColTX - 1) / kColTX;
  tiles_y = (g.n[1] + tile_y - 1) / tile_y;
  blocks = (int)g.nblocks;
  const int64_t cols = (int64_t)tiles_x * tiles_y;
  const int64_t want = std::max<int64_t>(1, blocks / cols);
  zc = (int)std::max<int64_t>(4, (g.n[2] + want - 1) / want);
  const int64_t nch = (g.n[2] + zc - 1) / zc;
  items = cols * nch;
}

void run_setup(const Launch &L, const Bufs &B, int cur, int tag) {
  if (L.prec == 1 && L.refine32 && L.g.dim == 3 && L.cg_col) {
    int tx, ty, zc, nbk;
    int64_t items;
    col_plan(L.g, tx, ty, zc, items, nbk, kColTY);
    hipLaunchKernelGGL((k_setup_col<float, true>), dim3((unsigned)nbk), dim3(kColThreads), 0,
                       L.st, L.g, tx, ty, zc, items, (const float *)B.rho[cur],
                       (const float *)B.mhat[0], (const float *)B.mhat[1],
                       (const float *)B.mhat[2], (float *)B.Fhat[0], (float *)B.Fhat[1],
                       (float *)B.Fhat[2], (const float *)B.psi, (const double *)B.x, B.b,
                       (double *)nullptr, B.rv32[0], B.partials, B.cg, tag);
    return;
  }
  if (L.prec == 1 && L.refine32) {
    if (L.g.dim == 2)
      hipLaunchKernelGGL((k_setup2m<2>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0, L.st,
                         L.g, (const float *)B.rho[cur], (const float *)B.mhat[0],
                         (const float *)B.mhat[1], (const float *)B.mhat[2], (float *)B.Fhat[0],
                         (float *)B.Fhat[1], (float *)B.Fhat[2], (const float *)B.psi,
                         (const double *)B.x, B.b, B.rv32[0], B.partials, B.cg, tag);
    else
      hipLaunchKernelGGL((k_setup2m<3>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0, L.st,
                         L.g, (const float *)B.rho[cur], (const float *)B.mhat[0],
                         (const float *)B.mhat[1], (const float *)B.mhat[2], (float *)B.Fhat[0],
                         (float *)B.Fhat[1], (float *)B.Fhat[2], (const float *)B.psi,
                         (const double *)B.x, B.b, B.rv32[0], B.partials, B.cg, tag);
    return;
  }
  if (L.g.dim == 3 && L.cg_col) {
    int tx, ty, zc, nbk;
    int64_t items;
    col_plan(L.g, tx, ty, zc, items, nbk, kColTY);
    auto go = [&](auto sdum) {
      using S = decltype(sdum);
      hipLaunchKernelGGL((k_setup_col<S>), dim3((unsigned)nbk), dim3(kColThreads), 0, L.st, L.g,
                         tx, ty, zc, items, (const S *)B.rho[cur], (const S *)B.mhat[0],
                         (const S *)B.mhat[1], (const S *)B.mhat[2], (S *)B.Fhat[0],
                         (S *)B.Fhat[1], (S *)B.Fhat[2], (const S *)B.psi, (const double *)B.x,
                         B.b, B.rv[0], (float *)nullptr, B.partials, B.cg, tag);
    };
    if (L.prec == 0) go(double{}); else go(float{});
    run_cg_start(L, B);
    return;
  }
  IBM_DISPATCH(L, {
    hipLaunchKernelGGL((k_setup2<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0,
                       L.st, L.g, (const S *)B.rho[cur], (const S *)B.mhat[0],
                       (const S *)B.mhat[1], (const S *)B.mhat[2], (S *)B.Fhat[0], (S *)B.Fhat[1],
                       (S *)B.Fhat[2], (const S *)B.psi, (const double *)B.x, B.b, B.rv[0],
                       B.partials, B.cg, tag);
  });
  run_cg_start(L, B);
}

void run_cg_start(const Launch &L, const Bufs &B) {
  if (L.prec == 1 && L.refine32) return;  // the refinement's first kernel starts its solve
  run_cg64_start(L, B);
}

void run_cg64_start(const Launch &L, const Bufs &B) {
  if (L.g.dim == 3 && L.cg_col) {
    int tx, ty, zc, nbk;
    int64_t items;
    col_plan(L.g, tx, ty, zc, items, nbk, kCgTY);
    auto go = [&](auto sdum) {
      using S = decltype(sdum);
      hipLaunchKernelGGL((k_cg_col<COL_START, S>), dim3((unsigned)nbk), dim3(kColTX * kCgTY), 0,
                         L.st, L.g, 0, tx, ty, zc, items, (const S *)B.psi,
                         (const double *)B.rv[0], (const double *)nullptr,
                         (const double *)nullptr, (double *)nullptr, B.wv[0], (double *)nullptr,
                         (double *)nullptr, (double *)nullptr, B.partials, B.cg,
                         (const int *)B.flags, B.progress);
    };
    if (L.prec == 0) go(double{}); else go(float{});
    return;
  }
  IBM_DISPATCH(L, {
    hipLaunchKernelGGL((k_cg_start<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0,
                       L.st, L.g, (const S *)B.psi, (const double *)B.rv[0], B.wv[0], B.partials);
  });
}

int cg_parts(const Launch &) { return 1; }

template <int DIM>
static void run_mcg_iter(const Launch &L, const Bufs &B, int it) {
  const int a = it & 1, b = a ^ 1;
  if (DIM == 3 && L.cg_col) {
    int tx, ty, zc, nbk;
    int64_t items;
    col_plan(L.g, tx, ty, zc, items, nbk, kColTY);
    hipLaunchKernelGGL(k_mcg_col, dim3((unsigned)nbk), dim3(kColThreads), 0, L.st, L.g, it, tx,
                       ty, zc, items, (const float *)B.psi, (const double *)B.b, B.x, B.x2,
                       (const float *)B.rv32[a], (const float *)B.wv32[a],
                       (const float *)B.sv32[a], B.rv32[b], B.wv32[b], B.sv32[b], B.pv32, B.d32,
                       B.partials, B.cg, (const int *)B.flags, B.progress);
    return;
  }
  hipLaunchKernelGGL((k_mcg_iter<DIM>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0, L.st, L.g,
                     it, (const float *)B.psi, (const double *)B.b, B.x, B.x2,
                     (const float *)B.rv32[a], (const float *)B.wv32[a], (const float *)B.sv32[a],
                     B.rv32[b], B.wv32[b], B.sv32[b], B.pv32, B.d32, B.partials, B.cg,
                     (const int *)B.flags, B.progress);
}

void run_cg_half(const Launch &L, const Bufs &B, int it, int part) {
  if (part != 0) return;
  if (L.prec == 1 && L.refine32) {
    if (L.g.dim == 2)
      run_mcg_iter<2>(L, B, it);
    else
      run_mcg_iter<3>(L, B, it);
    return;
  }
  run_cg64_iteration(L, B, it);
}

void run_cg64_iteration(const Launch &L, const Bufs &B, int it) {
  if (L.g.dim == 3 && L.cg_col) {
    int tx, ty, zc, nbk;
    int64_t items;
    col_plan(L.g, tx, ty, zc, items, nbk, kCgTY);
    const int a = it & 1, bb = a ^ 1;
    auto go = [&](auto mode, auto sdum) {
      using S = decltype(sdum);
      constexpr int M = decltype(mode)::value;
      hipLaunchKernelGGL((k_cg_col<M, S>), dim3((unsigned)nbk), dim3(kColTX * kCgTY), 0, L.st, L.g,
                         it, tx, ty, zc, items, (const S *)B.psi, (const double *)B.rv[a],
                         (const double *)B.wv[a], (const double *)B.sv[a], B.rv[bb], B.wv[bb],
                         B.sv[bb], B.pv, B.x, B.partials, B.cg, (const int *)B.flags, B.progress);
    };
    using F1 = std::integral_constant<int, COL_FIRST>;
    using F2 = std::integral_constant<int, COL_ITER>;
    if (L.prec == 0) {
      if (it == 0) go(F1{}, double{}); else go(F2{}, double{});
    } else {
      if (it == 0) go(F1{}, float{}); else go(F2{}, float{});
    }
    return;
  }
  IBM_DISPATCH(L, {
    const int a = it & 1, b = a ^ 1;
    hipLaunchKernelGGL((k_cg_iter<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0,
                       L.st, L.g, it, (const S *)B.psi, (const double *)B.rv[a],
                       (const double *)B.wv[a], (const double *)B.sv[a], B.rv[b], B.wv[b], B.sv[b],
                       B.pv, B.x, B.partials, B.cg, (const int *)B.flags, B.progress);
  });
}

void run_cg_iteration(const Launch &L, const Bufs &B, int it) {
  for (int part = 0; part < cg_parts(L); ++part) run_cg_half(L, B, it, part);
}

void run_correct(const Launch &L, const Bufs &B, int cur, int tag) {
  if (L.g.dim == 3 && L.cg_col) {
    int tx, ty, zc, nbk;
    int64_t items;
    col_plan(L.g, tx, ty, zc, items, nbk, kColTY);
    auto go = [&](auto sdum) {
      using S = decltype(sdum);
      hipLaunchKernelGGL((k_correct_col<S>), dim3((unsigned)nbk), dim3(kColThreads), 0, L.st,
                         L.g, tx, ty, zc, items, state_of<S>(B, cur), state_of<S>(B, cur ^ 1),
                         (const S *)B.rho_s, (const S *)B.E_s, (const S *)B.mhat[0],
                         (const S *)B.mhat[1], (const S *)B.mhat[2], (const S *)B.Fhat[0],
                         (const S *)B.Fhat[1], (const S *)B.Fhat[2], (const double *)B.x,
                         (const double *)(B.x2 ? B.x2 : B.x), B.partials, B.flags,
                         (const CgScal *)B.cg, tag);
    };
    if (L.prec == 0) go(double{}); else go(float{});
    return;
  }
  IBM_DISPATCH(L, {
    hipLaunchKernelGGL((k_correct<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0,
                       L.st, L.g, state_of<S>(B, cur), state_of<S>(B, cur ^ 1),
                       (const S *)B.rho_s, (const S *)B.E_s, (const S *)B.mhat[0],
                       (const S *)B.mhat[1], (const S *)B.mhat[2], (const S *)B.Fhat[0],
                       (const S *)B.Fhat[1], (const S *)B.Fhat[2], (const double *)B.x,
                       (const double *)(B.x2 ? B.x2 : B.x), B.partials, B.flags,
                       (const CgScal *)B.cg, tag);
  });
}

// The diffusion systems' buffers for solution ring slot `ring`: x = slot ring,
// y1 = the previous step's solution, y2 = the one before.
static DiffSys diff_sys(const Launch &L, const Bufs &B, int ring) {
  DiffSys D;
  for (int d = 0; d < 3; ++d) D.mf[d] = B.muf[d];
  for (int v = 0; v < kDiffVars; ++v) {
    D.x[v] = B.dring[ring][v];
    D.y1[v] = B.dring[(ring + 2) % 3][v];
    D.y2[v] = B.dring[(ring + 1) % 3][v];
    D.p[v] = B.dp[v];
    for (int s = 0; s < 2; ++s) {
      D.r[s][v] = B.dr[s][v];
      D.w[s][v] = B.dw[s][v];
      D.s[s][v] = B.ds[s][v];
    }
  }
  D.part = B.dpart;
  D.sc = B.dsc;
  D.kap_th = L.g.cp_Pr * L.g.inv_cv;  // lambda_f / (c_v mu_f) = gamma / Pr
  return D;
}

void run_diff_coef(const Launch &L, const Bufs &B, int cur) {
  IBM_DISPATCH(L, {
    for (int d = 0; d < DIM; ++d) {
      const int64_t nb = (L.g.NF[d] + 255) / 256;
      hipLaunchKernelGGL((k_diff_coef<DIM, S>), dim3((unsigned)nb), dim3(256), 0, L.st, L.g, d,
                         state_of<S>(B, cur), B.muf[d]);
    }
  });
}

void run_diff_start(const Launch &L, const Bufs &B, int cur, int ring, int order, int tag) {
  const DiffSys D = diff_sys(L, B, ring);
  IBM_DISPATCH(L, {
    hipLaunchKernelGGL((k_dsys_init<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0,
                       L.st, L.g, D, state_of<S>(B, cur), (const S *)B.rho_s,
                       (const S *)B.mom_s[0], (const S *)B.mom_s[1], (const S *)B.mom_s[2],
                       (const S *)B.E_s, order, tag);
    hipLaunchKernelGGL((k_dsys_start<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0,
                       L.st, L.g, D, (const S *)B.rho_s);
  });
}

void run_diff_iteration(const Launch &L, const Bufs &B, int ring, int it) {
  const DiffSys D = diff_sys(L, B, ring);
  IBM_DISPATCH(L, {
    hipLaunchKernelGGL((k_dsys_iter<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads), 0,
                       L.st, L.g, it, D, (const S *)B.rho_s, (const int *)B.flags, B.progress);
  });
}

void run_diff_finish(const Launch &L, const Bufs &B, int ring) {
  const DiffSys D = diff_sys(L, B, ring);
  IBM_DISPATCH(L, {
    const int64_t nb = (L.g.N + 255) / 256;
    hipLaunchKernelGGL((k_dsys_finish<DIM, S>), dim3((unsigned)nb), dim3(256), 0, L.st, L.g, D,
                       (const S *)B.rho_s, (S *)B.mom_s[0], (S *)B.mom_s[1], (S *)B.mom_s[2],
                       (S *)B.mhat[0], (S *)B.mhat[1], (S *)B.mhat[2], (S *)B.E_s, (S *)B.psi);
  });
}

template <typename S>
static DensPrim<S> dens_prim(void *const *a) {
  DensPrim<S> p;
  for (int v = 0; v < 5; ++v) p.v[v] = (S *)a[v];
  return p;
}

// dynamic LDS of the inviscid kernel: the slabs' primitives and one direction's face
// fluxes
template <int DIM, typename S>
static size_t dens_lds_bytes() {
  using X = DCross<DIM>;
  return sizeof(S) * (size_t)(DIM + 2) * (X::NP + X::T::NFD);
}
template <int DIM, typename S>
static void enable_dens_lds() {
  const size_t b = dens_lds_bytes<DIM, S>();
  if (b > 65536)
    (void)hipFuncSetAttribute((const void *)k_dens_inviscid<DIM, S>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
}
void enable_density_lds(int dim, int prec) {
  if (dim == 2 && prec == 0)
    enable_dens_lds<2, double>();
  else if (dim == 2)
    enable_dens_lds<2, float>();
  else if (prec == 0)
    enable_dens_lds<3, double>();
  else
    enable_dens_lds<3, float>();
}

void run_density_predictor(const Launch &L, const Bufs &B, int cur) {
  IBM_DISPATCH(L, {
    const StateV<S> st = state_of<S>(B, cur), nx = state_of<S>(B, cur ^ 1);
    const DensPrim<S> p1 = dens_prim<S>(B.dprim1);
    using X = DCross<DIM>;
    const unsigned nt2 = (unsigned)X::T::tiles(L.g), nt1 = (unsigned)DVTile<DIM>::tiles(L.g);
    const size_t shm = dens_lds_bytes<DIM, S>();
    hipLaunchKernelGGL((k_dens_inviscid<DIM, S>), dim3(nt2), dim3(X::NT), shm, L.st, L.g, st, nx,
                       (S *)B.rho_s, (S *)B.mhat[0], (S *)B.mhat[1], (S *)B.mhat[2], p1,
                       (const int *)B.flags);
    constexpr int nv = DVTile<DIM>::TX * DVTile<DIM>::TY * DVTile<DIM>::TZ;
    hipLaunchKernelGGL((k_dens_viscous<DIM, S>), dim3(nt1), dim3(nv), 0, L.st, L.g,
                       (const S *)B.rho_s, (const S *)B.mhat[0], (const S *)B.mhat[1],
                       (const S *)B.mhat[2], p1, (S *)B.mom_s[0], (S *)B.mom_s[1],
                       (S *)B.mom_s[2], (S *)B.E_s, (const int *)B.flags);
  });
}

void run_density_finish(const Launch &L, const Bufs &B, int cur, int tag) {
  IBM_DISPATCH(L, {
    hipLaunchKernelGGL((k_dens_finish<DIM, S>), dim3((unsigned)L.g.nblocks), dim3(kBlockThreads),
                       0, L.st, L.g, (const S *)B.rho_s, (const S *)B.mom_s[0],
                       (const S *)B.mom_s[1], (const S *)B.mom_s[2], (const S *)B.E_s,
                       state_of<S>(B, cur ^ 1), B.partials, B.flags, tag);
  });
}

void run_mass(const Launch &L, const Bufs &B) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, L.st,
                     (const double *)B.partials + PART_MASS * kMaxBlocks, (int)L.g.nblocks,
                     B.scal);
}

}  // namespace ibmk
