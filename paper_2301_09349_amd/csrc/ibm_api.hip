// ibm_api.hip -- host side of the C ABI declared in include/ibm.h: descriptor
// validation, workspace carving (the library never allocates device memory),
// marker set-up and the step loop with the pressure-CG convergence probe.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ibm.h"
#include "ibm_launch.h"

using ibmk::Bufs;
using ibmk::CgScal;
using ibmk::GridK;
using ibmk::Launch;

// Event-pair timing of kernel classes (measurement only). A pair brackets the
// launches of one class in a step; the CG's pairs bracket a batch of back-to-back
// iterations (it0 .. it0 + nl - 1) and count only the iterations that did work.
struct Prof {
  bool on = false;
  double ms[IBM_PROF_CLASSES] = {};
  int64_t n[IBM_PROF_CLASSES] = {};
  struct Pair {
    int cls, it0, nl;
    hipEvent_t a, b;
    int count = 1;
  };
  std::vector<hipEvent_t> pool, used;
  std::vector<Pair> pending;
  size_t step_first = 0;  // first pending pair of the current step
  hipEvent_t get() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      return nullptr;
    }
    used.push_back(e);
    return e;
  }
  hipEvent_t mark(hipStream_t st) {
    hipEvent_t e = get();
    if (e) (void)hipEventRecord(e, st);
    return e;
  }
  // the CG batches of the current step: count the iterations that did work (a
  // solve of n iterations also launches the test that ends it, and a batch may run
  // past the end; that time stays in the total)
  void count_cg(int cg_iters) {
    for (size_t i = step_first; i < pending.size(); ++i) {
      Pair &p = pending[i];
      if (p.cls != IBM_PROF_CG) continue;
      const int hi = std::min(p.it0 + p.nl, cg_iters);
      p.count = std::max(0, hi - p.it0);
    }
  }
  // after a synchronisation: accumulate the recorded durations
  void settle() {
    for (const Pair &p : pending) {
      if (!p.a || !p.b) continue;
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
        ms[p.cls] += t;
        n[p.cls] += p.count;
      }
    }
    pending.clear();
    pool.insert(pool.end(), used.begin(), used.end());
    used.clear();
  }
  ~Prof() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : used) (void)hipEventDestroy(e);
  }
};

struct ibm_ctx {
  ibm_grid_desc desc;
  Launch L;
  Bufs B;
  int cur = 0;
  int64_t step = 0;
  int nc = 0;  // candidate markers (0: no body)
  int dedupe = 0;
  int motion_axis = -1;
  double motion_amp = 0.0, motion_freq = 0.0;
  int cg_hint = 8;
  int adj_hint = 8;  // iterations of the last adjoint pressure solve
  int diff_hint = 8;  // iterations of the last implicit diffusion solves
  int diff_ring = 0;  // solution ring slot of the next step's diffusion solves
  // previous steps' diffusion solutions held in the ring (0..2); cleared with
  // prev_valid
  int diff_hist = 0;
  int tape_cap = 0;
  int tape_len = 0;  // steps recorded by the last IBM_RECORD call
  // the other state slot holds the state of the step before the current one (the CG
  // start is then extrapolated); cleared whenever the state is set from outside
  bool prev_valid = false;
  // E_hist holds the energy of the state before the other slot's (the three-point
  // start is then possible); cleared with prev_valid
  bool hist_valid = false;
  // E_hist2 holds the energy of the state before E_hist's (the four-point start is
  // then possible); cleared with hist_valid
  bool hist2_valid = false;
  // highest order of the extrapolated CG start: 3 (default), 2 with
  // IBM_CG_START=quadratic, 1 with IBM_CG_START=linear, 0 with IBM_CG_START=plain
  int cg_order = 3;
  int tag = 0;  // solve tag, one per pass of a step launched
  // device whose static scratch array holds this context's buffers
  // (ibm_create_grid_noalloc), -1 for a caller's workspace
  int scratch_dev = -1;
  // A moving body's markers are set up ahead of the steps that use them, on side
  // streams, into the two marker sets (Bufs and Bufs::alt): a step reads the set in
  // Bufs, while the set-ups for the next step (in the other set) and for the step
  // after it (in this step's set, once its last marker kernel is done: event
  // ev_used) run; a step's first marker kernel waits for its set's ev_built. Set k
  // has its own side stream, so the two set-ups in flight overlap. Only within one
  // call: the first step of a call sets its markers up in place. Not with
  // IBM_REBUILD=inline or on the static scratch array; created at the first moving
  // step.
  bool side_ok = true;
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t ev_used[2] = {nullptr, nullptr}, ev_built[2] = {nullptr, nullptr};
  int aset = 0;                     // the set in Bufs (the other is in Bufs::alt)
  int64_t set_step[2] = {-1, -1};  // the step whose markers set k holds or will hold
  bool pending[2] = {false, false};  // a set-up queued into set k not yet waited for
  // adjoint steps accumulate the marker-position cotangents (between a NULL call of
  // ibm_shape_gradient and the call that reads them)
  bool shape_acc = false;
  std::string err;
  CgScal cgh;
  Prof prof;
  ~ibm_ctx() {
    for (int k = 0; k < 2; ++k) {
      if (side[k]) {
        (void)hipStreamSynchronize(side[k]);
        (void)hipStreamDestroy(side[k]);
      }
      if (ev_used[k]) (void)hipEventDestroy(ev_used[k]);
      if (ev_built[k]) (void)hipEventDestroy(ev_built[k]);
    }
    if (B.progress) (void)hipHostFree(B.progress);
  }
};

namespace {

constexpr double kPi = 3.14159265358979323846;

ibm_status fail(ibm_ctx *ctx, ibm_status s, const char *msg) {
  if (ctx) ctx->err = msg;
  return s;
}

#define HIPCHECK(ctx, expr)                                              \
  do {                                                                   \
    hipError_t e_ = (expr);                                              \
    if (e_ != hipSuccess) {                                              \
      if (ctx) (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_); \
      return IBM_E_HIP;                                                  \
    }                                                                    \
  } while (0)

const char *check_desc(const ibm_grid_desc *d) {
  if (!d) return "descriptor is NULL";
  if (d->dim != 2 && d->dim != 3) return "dim must be 2 or 3";
  for (int a = 0; a < d->dim; ++a) {
    if (d->n[a] < 3) return "each n[d] must be >= 3";
    if (!(d->hi[a] > d->lo[a])) return "hi must exceed lo";
    for (int s = 0; s < 2; ++s)
      if (d->bc[a][s] < IBM_PERIODIC || d->bc[a][s] > IBM_SUPERSONIC_OUTFLOW)
        return "unknown boundary type";
    if ((d->bc[a][0] == IBM_PERIODIC) != (d->bc[a][1] == IBM_PERIODIC))
      return "periodic must be set on both sides";
  }
  if (d->dim == 2 && d->n[2] != 1) return "n[2] must be 1 in 2D";
  if (d->precision != IBM_FP64 && d->precision != IBM_FP32) return "unknown precision";
  if (d->convection != IBM_CONV_VANLEER && d->convection != IBM_CONV_LINEAR)
    return "unknown convection scheme";
  if (d->viscosity_law != IBM_MU_SUTHERLAND && d->viscosity_law != IBM_MU_CONSTANT)
    return "unknown viscosity law";
  if (d->diffusion != IBM_DIFF_EXPLICIT && d->diffusion != IBM_DIFF_IMPLICIT)
    return "unknown diffusion treatment";
  if (d->n_outer < 0 || d->n_outer > 64) return "n_outer must be in 0..64";
  if (d->scheme != IBM_SCHEME_PRESSURE && d->scheme != IBM_SCHEME_DENSITY) return "unknown scheme";
  for (int a = 0; a < d->dim; ++a)
    for (int s = 0; s < 2; ++s)
      if (d->bc[a][s] >= IBM_SUPERSONIC_INFLOW && d->scheme != IBM_SCHEME_DENSITY)
        return "supersonic sides need the density-based step";
  if (d->scheme == IBM_SCHEME_DENSITY && (d->diffusion != IBM_DIFF_EXPLICIT || d->n_outer > 1))
    return "the density-based step takes explicit diffusion and one pass";
  if (!(d->Re > 0) || !(d->Ma > 0) || !(d->Pr > 0) || !(d->gamma > 1.0))
    return "Re, Ma, Pr must be > 0 and gamma > 1";
  if (!(d->sutherland_S >= 0)) return "sutherland_S must be >= 0";
  if (!(d->dt > 0) && !(d->cfl > 0)) return "need dt > 0 or cfl > 0";
  if (!(d->cg_rtol > 0) || d->cg_maxit < 1) return "cg_rtol > 0 and cg_maxit >= 1 required";
  if (d->max_markers < 0) return "max_markers must be >= 0";
  int64_t N = 1;
  for (int a = 0; a < d->dim; ++a) N *= d->n[a];
  if (N > (int64_t)1 << 31) return "grid too large";
  return nullptr;
}

double mu_law(const ibm_grid_desc &d, double th) {
  double mu_inf = 1.0 / d.Re;
  if (d.viscosity_law == IBM_MU_CONSTANT) return mu_inf;
  return mu_inf * th * std::sqrt(th) * (1.0 + d.sutherland_S) / (th + d.sutherland_S);
}

GridK make_grid(const ibm_grid_desc &d) {
  GridK g;
  std::memset(&g, 0, sizeof(g));
  g.dim = d.dim;
  g.N = 1;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = (a < d.dim) ? d.n[a] : 1;
    g.lo[a] = (a < d.dim) ? d.lo[a] : 0.0;
    g.h[a] = (a < d.dim) ? (d.hi[a] - d.lo[a]) / double(g.n[a]) : 1.0;
    g.ih[a] = 1.0 / g.h[a];
    g.N *= g.n[a];
    for (int s = 0; s < 2; ++s) g.bc[a][s] = (a < d.dim) ? d.bc[a][s] : IBM_PERIODIC;
    g.U_inf[a] = d.U_inf[a];
  }
  for (int a = 0; a < 3; ++a) {
    g.NF[a] = 1;
    for (int b = 0; b < 3; ++b) {
      g.fn[a][b] = g.n[b] + (a == b ? 1 : 0);
      g.NF[a] *= g.fn[a][b];
    }
    if (a >= d.dim) g.NF[a] = 0;
  }
  g.conv = d.convection;
  g.visc = d.viscosity_law;
  g.R = 1.0 / (d.gamma * d.Ma * d.Ma);
  g.cv = g.R / (d.gamma - 1.0);
  g.inv_cv = 1.0 / g.cv;
  g.cp = d.gamma * g.cv;
  g.gm1 = d.gamma - 1.0;
  g.mu_inf = 1.0 / d.Re;
  g.S = d.sutherland_S;
  g.Pr = d.Pr;
  g.cp_Pr = g.cp / d.Pr;
  g.p_inf = g.R;
  g.dV = g.h[0] * g.h[1] * (d.dim == 3 ? g.h[2] : 1.0);
  if (d.dt > 0.0) {
    g.dt = d.dt;
  } else {
    // half of the combined explicit limit of convection and conduction, with the
    // thermal diffusivity gamma mu / (Pr rho) at theta_max and rho = 1/theta_max
    double thm = std::max(1.0, d.dt_theta_max);
    double uref = std::sqrt(d.U_inf[0] * d.U_inf[0] + d.U_inf[1] * d.U_inf[1] +
                            d.U_inf[2] * d.U_inf[2]) + d.dt_u_max;
    double alpha = d.gamma * mu_law(d, thm) * thm / d.Pr;
    double sc = 0.0, sd = 0.0;
    for (int a = 0; a < d.dim; ++a) {
      sc += uref / g.h[a];
      sd += 1.0 / (g.h[a] * g.h[a]);
    }
    // the density-based step is explicit in the acoustic waves too: the sound
    // speed at theta_max is added to the flow speed
    if (d.scheme == IBM_SCHEME_DENSITY) {
      const double c = std::sqrt(d.gamma * g.R * thm);
      sc = 0.0;
      for (int a = 0; a < d.dim; ++a) sc += (uref + c) / g.h[a];
    }
    // with implicit diffusion only convection limits the step (without any flow
    // speed the explicit limit is kept)
    if (d.diffusion == IBM_DIFF_IMPLICIT && sc > 0.0)
      g.dt = d.cfl / sc;
    else
      g.dt = d.cfl / (sc + 2.0 * alpha * sd);
  }
  g.implicit_diff = d.diffusion == IBM_DIFF_IMPLICIT ? 1 : 0;
  if (d.dim == 2) {
    g.tiles[0] = (g.n[0] + 63) / 64;
    g.tiles[1] = (g.n[1] + 3) / 4;
    g.tiles[2] = 1;
  } else {
    g.tiles[0] = (g.n[0] + 63) / 64;
    g.tiles[1] = (g.n[1] + 3) / 4;
    g.tiles[2] = g.n[2];
  }
  g.ntiles = (int64_t)g.tiles[0] * g.tiles[1] * g.tiles[2];
  const int64_t groups = ibmk::kBlockThreads / ibmk::kTile;
  g.nblocks = std::min<int64_t>(((g.ntiles + groups - 1) / groups + 7) / 8 * 8, ibmk::kMaxBlocks);
  return g;
}

int next_pow2(int64_t v) {
  int64_t p = 2;
  while (p < v) p <<= 1;
  return (int)p;
}

struct Carver {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

// Lays the buffers out in the workspace (or only measures when base == NULL).
size_t plan(const ibm_grid_desc &d, const GridK &g, int max_markers, int tape_steps, char *base,
            Bufs &B, int &npairs_pad) {
  Carver C{base};
  const size_t w = (d.precision == IBM_FP32) ? 4 : 8;
  const int dim = d.dim;
  const size_t N = (size_t)g.N;
  auto field = [&](size_t n) { return (void *)C.take<char>(n * w); };
  for (int s = 0; s < 2; ++s) {
    B.rho[s] = field(N);
    B.E[s] = field(N);
    for (int q = 0; q < 3; ++q) {
      B.mom[s][q] = q < dim ? field(N) : nullptr;
      B.F[s][q] = q < dim ? field((size_t)g.NF[q]) : nullptr;
    }
  }
  B.rho_s = field(N);
  B.E_s = field(N);
  B.E_hist = field(N);
  B.E_hist2 = field(N);
  B.psi = field(N);
  for (int q = 0; q < 3; ++q) {
    B.mom_s[q] = q < dim ? field(N) : nullptr;
    B.mhat[q] = q < dim ? field(N) : nullptr;
    B.Fhat[q] = q < dim ? field((size_t)g.NF[q]) : nullptr;
  }
  B.b = C.take<double>(N);
  B.x = C.take<double>(N);
  B.x2 = nullptr;
  for (int s = 0; s < 2; ++s) B.rv32[s] = B.wv32[s] = B.sv32[s] = nullptr;
  B.pv32 = B.d32 = nullptr;
  if (d.precision == IBM_FP32) {
    // FP32 form: x ping-pong for the refinement; inner CG vectors in FP32
    B.x2 = C.take<double>(N);
    for (int s = 0; s < 2; ++s) {
      B.rv32[s] = C.take<float>(N);
      B.wv32[s] = C.take<float>(N);
      B.sv32[s] = C.take<float>(N);
    }
    B.pv32 = C.take<float>(N);
    B.d32 = C.take<float>(N);
  }
  {
    // FP64 CG vectors (the FP32 form's default solve and every adjoint solve)
    B.pv = C.take<double>(N);
    for (int s = 0; s < 2; ++s) {
      B.rv[s] = C.take<double>(N);
      B.wv[s] = C.take<double>(N);
      B.sv[s] = C.take<double>(N);
    }
  }
  {
    const bool imp = d.diffusion == IBM_DIFF_IMPLICIT;
    const int nv = dim + 1;
    for (int q = 0; q < 3; ++q) B.muf[q] = (imp && q < dim) ? C.take<double>((size_t)g.NF[q]) : nullptr;
    for (int v = 0; v < ibmk::kDiffVars; ++v) {
      const bool on = imp && v < nv;
      for (int r = 0; r < 3; ++r) B.dring[r][v] = on ? C.take<double>(N) : nullptr;
      for (int s = 0; s < 2; ++s) {
        B.dr[s][v] = on ? C.take<double>(N) : nullptr;
        B.dw[s][v] = on ? C.take<double>(N) : nullptr;
        B.ds[s][v] = on ? C.take<double>(N) : nullptr;
      }
      B.dp[v] = on ? C.take<double>(N) : nullptr;
    }
    B.dpart = imp ? C.take<double>((size_t)ibmk::kDiffVars * ibmk::DP_REGIONS * ibmk::kMaxBlocks)
                  : nullptr;
    B.dsc = imp ? C.take<ibmk::DiffScal>(1) : nullptr;
    const bool dens = d.scheme == IBM_SCHEME_DENSITY;
    for (int v = 0; v < 5; ++v) {
      B.dprim1[v] = (dens && (v < dim || v == 3)) ? field(N) : nullptr;
    }
  }
  B.partials = C.take<double>((size_t)ibmk::PART_REGIONS * ibmk::kMaxBlocks);
  B.cg = C.take<CgScal>(1);
  B.scal = C.take<double>(8);
  B.flags = C.take<int>(8);
  const size_t nc = std::max(max_markers, 1);
  const int nslot = dim == 3 ? 27 : 9;
  npairs_pad = next_pow2((int64_t)nc * nslot);
  B.cX0 = C.take<double>(3 * nc);
  B.cUd0 = C.take<double>(3 * nc);
  B.cTw = C.take<double>(nc);
  B.cdA = C.take<double>(nc);
  B.ceps = C.take<double>(nc);
  // the two marker sets
  auto carve_set = [&]() {
    ibmk::MarkerSet m;
    m.cXc = C.take<double>(3 * nc);
    m.cUdc = C.take<double>(3 * nc);
    m.ckey = C.take<int64_t>(nc);
    m.cd2 = C.take<double>(nc);
    m.ckeep = C.take<int>(nc);
    m.mcount = C.take<int>(8);
    m.ids = C.take<int>(nc);
    m.X = C.take<double>(3 * nc);
    m.Ud = C.take<double>(3 * nc);
    m.Tw = C.take<double>(nc);
    m.dA = C.take<double>(nc);
    m.eps = C.take<double>(nc);
    m.sidx = C.take<int>(9 * nc);
    m.sw1 = C.take<double>(9 * nc);
    m.pcell = C.take<int64_t>(27 * nc);
    m.pw = C.take<double>(27 * nc);
    m.keys = C.take<uint64_t>((size_t)npairs_pad);
    m.keys_in = C.take<uint64_t>((size_t)npairs_pad);
    m.seg = C.take<int>(27 * nc + 1);
    m.ell_col = C.take<int>((size_t)ibmk::kMaxNbr * nc);
    m.ell_val = C.take<double>((size_t)ibmk::kMaxNbr * nc);
    m.ell_cnt = C.take<int>(nc);
    for (int v = 0; v < 4; ++v) m.ev[v] = C.take<double>(nc);
    return m;
  };
  ibmk::put_marker_set(B, carve_set());
  B.alt = carve_set();
  B.mk = C.take<double>(9 * nc);
  B.mforce = C.take<double>(3 * nc);
  B.mheat = C.take<double>(nc);
  B.totals = C.take<double>(8);
  // tape and adjoint work buffers (contexts with a tape only)
  B.tape = nullptr;
  B.tape_stride = B.tape_xoff = 0;
  B.pprim = B.pbar = B.fo = B.co = B.rs_bar = B.Es_bar = B.fbar = B.tbar = B.lam = B.rhs = nullptr;
  B.mkbar = nullptr;
  B.wbar = B.epsbar = B.pfld = B.gsum = B.lam_g = nullptr;
  for (int q = 0; q < 3; ++q) B.ms_bar[q] = nullptr;
  if (tape_steps > 0) {
    const size_t NFt = (size_t)(g.NF[0] + g.NF[1] + g.NF[2]);
    const size_t Np = (size_t)ibmk::padded_cells(g);
    B.tape_xoff = (((size_t)(dim + 2) * N + NFt) * w + 255) & ~size_t(255);
    B.tape_stride = (B.tape_xoff + N * sizeof(double) + 255) & ~size_t(255);
    B.tape = C.take<char>(B.tape_stride * (size_t)tape_steps);
    B.pprim = C.take<double>((size_t)(dim + 4) * Np);
    B.pbar = C.take<double>((size_t)(dim + 3) * Np);
    const int nfo = (d.convection == IBM_CONV_VANLEER) ? 5 * dim + 3 : 4 * dim + 2;
    B.fo = C.take<double>((size_t)nfo * NFt);
    B.co = C.take<double>((size_t)(dim * dim + dim + 2) * N);
    B.rs_bar = C.take<double>(N);
    B.Es_bar = C.take<double>(N);
    for (int q = 0; q < dim; ++q) B.ms_bar[q] = C.take<double>(N);
    B.fbar = C.take<double>(NFt);
    B.tbar = C.take<double>(N);
    B.lam = C.take<double>(N);
    B.rhs = C.take<double>(N);
    B.mkbar = C.take<double>((size_t)(2 * dim + 3) * nc);
    B.wbar = C.take<double>((size_t)27 * nc);
    B.epsbar = C.take<double>(nc);
    B.pfld = C.take<double>((size_t)27 * (dim + 2) * nc);
    B.gsum = C.take<double>((size_t)54 * nc);
    B.lam_g = C.take<double>(nc);
  }
  return (C.off + 255) & ~size_t(255);
}

ibm_status sync_read(ibm_ctx *ctx, void *dst, const void *src, size_t bytes) {
  HIPCHECK(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->L.st));
  HIPCHECK(ctx, hipStreamSynchronize(ctx->L.st));
  return IBM_OK;
}

// marker positions at time t, supports, sort, eps, on `stream` (NULL: the context's).
// Only the set-up of a new body saves eps per candidate (the start of every later
// solve), so that a rebuild depends on t alone and may run ahead on a side stream.
ibm_status rebuild_markers(ibm_ctx *ctx, double t, bool save_eps = false,
                           hipStream_t stream = nullptr, const Bufs *into = nullptr) {
  double off = 0.0, vel = 0.0;
  int axis = -1;
  if (ctx->motion_axis >= 0) {
    axis = ctx->motion_axis;
    off = ctx->motion_amp * std::sin(2.0 * kPi * ctx->motion_freq * t);
    vel = ctx->motion_amp * 2.0 * kPi * ctx->motion_freq * std::cos(2.0 * kPi * ctx->motion_freq * t);
  }
  Launch L = ctx->L;
  if (stream) L.st = stream;
  ibmk::run_rebuild_markers(L, into ? *into : ctx->B, ctx->nc, off, vel, axis, ctx->dedupe,
                            save_eps);
  HIPCHECK(ctx, hipGetLastError());
  return IBM_OK;
}

// Waits until the CG of step `tag` has posted a finished solve or its test at
// iteration `target` (see pack_progress). The host spins on the progress word in
// pinned memory; if the stream drains without it, or after a long stall, it
// stops with an error instead of waiting for ever. Without pinned memory the
// stream is synchronised and the scalars are read back.
ibm_status wait_progress(ibm_ctx *ctx, int tag, int target, uint64_t *out) {
  hipStream_t st = ctx->L.st;
  if (!ctx->B.progress) {
    HIPCHECK(ctx, hipStreamSynchronize(st));
    CgScal c;
    HIPCHECK(ctx, hipMemcpy(&c, ctx->B.cg, sizeof(c), hipMemcpyDeviceToHost));
    int f[8];
    HIPCHECK(ctx, hipMemcpy(f, ctx->B.flags, sizeof(f), hipMemcpyDeviceToHost));
    const int err = (f[0] ? 1 : 0) | (f[1] ? 2 : 0) | (f[2] ? 4 : 0) | (f[3] ? 8 : 0);
    *out = ibmk::pack_progress(c.step_tag, c.iters, err, c.done);
    return IBM_OK;
  }
  const auto t0 = std::chrono::steady_clock::now();
  for (uint64_t spin = 1;; ++spin) {
    const uint64_t w = __atomic_load_n(ctx->B.progress, __ATOMIC_ACQUIRE);
    if ((int)(uint32_t)(w >> 32) == tag) {
      const int it = (int)((w >> 8) & 0xFFFFFF);
      if ((w & 0xF) != 0 || it >= target) {
        *out = w;
        return IBM_OK;
      }
    }
    if ((spin & 4095) == 0) {
      hipError_t q = hipStreamQuery(st);
      if (q == hipSuccess) {
        const uint64_t w2 = __atomic_load_n(ctx->B.progress, __ATOMIC_ACQUIRE);
        if (w2 != w) continue;
        return fail(ctx, IBM_E_HIP, "pressure CG finished without reporting its progress");
      }
      if (q != hipErrorNotReady) {
        ctx->err = std::string("stream error while waiting for the CG: ") + hipGetErrorString(q);
        return IBM_E_HIP;
      }
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120))
        return fail(ctx, IBM_E_HIP, "no CG progress for 120 s");
    }
  }
}

ibm_status marker_flags(ibm_ctx *ctx, const int *f) {
  if (f[1]) return fail(ctx, IBM_E_ARG, "a marker support leaves the (non-periodic) box");
  if (f[3]) return fail(ctx, IBM_E_SIZE, "too many overlapping markers for one Gram row");
  if (f[2]) return fail(ctx, IBM_E_NOT_CONVERGED, "the quadrature solve A eps = 1 did not converge");
  return IBM_OK;
}

// Copies state slot `slot` to tape record `rec` (to_tape) or back, in one launch.
ibm_status tape_copy(ibm_ctx *ctx, int rec, int slot, bool to_tape) {
  const GridK &g = ctx->L.g;
  Bufs &B = ctx->B;
  hipStream_t st = ctx->L.st;
  char *base = B.tape + B.tape_stride * (size_t)rec;
  const size_t N = (size_t)g.N;
  const size_t w = ctx->L.prec ? sizeof(float) : sizeof(double);
  void *parts[9];
  size_t sizes[9];
  int np = 0;
  parts[np] = B.rho[slot];
  sizes[np++] = N;
  for (int q = 0; q < g.dim; ++q) {
    parts[np] = B.mom[slot][q];
    sizes[np++] = N;
  }
  parts[np] = B.E[slot];
  sizes[np++] = N;
  for (int q = 0; q < g.dim; ++q) {
    parts[np] = B.F[slot][q];
    sizes[np++] = (size_t)g.NF[q];
  }
  ibmk::CopyParts cp;
  size_t off = 0;
  for (int i = 0; i < np; ++i) {
    void *dst = to_tape ? (void *)(base + off) : parts[i];
    const void *src = to_tape ? (const void *)parts[i] : (const void *)(base + off);
    cp.add(dst, src, sizes[i] * w);
    off += sizes[i] * w;
  }
  Launch L = ctx->L;
  L.st = st;
  ibmk::run_copy_parts(L, cp);
  HIPCHECK(ctx, hipGetLastError());
  return IBM_OK;
}

// Runs a pressure-type CG whose set-up has been queued (tag posted by its
// iterations) to completion with the buffers of `Bc`; returns its iterations.
ibm_status run_cg_to_end(ibm_ctx *ctx, const Bufs &Bc, int tag, int *iters) {
  // every such solve (the adjoint's) runs the FP64 CG, whatever the context's form
  const Launch &L = ctx->L;
  int launched = 0;
  const int first = std::max(1, ctx->adj_hint + 1);
  for (int c = 0; c < first; ++c) ibmk::run_cg64_iteration(L, Bc, launched++);
  HIPCHECK(ctx, hipGetLastError());
  uint64_t w = 0;
  for (;;) {
    ibm_status r = wait_progress(ctx, tag, launched - 1, &w);
    if (r) return r;
    if (w & 0xF) break;
    for (int c = 0; c < 4; ++c) ibmk::run_cg64_iteration(L, Bc, launched++);
    HIPCHECK(ctx, hipGetLastError());
  }
  const int dstate = (int)(w & 0xF), err = (int)((w >> 4) & 0xF);
  *iters = (int)((w >> 8) & 0xFFFFFF);
  ctx->adj_hint = std::max(1, *iters);
  if (err) return fail(ctx, IBM_E_NONFINITE, "adjoint pressure solve stopped on an error flag");
  if (dstate != 1) return fail(ctx, IBM_E_NOT_CONVERGED, "adjoint pressure CG reached cg_maxit");
  return IBM_OK;
}

// Implicit diffusion of one pass of a step, after its predictor: the face
// viscosities of the state in slot `flux`, then the dim + 1 solves side by side
// (one kernel per iteration), started in the first pass from the linear
// extrapolation of the last two steps' solutions when both are held (and
// IBM_CG_START is not plain), else from that state; in a later pass from the
// previous pass's solution. Progress is posted under -(8 tag + 1), apart from
// step tags. Returns the iterations in *iters.
ibm_status diffusion_solves(ibm_ctx *ctx, int tag, int flux, int pass, bool last, int *iters) {
  const Launch &L = ctx->L;
  const Bufs &B = ctx->B;
  const int ring = ctx->diff_ring;
  const int order = pass > 0 ? 2 : (ctx->cg_order >= 1 && ctx->diff_hist >= 2) ? 1 : 0;
  const int dtag = -(tag * 8 + 1);
  ibmk::run_diff_coef(L, B, flux);
  ibmk::run_diff_start(L, B, flux, ring, order, dtag);
  int launched = 0;
  const int first = std::max(1, ctx->diff_hint + 1);
  for (; launched < first; ++launched) ibmk::run_diff_iteration(L, B, ring, launched);
  HIPCHECK(ctx, hipGetLastError());
  uint64_t w = 0;
  for (;;) {
    ibm_status r = wait_progress(ctx, dtag, launched - 1, &w);
    if (r) return r;
    if (w & 0xF) break;
    for (int c = 0; c < 2; ++c) ibmk::run_diff_iteration(L, B, ring, launched++);
    HIPCHECK(ctx, hipGetLastError());
  }
  const int dstate = (int)(w & 0xF), err = (int)((w >> 4) & 0xF);
  *iters = (int)((w >> 8) & 0xFFFFFF);
  ctx->diff_hint = std::max(1, *iters);
  if (err) {
    const ibm_status s = (err & 1) ? IBM_E_NONFINITE : (err & 2) ? IBM_E_ARG
                       : (err & 8) ? IBM_E_SIZE : IBM_E_NOT_CONVERGED;
    return fail(ctx, s, "implicit diffusion solve stopped on an error flag");
  }
  if (dstate != 1) return fail(ctx, IBM_E_NOT_CONVERGED, "implicit diffusion CG reached cg_maxit");
  ibmk::run_diff_finish(L, B, ring);
  HIPCHECK(ctx, hipGetLastError());
  if (last) {
    // this step's solutions now head the ring
    ctx->diff_ring = (ring + 1) % 3;
    ctx->diff_hist = std::min(ctx->diff_hist + 1, 2);
  }
  return IBM_OK;
}

}  // namespace

// ======================================================================== ABI
extern "C" {

size_t ibm_workspace_bytes(const ibm_grid_desc *desc, int32_t max_markers, int32_t tape_steps) {
  if (check_desc(desc) || max_markers < 0 || tape_steps < 0) return 0;
  GridK g = make_grid(*desc);
  Bufs B;
  int np;
  return plan(*desc, g, max_markers, tape_steps, nullptr, B, np);
}

}  // extern "C"

namespace {

// Context creation on a workspace; `pinned` asks for the pinned host word through which
// the CG reports its progress (without it the step loop synchronises instead).
ibm_status create_ctx(const ibm_grid_desc *desc, void *dev_workspace, size_t bytes,
                      int32_t tape_steps, void *hip_stream, bool pinned, ibm_ctx **out) {
  if (!out) return IBM_E_ARG;
  *out = nullptr;
  if (check_desc(desc)) return IBM_E_ARG;
  if (tape_steps < 0) return IBM_E_ARG;
  if (!dev_workspace || (reinterpret_cast<uintptr_t>(dev_workspace) & 255)) return IBM_E_ARG;
  const int nslot = desc->dim == 3 ? 27 : 9;
  if ((int64_t)desc->max_markers * nslot >= ((int64_t)1 << ibmk::kPairBits)) return IBM_E_SIZE;
  ibm_ctx *ctx = new (std::nothrow) ibm_ctx();
  if (!ctx) return IBM_E_HIP;
  ctx->desc = *desc;
  ctx->L.g = make_grid(*desc);
  ctx->L.prec = desc->precision;
  ctx->L.nc_cap = std::max(desc->max_markers, 1);
  ctx->L.st = (hipStream_t)hip_stream;
  {
    // LDS-tiled predictor when its tile fits the device's LDS per workgroup;
    // IBM_PREDICTOR=plain selects the per-cell variant (for comparisons).
    int dev = 0, maxsh = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const size_t need = ibmk::predictor_lds_bytes(desc->dim, desc->precision);
    const char *env = std::getenv("IBM_PREDICTOR");
    ctx->L.pred_lds = (need <= (size_t)maxsh) && !(env && std::strcmp(env, "plain") == 0);
    // FP32 form: iterative refinement around an FP32 inner CG by default in 3D (its
    // column kernels halve the bytes of an iteration), the FP64 CG on the FP32 psi in
    // 2D (there the extra launches of the refinement cost more than the bytes it
    // saves); IBM_FP32_SOLVE=refine or =fp64 chooses either
    const char *fs = std::getenv("IBM_FP32_SOLVE");
    ctx->L.refine32 = (fs && std::strcmp(fs, "refine") == 0) ? 1
                      : (fs && std::strcmp(fs, "fp64") == 0) ? 0
                      : (desc->dim == 3 ? 1 : 0);
    // 3D pressure CG by z-columns; IBM_CG3D=tile selects the tile-wise iteration
    const char *c3 = std::getenv("IBM_CG3D");
    ctx->L.cg_col = (c3 && std::strcmp(c3, "tile") == 0) ? 0 : 1;
    const char *cgs = std::getenv("IBM_CG_START");
    ctx->cg_order = !cgs ? 3 : std::strcmp(cgs, "plain") == 0 ? 0
                             : std::strcmp(cgs, "linear") == 0 ? 1
                             : std::strcmp(cgs, "quadratic") == 0 ? 2 : 3;
    if (ctx->L.pred_lds && need > 65536) ibmk::enable_predictor_lds(desc->dim, desc->precision);
    if (desc->scheme == IBM_SCHEME_DENSITY) ibmk::enable_density_lds(desc->dim, desc->precision);
    // a moving body's markers set up ahead on side streams; IBM_REBUILD=inline
    // keeps them on the context's stream (a context without its own allocations
    // always does)
    const char *rb = std::getenv("IBM_REBUILD");
    ctx->side_ok = pinned && !(rb && std::strcmp(rb, "inline") == 0);
  }
  ctx->tape_cap = tape_steps;
  size_t need = plan(*desc, ctx->L.g, desc->max_markers, tape_steps, (char *)dev_workspace, ctx->B,
                     ctx->L.npairs_pad);
  if (bytes < need) {
    delete ctx;
    return IBM_E_SIZE;
  }
  // one word of pinned, coherent host memory through which the CG reports its
  // progress (without it the step loop synchronises instead)
  if (pinned) {
    void *hp = nullptr;
    if (hipHostMalloc(&hp, 64, hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess && hp) {
      ctx->B.progress = static_cast<uint64_t *>(hp);
      *ctx->B.progress = 0;
    } else {
      (void)hipGetLastError();
      ctx->B.progress = nullptr;
    }
  }
  CgScal c0;
  std::memset(&c0, 0, sizeof(c0));
  c0.tol2 = desc->cg_rtol * desc->cg_rtol;
  c0.maxit = desc->cg_maxit;
  hipError_t e = hipMemcpyAsync(ctx->B.cg, &c0, sizeof(c0), hipMemcpyHostToDevice, ctx->L.st);
  if (e == hipSuccess && ctx->B.dsc) {
    ibmk::DiffScal d0;
    std::memset(&d0, 0, sizeof(d0));
    d0.tol2 = c0.tol2;
    d0.maxit = c0.maxit;
    e = hipMemcpyAsync(ctx->B.dsc, &d0, sizeof(d0), hipMemcpyHostToDevice, ctx->L.st);
  }
  if (e == hipSuccess) e = hipMemsetAsync(ctx->B.flags, 0, 8 * sizeof(int), ctx->L.st);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->B.mcount, 0, 8 * sizeof(int), ctx->L.st);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->B.totals, 0, 8 * sizeof(double), ctx->L.st);
  if (e == hipSuccess) {
    ibmk::run_uniform_state(ctx->L, ctx->B, 0);
    if (ctx->B.wbar) ibmk::run_shape_clear(ctx->L, ctx->B, ctx->L.nc_cap);
    // the adjoint pressure solve starts from the previous one's solution
    if (ctx->B.lam) ibmk::run_fill(ctx->L, ctx->B.lam, ctx->L.g.N, 0.0);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->L.st);
  if (e != hipSuccess) {
    delete ctx;
    return IBM_E_HIP;
  }
  *out = ctx;
  return IBM_OK;
}

}  // namespace

extern "C" {

ibm_status ibm_create_grid(const ibm_grid_desc *desc, void *dev_workspace, size_t bytes,
                           int32_t tape_steps, void *hip_stream, ibm_ctx **out) {
  return create_ctx(desc, dev_workspace, bytes, tape_steps, hip_stream, true, out);
}

}  // extern "C"

// Device memory of ibm_create_grid_noalloc: one fixed array per GPU the library runs
// on (each device holds its own copy until the process ends). Host code never uses the
// array's name as an address: its device address is looked up once per device and kept.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];   // device address of `scratch`, per device
bool g_scratch_busy[kScratchDevices];  // a live context holds the device's array
}  // namespace

extern "C" {

ibm_status ibm_create_grid_noalloc(const ibm_grid_desc *desc, int32_t tape_steps,
                                   void *hip_stream, ibm_ctx **out) {
  if (!out) return IBM_E_ARG;
  *out = nullptr;
  if (check_desc(desc) || tape_steps < 0) return IBM_E_ARG;
  const size_t need = ibm_workspace_bytes(desc, desc->max_markers, tape_steps);
  if (need == 0) return IBM_E_ARG;
  if (need > kScratchBytes) return IBM_E_SIZE;  // beyond the fixed array (64 MiB)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return IBM_E_HIP;
  void *ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void *p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return IBM_E_HIP;
      }
      g_scratch_ptr[dev] = p;
    }
    if (g_scratch_busy[dev]) return IBM_E_STATE;  // one live context per device
    g_scratch_busy[dev] = true;
    ptr = g_scratch_ptr[dev];
  }
  // no pinned progress word either: the step loop synchronises instead
  ibm_status st = create_ctx(desc, ptr, kScratchBytes, tape_steps, hip_stream, false, out);
  if (st != IBM_OK) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    g_scratch_busy[dev] = false;
    return st;
  }
  (*out)->scratch_dev = dev;
  return IBM_OK;
}

void ibm_destroy(ibm_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->L.st);
  const int sd = ctx->scratch_dev;
  delete ctx;
  if (sd >= 0) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    g_scratch_busy[sd] = false;
  }
}

const char *ibm_last_error(const ibm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

double ibm_dt(const ibm_ctx *ctx) { return ctx ? ctx->L.g.dt : 0.0; }

ibm_status ibm_init_primitive(ibm_ctx *ctx, const void *rho, const void *u, const void *theta) {
  if (!ctx) return IBM_E_ARG;
  if (!rho || !u || !theta) return fail(ctx, IBM_E_ARG, "init_primitive: NULL field");
  ibmk::run_init_primitive(ctx->L, ctx->B, ctx->cur, rho, u, theta);
  HIPCHECK(ctx, hipGetLastError());
  ctx->step = 0;
  ctx->prev_valid = ctx->hist_valid = ctx->hist2_valid = false;
  ctx->diff_hist = 0;
  if (ctx->nc > 0 && ctx->motion_axis >= 0) {
    ibm_status s = rebuild_markers(ctx, 0.0);
    if (s) return s;
  }
  HIPCHECK(ctx, hipStreamSynchronize(ctx->L.st));
  return IBM_OK;
}

ibm_status ibm_set_state(ibm_ctx *ctx, const void *rho, const void *mom, const void *eint,
                         const void *face_flux, int64_t step) {
  if (!ctx) return IBM_E_ARG;
  if (!rho || !mom || !eint) return fail(ctx, IBM_E_ARG, "set_state: NULL field");
  if (step < 0) return fail(ctx, IBM_E_ARG, "set_state: negative step");
  const GridK &g = ctx->L.g;
  const size_t w = ctx->L.prec ? 4 : 8;
  const int c = ctx->cur;
  hipStream_t st = ctx->L.st;
  HIPCHECK(ctx, hipMemcpyAsync(ctx->B.rho[c], rho, g.N * w, hipMemcpyDeviceToDevice, st));
  HIPCHECK(ctx, hipMemcpyAsync(ctx->B.E[c], eint, g.N * w, hipMemcpyDeviceToDevice, st));
  for (int q = 0; q < g.dim; ++q)
    HIPCHECK(ctx, hipMemcpyAsync(ctx->B.mom[c][q], (const char *)mom + q * g.N * w, g.N * w,
                                 hipMemcpyDeviceToDevice, st));
  if (face_flux) {
    size_t off = 0;
    for (int q = 0; q < g.dim; ++q) {
      HIPCHECK(ctx, hipMemcpyAsync(ctx->B.F[c][q], (const char *)face_flux + off * w, g.NF[q] * w,
                                   hipMemcpyDeviceToDevice, st));
      off += g.NF[q];
    }
  } else {
    ibmk::run_flux_from_momentum(ctx->L, ctx->B, c);
    HIPCHECK(ctx, hipGetLastError());
  }
  ctx->step = step;
  ctx->prev_valid = ctx->hist_valid = ctx->hist2_valid = false;
  ctx->diff_hist = 0;
  if (ctx->nc > 0 && ctx->motion_axis >= 0) {
    ibm_status s = rebuild_markers(ctx, double(step) * g.dt);
    if (s) return s;
  }
  HIPCHECK(ctx, hipStreamSynchronize(st));
  return IBM_OK;
}

ibm_status ibm_get_state(const ibm_ctx *cctx, void *rho, void *mom, void *eint, void *face_flux) {
  ibm_ctx *ctx = const_cast<ibm_ctx *>(cctx);
  if (!ctx) return IBM_E_ARG;
  const GridK &g = ctx->L.g;
  const size_t w = ctx->L.prec ? 4 : 8;
  const int c = ctx->cur;
  hipStream_t st = ctx->L.st;
  if (rho) HIPCHECK(ctx, hipMemcpyAsync(rho, ctx->B.rho[c], g.N * w, hipMemcpyDeviceToDevice, st));
  if (eint) HIPCHECK(ctx, hipMemcpyAsync(eint, ctx->B.E[c], g.N * w, hipMemcpyDeviceToDevice, st));
  if (mom)
    for (int q = 0; q < g.dim; ++q)
      HIPCHECK(ctx, hipMemcpyAsync((char *)mom + q * g.N * w, ctx->B.mom[c][q], g.N * w,
                                   hipMemcpyDeviceToDevice, st));
  if (face_flux) {
    size_t off = 0;
    for (int q = 0; q < g.dim; ++q) {
      HIPCHECK(ctx, hipMemcpyAsync((char *)face_flux + off * w, ctx->B.F[c][q], g.NF[q] * w,
                                   hipMemcpyDeviceToDevice, st));
      off += g.NF[q];
    }
  }
  return IBM_OK;
}

ibm_status ibm_set_markers(ibm_ctx *ctx, int32_t n, const double *X, const double *U_d,
                           const double *T_w, const double *dA, uint32_t flags) {
  if (!ctx) return IBM_E_ARG;
  if (n < 0) return fail(ctx, IBM_E_ARG, "set_markers: n < 0");
  if (n > ctx->desc.max_markers) return fail(ctx, IBM_E_SIZE, "set_markers: n exceeds max_markers");
  if (flags & ~(IBM_DEDUPE | IBM_NO_HEAT)) return fail(ctx, IBM_E_ARG, "set_markers: unknown flag");
  if (n > 0 && !X) return fail(ctx, IBM_E_ARG, "set_markers: X is NULL");
  const int dim = ctx->desc.dim;
  hipStream_t st = ctx->L.st;
  Bufs &B = ctx->B;
  ctx->nc = 0;
  ctx->tape_len = 0;
  if (n == 0) {
    HIPCHECK(ctx, hipMemsetAsync(B.mcount, 0, 8 * sizeof(int), st));
    HIPCHECK(ctx, hipStreamSynchronize(st));
    return IBM_OK;
  }
  const size_t pitch_dst = 3 * sizeof(double), pitch_src = dim * sizeof(double);
  HIPCHECK(ctx, hipMemsetAsync(B.cX0, 0, 3 * n * sizeof(double), st));
  HIPCHECK(ctx, hipMemsetAsync(B.cUd0, 0, 3 * n * sizeof(double), st));
  HIPCHECK(ctx, hipMemcpy2DAsync(B.cX0, pitch_dst, X, pitch_src, pitch_src, n,
                                 hipMemcpyDeviceToDevice, st));
  if (U_d)
    HIPCHECK(ctx, hipMemcpy2DAsync(B.cUd0, pitch_dst, U_d, pitch_src, pitch_src, n,
                                   hipMemcpyDeviceToDevice, st));
  if (T_w)
    HIPCHECK(ctx, hipMemcpyAsync(B.cTw, T_w, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    ibmk::run_fill(ctx->L, B.cTw, n, 1.0);
  if (dA)
    HIPCHECK(ctx, hipMemcpyAsync(B.cdA, dA, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    HIPCHECK(ctx, hipMemsetAsync(B.cdA, 0, n * sizeof(double), st));
  ibmk::run_fill(ctx->L, B.ceps, n, dim == 3 ? 8.0 : 4.0);
  HIPCHECK(ctx, hipMemsetAsync(B.flags, 0, 8 * sizeof(int), st));
  ctx->nc = n;
  ctx->dedupe = (flags & IBM_DEDUPE) ? 1 : 0;
  ctx->L.g.no_heat = (flags & IBM_NO_HEAT) ? 1 : 0;
  ibm_status s = rebuild_markers(ctx, double(ctx->step) * ctx->L.g.dt, true);
  if (s) {
    ctx->nc = 0;
    return s;
  }
  int f[8];
  s = sync_read(ctx, f, B.flags, sizeof(f));
  if (s) return s;
  s = marker_flags(ctx, f);
  if (s) ctx->nc = 0;
  return s;
}

ibm_status ibm_set_motion(ibm_ctx *ctx, int32_t axis, double amplitude, double frequency) {
  if (!ctx) return IBM_E_ARG;
  if (axis >= ctx->desc.dim) return fail(ctx, IBM_E_ARG, "set_motion: axis >= dim");
  if (!std::isfinite(amplitude) || !std::isfinite(frequency))
    return fail(ctx, IBM_E_ARG, "set_motion: non-finite parameter");
  ctx->motion_axis = axis < 0 ? -1 : axis;
  ctx->tape_len = 0;
  ctx->motion_amp = amplitude;
  ctx->motion_freq = frequency;
  if (ctx->nc > 0) {
    hipStream_t st = ctx->L.st;
    HIPCHECK(ctx, hipMemsetAsync(ctx->B.flags, 0, 8 * sizeof(int), st));
    ibm_status s = rebuild_markers(ctx, double(ctx->step) * ctx->L.g.dt);
    if (s) return s;
    int f[8];
    s = sync_read(ctx, f, ctx->B.flags, sizeof(f));
    if (s) return s;
    return marker_flags(ctx, f);
  }
  return IBM_OK;
}

ibm_status ibm_set_wall_temperature(ibm_ctx *ctx, const double *T_w) {
  if (!ctx) return IBM_E_ARG;
  if (ctx->nc == 0) return fail(ctx, IBM_E_STATE, "set_wall_temperature: no markers");
  if (!T_w) return fail(ctx, IBM_E_ARG, "set_wall_temperature: NULL");
  ctx->tape_len = 0;
  hipStream_t st = ctx->L.st;
  HIPCHECK(ctx, hipMemcpyAsync(ctx->B.cTw, T_w, ctx->nc * sizeof(double), hipMemcpyDeviceToDevice,
                               st));
  // re-gather the markers in use (same time, same selection; eps unchanged)
  double off = 0.0, vel = 0.0;
  const double t = double(ctx->step) * ctx->L.g.dt;
  if (ctx->motion_axis >= 0) {
    off = ctx->motion_amp * std::sin(2.0 * kPi * ctx->motion_freq * t);
    vel = ctx->motion_amp * 2.0 * kPi * ctx->motion_freq * std::cos(2.0 * kPi * ctx->motion_freq * t);
  }
  ibmk::run_place_markers(ctx->L, ctx->B, ctx->nc, off, vel, ctx->motion_axis, ctx->dedupe);
  HIPCHECK(ctx, hipGetLastError());
  HIPCHECK(ctx, hipStreamSynchronize(st));
  return IBM_OK;
}

ibm_status ibm_step(ibm_ctx *ctx, int32_t n_steps, uint32_t flags, double *hist,
                    ibm_step_info *info) {
  if (!ctx) return IBM_E_ARG;
  if (n_steps < 0) return fail(ctx, IBM_E_ARG, "step: n_steps < 0");
  if (flags & ~IBM_RECORD) return fail(ctx, IBM_E_ARG, "step: unknown flag");
  const bool record = (flags & IBM_RECORD) != 0;
  if (record && n_steps > ctx->tape_cap)
    return fail(ctx, IBM_E_SIZE, "step: IBM_RECORD of more steps than the tape holds");
  if (record) ctx->tape_len = 0;
  const Launch &L = ctx->L;
  Bufs &B = ctx->B;
  hipStream_t st = L.st;
  ibm_status rc = IBM_OK;
  int64_t done = 0;
  int total_it = 0, last_it = 0, diff_it = 0;
  Prof &P = ctx->prof;
  auto timed = [&](int cls, int it, auto &&launch) {
    if (!P.on) {
      launch();
      return;
    }
    hipEvent_t a = P.mark(st);
    launch();
    hipEvent_t b = P.mark(st);
    P.pending.push_back({cls, it, 1, a, b});
  };
  // a batch of `count` CG iterations from `it0`, back to back
  auto cg_batch = [&](int it0, int count) {
    hipEvent_t a = P.on ? P.mark(st) : nullptr;
    for (int it = it0; it < it0 + count; ++it) ibmk::run_cg_iteration(L, B, it);
    if (P.on) {
      hipEvent_t b = P.mark(st);
      P.pending.push_back({IBM_PROF_CG, it0, count, a, b});
    }
  };
  // A moving body: the first step of the call sets its markers up on the main
  // stream and queues the next step's into the other set; every step queues, after
  // its last marker kernel, the set-up of the step two ahead into its own set (see
  // ibm_ctx::side), within the call.
  const bool moving = ctx->nc > 0 && ctx->motion_axis >= 0;
  if (moving && ctx->side_ok && !ctx->side[0]) {
    for (int k = 0; k < 2; ++k) {
      HIPCHECK(ctx, hipStreamCreateWithFlags(&ctx->side[k], hipStreamNonBlocking));
      HIPCHECK(ctx, hipEventCreateWithFlags(&ctx->ev_used[k], hipEventDisableTiming));
      HIPCHECK(ctx, hipEventCreateWithFlags(&ctx->ev_built[k], hipEventDisableTiming));
    }
  }
  const bool use_side = moving && ctx->side[0] != nullptr;
  ctx->set_step[0] = ctx->set_step[1] = -1;
  // the main stream waits for the set-ups queued and not yet waited for
  auto join_all = [&]() -> hipError_t {
    for (int k = 0; k < 2; ++k) {
      if (!ctx->pending[k]) continue;
      ctx->pending[k] = false;
      hipError_t e = hipStreamWaitEvent(st, ctx->ev_built[k], 0);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  // an early return still leaves the main stream behind the side streams' work
  struct AheadGuard {
    ibm_ctx *c;
    ~AheadGuard() {
      for (int k = 0; k < 2; ++k) {
        if (!c->pending[k]) continue;
        c->pending[k] = false;
        (void)hipStreamWaitEvent(c->L.st, c->ev_built[k], 0);
      }
    }
  } ahead_guard{ctx};
  // queues the set-up of `step`'s markers (time (step + 1) dt) into set k on side[k],
  // behind the main stream's work so far (its last use of set k)
  auto queue_setup = [&](int64_t step, int k) -> ibm_status {
    HIPCHECK(ctx, hipEventRecord(ctx->ev_used[k], st));
    HIPCHECK(ctx, hipStreamWaitEvent(ctx->side[k], ctx->ev_used[k], 0));
    Bufs Bk = B;
    if (k != ctx->aset) ibmk::put_marker_set(Bk, B.alt);
    ctx->set_step[k] = -1;
    hipEvent_t a = P.on ? P.mark(ctx->side[k]) : nullptr;
    ibm_status ms = rebuild_markers(ctx, double(step + 1) * L.g.dt, false, ctx->side[k], &Bk);
    if (P.on) P.pending.push_back({IBM_PROF_REBUILD, 0, 1, a, P.mark(ctx->side[k])});
    if (ms) return ms;
    HIPCHECK(ctx, hipEventRecord(ctx->ev_built[k], ctx->side[k]));
    ctx->pending[k] = true;
    ctx->set_step[k] = step;
    return IBM_OK;
  };
  // the markers of the step starting now (s-th of the call) into Bufs: the set
  // queued for it, or set up here (then the next step's are queued)
  auto step_markers = [&](int s) -> ibm_status {
    if (!moving) return IBM_OK;
    const int64_t step = ctx->step;
    const int k = ctx->set_step[0] == step ? 0 : ctx->set_step[1] == step ? 1 : -1;
    if (k >= 0) {
      if (k != ctx->aset) {
        const ibmk::MarkerSet held = ibmk::marker_set_of(B);
        ibmk::put_marker_set(B, B.alt);
        B.alt = held;
        ctx->aset = k;
      }
      return IBM_OK;
    }
    ibm_status ms = IBM_OK;
    timed(IBM_PROF_MARKERS, 0, [&] { ms = rebuild_markers(ctx, double(step + 1) * L.g.dt); });
    if (ms) return ms;
    ctx->set_step[ctx->aset] = step;
    if (use_side && s + 1 < n_steps) return queue_setup(step + 1, ctx->aset ^ 1);
    return IBM_OK;
  };
  // before the step's first marker kernel: its set is ready
  auto join_markers = [&]() -> hipError_t {
    const int k = ctx->aset;
    if (!ctx->pending[k]) return hipSuccess;
    ctx->pending[k] = false;
    return hipStreamWaitEvent(st, ctx->ev_built[k], 0);
  };
  // after the step's last marker kernel: the step two ahead into this step's set
  auto queue_after = [&](int s) -> ibm_status {
    if (!use_side || s + 2 >= n_steps) return IBM_OK;
    return queue_setup(ctx->step + 2, ctx->aset);
  };
  // Flags are sticky for the whole call: a step that fails keeps every later step
  // from writing the state, so the state it started from survives.
  HIPCHECK(ctx, hipMemsetAsync(B.flags, 0, 8 * sizeof(int), st));
  const int cur0 = ctx->cur;
  const int64_t step0 = ctx->step;
  const int first_tag = ctx->tag + 1;
  if (ctx->desc.scheme == IBM_SCHEME_DENSITY) {
    if (record) return fail(ctx, IBM_E_ARG, "step: the density-based step has no adjoint tape");
    // App. B: the explicit step without the body, the marker sources from its
    // result, the new state; nothing waits for the host
    for (int s = 0; s < n_steps; ++s) {
      const int tag = ++ctx->tag;
      {
        ibm_status ms = step_markers(s);
        if (ms) return ms;
      }
      timed(IBM_PROF_PREDICTOR, 0, [&] { ibmk::run_density_predictor(L, B, ctx->cur); });
      double *hrow = hist ? hist + 4 * (size_t)s : nullptr;
      if (ctx->nc > 0) {
        HIPCHECK(ctx, join_markers());
        timed(IBM_PROF_MARKERS, 0, [&] { ibmk::run_markers_step(L, B, hrow); });
        {
          ibm_status ms = queue_after(s);
          if (ms) return ms;
        }
      } else if (hrow) {
        HIPCHECK(ctx, hipMemsetAsync(hrow, 0, 4 * sizeof(double), st));
      }
      timed(IBM_PROF_CORRECT, 0, [&] { ibmk::run_density_finish(L, B, ctx->cur, tag); });
      HIPCHECK(ctx, hipGetLastError());
      ctx->cur ^= 1;
      ctx->prev_valid = ctx->hist_valid = ctx->hist2_valid = false;
      ctx->step += 1;
      ++done;
    }
  }
  // App. A step 3 is run `passes` times per step: every pass after the first
  // re-evaluates the predictor at the latest iterate (the other state slot) with
  // the step's start (slot cur) for the time derivative, re-spreads the marker
  // sources of the first pass, and solves the pressure equation again from the
  // previous pass's solution. Each pass has its own tag.
  const int passes = std::max(1, ctx->desc.n_outer);
  for (int s = 0; s < (ctx->desc.scheme == IBM_SCHEME_DENSITY ? 0 : n_steps); ++s) {
    {
      ibm_status ms = step_markers(s);
      if (ms) return ms;
    }
    if (record) {
      ibm_status ts = tape_copy(ctx, s, ctx->cur, true);
      if (ts) return ts;
    }
    const int order = std::min(
        ctx->cg_order, ctx->prev_valid ? (ctx->hist_valid ? (ctx->hist2_valid ? 3 : 2) : 1) : 0);
    double *hrow = hist ? hist + 4 * (size_t)s : nullptr;
    bool failed = false, maxit = false;
    int iters = 0;
    for (int pass = 0; pass < passes; ++pass) {
      const int tag = ++ctx->tag;
      const bool first = pass == 0;
      const int flux = first ? ctx->cur : ctx->cur ^ 1;
      P.step_first = P.pending.size();
      timed(IBM_PROF_PREDICTOR, 0, [&] {
        ibmk::run_predictor(L, B, ctx->cur, flux, first ? order : -1,
                            first ? ctx->cg_order - 1 : 0);
      });
      // the FP32 refinement may have finished in its second x buffer
      if (!first && L.prec == 1 && L.refine32) ibmk::run_copy_solution(L, B, B.x);
      if (L.g.implicit_diff) {
        ibm_status ds = IBM_OK;
        int dit = 0;
        timed(IBM_PROF_DIFFUSION, 0,
              [&] { ds = diffusion_solves(ctx, tag, flux, pass, pass == passes - 1, &dit); });
        diff_it += dit;
        if (ds) {
          // E_hist may already hold this step's E^{n-1}
          ctx->prev_valid = ctx->hist_valid = ctx->hist2_valid = false;
          ctx->diff_hist = 0;
          rc = ds;
          failed = true;
          break;
        }
      }
      if (ctx->nc > 0) {
        HIPCHECK(ctx, join_markers());
        if (first)
          timed(IBM_PROF_MARKERS, 0, [&] { ibmk::run_markers_step(L, B, hrow); });
        else
          timed(IBM_PROF_MARKERS, 0, [&] { ibmk::run_spread(L, B); });
        if (pass == passes - 1) {
          ibm_status ms = queue_after(s);
          if (ms) return ms;
        }
      } else if (hrow && first) {
        HIPCHECK(ctx, hipMemsetAsync(hrow, 0, 4 * sizeof(double), st));
      }
      timed(IBM_PROF_SETUP, 0, [&] { ibmk::run_setup(L, B, ctx->cur, tag); });
      // Iteration `it` tests convergence after `it` updates at its start, so a solve
      // of n iterations takes n + 1 launches; launches past convergence return at
      // once. The first batch follows the last solve's count, and the correction is
      // queued behind it (it runs only once the solve has finished), so the device
      // does not wait for the host unless the batch falls short.
      int launched = 0;
      const int nfirst = std::max(1, ctx->cg_hint + 1);
      cg_batch(launched, nfirst);
      launched += nfirst;
      timed(IBM_PROF_CORRECT, 0, [&] { ibmk::run_correct(L, B, ctx->cur, tag); });
      HIPCHECK(ctx, hipGetLastError());
      uint64_t w = 0;
      for (;;) {
        ibm_status r = wait_progress(ctx, tag, launched - 1, &w);
        if (r) return r;
        if (w & 0xF) break;
        cg_batch(launched, 2);
        launched += 2;
        timed(IBM_PROF_CORRECT, 0, [&] { ibmk::run_correct(L, B, ctx->cur, tag); });
        HIPCHECK(ctx, hipGetLastError());
      }
      const int dstate = (int)(w & 0xF), err = (int)((w >> 4) & 0xF);
      iters = (int)((w >> 8) & 0xFFFFFF);
      if (P.on) P.count_cg(iters);
      if (err) {
        ctx->prev_valid = ctx->hist_valid = ctx->hist2_valid = false;
        ctx->diff_hist = 0;
        // this pass's correction did not run; an earlier failure is sorted out below
        rc = (err & 1) ? IBM_E_NONFINITE : (err & 2) ? IBM_E_ARG : (err & 8) ? IBM_E_SIZE
                                                                           : IBM_E_NOT_CONVERGED;
        failed = true;
        break;
      }
      total_it += iters;
      ctx->cg_hint = std::max(1, iters);
      if (dstate != 1) {  // the correction ran; the step ends here
        maxit = true;
        break;
      }
    }
    if (failed) break;
    if (record) {
      ibmk::run_copy_solution(L, B, (double *)(B.tape + B.tape_stride * (size_t)s + B.tape_xoff));
      HIPCHECK(ctx, hipGetLastError());
    }
    ctx->cur ^= 1;
    ctx->hist2_valid = ctx->hist_valid && ctx->cg_order >= 3;
    ctx->hist_valid = ctx->prev_valid && ctx->cg_order >= 2;
    ctx->prev_valid = true;
    ctx->step += 1;
    ++done;
    last_it = iters;
    if (maxit) {
      rc = fail(ctx, IBM_E_NOT_CONVERGED, "pressure CG reached cg_maxit");
      break;
    }
  }
  if (done > 0) ibmk::run_mass(L, B);
  HIPCHECK(ctx, join_all());  // a step that failed may leave later steps' markers queued
  HIPCHECK(ctx, hipStreamSynchronize(st));
  int f[8];
  {
    ibm_status r = sync_read(ctx, f, B.flags, sizeof(f));
    if (r) return r;
    r = sync_read(ctx, &ctx->cgh, B.cg, sizeof(CgScal));
    if (r) return r;
  }
  if (P.on) P.settle();
  if (f[ibmk::FLAG_NONFINITE]) {
    // the first failing step and every later one left their input in place
    const int s_bad = ((f[ibmk::FLAG_BAD_STEP] - 1) - first_tag) / passes;
    if (s_bad >= 0 && s_bad <= n_steps) {
      ctx->cur = cur0 ^ (s_bad & 1);
      ctx->prev_valid = ctx->hist_valid = ctx->hist2_valid = false;
      ctx->diff_hist = 0;
      ctx->step = step0 + s_bad;
      done = s_bad;
    }
    rc = fail(ctx, IBM_E_NONFINITE, "step produced a non-finite or non-positive value");
  } else if (f[ibmk::FLAG_SUPPORT] || f[ibmk::FLAG_EPS] || f[ibmk::FLAG_GRAM]) {
    rc = marker_flags(ctx, f);
  }
  if (info) {
    info->steps_done = done;
    info->step = ctx->step;
    info->cg_iters_last = last_it;
    info->cg_iters_total = total_it;
    info->diff_iters_total = diff_it;
    info->cg_residual = ctx->cgh.res;
    info->dt = L.g.dt;
    info->time = double(ctx->step) * L.g.dt;
    double m = 0.0;
    if (done > 0) {
      ibm_status r = sync_read(ctx, &m, B.scal, sizeof(double));
      if (r) return r;
    }
    info->mass = m;
  }
  if (record) ctx->tape_len = (int)done;
  return rc;
}

ibm_status ibm_wall_fluxes(const ibm_ctx *cctx, double *force, double *heat, double *totals) {
  ibm_ctx *ctx = const_cast<ibm_ctx *>(cctx);
  if (!ctx) return IBM_E_ARG;
  hipStream_t st = ctx->L.st;
  int nu = 0;
  if (ctx->nc > 0) {
    ibm_status r = sync_read(ctx, &nu, ctx->B.mcount, sizeof(int));
    if (r) return r;
  }
  const int dim = ctx->desc.dim;
  if (force && nu > 0)
    HIPCHECK(ctx, hipMemcpy2DAsync(force, dim * sizeof(double), ctx->B.mforce, 3 * sizeof(double),
                                   dim * sizeof(double), nu, hipMemcpyDeviceToDevice, st));
  if (heat && nu > 0)
    HIPCHECK(ctx, hipMemcpyAsync(heat, ctx->B.mheat, nu * sizeof(double), hipMemcpyDeviceToDevice,
                                 st));
  if (totals) {
    if (ctx->nc > 0) {
      ibm_status r = sync_read(ctx, totals, ctx->B.totals, 4 * sizeof(double));
      if (r) return r;
    } else {
      for (int q = 0; q < 4; ++q) totals[q] = 0.0;
    }
  }
  return IBM_OK;
}

ibm_status ibm_wall_heat_flux(const ibm_ctx *cctx, double *q) {
  ibm_ctx *ctx = const_cast<ibm_ctx *>(cctx);
  if (!ctx) return IBM_E_ARG;
  if (!q) return fail(ctx, IBM_E_ARG, "wall_heat_flux: NULL destination");
  if (ctx->nc == 0) return fail(ctx, IBM_E_STATE, "wall_heat_flux: no markers");
  hipStream_t st = ctx->L.st;
  // status word: the last of the 8 flag slots (FLAG_* use 0..4)
  int *status = ctx->B.flags + 7;
  ibmk::run_heat_flux(ctx->L, ctx->B, ctx->nc, q, status);
  HIPCHECK(ctx, hipGetLastError());
  int stv = 0;
  ibm_status r = sync_read(ctx, &stv, status, sizeof(int));
  if (r) return r;
  if (stv) return fail(ctx, IBM_E_STATE, "wall_heat_flux: the markers in use carry no surface (dA)");
  return IBM_OK;
}

ibm_status ibm_markers_in_use(const ibm_ctx *cctx, int32_t *n_used, int32_t *ids, double *eps) {
  ibm_ctx *ctx = const_cast<ibm_ctx *>(cctx);
  if (!ctx) return IBM_E_ARG;
  int nu = 0;
  if (ctx->nc > 0) {
    ibm_status r = sync_read(ctx, &nu, ctx->B.mcount, sizeof(int));
    if (r) return r;
  }
  if (n_used) *n_used = nu;
  hipStream_t st = ctx->L.st;
  if (ids && nu > 0)
    HIPCHECK(ctx, hipMemcpyAsync(ids, ctx->B.ids, nu * sizeof(int), hipMemcpyDeviceToDevice, st));
  if (eps && nu > 0)
    HIPCHECK(ctx, hipMemcpyAsync(eps, ctx->B.eps, nu * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHECK(ctx, hipStreamSynchronize(st));
  return IBM_OK;
}

ibm_status ibm_get_field(const ibm_ctx *cctx, int32_t which, void *dst) {
  ibm_ctx *ctx = const_cast<ibm_ctx *>(cctx);
  if (!ctx) return IBM_E_ARG;
  if (!dst) return fail(ctx, IBM_E_ARG, "get_field: NULL destination");
  const GridK &g = ctx->L.g;
  const size_t w = ctx->L.prec ? 4 : 8;
  hipStream_t st = ctx->L.st;
  const Bufs &B = ctx->B;
  switch (which) {
    case 0:
      HIPCHECK(ctx, hipMemcpyAsync(dst, B.rho_s, g.N * w, hipMemcpyDeviceToDevice, st));
      break;
    case 1:
      for (int q = 0; q < g.dim; ++q)
        HIPCHECK(ctx, hipMemcpyAsync((char *)dst + q * g.N * w, B.mom_s[q], g.N * w,
                                     hipMemcpyDeviceToDevice, st));
      break;
    case 2:
      HIPCHECK(ctx, hipMemcpyAsync(dst, B.E_s, g.N * w, hipMemcpyDeviceToDevice, st));
      break;
    case 3:
      HIPCHECK(ctx, hipMemcpyAsync(dst, B.psi, g.N * w, hipMemcpyDeviceToDevice, st));
      break;
    case 4:
      HIPCHECK(ctx, hipMemcpyAsync(dst, B.b, g.N * 8, hipMemcpyDeviceToDevice, st));
      break;
    case 5: {
      ibm_status r = sync_read(ctx, &ctx->cgh, B.cg, sizeof(CgScal));
      if (r) return r;
      const double *xs = (ctx->cgh.xfinal && B.x2) ? B.x2 : B.x;
      HIPCHECK(ctx, hipMemcpyAsync(dst, xs, g.N * 8, hipMemcpyDeviceToDevice, st));
      break;
    }
    case 6: {
      int nu = 0;
      if (ctx->nc > 0) {
        ibm_status r = sync_read(ctx, &nu, B.mcount, sizeof(int));
        if (r) return r;
      }
      if (nu > 0)
        HIPCHECK(ctx, hipMemcpyAsync(dst, B.mk, (size_t)nu * (2 * g.dim + 3) * sizeof(double),
                                     hipMemcpyDeviceToDevice, st));
      break;
    }
    default:
      return fail(ctx, IBM_E_ARG, "get_field: unknown field");
  }
  HIPCHECK(ctx, hipStreamSynchronize(st));
  return IBM_OK;
}

int32_t ibm_tape_length(const ibm_ctx *ctx) { return ctx ? ctx->tape_len : 0; }

ibm_status ibm_shape_gradient(ibm_ctx *ctx, double *X_bar) {
  if (!ctx) return IBM_E_ARG;
  if (!ctx->B.wbar) return fail(ctx, IBM_E_STATE, "shape_gradient: no adjoint workspace");
  if (ctx->motion_axis >= 0)
    return fail(ctx, IBM_E_ARG, "shape_gradient: markers must be at rest");
  if (ctx->nc == 0) return fail(ctx, IBM_E_STATE, "shape_gradient: no markers");
  const Launch &L = ctx->L;
  hipStream_t st = L.st;
  if (!X_bar) {
    ibmk::run_shape_clear(L, ctx->B, ctx->nc);
    HIPCHECK(ctx, hipGetLastError());
    HIPCHECK(ctx, hipStreamSynchronize(st));
    ctx->shape_acc = true;
    return IBM_OK;
  }
  ctx->shape_acc = false;
  if (!ibmk::shape_supported(ctx->nc))
    return fail(ctx, IBM_E_SIZE, "shape_gradient: more candidate markers than supported");
  HIPCHECK(ctx, hipMemsetAsync(ctx->B.flags, 0, 8 * sizeof(int), st));
  ibmk::run_shape_gradient(L, ctx->B, ctx->nc, X_bar);
  HIPCHECK(ctx, hipGetLastError());
  int fl[8];
  HIPCHECK(ctx, hipMemcpyAsync(fl, ctx->B.flags, sizeof(fl), hipMemcpyDeviceToHost, st));
  HIPCHECK(ctx, hipStreamSynchronize(st));
  if (fl[2]) return fail(ctx, IBM_E_NOT_CONVERGED, "shape_gradient: quadrature adjoint solve");
  return IBM_OK;
}

ibm_status ibm_adjoint_step(ibm_ctx *ctx, int32_t tape_index, const double *state_bar_in,
                            double *state_bar_out, const double *out_bar, double *Tw_bar) {
  if (!ctx) return IBM_E_ARG;
  if (ctx->motion_axis >= 0) return fail(ctx, IBM_E_ARG, "adjoint_step: markers must be at rest");
  if (ctx->L.g.implicit_diff)
    return fail(ctx, IBM_E_ARG, "adjoint_step: implicit diffusion has no adjoint");
  if (ctx->desc.n_outer > 1)
    return fail(ctx, IBM_E_ARG, "adjoint_step: outer passes have no adjoint");
  if (ctx->desc.scheme == IBM_SCHEME_DENSITY)
    return fail(ctx, IBM_E_ARG, "adjoint_step: the density-based step has no adjoint");
  if (ctx->L.g.no_heat)
    return fail(ctx, IBM_E_ARG, "adjoint_step: markers without heat exchange have no adjoint");
  if (!state_bar_in || !state_bar_out) return fail(ctx, IBM_E_ARG, "adjoint_step: NULL cotangent");
  if (state_bar_in == state_bar_out)
    return fail(ctx, IBM_E_ARG, "adjoint_step: state_bar_in and state_bar_out must differ");
  if (ctx->nc > 0 && (!out_bar || !Tw_bar))
    return fail(ctx, IBM_E_ARG, "adjoint_step: out_bar and Tw_bar are needed with markers");
  if (tape_index < 0 || tape_index >= ctx->tape_len)
    return fail(ctx, IBM_E_STATE, "adjoint_step: tape_index is not a recorded step");
  const Launch &L = ctx->L;
  Bufs &B = ctx->B;
  hipStream_t st = L.st;
  const int slot = ctx->cur ^ 1;
  // the other slot now holds the recorded state
  ctx->prev_valid = ctx->hist_valid = ctx->hist2_valid = false;
  ctx->diff_hist = 0;
  const double zero4[4] = {0.0, 0.0, 0.0, 0.0};
  const double *ob = out_bar ? out_bar : zero4;
  // forward pieces of the step, recomputed from its record
  HIPCHECK(ctx, hipMemsetAsync(B.flags, 0, 8 * sizeof(int), st));
  {
    ibm_status r = tape_copy(ctx, tape_index, slot, false);
    if (r) return r;
  }
  ibmk::run_predictor(L, B, slot, slot, 0, 0);
  if (ctx->nc > 0) {
    // the interpolated fields, for the position gradient while one is accumulated
    if (ctx->shape_acc) ibmk::run_pair_fields(L, B);
    ibmk::run_markers_step(L, B, nullptr);
  }
  ibmk::run_setup(L, B, slot, ++ctx->tag);
  {
    // the recorded solution replaces the solve (the set-up's CG start is overwritten)
    ibmk::CopyParts cp;
    cp.add(B.x, B.tape + B.tape_stride * (size_t)tape_index + B.tape_xoff,
           (size_t)L.g.N * sizeof(double));
    ibmk::run_copy_parts(L, cp);
  }
  // reverse: correction, pressure solve, set-up, forcing and spreading, predictor
  ibmk::run_adj_correction(L, B, slot, state_bar_in, state_bar_out);
  const int tag = ++ctx->tag;
  ibmk::run_adj_cg_init(L, B, tag);
  HIPCHECK(ctx, hipGetLastError());
  Bufs Ba = B;
  Ba.x = B.lam;
  int iters = 0;
  {
    ibm_status r = run_cg_to_end(ctx, Ba, tag, &iters);
    if (r) return r;
  }
  ibmk::run_adj_setup(L, B, slot, state_bar_in, state_bar_out);
  if (ctx->nc > 0) ibmk::run_adj_markers(L, B, ob, Tw_bar, ctx->shape_acc);
  ibmk::run_adj_predictor(L, B, slot, state_bar_out);
  HIPCHECK(ctx, hipGetLastError());
  return IBM_OK;
}

ibm_status ibm_profile(ibm_ctx *ctx, int32_t enable) {
  if (!ctx) return IBM_E_ARG;
  HIPCHECK(ctx, hipStreamSynchronize(ctx->L.st));
  ctx->prof.settle();
  ctx->prof.on = enable != 0;
  if (enable) {
    for (int c = 0; c < IBM_PROF_CLASSES; ++c) {
      ctx->prof.ms[c] = 0.0;
      ctx->prof.n[c] = 0;
    }
  }
  return IBM_OK;
}

ibm_status ibm_profile_read(const ibm_ctx *ctx, double *ms, int64_t *launches) {
  if (!ctx) return IBM_E_ARG;
  for (int c = 0; c < IBM_PROF_CLASSES; ++c) {
    if (ms) ms[c] = ctx->prof.ms[c];
    if (launches) launches[c] = ctx->prof.n[c];
  }
  return IBM_OK;
}

}  // extern "C"
