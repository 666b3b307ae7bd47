// C ABI of the limited CG-WENO stage (declarations and documentation in
// include/cem.h).  Host orchestration of the gfx950 kernels of kernels.hpp.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/cem.h"
#include "kernels.hpp"
#include "kernels_sys.hpp"
#include "kernels_batch.hpp"
#include "tables.hpp"

using namespace cem;

namespace {

// up to this many per-block dt_e minima every node-update block reduces them
// itself; above it one block does it once (k_stage_dt)
constexpr int kDtFusedMax = 1024;

// 2D Euler element pass 1 on the system kernels instead of the one-thread
// tile: measured slower (512^2 Q3 float64 3.23 against 3.16 ms per step;
// 512 Q2 problems 90.7 against 81.9 ms float64, 72.2 against 69.0 mixed)
constexpr bool kSys2D = false;

// 2D element pass 1 with two threads (roles) per element: scalar problems.
// Measured per stage: KPP 256^2 Q2 22.7 -> 17.3 us; for 512^2 Q3 Euler the
// one-thread tile stays faster (0.46 against 0.47 ms, mixed 0.36 against
// 0.45 ms).  The mixed form takes three roles (sensor, residual, facets:
// KPP 13.3 -> 11.9 us); in float64 three roles measured slower (13.0 ->
// 16.2 us).
template <int PH> constexpr bool tile2_roles() { return Phys<2, PH>::M == 1; }

// Euler element pass 1: the system kernels (one thread per element and
// component, two launches) rather than the one-thread LDS tile.  3D Euler
// always takes them; 2D Euler can take either (cem_ctx::elem1_sys, a knob of
// the batch autotuner; kSys2D is the default), so both are compiled for it.
template <int D, int PH> constexpr bool sys_capable() { return PH == EUL && D >= 2; }

thread_local std::string g_err;

cem_status fail(cem_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t _e = (call);                                                            \
    if (_e != hipSuccess) return fail(CEM_EHIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
// log2 of a power of two
constexpr int ilog2_exact(int v) { return v <= 1 ? 0 : 1 + ilog2_exact(v / 2); }
}  // namespace

struct cem_ctx {
  int d = 0, p = 0, kind = 0, m = 0, nl = 0;
  int n[3] = {1, 1, 1}, L[3] = {1, 1, 1};
  int64_t N = 0, E = 0;
  double h = 0.0;
  cem_params prm{};
  PhysParams ph{};
  hipStream_t stream = nullptr;
  HostTables tabs;
  std::vector<double> tabblob;     // all tables, packed
  size_t off_kg[3] = {0, 0, 0}, off_km[3] = {0, 0, 0}, off_kgf[3] = {0, 0, 0},
         off_kmf[3] = {0, 0, 0}, off_sf = 0;
  // float copies (mixed precision), byte offsets into the table region
  size_t boff_kg32[3] = {0, 0, 0}, boff_km32[3] = {0, 0, 0}, boff_kgf32[3] = {0, 0, 0},
         boff_kmf32[3] = {0, 0, 0}, boff_sf32 = 0;
  bool mixed = false;
  // non-periodic 1D line: boundary conditions and line-operator tables
  bool bounded = false;
  int bc[2] = {0, 0};
  double bc_u[2][5] = {{0.0}};
  size_t off_bm[3] = {0, 0, 0}, off_bg[3] = {0, 0, 0};   // wi, lo, hi (doubles)
  // bound memory
  double* u = nullptr;
  double* u0 = nullptr;
  char* ws = nullptr;
  size_t ws_need = 0;
  // workspace carve-up (byte offsets)
  size_t o_g, o_r, o_udot, o_tmp, o_tmp2, o_relem, o_ue, o_ubarL, o_ubar, o_fahi, o_dte, o_gam,
      o_nu, o_beta, o_bnd, o_fdiv, o_dtbuf, o_counts, o_inv, o_tab, o_dtpart, o_fnode, o_fbnd;
  size_t o_g32 = 0, o_r32 = 0, o_udot32 = 0, o_tmp32 = 0, o_tmp2_32 = 0;
  bool fnode_valid = false;   // nodal fluxes match the bound state
  int lds_max = 65536;        // LDS bytes one block may use on the bound device
  int upd_blocks = 0, inv_blocks = 0;
  size_t ndtp = 0;                 // capacity of the per-block dt_e minima
  int elem1_sys = kSys2D ? 1 : 0;  // 2D Euler: element pass 1 on the system kernels
  int line_mfma = 2;               // float64 line passes: 0 vector, 1 matrix cores, 2 by size
  bool fuse_update = false;        // 2D Euler: pass 2 updates the nodes inside its blocks
  int cnt_slots = 0;               // per-block counter pairs: update blocks, then pass-2 blocks
  bool bound = false, bounds_set = false;
  // whole-step HIP graph (captured on a private stream, launched on stream)
  bool use_graphs = true;
  bool copy_base_next = false;   // the next stage 0 also writes u_base = u
  bool in_step = false;          // stages of cem_step: the fused assembly skips storing r
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  double graph_dt = -1.0, graph_cfl = -1.0;
  // optional per-kernel event timing
  unsigned timing_mask = 0;
  struct Rec { int id; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;

  template <class T> T* W(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

// batched form: launches of one stage over all problems (see kernels_batch.hpp)
enum BKind { B_LINE, B_LINE_X, B_LINE_Y, B_LINE_MX, B_LINE_MY, B_STAGE_DT, B_ELEM1_TILE, B_ELEM1_TILE2, B_ELEM1_SYS, B_RESID_SYS, B_GATHER_LX,
             B_GATHER_R, B_ELEM2, B_ELEM2_SYS, B_UPDATE, B_LINE_BND, B_LINE_BND_RUNS, B_ELEM1 };

struct BLaunch {
  int kind = 0;
  bool grad = false;       // line kernels: float64 input (u) rather than RT
  int re = 1;              // line kernels: runs of re P outputs
  int nprob = 0, blocks = 0;
  size_t lds = 0;
  size_t o_first = 0, o_args = 0, o_args2 = 0;   // byte offsets in the plan region
};

struct cem_batch {
  int count = 0, d = 0, p = 0, kind = 0, m = 0;
  bool mixed = false;
  hipStream_t stream = nullptr;
  std::vector<cem_ctx*> pr;
  std::vector<long long> uoff;     // [count + 1] start of each problem in the state arrays
  std::vector<size_t> wsoff;       // start of each problem's workspace (bytes)
  size_t ws_need = 0, o_plan = 0, plan_cap = 0;
  char* ws = nullptr;
  double* u = nullptr;
  double* u0 = nullptr;
  bool bound = false;
  std::vector<BLaunch> launches[3];
  double plan_dt = -1.0, plan_cfl = -1.0;
  bool use_graphs = true;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  // tuning knobs of the plan (cem_batch_autotune)
  int xlines_cap = 2048;           // axis-0 line kernels: cap on values staged per block
  int order = 0;                   // 0: problems in input order, 1: largest first
  int ytile_cap = 40960;           // strided line kernels: LDS bytes of a tile (sets the runs per thread)
  int elem1_sys = kSys2D ? 1 : 0;  // 2D Euler: element pass 1 on the system kernels (else the LDS tile)
  int line_mfma = 1;               // float64 line passes on the matrix cores (else the vector kernels)
  int fuse_update = 0;             // 2D Euler: pass 2 updates the nodes inside its blocks
};

namespace {

void pack_tables(cem_ctx* c) {
  const HostTables& T = c->tabs;
  std::vector<double>& B = c->tabblob;
  B.clear();
  auto put = [&](const std::vector<double>& v) {
    size_t off = B.size();
    B.insert(B.end(), v.begin(), v.end());
    while (B.size() % 32) B.push_back(0.0);
    return off;
  };
  const int P1 = T.p + 1, D = T.d;
  {
    // compact tables of the sum-factorised element kernels (SFLayout order)
    std::vector<double> sf;
    const int PP = P1 * P1;
    auto app = [&](const std::vector<double>& v, int n) {
      for (int i = 0; i < n; ++i) sf.push_back(i < (int)v.size() ? v[i] : 0.0);
    };
    app(T.vq, PP);
    app(T.dq, PP);
    app(T.wq, PP);
    app(T.g1, PP);
    app(T.k1, PP);
    app(T.ct1, PP);
    app(T.ext, 2 * PP);
    app(T.qp, (int)T.qp.size());
    c->off_sf = put(sf);
  }
  if (c->bounded) {
    c->off_bm[0] = put(T.bmass.wi);
    c->off_bm[1] = put(T.bmass.lo);
    c->off_bm[2] = put(T.bmass.hi);
    c->off_bg[0] = put(T.bgrad.wi);
    c->off_bg[1] = put(T.bgrad.lo);
    c->off_bg[2] = put(T.bgrad.hi);
  }
  for (int k = 0; k < D; ++k) {
    c->off_kg[k] = put(T.kgrad[k].w);
    c->off_km[k] = put(T.kmass[k].w);
    c->off_kgf[k] = put(T.kgrad[k].wf);
    c->off_kmf[k] = put(T.kmass[k].wf);
  }
  // float copies of every table (the mixed-precision contractions), stored
  // two per double word; offsets in bytes from the start of the blob
  auto put32 = [&](size_t off, size_t n) {
    std::vector<float> f(n);
    for (size_t i = 0; i < n; ++i) f[i] = (float)B[off + i];
    std::vector<double> packed((n + 1) / 2, 0.0);
    std::memcpy(packed.data(), f.data(), n * sizeof(float));
    return put(packed) * sizeof(double);
  };
  {
    const int PP = P1 * P1;
    const size_t nsf = 8 * (size_t)PP + T.qp.size();
    c->boff_sf32 = put32(c->off_sf, nsf);
  }
  for (int k = 0; k < D; ++k) {
    c->boff_kg32[k] = put32(c->off_kg[k], T.kgrad[k].w.size());
    c->boff_km32[k] = put32(c->off_km[k], T.kmass[k].w.size());
    // the fast float kernels use their own, narrower rows
    c->boff_kgf32[k] = put32(put(T.kgrad[k].wf32), T.kgrad[k].wf32.size());
    c->boff_kmf32[k] = put32(put(T.kmass[k].wf32), T.kmass[k].wf32.size());
  }
}

hipEvent_t get_event(cem_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Timing of single kernels: when the kernel id is selected, the launch goes
// through hipExtLaunchKernelGGL with a start and a stop event, which take the
// dispatch's own begin and end timestamps (no event-packet or dispatch latency
// in the interval); otherwise it is an ordinary launch.
bool timing_events(cem_ctx* c, int id, hipEvent_t* a, hipEvent_t* b) {
  *a = *b = nullptr;
  if (!(c->timing_mask & (1u << id))) return false;
  *a = get_event(c);
  *b = get_event(c);
  if (!*a || !*b) {
    if (*a) c->pool.push_back(*a);
    if (*b) c->pool.push_back(*b);
    return false;
  }
  c->recs.push_back({id, *a, *b});
  return true;
}

#define CEM_LAUNCH(c, id, K, grid, block, lds, st, ...)                                        \
  do {                                                                                         \
    hipEvent_t ev0_, ev1_;                                                                     \
    if (timing_events(c, id, &ev0_, &ev1_))                                                    \
      hipExtLaunchKernelGGL(K, dim3(grid), dim3(block), (std::uint32_t)(lds), st, ev0_, ev1_, \
                            0u, __VA_ARGS__);                                                  \
    else                                                                                       \
      hipLaunchKernelGGL(K, dim3(grid), dim3(block), lds, st, __VA_ARGS__);                    \
  } while (0)

// fixed widths of the register-blocked line kernel per degree (device
// templates LineTaps<P>)
const int kWfast[5] = {0, LineTaps<1>::W, LineTaps<2>::W, LineTaps<3>::W, 0};
const int kRfast[5] = {0, 1, 2, 3, 0};   // shortest run: RE = 1
const int kSfast[5] = {0, LineTaps<1>::S, LineTaps<2>::S, LineTaps<3>::S, 0};
const int kWfast32[5] = {0, LineTaps32<1>::W, LineTaps32<2>::W, LineTaps32<3>::W, 0};
const int kSfast32[5] = {0, LineTaps32<1>::S, LineTaps32<2>::S, LineTaps32<3>::S, 0};

// line passes on the matrix cores: always (mode 1), never (0), or from
// 2^20 values per pass (2; smaller meshes keep the one-launch vector
// gradient passes, whose launch count matters more there)
inline bool use_mfma(const cem_ctx* c) {
  return c->line_mfma == 1 || (c->line_mfma == 2 && (int64_t)c->m * c->N >= (int64_t(1) << 20));
}

template <int P, class TI, class TO>
void launch_line_fast(cem_ctx* c, int id, LineFastArgs la, hipStream_t st) {
  constexpr int W = LineTapsV<P, TO>::W;
  if (use_mfma(c)) {
    la.ky = line_mfma_chunks(la.ntrans, la.L, 2048);
    const int seg = kMfmaTY * la.ky;
    dim3 grid((unsigned)((la.ntrans + kMfmaLines - 1) / kMfmaLines), (unsigned)((la.L + seg - 1) / seg));
    const size_t lds = line_mfma_lds<P, TO>();
    if (la.axis == 0)
      CEM_LAUNCH(c, id, (k_line_mfma<P, true, TI, TO>), grid, 256, lds, st, la);
    else
      CEM_LAUNCH(c, id, (k_line_mfma<P, false, TI, TO>), grid, 256, lds, st, la);
    return;
  }
  if (la.axis == 0 && la.L <= 4096) {
    // whole lines in LDS; one line per block unless lines are short
    const int re = la.L >= 2 * P + 2 * W ? 2 : 1;
    la.nlb = line_rows_per_block<P, TO>(la.L, la.ntrans, 4096, re * P);
    const size_t lds = (size_t)la.nlb * line_row_pitch<P, TO>(la.L) * sizeof(TO);
    const unsigned grid = (unsigned)((la.ntrans + la.nlb - 1) / la.nlb);
    if (re == 2)
      CEM_LAUNCH(c, id, (k_line_x<P, 2, TI, TO>), grid, 256, lds, st, la);
    else
      CEM_LAUNCH(c, id, (k_line_x<P, 1, TI, TO>), grid, 256, lds, st, la);
    return;
  }
  if (la.axis > 0) {
    const int R = P * la.re, TY = 8 * R * la.ky;
    const size_t lds = (size_t)(TY + LineTapsV<P, TO>::S) * kTileX * sizeof(TO);
    dim3 grid(nblocks(la.ntrans, kTileX), (unsigned)((la.L + TY - 1) / TY));
    if (la.re == 2)
      CEM_LAUNCH(c, id, (k_line_y<P, 2, TI, TO>), grid, 256, lds, st, la);
    else
      CEM_LAUNCH(c, id, (k_line_y<P, 1, TI, TO>), grid, 256, lds, st, la);
    return;
  }
  // longest run that still gives >= 2^17 threads (2 waves per SIMD)
  int re = kLineMaxRE;
  while (re > 1 && (la.L < P * re + 2 * LineTapsV<P, TO>::W ||
                    la.ntrans * ((la.L + P * re - 1) / (P * re)) < (int64_t(1) << 17)))
    re /= 2;
  const int R = P * re;
  dim3 grid(nblocks(la.ntrans, 256), (unsigned)((la.L + R - 1) / R));
  switch (re) {
    case 4: CEM_LAUNCH(c, id, (k_line_fast<P, 4, TI, TO>), grid, 256, 0, st, la); break;
    case 2: CEM_LAUNCH(c, id, (k_line_fast<P, 2, TI, TO>), grid, 256, 0, st, la); break;
    default: CEM_LAUNCH(c, id, (k_line_fast<P, 1, TI, TO>), grid, 256, 0, st, la); break;
  }
}

StageArgs make_args(const cem_ctx* c) {
  StageArgs a{};
  a.mesh.n[0] = c->n[0];
  a.mesh.n[1] = c->n[1];
  a.mesh.n[2] = c->n[2];
  a.mesh.L[0] = c->L[0];
  a.mesh.L[1] = c->L[1];
  a.mesh.L[2] = c->L[2];
  a.mesh.N = c->N;
  a.mesh.E = c->E;
  a.mesh.h = c->h;
  a.mesh.bnd1d = c->bounded ? 1 : 0;
  for (int s = 0; s < 2; ++s) {
    a.bc_kind[s] = c->bc[s];
    for (int q = 0; q < 5; ++q) a.bc_u[s][q] = c->bc_u[s][q];
  }
  a.fbnd = c->W<double>(c->o_fbnd);
  const double* tb = c->W<double>(c->o_tab);
  a.tab.sf = tb + c->off_sf;
  a.tab.sf32 = reinterpret_cast<const float*>(reinterpret_cast<const char*>(tb) + c->boff_sf32);
  if (c->mixed) {
    a.g32 = c->W<float>(c->o_g32);
    a.r32 = c->W<float>(c->o_r32);
    a.udot32 = c->W<float>(c->o_udot32);
  }
  a.ph = c->ph;
  a.q = c->prm.q;
  a.rexp = c->prm.r;
  a.eps = c->prm.eps;
  a.w_lin = c->prm.w_lin;
  a.eps_pos = c->prm.eps_pos;
  a.gamma_mode = c->prm.gamma_mode;
  a.alpha_mode = c->prm.alpha_mode;
  a.beta_mode = c->prm.beta_mode;
  a.flux_mode = c->prm.flux_mode;
  a.umin = c->prm.u_min;
  a.umax = c->prm.u_max;
  a.clamp_tol = c->prm.clamp_ulps * DBL_EPSILON * std::fmax(std::fabs(c->prm.u_min), std::fabs(c->prm.u_max));
  a.bounds_local = c->kind != CEM_EULER && c->prm.bounds == CEM_BOUNDS_LOCAL;
  a.bnd = c->W<double>(c->o_bnd);
  a.contrib_q1 = c->prm.contrib == CEM_CONTRIB_Q1;
  a.store_r = c->in_step ? 0 : 1;
  a.fdiv = c->W<double>(c->o_fdiv);
  a.u = c->u;
  a.u0 = c->u0;
  a.uout = c->u;
  a.g = c->W<double>(c->o_g);
  a.fnode = c->W<double>(c->o_fnode);
  a.r = c->W<double>(c->o_r);
  a.udot = c->W<double>(c->o_udot);
  a.relem = c->W<double>(c->o_relem);
  a.ue = c->W<double>(c->o_ue);
  a.ubarL = c->W<double>(c->o_ubarL);
  a.ubar = c->W<double>(c->o_ubar);
  a.fahi = c->W<double>(c->o_fahi);
  a.dte = c->W<double>(c->o_dte);
  a.gam = c->W<double>(c->o_gam);
  a.nu = c->W<double>(c->o_nu);
  a.beta = c->W<double>(c->o_beta);
  a.dtbuf = c->W<double>(c->o_dtbuf);
  a.counts = c->W<int>(c->o_counts);
  a.dtpart = c->W<double>(c->o_dtpart);
  return a;
}


// line operator arguments; weights of the output type (float copies in the
// mixed-precision form)
// wide: the strided kernel may take runs of 2P (single-problem launches)
template <class TO>
LineFastArgs line_args(const cem_ctx* c, const void* in, void* out, int axis, bool grad, bool wide = true) {
  LineFastArgs la{};
  la.in = in;
  la.out = out;
  const char* tb = c->ws + c->o_tab;
  if (sizeof(TO) == 4)
    la.w = tb + (grad ? c->boff_kgf32[axis] : c->boff_kmf32[axis]);
  else
    la.w = tb + 8 * (grad ? c->off_kgf[axis] : c->off_kmf[axis]);
  la.L = c->L[axis];
  la.axis = axis;
  la.L0 = c->L[0];
  la.L1 = c->L[1];
  la.N = c->N;
  la.NT = c->N / c->L[axis];
  la.ntrans = (int64_t)c->m * la.NT;
  la.re = 1;
  la.ky = 1;
  if (axis > 0) {
    const int W = sizeof(TO) == 4 ? kWfast32[c->p] : kWfast[c->p];
    const int S = sizeof(TO) == 4 ? kSfast32[c->p] : kSfast[c->p];
    if (wide) la.re = line_y_re(la.ntrans, la.L, c->p, W);
    la.ky = line_y_runs(la.ntrans, la.L, c->p * la.re, S, (int)sizeof(TO));
  }
  return la;
}

template <class TI, class TO>
cem_status launch_line(cem_ctx* c, const TI* in, TO* out, int axis, bool grad) {
  const int id = grad ? 0 : 4;
  const LineKernel& K = grad ? c->tabs.kgrad[axis] : c->tabs.kmass[axis];
  const char* tb = c->ws + c->o_tab;
  if (K.wfast > 0) {
    LineFastArgs la = line_args<TO>(c, in, out, axis, grad);
    switch (c->p) {
      case 1: launch_line_fast<1, TI, TO>(c, id, la, c->stream); break;
      case 2: launch_line_fast<2, TI, TO>(c, id, la, c->stream); break;
      case 3: launch_line_fast<3, TI, TO>(c, id, la, c->stream); break;
      default: return fail(CEM_EINVAL, "no fast line kernel for this degree");
    }
    HIPCHK(hipGetLastError());
    return CEM_OK;
  }
  LineArgs la{};
  la.in = in;
  la.out = out;
  if (sizeof(TO) == 4)
    la.w = tb + (grad ? c->boff_kg32[axis] : c->boff_km32[axis]);
  else
    la.w = tb + 8 * (grad ? c->off_kg[axis] : c->off_km[axis]);
  la.taps = K.taps;
  la.first = K.first;
  la.L = c->L[axis];
  la.P = c->p;
  la.stride = axis == 0 ? 1 : (axis == 1 ? (int64_t)c->L[0] : (int64_t)c->L[0] * c->L[1]);
  la.N = c->N;
  la.total = (int64_t)c->m * c->N;
  la.scale = 1.0;
  CEM_LAUNCH(c, id, (k_line<TI, TO>), nblocks(la.total, 256), 256, 0, c->stream, la);
  HIPCHK(hipGetLastError());
  return CEM_OK;
}

// arguments of a line operator of a non-periodic line (grad: Mb^{-1} Cb,
// else Mb^{-1}); false when its blocks would not cover the line
bool bnd_line_args(const cem_ctx* c, const double* in, double* out, bool grad, BndLineArgs& la) {
  const BoundedLine& K = grad ? c->tabs.bgrad : c->tabs.bmass;
  const size_t* off = grad ? c->off_bg : c->off_bm;
  const double* tb = c->W<double>(c->o_tab);
  la = BndLineArgs{};
  la.in = in;
  la.out = out;
  la.wi = tb + off[0];
  la.lo = tb + off[1];
  la.hi = tb + off[2];
  la.N = c->N;
  la.total = (int64_t)c->m * c->N;
  la.P = c->p;
  la.W = K.W;
  la.blo = K.blo;
  la.bhi = K.bhi;
  la.cw = K.cw;
  // the kernel's reads stay in the line: end blocks of at least W rows, or
  // one exact block over the whole line
  return (K.blo >= K.W && K.bhi >= K.W && 2 * (int64_t)K.W < c->N && K.cw <= c->N) ||
         (K.blo == c->N && K.bhi == 0 && K.cw == c->N);
}

cem_status launch_line_bnd(cem_ctx* c, const double* in, double* out, bool grad) {
  const BoundedLine& K = grad ? c->tabs.bgrad : c->tabs.bmass;
  const double* tb = c->W<double>(c->o_tab);
  BndLineArgs la;
  if (!bnd_line_args(c, in, out, grad, la))
    return fail(CEM_EINVAL, "internal: line operator blocks do not cover the line");
  const int id = grad ? 0 : 4;
  // long lines: LDS tiles with register-blocked runs of 2P outputs, on the
  // padded interior rows of the periodic fast tables (the same infinite-line
  // rows, built for the periodic line of the same cells)
  const LineKernel& F = grad ? c->tabs.kgrad[0] : c->tabs.kmass[0];
  if (K.blo < c->N && F.wfast == K.W && kWfast[c->p] == K.W) {
    la.wf = tb + (grad ? c->off_kgf[0] : c->off_kmf[0]);
    const int R = 2 * c->p, LW = 256 * R + kSfast[c->p];
    const size_t lds = (size_t)(LW + (R % 2 == 0 ? (LW - 1) / R : 0)) * sizeof(double);
    dim3 grid(nblocks(c->N, 256 * R), (unsigned)c->m);
    switch (c->p) {
      case 1: CEM_LAUNCH(c, id, (k_line_bnd_runs<1, 2>), grid, 256, lds, c->stream, la); break;
      case 2: CEM_LAUNCH(c, id, (k_line_bnd_runs<2, 2>), grid, 256, lds, c->stream, la); break;
      case 3: CEM_LAUNCH(c, id, (k_line_bnd_runs<3, 2>), grid, 256, lds, c->stream, la); break;
      default: return fail(CEM_EINVAL, "no line kernel for this degree");
    }
  } else {
    CEM_LAUNCH(c, id, k_line_bnd, nblocks(la.total, 256), 256, 0, c->stream, la);
  }
  HIPCHK(hipGetLastError());
  return CEM_OK;
}

// element passes of systems (one thread per element and component)
template <int D, int P, int PH, class RT>
cem_status launch_sys(cem_ctx* c, StageArgs& a, bool first) {
  using TL = SysTile<D, P, PH>;
  constexpr int M = Phys<D, PH>::M, EB = TL::EB;
  const size_t lds = TL::LY::bytes;
  if (lds > (size_t)c->lds_max) return fail(CEM_EINVAL, "element tile does not fit the LDS of a block");
  const unsigned nb = (unsigned)TL::blocks(c->n);
  if (nb > c->ndtp) return fail(CEM_EINVAL, "internal: more element blocks than dt_e minima slots");
  if (first) {
    a.ndtpart = (int)nb;
    CEM_LAUNCH(c, 1, (k_elem1_sys<D, P, PH, RT>), nb, M * EB, lds, c->stream, a);
    HIPCHK(hipGetLastError());
    CEM_LAUNCH(c, 7, (k_resid_sys<D, P, PH, RT>), nb, M * EB, lds, c->stream, a);
  } else {
    CEM_LAUNCH(c, 5, (k_elem2_sys<D, P, PH, RT>), nb, M * EB, lds, c->stream, a);
  }
  HIPCHK(hipGetLastError());
  return CEM_OK;
}

// RT: value type of the contractions (double; float in the mixed form,
// where g, r, udot and the residual vectors are float arrays)
template <int D, int P, int PH, class RT>
cem_status stage_impl(cem_ctx* c, int stage, double dt, double cfl) {
  constexpr int M = Phys<D, PH>::M;
  constexpr bool MIX = sizeof(RT) == 4;
  StageArgs a = make_args(c);
  if constexpr (Phys<D, PH>::kNodal) {
    if (!c->fnode_valid) {
      hipLaunchKernelGGL((k_nodal_flux<D, PH>), dim3(nblocks(c->N, 256)), dim3(256), 0, c->stream, a);
      HIPCHK(hipGetLastError());
    }
  }
  c->fnode_valid = true;    // the update at the end of the stage refreshes them
  const double rka[3] = {0.0, 0.75, 1.0 / 3.0}, rkb[3] = {1.0, 0.25, 2.0 / 3.0};
  a.rk_a = rka[stage];
  a.rk_b = rkb[stage];
  a.stage = stage;
  a.copy_base = (stage == 0 && c->copy_base_next) ? 1 : 0;
  a.ndtpart = (int)nblocks(c->E, 128);
  a.dt_fixed = dt;
  a.cfl = cfl;
  RT* g = MIX ? (RT*)a.g32 : (RT*)a.g;
  RT* r = MIX ? (RT*)a.r32 : (RT*)a.r;
  RT* udot = MIX ? (RT*)a.udot32 : (RT*)a.udot;
  RT* tmp = c->W<RT>(MIX ? c->o_tmp32 : c->o_tmp);
  RT* tmp2 = c->W<RT>(MIX ? c->o_tmp2_32 : c->o_tmp2);
  // projected gradient g_k = M_1D^{-1} C_1D u along axis k (Sec. 2.2): the
  // passes are independent, so on fast-kernel lines they share one launch
  bool multi = D >= 2 && c->L[0] <= 4096 && !use_mfma(c);
  for (int k = 0; k < D; ++k) multi = multi && c->tabs.kgrad[k].wfast > 0;
  if (multi) {
    constexpr int W = LineTapsV<P, RT>::W, S = LineTapsV<P, RT>::S;
    MultiLineArgs ml{};
    ml.naxes = D;
    // one run length for all strided axes (a template argument of the launch)
    bool wide = true;
    for (int k = 1; k < D; ++k) wide = wide && line_args<RT>(c, c->u, g, k, true).re == 2;
    const int TY = 8 * P * (wide ? 2 : 1);
    // axis 0: runs of 2P where the lines allow (4P measured slower)
    const int rex = c->L[0] >= 2 * P + 2 * W ? 2 : 1;
    size_t lds = (size_t)(TY + S) * kTileX * sizeof(RT);
    for (int k = 0; k < D; ++k) {
      LineFastArgs la = line_args<RT>(c, c->u, g + (int64_t)k * M * c->N, k, true, wide);
      if (k == 0) {
        la.nlb = line_rows_per_block<P, RT>(la.L, la.ntrans, 4096, rex * P);
        ml.nb[0] = (int)((la.ntrans + la.nlb - 1) / la.nlb);
        lds = std::max(lds, (size_t)la.nlb * line_row_pitch<P, RT>(la.L) * sizeof(RT));
      } else {
        const int TYk = TY * la.ky;
        la.gx = (int)nblocks(la.ntrans, kTileX);
        ml.nb[k] = la.gx * ((la.L + TYk - 1) / TYk);
        lds = std::max(lds, (size_t)(TYk + S) * kTileX * sizeof(RT));
      }
      ml.a[k] = la;
    }
    int nb = 0;
    for (int k = 0; k < D; ++k) nb += ml.nb[k];
    if (rex == 2 && wide)
      CEM_LAUNCH(c, 0, (k_line_multi<P, 2, 2, double, RT>), nb, 256, lds, c->stream, ml);
    else if (rex == 2)
      CEM_LAUNCH(c, 0, (k_line_multi<P, 2, 1, double, RT>), nb, 256, lds, c->stream, ml);
    else if (wide)
      CEM_LAUNCH(c, 0, (k_line_multi<P, 1, 2, double, RT>), nb, 256, lds, c->stream, ml);
    else
      CEM_LAUNCH(c, 0, (k_line_multi<P, 1, 1, double, RT>), nb, 256, lds, c->stream, ml);
    HIPCHK(hipGetLastError());
  } else {
    for (int k = 0; k < D; ++k) {
      cem_status s = launch_line(c, (const double*)c->u, g + (int64_t)k * M * c->N, k, true);
      if (s != CEM_OK) return s;
    }
  }
  // element pass: sensor, residual (with the stabilisation), facet data.
  // (Running the g-independent part concurrently with the gradient passes on
  // a second stream was measured slower on the 256^2 KPP mesh.)
  {
    // 3D systems: one thread per (element, component), in two launches
    // (sensor and facets; residual).  2D: the LDS element tile with one
    // thread per element measured faster for both physics (512^2 Q3 Euler:
    // 0.46 ms per stage against 0.52 for the two system launches)
    bool sys_done = false;
    if constexpr (sys_capable<D, PH>()) {
      if (D == 3 || c->elem1_sys) {
        cem_status st = launch_sys<D, P, PH, RT>(c, a, true);
        if (st != CEM_OK) return st;
        sys_done = true;
      }
    }
    if (sys_done) {
    } else if constexpr (sys_capable<D, PH>() && D == 3) {
    } else if constexpr (D == 2) {
      using TT = Tile2<P, M>;
      const int nb = ((c->n[0] + TT::TEX - 1) / TT::TEX) * ((c->n[1] + TT::TEY - 1) / TT::TEY);
      a.ndtpart = nb;
      if ((size_t)nb > c->ndtp) return fail(CEM_EINVAL, "internal: more element blocks than dt_e minima slots");
      if constexpr (tile2_roles<PH>() && MIX)
        CEM_LAUNCH(c, 1, (k_elem1_tile3<P, PH, true, RT>), nb, 384, (TT::words + 256) * sizeof(double),
                   c->stream, a);
      else if constexpr (tile2_roles<PH>())
        CEM_LAUNCH(c, 1, (k_elem1_tile2<P, PH, true, RT>), nb, 256, (TT::words + 256) * sizeof(double),
                   c->stream, a);
      else
        CEM_LAUNCH(c, 1, (k_elem1_tile<P, PH, true, RT>), nb, 128, TT::words * sizeof(double), c->stream, a);
    } else {
      CEM_LAUNCH(c, 1, (k_elem1<D, P, PH, true, RT>), nblocks(c->E, 128), 128, 0, c->stream, a);
    }
  }
  HIPCHK(hipGetLastError());
  // udot = M_C^{-1} r, one line pass per axis (Sec. 4.3, step 2); the
  // assembly of r is fused into the first pass when it runs on whole x-lines
  const RT* src = r;
  int k0 = 0;
  if (c->tabs.kmass[0].wfast > 0 && c->L[0] <= 4096) {
    LineFastArgs la = line_args<RT>(c, r, D == 1 ? udot : tmp, 0, false);
    constexpr int W = LineTapsV<P, RT>::W;
    const int re = line_x_re(la.ntrans, la.L, P, W, 1, 2);
    la.nlb = line_rows_per_block<P, RT>(la.L, la.ntrans, 4096, re * P);
    const size_t lds = (size_t)la.nlb * line_row_pitch<P, RT>(la.L) * sizeof(RT) +
                       (size_t)la.nlb * kGatherLineInts * sizeof(int);
    const unsigned grid = (unsigned)((la.ntrans + la.nlb - 1) / la.nlb);
    if (re == 2)
      CEM_LAUNCH(c, 3, (k_gather_line_x<D, P, M, 2, RT>), grid, 256, lds, c->stream, a, la);
    else
      CEM_LAUNCH(c, 3, (k_gather_line_x<D, P, M, 1, RT>), grid, 256, lds, c->stream, a, la);
    HIPCHK(hipGetLastError());
    src = D == 1 ? udot : tmp;
    k0 = 1;
  } else {
    CEM_LAUNCH(c, 3, (k_gather_r<D, P, M, RT>), nblocks(c->N, 256), 256, 0, c->stream, a);
    HIPCHK(hipGetLastError());
  }
  for (int k = k0; k < D; ++k) {
    RT* dst = (k == D - 1) ? udot : (k % 2 == 0 ? tmp : tmp2);
    cem_status s = launch_line(c, src, dst, k, false);
    if (s != CEM_OK) return s;
    src = dst;
  }
  if constexpr (P == 1 && PH != EUL && !MIX) {
    // Q1 contributions: udot becomes the low-order time derivative
    if (a.contrib_q1) {
      hipLaunchKernelGGL((k_udot_lo<D, P>), dim3(nblocks(c->N, 256)), dim3(256), 0, c->stream, a);
      HIPCHK(hipGetLastError());
    }
  }
  bool fused = false;
  if constexpr (PH == EUL && D == 2) fused = c->fuse_update;
  if (fused) {
    // pass 2 updates the nodes inside its blocks: the stage dt first
    a.fuse_upd = ilog2_exact(SysTile<D, P, PH>::EB);
    a.cnt_off = c->upd_blocks;
    a.dt_ready = 1;
    CEM_LAUNCH(c, 2, k_stage_dt, 1, 1024, 0, c->stream, a);
    HIPCHK(hipGetLastError());
  }
  if constexpr (PH == EUL && D >= 2) {
    cem_status st = launch_sys<D, P, PH, RT>(c, a, false);
    if (st != CEM_OK) return st;
  } else {
    CEM_LAUNCH(c, 5, (k_elem2<D, P, PH, RT>), nblocks(c->E, 128), 128, 0, c->stream, a);
  }
  HIPCHK(hipGetLastError());
  if (!fused && a.ndtpart > kDtFusedMax) {
    // many per-block minima: one block reduces them once for the update
    a.dt_ready = 1;
    CEM_LAUNCH(c, 2, k_stage_dt, 1, 1024, 0, c->stream, a);
    HIPCHK(hipGetLastError());
  }
  CEM_LAUNCH(c, 6, (k_update<D, P, PH>), c->upd_blocks, 256, 0, c->stream, a);
  HIPCHK(hipGetLastError());
  return CEM_OK;
}

// One stage on a non-periodic 1D line (float64): the same five steps with
// the line operators of the bounded line, the boundary facets in the
// element passes and the end nodes gathered from their one element.
template <int P, int PH>
cem_status stage_line_impl(cem_ctx* c, int stage, double dt, double cfl) {
  constexpr int M = Phys<1, PH>::M;
  static_assert(!Phys<1, PH>::kNodal, "no nodal-flux physics on lines");
  StageArgs a = make_args(c);
  const double rka[3] = {0.0, 0.75, 1.0 / 3.0}, rkb[3] = {1.0, 0.25, 2.0 / 3.0};
  a.rk_a = rka[stage];
  a.rk_b = rkb[stage];
  a.stage = stage;
  a.copy_base = (stage == 0 && c->copy_base_next) ? 1 : 0;
  a.ndtpart = (int)nblocks(c->E, 128);
  a.dt_fixed = dt;
  a.cfl = cfl;
  if ((size_t)a.ndtpart > c->ndtp) return fail(CEM_EINVAL, "internal: more element blocks than dt_e minima slots");
  // projected gradient g = Mb^{-1} Cb u (Sec. 2.2)
  cem_status st = launch_line_bnd(c, c->u, a.g, true);
  if (st != CEM_OK) return st;
  // element pass: sensor, residual with the boundary flux at the end
  // nodes, facets (boundary facets at the ends)
  CEM_LAUNCH(c, 1, (k_elem1<1, P, PH, true, double>), nblocks(c->E, 128), 128, 0, c->stream, a);
  HIPCHK(hipGetLastError());
  // r, then udot = Mb^{-1} r (Sec. 4.3, step 2)
  CEM_LAUNCH(c, 3, (k_gather_r<1, P, M, double>), nblocks(c->N, 256), 256, 0, c->stream, a);
  HIPCHK(hipGetLastError());
  st = launch_line_bnd(c, a.r, a.udot, false);
  if (st != CEM_OK) return st;
  CEM_LAUNCH(c, 5, (k_elem2<1, P, PH, double>), nblocks(c->E, 128), 128, 0, c->stream, a);
  HIPCHK(hipGetLastError());
  if (a.ndtpart > kDtFusedMax) {
    a.dt_ready = 1;
    CEM_LAUNCH(c, 2, k_stage_dt, 1, 1024, 0, c->stream, a);
    HIPCHK(hipGetLastError());
  }
  CEM_LAUNCH(c, 6, (k_update<1, P, PH>), c->upd_blocks, 256, 0, c->stream, a);
  HIPCHK(hipGetLastError());
  return CEM_OK;
}

// ---------------------------------------------------------------------------
// batched form: plan (per-stage launch list with per-problem arguments in
// device memory) and dispatch
// ---------------------------------------------------------------------------
template <int D, int P, int PH, class RT>
StageArgs batch_stage_args(cem_ctx* c, int stage, double dt, double cfl) {
  StageArgs a = make_args(c);
  a.store_r = 0;
  const double rka[3] = {0.0, 0.75, 1.0 / 3.0}, rkb[3] = {1.0, 0.25, 2.0 / 3.0};
  a.rk_a = rka[stage];
  a.rk_b = rkb[stage];
  a.stage = stage;
  a.copy_base = stage == 0 ? 1 : 0;
  a.dt_fixed = dt;
  a.cfl = cfl;
  constexpr int M = Phys<D, PH>::M;
  bool sys = false;
  if constexpr (sys_capable<D, PH>()) sys = D == 3 || c->elem1_sys;
  if (sys) {
    if constexpr (sys_capable<D, PH>()) a.ndtpart = (int)SysTile<D, P, PH>::blocks(c->n);
  } else if constexpr (D == 2) {
    using TT = Tile2<P, M>;
    a.ndtpart = ((c->n[0] + TT::TEX - 1) / TT::TEX) * ((c->n[1] + TT::TEY - 1) / TT::TEY);
  } else {
    a.ndtpart = (int)nblocks(c->E, 128);
  }
  if constexpr (PH == EUL && D == 2) {
    if (c->fuse_update) {
      // pass 2 updates the nodes inside its blocks (the stage dt reduced
      // ahead of it by kb_stage_dt)
      a.fuse_upd = ilog2_exact(SysTile<D, P, PH>::EB);
      a.cnt_off = c->upd_blocks;
      a.dt_ready = 1;
    }
  }
  return a;
}

template <int D, int P, int PH, class RT>
cem_status batch_plan(cem_batch* b, double dt, double cfl) {
  constexpr int M = Phys<D, PH>::M;
  // problems in launch order (largest first puts the long-running blocks at
  // the front of every grid)
  std::vector<cem_ctx*> all = b->pr;
  for (cem_ctx* c : all) {
    c->elem1_sys = b->elem1_sys;
    c->fuse_update = b->fuse_update != 0;
  }
  if (b->order == 1)
    std::stable_sort(all.begin(), all.end(), [](const cem_ctx* x, const cem_ctx* y) { return x->N > y->N; });
  constexpr bool MIX = sizeof(RT) == 4;
  constexpr int W = LineTapsV<P, RT>::W, S = LineTapsV<P, RT>::S;
  std::vector<char> blob;
  auto put = [&](const void* p, size_t n) {
    const size_t off = blob.size();
    blob.insert(blob.end(), static_cast<const char*>(p), static_cast<const char*>(p) + n);
    while (blob.size() % 256) blob.push_back(0);
    return off;
  };
  struct Group {
    BLaunch l;
    std::vector<int> first{0};
    std::vector<StageArgs> sa;
    std::vector<LineFastArgs> lf;
    std::vector<LineArgs> la;
    std::vector<BndLineArgs> bl;
  };
  auto close = [&](Group& g, std::vector<BLaunch>& out) {
    if (g.first.size() <= 1) return;
    g.l.nprob = (int)g.first.size() - 1;
    g.l.blocks = g.first.back();
    g.l.o_first = put(g.first.data(), g.first.size() * sizeof(int));
    if (!g.sa.empty()) g.l.o_args = put(g.sa.data(), g.sa.size() * sizeof(StageArgs));
    if (!g.lf.empty()) (g.sa.empty() ? g.l.o_args : g.l.o_args2) = put(g.lf.data(), g.lf.size() * sizeof(LineFastArgs));
    if (!g.la.empty()) g.l.o_args = put(g.la.data(), g.la.size() * sizeof(LineArgs));
    if (!g.bl.empty()) g.l.o_args = put(g.bl.data(), g.bl.size() * sizeof(BndLineArgs));
    out.push_back(g.l);
  };
  // one line pass of every problem (axis k), grouped by kernel variant
  auto lines = [&](std::vector<BLaunch>& out, const std::vector<cem_ctx*>& probs, bool grad, int k, auto src_of,
                   auto dst_of) -> cem_status {
    // runs of 2P wherever the line allows (the whole batch fills the chip,
    // so the strided tiles are as long as 40 KB of LDS allows)
    Group gx[2], gy[2], gg, gm, gb, gbr;
    for (int v = 0; v < 2; ++v) {
      gx[v].l.kind = B_LINE_X;
      gy[v].l.kind = B_LINE_Y;
      gx[v].l.re = gy[v].l.re = v + 1;
      gx[v].l.grad = gy[v].l.grad = grad;
    }
    gg.l.kind = B_LINE;
    gg.l.grad = grad;
    gm.l.kind = k == 0 ? B_LINE_MX : B_LINE_MY;
    gm.l.grad = grad;
    gb.l.kind = B_LINE_BND;
    gb.l.grad = grad;
    gbr.l.kind = B_LINE_BND_RUNS;
    gbr.l.grad = grad;
    for (cem_ctx* c : probs) {
      const LineKernel& K = grad ? c->tabs.kgrad[k] : c->tabs.kmass[k];
      const void* in = src_of(c);
      void* out_p = dst_of(c);
      if (c->bounded) {
        // non-periodic lines (float64): LDS tiles of runs on long lines,
        // one output per thread on short ones (every row exact)
        BndLineArgs a;
        if (!bnd_line_args(c, static_cast<const double*>(in), static_cast<double*>(out_p), grad, a))
          return fail(CEM_EINVAL, "internal: line operator blocks do not cover the line");
        const BoundedLine& BK = grad ? c->tabs.bgrad : c->tabs.bmass;
        if (BK.blo < c->N && K.wfast == BK.W && kWfast[P] == BK.W) {
          a.wf = c->W<double>(c->o_tab) + (grad ? c->off_kgf[0] : c->off_kmf[0]);
          constexpr int R = 2 * P, LW = 256 * R + LineTaps<P>::S;
          gbr.bl.push_back(a);
          gbr.first.push_back(gbr.first.back() + (int)nblocks(c->N, 256 * R) * c->m);
          gbr.l.lds = (size_t)(LW + (R % 2 == 0 ? (LW - 1) / R : 0)) * sizeof(double);
        } else {
          gb.bl.push_back(a);
          gb.first.push_back(gb.first.back() + (int)nblocks(a.total, 256));
        }
      } else if (K.wfast > 0 && b->line_mfma) {
        // matrix-core blocks of 16 whole lines (the batch fills the chip)
        LineFastArgs a = line_args<RT>(c, in, out_p, k, grad, false);
        a.ky = line_mfma_chunks(a.ntrans, a.L, 0);
        a.gx = (int)((a.ntrans + kMfmaLines - 1) / kMfmaLines);
        const int seg = kMfmaTY * a.ky;
        gm.lf.push_back(a);
        gm.first.push_back(gm.first.back() + a.gx * ((a.L + seg - 1) / seg));
        gm.l.lds = line_mfma_lds<P, RT>();
      } else if (K.wfast > 0) {
        LineFastArgs a = line_args<RT>(c, in, out_p, k, grad, false);
        const int re = a.L >= 2 * P + 2 * W ? 2 : 1;
        if (k == 0) {
          if (a.L > 4096) return fail(CEM_EINVAL, "batched form: x-lines longer than 4096 nodes");
          a.nlb = line_rows_per_block<P, RT>(a.L, a.ntrans, b->xlines_cap, re * P);
          Group& G = gx[re - 1];
          G.lf.push_back(a);
          G.first.push_back(G.first.back() + (int)((a.ntrans + a.nlb - 1) / a.nlb));
          G.l.lds = std::max(G.l.lds, (size_t)a.nlb * line_row_pitch<P, RT>(a.L) * sizeof(RT));
        } else {
          a.re = re;
          a.ky = 1;
          while (a.ky < 4 && (8 * P * re * 2 * a.ky + S) * kTileX * (int)sizeof(RT) <= b->ytile_cap) a.ky *= 2;
          const int TY = 8 * P * re * a.ky;
          a.gx = (int)nblocks(a.ntrans, kTileX);
          Group& G = gy[re - 1];
          G.lf.push_back(a);
          G.first.push_back(G.first.back() + a.gx * ((a.L + TY - 1) / TY));
          G.l.lds = std::max(G.l.lds, (size_t)(TY + S) * kTileX * sizeof(RT));
        }
      } else {
        LineArgs a{};
        const char* tb = c->ws + c->o_tab;
        a.in = in;
        a.out = out_p;
        a.w = MIX ? (const void*)(tb + (grad ? c->boff_kg32[k] : c->boff_km32[k]))
                  : (const void*)(tb + 8 * (grad ? c->off_kg[k] : c->off_km[k]));
        a.taps = K.taps;
        a.first = K.first;
        a.L = c->L[k];
        a.P = c->p;
        a.stride = k == 0 ? 1 : (k == 1 ? (int64_t)c->L[0] : (int64_t)c->L[0] * c->L[1]);
        a.N = c->N;
        a.total = (int64_t)c->m * c->N;
        a.scale = 1.0;
        gg.la.push_back(a);
        gg.first.push_back(gg.first.back() + (int)nblocks(a.total, 256));
      }
    }
    for (int v = 0; v < 2; ++v) {
      close(gx[v], out);
      close(gy[v], out);
    }
    close(gm, out);
    close(gg, out);
    close(gb, out);
    close(gbr, out);
    return CEM_OK;
  };
  auto gbuf = [&](cem_ctx* c) -> RT* { return c->W<RT>(MIX ? c->o_g32 : c->o_g); };
  auto rbuf = [&](cem_ctx* c) -> RT* { return c->W<RT>(MIX ? c->o_r32 : c->o_r); };
  auto ubuf = [&](cem_ctx* c) -> RT* { return c->W<RT>(MIX ? c->o_udot32 : c->o_udot); };
  auto tbuf = [&](cem_ctx* c, int i) -> RT* {
    return c->W<RT>(i == 0 ? (MIX ? c->o_tmp32 : c->o_tmp) : (MIX ? c->o_tmp2_32 : c->o_tmp2));
  };
  // mass pass k of problem c: (source, destination) as in the single-problem stage
  auto fused = [&](cem_ctx* c) { return !c->bounded && c->tabs.kmass[0].wfast > 0 && c->L[0] <= 4096; };
  auto mass_dst = [&](cem_ctx* c, int k) -> RT* { return k == D - 1 ? ubuf(c) : tbuf(c, k % 2); };
  auto mass_src = [&](cem_ctx* c, int k) -> const RT* { return k == 0 ? rbuf(c) : mass_dst(c, k - 1); };
  for (int st = 0; st < 3; ++st) {
    std::vector<BLaunch>& L = b->launches[st];
    L.clear();
    std::vector<StageArgs> sa(b->count);
    for (int q = 0; q < b->count; ++q) sa[q] = batch_stage_args<D, P, PH, RT>(all[q], st, dt, cfl);
    // projected gradient, one pass per axis
    for (int k = 0; k < D; ++k) {
      cem_status s = lines(L, all, true, k, [&](cem_ctx* c) -> const void* { return c->u; },
                           [&](cem_ctx* c) -> void* { return gbuf(c) + (int64_t)k * M * c->N; });
      if (s != CEM_OK) return s;
    }
    // element pass 1
    {
      Group g;
      bool sys = false;
      if constexpr (sys_capable<D, PH>()) {
        sys = D == 3 || b->elem1_sys;
        if (sys) {
          g.l.kind = B_ELEM1_SYS;
          g.l.lds = SysTile<D, P, PH>::LY::bytes;
        }
      }
      if (sys) {
      } else if constexpr (D == 2) {
        using TT = Tile2<P, M>;
        g.l.kind = tile2_roles<PH>() ? B_ELEM1_TILE2 : B_ELEM1_TILE;
        g.l.lds = (TT::words + (tile2_roles<PH>() ? 256 : 0)) * sizeof(double);
      } else if constexpr (D == 1) {
        g.l.kind = B_ELEM1;
      } else {
        return fail(CEM_EINVAL, "batched form: 1D lines, 2D problems or 3D Euler only");
      }
      for (int q = 0; q < b->count; ++q) {
        g.sa.push_back(sa[q]);
        g.first.push_back(g.first.back() + sa[q].ndtpart);
      }
      if (sys) {
        // the residual half of the system pass: the same blocks
        Group gr = g;
        gr.l.kind = B_RESID_SYS;
        close(g, L);
        close(gr, L);
      } else {
        close(g, L);
      }
    }
    // assembly of r fused with the first mass pass where the x-lines allow it
    {
      Group gf[2], gr;
      for (int v = 0; v < 2; ++v) {
        gf[v].l.kind = B_GATHER_LX;
        gf[v].l.re = v + 1;
      }
      gr.l.kind = B_GATHER_R;
      for (int q = 0; q < b->count; ++q) {
        cem_ctx* c = all[q];
        if (fused(c)) {
          LineFastArgs a = line_args<RT>(c, rbuf(c), mass_dst(c, 0), 0, false);
          const int re = a.L >= 2 * P + 2 * W ? 2 : 1;
          a.nlb = line_rows_per_block<P, RT>(a.L, a.ntrans, b->xlines_cap, re * P);
          Group& G = gf[re - 1];
          G.sa.push_back(sa[q]);
          G.lf.push_back(a);
          G.first.push_back(G.first.back() + (int)((a.ntrans + a.nlb - 1) / a.nlb));
          G.l.lds = std::max(G.l.lds, (size_t)a.nlb * line_row_pitch<P, RT>(a.L) * sizeof(RT) +
                                          (size_t)a.nlb * kGatherLineInts * sizeof(int));
        } else {
          gr.sa.push_back(sa[q]);
          gr.first.push_back(gr.first.back() + (int)nblocks(c->N, 256));
        }
      }
      close(gf[0], L);
      close(gf[1], L);
      close(gr, L);
    }
    // remaining mass passes (axis 0 of the unfused problems, then axes >= 1)
    for (int k = 0; k < D; ++k) {
      std::vector<cem_ctx*> sel;        // axis 0: only the problems whose first pass was not fused
      for (cem_ctx* c : all)
        if (k > 0 || !fused(c)) sel.push_back(c);
      if (sel.empty()) continue;
      cem_status s = lines(L, sel, false, k, [&](cem_ctx* c) -> const void* { return mass_src(c, k); },
                           [&](cem_ctx* c) -> void* { return mass_dst(c, k); });
      if (s != CEM_OK) return s;
    }
    // element pass 2 and the update; with the fused update, the stage dt
    // of every problem first (one block each)
    if constexpr (PH == EUL && D == 2) {
      if (b->fuse_update) {
        Group gd;
        gd.l.kind = B_STAGE_DT;
        for (int q = 0; q < b->count; ++q) {
          gd.sa.push_back(sa[q]);
          gd.first.push_back(gd.first.back() + 1);
        }
        close(gd, L);
      }
    }
    {
      Group g2, gu;
      if constexpr (PH == EUL && D >= 2) {
        g2.l.kind = B_ELEM2_SYS;
        g2.l.lds = SysTile<D, P, PH>::LY::bytes;
      } else {
        g2.l.kind = B_ELEM2;
      }
      gu.l.kind = B_UPDATE;
      for (int q = 0; q < b->count; ++q) {
        cem_ctx* c = all[q];
        g2.sa.push_back(sa[q]);
        if constexpr (PH == EUL && D >= 2)
          g2.first.push_back(g2.first.back() + (int)SysTile<D, P, PH>::blocks(c->n));
        else
          g2.first.push_back(g2.first.back() + (int)nblocks(c->E, 128));
        gu.sa.push_back(sa[q]);
        gu.first.push_back(gu.first.back() + c->upd_blocks);
      }
      close(g2, L);
      close(gu, L);
    }
  }
  if (blob.size() > b->plan_cap) return fail(CEM_EINVAL, "batched form: plan region too small");
  HIPCHK(hipMemcpyAsync(b->ws + b->o_plan, blob.data(), blob.size(), hipMemcpyHostToDevice, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  b->plan_dt = dt;
  b->plan_cfl = cfl;
  return CEM_OK;
}

template <int D, int P, int PH, class RT>
cem_status batch_stage(cem_batch* b, int st, hipStream_t stream) {
  constexpr int M = Phys<D, PH>::M;
  constexpr bool MIX = sizeof(RT) == 4;
  const char* base = b->ws + b->o_plan;
  // per-kernel timing (cem_batch_set_timing) goes through the first
  // problem's context: one record per batched launch
  cem_ctx* c0 = b->pr[0];
  for (const BLaunch& l : b->launches[st]) {
    const int LID = l.grad ? 0 : 4;     // line kernels: gradient or mass pass
    const BatchMap mp{reinterpret_cast<const int*>(base + l.o_first), l.nprob};
    const StageArgs* sa = reinterpret_cast<const StageArgs*>(base + l.o_args);
    const LineFastArgs* lf = reinterpret_cast<const LineFastArgs*>(base + l.o_args);
    const LineArgs* la = reinterpret_cast<const LineArgs*>(base + l.o_args);
    const dim3 g(l.blocks);
    switch (l.kind) {
      case B_LINE:
        if (l.grad) CEM_LAUNCH(c0, LID, (kb_line<double, RT>), g, dim3(256), 0, stream, la, mp);
        else CEM_LAUNCH(c0, LID, (kb_line<RT, RT>), g, dim3(256), 0, stream, la, mp);
        break;
      case B_LINE_X:
        if (l.re == 2) {
          if (l.grad) CEM_LAUNCH(c0, LID, (kb_line_x<P, 2, double, RT>), g, dim3(256), l.lds, stream, lf, mp);
          else CEM_LAUNCH(c0, LID, (kb_line_x<P, 2, RT, RT>), g, dim3(256), l.lds, stream, lf, mp);
        } else {
          if (l.grad) CEM_LAUNCH(c0, LID, (kb_line_x<P, 1, double, RT>), g, dim3(256), l.lds, stream, lf, mp);
          else CEM_LAUNCH(c0, LID, (kb_line_x<P, 1, RT, RT>), g, dim3(256), l.lds, stream, lf, mp);
        }
        break;
      case B_LINE_Y:
        if (l.re == 2) {
          if (l.grad) CEM_LAUNCH(c0, LID, (kb_line_y<P, 2, double, RT>), g, dim3(256), l.lds, stream, lf, mp);
          else CEM_LAUNCH(c0, LID, (kb_line_y<P, 2, RT, RT>), g, dim3(256), l.lds, stream, lf, mp);
        } else {
          if (l.grad) CEM_LAUNCH(c0, LID, (kb_line_y<P, 1, double, RT>), g, dim3(256), l.lds, stream, lf, mp);
          else CEM_LAUNCH(c0, LID, (kb_line_y<P, 1, RT, RT>), g, dim3(256), l.lds, stream, lf, mp);
        }
        break;
      case B_LINE_MX:
        if (l.grad) CEM_LAUNCH(c0, LID, (kb_line_mfma<P, true, double, RT>), g, dim3(256), l.lds, stream, lf, mp);
        else CEM_LAUNCH(c0, LID, (kb_line_mfma<P, true, RT, RT>), g, dim3(256), l.lds, stream, lf, mp);
        break;
      case B_LINE_MY:
        if (l.grad) CEM_LAUNCH(c0, LID, (kb_line_mfma<P, false, double, RT>), g, dim3(256), l.lds, stream, lf, mp);
        else CEM_LAUNCH(c0, LID, (kb_line_mfma<P, false, RT, RT>), g, dim3(256), l.lds, stream, lf, mp);
        break;
      case B_STAGE_DT:
        CEM_LAUNCH(c0, 2, kb_stage_dt, g, dim3(1024), 0, stream, sa, mp);
        break;
      case B_ELEM1_TILE:
        if constexpr (D == 2) CEM_LAUNCH(c0, 1, (kb_elem1_tile<P, PH, true, RT>), g, dim3(128), l.lds, stream, sa, mp);
        break;
      case B_ELEM1_TILE2:
        if constexpr (D == 2 && tile2_roles<PH>())
          CEM_LAUNCH(c0, 1, (kb_elem1_tile2<P, PH, true, RT>), g, dim3(256), l.lds, stream, sa, mp);
        break;
      case B_ELEM1_SYS:
        if constexpr (sys_capable<D, PH>())
          CEM_LAUNCH(c0, 1, (kb_elem1_sys<D, P, PH, RT>), g, dim3(M * SysTile<D, P, PH>::EB), l.lds, stream, sa, mp);
        break;
      case B_RESID_SYS:
        if constexpr (sys_capable<D, PH>())
          CEM_LAUNCH(c0, 7, (kb_resid_sys<D, P, PH, RT>), g, dim3(M * SysTile<D, P, PH>::EB), l.lds, stream, sa, mp);
        break;
      case B_GATHER_LX:
        if (l.re == 2)
          CEM_LAUNCH(c0, 3, (kb_gather_line_x<D, P, M, 2, RT>), g, dim3(256), l.lds, stream, sa,
                             reinterpret_cast<const LineFastArgs*>(base + l.o_args2), mp);
        else
          CEM_LAUNCH(c0, 3, (kb_gather_line_x<D, P, M, 1, RT>), g, dim3(256), l.lds, stream, sa,
                             reinterpret_cast<const LineFastArgs*>(base + l.o_args2), mp);
        break;
      case B_GATHER_R:
        CEM_LAUNCH(c0, 3, (kb_gather_r<D, P, M, RT>), g, dim3(256), 0, stream, sa, mp);
        break;
      case B_ELEM2:
        if constexpr (!(PH == EUL && D >= 2))
          CEM_LAUNCH(c0, 5, (kb_elem2<D, P, PH, RT>), g, dim3(128), 0, stream, sa, mp);
        break;
      case B_ELEM2_SYS:
        if constexpr (PH == EUL && D >= 2)
          CEM_LAUNCH(c0, 5, (kb_elem2_sys<D, P, PH, RT>), g, dim3(M * SysTile<D, P, PH>::EB), l.lds, stream, sa, mp);
        break;
      case B_UPDATE:
        CEM_LAUNCH(c0, 6, (kb_update<D, P, PH>), g, dim3(256), 0, stream, sa, mp);
        break;
      case B_LINE_BND:
        CEM_LAUNCH(c0, LID, kb_line_bnd, g, dim3(256), 0, stream,
                   reinterpret_cast<const BndLineArgs*>(base + l.o_args), mp);
        break;
      case B_LINE_BND_RUNS:
        if constexpr (D == 1 && !MIX)
          CEM_LAUNCH(c0, LID, (kb_line_bnd_runs<P, 2>), g, dim3(256), l.lds, stream,
                     reinterpret_cast<const BndLineArgs*>(base + l.o_args), mp);
        break;
      case B_ELEM1:
        if constexpr (D == 1) CEM_LAUNCH(c0, 1, (kb_elem1<D, P, PH, true, RT>), g, dim3(128), 0, stream, sa, mp);
        break;
      default:
        return fail(CEM_EINVAL, "batched form: unknown launch");
    }
    HIPCHK(hipGetLastError());
  }
  return CEM_OK;
}

struct BatchFns {
  cem_status (*plan)(cem_batch*, double, double);
  cem_status (*stage)(cem_batch*, int, hipStream_t);
};

// the batched form covers 1D problems (float64, periodic or non-periodic
// lines), 2D problems (every physics) and 3D Euler
BatchFns pick_batch(int d, int p, int kind, bool mixed) {
#define BCASE(D, P, PH)                                                                 \
  if (d == D && p == P && kind == PH)                                                   \
    return mixed ? BatchFns{&batch_plan<D, P, PH, float>, &batch_stage<D, P, PH, float>} \
                 : BatchFns{&batch_plan<D, P, PH, double>, &batch_stage<D, P, PH, double>};
  // 1D (periodic or non-periodic lines) in float64
#define BCASE1(P, PH)                              \
  if (d == 1 && p == P && kind == PH && !mixed)    \
    return BatchFns{&batch_plan<1, P, PH, double>, &batch_stage<1, P, PH, double>};
  BCASE1(1, ADV) BCASE1(2, ADV) BCASE1(3, ADV)
  BCASE1(1, EUL) BCASE1(2, EUL) BCASE1(3, EUL)
  BCASE1(1, NCV) BCASE1(2, NCV) BCASE1(3, NCV)
#undef BCASE1
  BCASE(2, 1, ADV) BCASE(2, 2, ADV) BCASE(2, 3, ADV)
  BCASE(2, 1, KPP) BCASE(2, 2, KPP) BCASE(2, 3, KPP)
  BCASE(2, 1, EUL) BCASE(2, 2, EUL) BCASE(2, 3, EUL)
  BCASE(3, 1, EUL) BCASE(3, 2, EUL)
#undef BCASE
  return BatchFns{nullptr, nullptr};
}

using StageFn = cem_status (*)(cem_ctx*, int, double, double);

void drop_graph(cem_ctx* c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
}

// float64 stages for every supported (d, p, physics); the mixed-precision
// form is built for d = 2, 3; non-periodic lines for 1D advection, Euler
// and the nonconvex flux
StageFn pick(int d, int p, int kind, bool mixed = false, bool bounded = false) {
  if (bounded) {
    if (d != 1 || mixed) return nullptr;
#define LCASE(P, PH) \
    if (p == P && kind == PH) return &stage_line_impl<P, PH>;
    LCASE(1, ADV) LCASE(2, ADV) LCASE(3, ADV)
    LCASE(1, EUL) LCASE(2, EUL) LCASE(3, EUL)
    LCASE(1, NCV) LCASE(2, NCV) LCASE(3, NCV)
#undef LCASE
    return nullptr;
  }
#define CASE(D, P, PH) \
  if (d == D && p == P && kind == PH && !mixed) return &stage_impl<D, P, PH, double>;
#define CASEM(D, P, PH) \
  if (d == D && p == P && kind == PH) return mixed ? &stage_impl<D, P, PH, float> : &stage_impl<D, P, PH, double>;
  CASE(1, 1, ADV) CASE(1, 2, ADV) CASE(1, 3, ADV)
  CASE(1, 1, EUL) CASE(1, 2, EUL) CASE(1, 3, EUL)
  CASE(1, 1, NCV) CASE(1, 2, NCV) CASE(1, 3, NCV)
  CASEM(2, 1, ADV) CASEM(2, 2, ADV) CASEM(2, 3, ADV)
  CASEM(2, 1, KPP) CASEM(2, 2, KPP) CASEM(2, 3, KPP)
  CASEM(2, 1, EUL) CASEM(2, 2, EUL) CASEM(2, 3, EUL)
  CASEM(3, 1, ADV) CASEM(3, 2, ADV)
  CASEM(3, 1, EUL) CASEM(3, 2, EUL)
#undef CASE
#undef CASEM
  return nullptr;
}

}  // namespace

extern "C" {

const char* cem_last_error(void) { return g_err.c_str(); }

cem_status cem_params_default(cem_params* p) {
  if (!p) return fail(CEM_EINVAL, "null params");
  std::memset(p, 0, sizeof(*p));
  p->q = 1.0;
  p->r = 2.0;
  p->eps = 1e-12;
  p->w_lin = 1e-3;
  p->eps_pos = 1e-10;
  p->clamp_ulps = 64.0;
  p->u_min = -INFINITY;
  p->u_max = INFINITY;
  return CEM_OK;
}

cem_status cem_create(const cem_mesh_desc* mesh, const cem_physics_desc* phys, const cem_params* prm,
                      void* stream, cem_ctx** out) {
  if (!mesh || !phys || !prm || !out) return fail(CEM_EINVAL, "null argument");
  const int d = mesh->dim, p = mesh->degree;
  if (d < 1 || d > 3) return fail(CEM_EINVAL, "dim must be 1, 2 or 3");
  if (prm->precision != CEM_FP64 && prm->precision != CEM_FP32_MIXED)
    return fail(CEM_EINVAL, "precision must be CEM_FP64 or CEM_FP32_MIXED");
  for (int s = 0; s < 2; ++s)
    if (mesh->bc[s] < CEM_BC_PERIODIC || mesh->bc[s] > CEM_BC_WALL) return fail(CEM_EINVAL, "bc must be a cem_bc_kind");
  const bool bounded = mesh->bc[0] != CEM_BC_PERIODIC || mesh->bc[1] != CEM_BC_PERIODIC;
  if (bounded) {
    if (mesh->bc[0] == CEM_BC_PERIODIC || mesh->bc[1] == CEM_BC_PERIODIC)
      return fail(CEM_EINVAL, "both ends periodic, or neither");
    if (d != 1) return fail(CEM_EINVAL, "non-periodic boundaries are provided for 1D lines");
    if (prm->precision != CEM_FP64) return fail(CEM_EINVAL, "non-periodic lines compute in float64");
    if (prm->flux_mode == CEM_FLUX_SUBCELL)
      return fail(CEM_EINVAL, "the subcell bound of Lemma 1 is not defined with boundary facets");
    if (prm->contrib == CEM_CONTRIB_Q1) return fail(CEM_EINVAL, "the Q1 contributions need a periodic mesh");
    const int mm = phys->kind == CEM_EULER ? 3 : 1;
    for (int s = 0; s < 2; ++s) {
      if (mesh->bc[s] == CEM_BC_WALL && phys->kind != CEM_EULER)
        return fail(CEM_EINVAL, "CEM_BC_WALL is an Euler condition");
      if (mesh->bc[s] != CEM_BC_STATE) continue;
      const double* st = mesh->bc_state[s];
      for (int q = 0; q < mm; ++q)
        if (!std::isfinite(st[q])) return fail(CEM_EINVAL, "boundary state not finite");
      if (phys->kind == CEM_EULER) {
        const double pr = (phys->gamma_gas - 1.0) * (st[2] - 0.5 * st[1] * st[1] / st[0]);
        if (!(st[0] > 0.0) || !(pr > 0.0)) return fail(CEM_EINVAL, "boundary state outside the invariant domain");
      } else if (!(st[0] >= prm->u_min && st[0] <= prm->u_max)) {
        return fail(CEM_EINVAL, "boundary state outside [u_min, u_max]");
      }
    }
  }
  if (!pick(d, p, phys->kind, prm->precision == CEM_FP32_MIXED, bounded))
    return fail(CEM_EINVAL, "unsupported (dim, degree, physics, precision)");
  if (prm->flux_mode < CEM_FLUX_LIMIT || prm->flux_mode > CEM_FLUX_SHRINK)
    return fail(CEM_EINVAL, "flux_mode must be CEM_FLUX_LIMIT, CEM_FLUX_SUBCELL or CEM_FLUX_SHRINK");
  if (prm->bounds != CEM_BOUNDS_GLOBAL && prm->bounds != CEM_BOUNDS_LOCAL)
    return fail(CEM_EINVAL, "bounds must be CEM_BOUNDS_GLOBAL or CEM_BOUNDS_LOCAL");
  if (prm->contrib != CEM_CONTRIB_AEC && prm->contrib != CEM_CONTRIB_Q1)
    return fail(CEM_EINVAL, "contrib must be CEM_CONTRIB_AEC or CEM_CONTRIB_Q1");
  if (prm->contrib == CEM_CONTRIB_Q1 && (p != 1 || phys->kind == CEM_EULER || prm->precision != CEM_FP64))
    return fail(CEM_EINVAL, "the Q1 contributions need degree 1, a scalar problem and float64");
  double h = 0.0;
  for (int k = 0; k < d; ++k) {
    if (mesh->n[k] < 2) return fail(CEM_EINVAL, "need at least 2 cells per axis");
    const double hk = (mesh->hi[k] - mesh->lo[k]) / mesh->n[k];
    if (!(hk > 0.0)) return fail(CEM_EINVAL, "empty box");
    if (k == 0) h = hk;
    else if (std::fabs(hk - h) > 1e-12 * h) return fail(CEM_EINVAL, "cells must be cubes");
  }
  if (prm->q < 1.0 || prm->r <= 0.0 || prm->eps <= 0.0 || prm->w_lin < 0.0 || 2 * d * prm->w_lin >= 1.0)
    return fail(CEM_EINVAL, "invalid WENO parameters");
  if (phys->kind == CEM_ADVECTION) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += std::fabs(phys->velocity[k]);
    if (s == 0.0) return fail(CEM_EINVAL, "zero advection velocity");
  }
  if (phys->kind == CEM_EULER && !(phys->gamma_gas > 1.0 && phys->gamma_gas <= 5.0 / 3.0))
    return fail(CEM_EINVAL, "gamma must lie in (1, 5/3]");
  cem_ctx* c = new cem_ctx();
  c->d = d;
  c->p = p;
  c->kind = phys->kind;
  c->m = phys->kind == CEM_EULER ? d + 2 : 1;
  c->h = h;
  c->N = 1;
  c->E = 1;
  c->bounded = bounded;
  for (int s = 0; s < 2; ++s) {
    c->bc[s] = mesh->bc[s];
    for (int q = 0; q < 5; ++q) c->bc_u[s][q] = mesh->bc_state[s][q];
  }
  for (int k = 0; k < d; ++k) {
    c->n[k] = mesh->n[k];
    c->L[k] = p * mesh->n[k] + (bounded ? 1 : 0);
    c->N *= c->L[k];
    c->E *= c->n[k];
  }
  if ((int64_t)c->m * c->N >= (int64_t(1) << 31)) {
    delete c;
    return fail(CEM_EINVAL, "mesh too large: m * N must stay below 2^31");
  }
  c->nl = 1;
  for (int k = 0; k < d; ++k) c->nl *= (p + 1);
  if ((int64_t)c->m * c->nl * c->E >= (int64_t(1) << 31)) {
    delete c;
    return fail(CEM_EINVAL, "mesh too large: the element vectors, m (p+1)^d E values, must stay below 2^31");
  }
  c->prm = *prm;
  c->mixed = prm->precision == CEM_FP32_MIXED;
  for (int k = 0; k < 3; ++k) c->ph.vel[k] = k < d ? phys->velocity[k] : 0.0;
  c->ph.vnorm = std::sqrt(c->ph.vel[0] * c->ph.vel[0] + c->ph.vel[1] * c->ph.vel[1] + c->ph.vel[2] * c->ph.vel[2]);
  c->ph.gam = phys->gamma_gas;
  c->ph.rn = 0;
  if (phys->kind == CEM_EULER) {
    // the integer 1 / ex of the two-rarefaction bound, when there is one
    const double r = 2.0 * phys->gamma_gas / (phys->gamma_gas - 1.0), rr = std::nearbyint(r);
    if (rr >= 2.0 && rr <= 32.0 && std::fabs(r - rr) <= 1e-9 * rr) c->ph.rn = (int)rr;
  }
  c->stream = (hipStream_t)stream;
  // (the periodic line tables of a non-periodic line are built for the
  // periodic line of the same cells and stay unused)
  const int Lper[3] = {p * c->n[0], c->L[1], c->L[2]};
  if (!build_tables(d, p, h, Lper, kWfast, kRfast, kSfast, kWfast32, kSfast32, c->tabs) ||
      (bounded && !build_bounded_line(p, c->n[0], h, c->tabs))) {
    delete c;
    return fail(CEM_EINVAL, "table construction failed");
  }
  pack_tables(c);
  // workspace carve-up
  const size_t mN = (size_t)c->m * c->N * 8, mE = (size_t)c->m * c->E * 8, E8 = (size_t)c->E * 8;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align256(bytes);
    return r;
  };
  c->o_g = take((size_t)d * mN);
  c->o_fnode = take((size_t)d * mN);
  c->o_r = take(mN);
  c->o_udot = take(mN);
  c->o_tmp = take(mN);
  c->o_tmp2 = take(mN);
  c->o_relem = take((size_t)c->nl * mE);
  c->o_ue = take(mE);
  c->o_ubarL = take(mE);
  c->o_ubar = take(mE);
  c->o_fahi = take((size_t)d * mE);
  c->o_dte = take(E8);
  c->o_gam = take(E8);
  c->o_nu = take(E8);
  c->o_beta = take(E8);
  c->o_bnd = take(2 * E8);
  c->o_fdiv = take(E8);
  c->o_fbnd = take((size_t)4 * c->m * 8);
  c->o_dtbuf = take(8 * 8);
  // per-block dt_e minima: one-thread-per-element blocks, 2D element tiles
  // or the 32- / 64-element blocks of the system passes
  size_t ndtp = nblocks(c->E, 32);
  if (d == 2) ndtp = std::max(ndtp, (size_t)((c->n[0] + 15) / 16) * (size_t)((c->n[1] + 7) / 8));
  c->ndtp = ndtp;
  c->o_dtpart = take(ndtp * 8);
  c->upd_blocks = (int)nblocks(c->N, 256);
  // counter pairs: one per update block, then one per pass-2 block of the
  // fused update (at most ndtp of them)
  c->cnt_slots = c->upd_blocks + (int)ndtp;
  c->o_counts = take((size_t)c->cnt_slots * 2 * sizeof(int));
  c->inv_blocks = 256;
  c->o_inv = take((size_t)c->inv_blocks * inv_nvals(c->m) * 8);
  if (c->mixed) {
    const size_t mN4 = (size_t)c->m * c->N * 4;
    c->o_g32 = take((size_t)d * mN4);
    c->o_r32 = take(mN4);
    c->o_udot32 = take(mN4);
    c->o_tmp32 = take(mN4);
    c->o_tmp2_32 = take(mN4);
  }
  c->o_tab = take(c->tabblob.size() * 8);
  c->ws_need = o;
  *out = c;
  return CEM_OK;
}

cem_status cem_sizes(const cem_ctx* c, long long* N, long long* E, int* m) {
  if (!c) return fail(CEM_EINVAL, "null context");
  if (N) *N = c->N;
  if (E) *E = c->E;
  if (m) *m = c->m;
  return CEM_OK;
}

cem_status cem_workspace_bytes(const cem_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(CEM_EINVAL, "null argument");
  *bytes = c->ws_need;
  return CEM_OK;
}

cem_status cem_reset_counters(cem_ctx* c) {
  if (!c || !c->bound) return fail(CEM_EINVAL, "context not bound");
  HIPCHK(hipMemsetAsync(c->ws + c->o_counts, 0, (size_t)c->cnt_slots * 2 * sizeof(int), c->stream));
  HIPCHK(hipMemsetAsync(c->ws + c->o_dtbuf, 0, 8 * 8, c->stream));
  return CEM_OK;
}

cem_status cem_bind(cem_ctx* c, double* u, double* u_base, void* workspace, size_t ws_bytes) {
  if (!c || !u || !u_base || !workspace) return fail(CEM_EINVAL, "null argument");
  if (u == u_base) return fail(CEM_EINVAL, "u and u_base must differ");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(CEM_EINVAL, "workspace not 256-byte aligned");
  if (ws_bytes < c->ws_need) return fail(CEM_ENOMEM, "workspace too small");
  drop_graph(c);
  c->fnode_valid = false;
  c->u = u;
  c->u0 = u_base;
  c->ws = static_cast<char*>(workspace);
  HIPCHK(hipMemcpyAsync(c->ws + c->o_tab, c->tabblob.data(), c->tabblob.size() * 8, hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));   // the host table blob stays alive, but keep bind simple
  {
    int dev = 0, v = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    c->lds_max = v;
  }
  c->bound = true;
  return cem_reset_counters(c);
}

cem_status cem_upload_state(cem_ctx* c, const double* host_u) {
  if (!c || !c->bound || !host_u) return fail(CEM_EINVAL, "context not bound / null");
  c->fnode_valid = false;
  HIPCHK(hipMemcpyAsync(c->u, host_u, (size_t)c->m * c->N * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CEM_OK;
}

cem_status cem_download_state(cem_ctx* c, double* host_u) {
  if (!c || !c->bound || !host_u) return fail(CEM_EINVAL, "context not bound / null");
  HIPCHK(hipMemcpyAsync(host_u, c->u, (size_t)c->m * c->N * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return CEM_OK;
}

cem_status cem_set_bounds(cem_ctx* c, int from_state, double u_min, double u_max) {
  if (!c || !c->bound) return fail(CEM_EINVAL, "context not bound");
  if (c->kind == CEM_EULER) return CEM_OK;
  if (from_state) {
    cem_invariants inv;
    const double keep_min = c->prm.u_min, keep_max = c->prm.u_max;
    c->prm.u_min = -INFINITY;
    c->prm.u_max = INFINITY;
    cem_status s = cem_check_invariants(c, &inv);
    c->prm.u_min = keep_min;          // restored on every path out
    c->prm.u_max = keep_max;
    if (s != CEM_OK && s != CEM_EIDP && s != CEM_ECFL) return s;
    if (inv.nonfinite) return fail(CEM_EINVAL, "state holds non-finite values");
    u_min = inv.u_min[0];
    u_max = inv.u_max[0];
    // the boundary data of a non-periodic line enters the scheme as well
    for (int s = 0; s < 2; ++s)
      if (c->bounded && c->bc[s] == CEM_BC_STATE) {
        u_min = std::fmin(u_min, c->bc_u[s][0]);
        u_max = std::fmax(u_max, c->bc_u[s][0]);
      }
  }
  if (!(u_min <= u_max)) return fail(CEM_EINVAL, "u_min > u_max");
  for (int s = 0; s < 2; ++s)
    if (c->bounded && c->bc[s] == CEM_BC_STATE && !(c->bc_u[s][0] >= u_min && c->bc_u[s][0] <= u_max))
      return fail(CEM_EINVAL, "boundary state outside [u_min, u_max]");
  c->prm.u_min = u_min;
  c->prm.u_max = u_max;
  c->bounds_set = true;
  drop_graph(c);            // the bounds are baked into captured launches
  return CEM_OK;
}

cem_status cem_rk_stage(cem_ctx* c, int stage, double dt, double cfl) {
  if (!c || !c->bound) return fail(CEM_EINVAL, "context not bound");
  if (stage < 0 || stage > 2) return fail(CEM_EINVAL, "stage must be 0, 1 or 2");
  if (stage == 0 && !(dt > 0.0) && !(cfl > 0.0)) return fail(CEM_EINVAL, "need dt > 0 or cfl > 0");
  if (c->kind != CEM_EULER && !c->bounds_set) return fail(CEM_EINVAL, "scalar bounds not set");
  return pick(c->d, c->p, c->kind, c->mixed, c->bounded)(c, stage, dt, cfl);
}

static cem_status step_direct(cem_ctx* c, double dt, double cfl) {
  c->copy_base_next = true;     // stage 0 writes u_base = u (no separate copy)
  c->in_step = true;
  cem_status st = CEM_OK;
  for (int s = 0; s < 3 && st == CEM_OK; ++s) st = pick(c->d, c->p, c->kind, c->mixed, c->bounded)(c, s, dt, cfl);
  c->copy_base_next = false;
  c->in_step = false;
  return st;
}

cem_status cem_step(cem_ctx* c, double dt, double cfl) {
  if (!c || !c->bound) return fail(CEM_EINVAL, "context not bound");
  if (!(dt > 0.0) && !(cfl > 0.0)) return fail(CEM_EINVAL, "need dt > 0 or cfl > 0");
  if (c->kind != CEM_EULER && !c->bounds_set) return fail(CEM_EINVAL, "scalar bounds not set");
  // direct launches with timing, without graphs, and whenever derived state
  // (nodal fluxes) must be rebuilt first so that captures stay replayable
  if (!c->use_graphs || c->timing_mask || !c->fnode_valid) return step_direct(c, dt, cfl);
  if (!c->graph || c->graph_dt != dt || c->graph_cfl != cfl) {
    // capture the three stages on the private stream, then replay the graph
    // on the caller's stream
    drop_graph(c);
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    cem_status st = step_direct(c, dt, cfl);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = user;
    if (st != CEM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(CEM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->graph = nullptr;
      return fail(CEM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    c->graph_dt = dt;
    c->graph_cfl = cfl;
  }
  HIPCHK(hipGraphLaunch(c->graph, c->stream));
  return CEM_OK;
}

cem_status cem_state_modified(cem_ctx* c) {
  if (!c) return fail(CEM_EINVAL, "null context");
  c->fnode_valid = false;
  return CEM_OK;
}

cem_status cem_set_line_kernels(cem_ctx* c, int mode) {
  if (!c) return fail(CEM_EINVAL, "null context");
  if (mode < 0 || mode > 2) return fail(CEM_EINVAL, "line kernel mode must be 0 (vector), 1 (matrix) or 2 (by size)");
  c->line_mfma = mode;
  drop_graph(c);
  return CEM_OK;
}

cem_status cem_set_fused_update(cem_ctx* c, int enable) {
  if (!c) return fail(CEM_EINVAL, "null context");
  c->fuse_update = enable != 0;
  drop_graph(c);
  return CEM_OK;
}

cem_status cem_set_graphs(cem_ctx* c, int enable) {
  if (!c) return fail(CEM_EINVAL, "null context");
  c->use_graphs = enable != 0;
  if (!c->use_graphs) drop_graph(c);
  return CEM_OK;
}

cem_status cem_check_invariants(cem_ctx* c, cem_invariants* out) {
  if (!c || !c->bound || !out) return fail(CEM_EINVAL, "context not bound / null");
  std::memset(out, 0, sizeof(*out));
  InvArgs ia{};
  ia.u = c->u;
  ia.N = c->N;
  ia.M = c->m;
  ia.D = c->d;
  ia.euler = c->kind == CEM_EULER;
  ia.gam = c->ph.gam;
  double hd = 1.0;
  for (int k = 0; k < c->d; ++k) hd *= c->h;
  ia.mnode = hd / c->nl;
  ia.P = c->p;
  ia.Lx = c->L[0];
  ia.Ly = c->L[1];
  ia.umin = c->prm.u_min;
  ia.umax = c->prm.u_max;
  ia.tol = c->prm.clamp_ulps * DBL_EPSILON * std::fmax(std::fabs(c->prm.u_min), std::fabs(c->prm.u_max));
  ia.part = c->W<double>(c->o_inv);
  hipLaunchKernelGGL(k_inv_partial, dim3(c->inv_blocks), dim3(256), 0, c->stream, ia);
  HIPCHK(hipGetLastError());
  const int nv = inv_nvals(c->m);
  std::vector<double> part((size_t)c->inv_blocks * nv);
  std::vector<int> cnt((size_t)c->cnt_slots * 2);
  double dtb[8];
  HIPCHK(hipMemcpyAsync(part.data(), ia.part, part.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(cnt.data(), c->ws + c->o_counts, cnt.size() * sizeof(int), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipMemcpyAsync(dtb, c->ws + c->o_dtbuf, sizeof(dtb), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  out->m = c->m;
  for (int v = 0; v < c->m; ++v) {
    out->u_min[v] = INFINITY;
    out->u_max[v] = -INFINITY;
    out->mass[v] = 0.0;
  }
  out->rho_min = INFINITY;
  out->p_min = INFINITY;
  // NaN-propagating extrema (std::fmin / fmax would drop a NaN)
  auto nmin = [](double x, double y) { return (x < y || x != x) ? x : y; };
  auto nmax = [](double x, double y) { return (x > y || x != x) ? x : y; };
  double nonfin = 0.0, sviol = 0.0;
  for (int b = 0; b < c->inv_blocks; ++b)
    for (int v = 0; v < nv; ++v) {
      const double x = part[(size_t)b * nv + v];
      if (v >= c->m * 3) {
        const int kind = v - c->m * 3;    // 0 rho_min, 1 p_min, 2 non-finite, 3 violations
        if (kind == 2) nonfin += x;
        else if (kind == 3) sviol += x;
        else if (!ia.euler) continue;
        else if (kind == 0) out->rho_min = nmin(out->rho_min, x);
        else out->p_min = nmin(out->p_min, x);
      } else if (v % 3 == 0) {
        out->u_min[v / 3] = nmin(out->u_min[v / 3], x);
      } else if (v % 3 == 1) {
        out->u_max[v / 3] = nmax(out->u_max[v / 3], x);
      } else {
        out->mass[v / 3] += x;
      }
    }
  for (int b = 0; b < c->cnt_slots; ++b) {
    out->clamped += cnt[2 * (size_t)b];
    out->violations += cnt[2 * (size_t)b + 1];
  }
  out->nonfinite = (long long)nonfin;
  out->state_violations = (long long)sviol;
  out->dt = dtb[0];
  out->min_dt_e = dtb[1];
  out->cfl_violated = dtb[2] != 0.0;
  // an invariant-domain failure is reported ahead of a CFL violation (the
  // latter is what made the former possible)
  if (out->violations || out->state_violations || out->nonfinite)
    return fail(CEM_EIDP, "invariant domain violated");
  if (out->cfl_violated) return fail(CEM_ECFL, "dt exceeded min_e dt_e");
  return CEM_OK;
}

size_t cem_tap_size(const cem_ctx* c, int tap) {
  if (!c) return 0;
  const size_t mN = (size_t)c->m * c->N, mE = (size_t)c->m * c->E, E = (size_t)c->E;
  switch (tap) {
    case 0: return (size_t)c->d * mN;
    case 1: case 2: return mN;
    case 3: case 4: case 5: case 9: return E;
    case 6: case 7: case 8: return mE;
    case 10: return (size_t)c->d * mE;
    case 11: return (size_t)c->nl * mE;
    case 12: return 2 * E;
    default: return 0;
  }
}

cem_status cem_debug_tap(cem_ctx* c, int tap, double* dst, size_t count) {
  if (!c || !c->bound || !dst) return fail(CEM_EINVAL, "context not bound / null");
  const size_t n = cem_tap_size(c, tap);
  if (n == 0 || count != n) return fail(CEM_EINVAL, "bad tap id or count");
  const size_t offs[13] = {c->o_g, c->o_r, c->o_udot, c->o_gam, c->o_nu, c->o_dte, c->o_ue,
                           c->o_ubarL, c->o_ubar, c->o_beta, c->o_fahi, c->o_relem, c->o_bnd};
  if (c->mixed && tap <= 2) {
    // g, r and udot are float arrays in the mixed form
    const size_t o32[3] = {c->o_g32, c->o_r32, c->o_udot32};
    hipLaunchKernelGGL(k_widen, dim3(nblocks(n, 256)), dim3(256), 0, c->stream,
                       c->W<const float>(o32[tap]), dst, (int64_t)n);
    HIPCHK(hipGetLastError());
    return CEM_OK;
  }
  HIPCHK(hipMemcpyAsync(dst, c->ws + offs[tap], n * 8, hipMemcpyDeviceToDevice, c->stream));
  return CEM_OK;
}

cem_status cem_set_timing(cem_ctx* c, unsigned mask) {
  if (!c) return fail(CEM_EINVAL, "null context");
  c->timing_mask = mask & ((1u << CEM_NUM_KERNELS) - 1);
  return CEM_OK;
}

cem_status cem_kernel_times(cem_ctx* c, double* total_ms, long long* launches, int n) {
  if (!c || !total_ms || !launches || n < 0) return fail(CEM_EINVAL, "null argument");
  for (int i = 0; i < n; ++i) {
    total_ms[i] = 0.0;
    launches[i] = 0;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  for (auto& r : c->recs) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    if (r.id < n) {
      total_ms[r.id] += ms;
      launches[r.id] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
  return CEM_OK;
}

void cem_destroy(cem_ctx* c) {
  if (!c) return;
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  delete c;
}

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
static void batch_drop_graph(cem_batch* b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
}

void cem_batch_destroy(cem_batch* b) {
  if (!b) return;
  batch_drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (cem_ctx* c : b->pr) cem_destroy(c);
  delete b;
}

cem_status cem_batch_create(int count, const cem_mesh_desc* meshes, const cem_physics_desc* phys,
                            const cem_params* prm, void* stream, cem_batch** out) {
  if (count < 1 || !meshes || !phys || !prm || !out) return fail(CEM_EINVAL, "null argument or count < 1");
  const int d = meshes[0].dim, p = meshes[0].degree;
  const bool mixed = prm->precision == CEM_FP32_MIXED;
  if (!pick_batch(d, p, phys->kind, mixed).plan)
    return fail(CEM_EINVAL, "batched form: 1D problems in float64, 2D problems or 3D Euler only");
  if (prm->contrib == CEM_CONTRIB_Q1)
    return fail(CEM_EINVAL, "batched form: the Q1 contributions run on single problems");
  cem_batch* b = new cem_batch();
  b->count = count;
  b->d = d;
  b->p = p;
  b->kind = phys->kind;
  b->mixed = mixed;
  b->stream = (hipStream_t)stream;
  b->uoff.assign(1, 0);
  size_t ws = 0;
  for (int k = 0; k < count; ++k) {
    if (meshes[k].dim != d || meshes[k].degree != p) {
      cem_batch_destroy(b);
      return fail(CEM_EINVAL, "batched form: every problem needs the same dimension and degree");
    }
    cem_ctx* c = nullptr;
    cem_status st = cem_create(&meshes[k], phys, prm, stream, &c);
    if (st != CEM_OK) {
      cem_batch_destroy(b);
      return st;
    }
    b->pr.push_back(c);
    b->m = c->m;
    b->uoff.push_back(b->uoff.back() + (long long)c->m * c->N);
    b->wsoff.push_back(ws);
    ws += align256(c->ws_need);
  }
  // plan region, per stage: StageArgs entries, one per problem in element
  // pass 1 (two with the system kernels' residual half), the assembly, the
  // stage dt of the fused update, pass 2 and the update; one line-argument
  // entry per problem and line pass (d gradient, d mass); at most 10 d + 8
  // launch groups, each with a block prefix of at most count + 1 ints and
  // up to three arrays padded to 256
  const size_t ngroups = 10 * (size_t)d + 8;
  const size_t per_stage = 6 * (size_t)count * sizeof(StageArgs) +
                           2 * (size_t)d * count * std::max(sizeof(LineFastArgs), sizeof(LineArgs)) +
                           ngroups * (size_t)(count + 1) * sizeof(int) + 3 * ngroups * 256;
  b->o_plan = ws;
  b->plan_cap = 3 * per_stage;
  b->ws_need = ws + align256(b->plan_cap);
  *out = b;
  return CEM_OK;
}

cem_status cem_batch_offsets(const cem_batch* b, long long* offsets, int n) {
  if (!b || !offsets || n != b->count + 1) return fail(CEM_EINVAL, "need count + 1 offsets");
  for (int k = 0; k <= b->count; ++k) offsets[k] = b->uoff[k];
  return CEM_OK;
}

cem_status cem_batch_workspace_bytes(const cem_batch* b, size_t* bytes) {
  if (!b || !bytes) return fail(CEM_EINVAL, "null argument");
  *bytes = b->ws_need;
  return CEM_OK;
}

cem_status cem_batch_bind(cem_batch* b, double* u, double* u_base, void* workspace, size_t ws_bytes) {
  if (!b || !u || !u_base || !workspace) return fail(CEM_EINVAL, "null argument");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(CEM_EINVAL, "workspace not 256-byte aligned");
  if (ws_bytes < b->ws_need) return fail(CEM_ENOMEM, "workspace too small");
  batch_drop_graph(b);
  char* ws = static_cast<char*>(workspace);
  for (int k = 0; k < b->count; ++k) {
    cem_status st = cem_bind(b->pr[k], u + b->uoff[k], u_base + b->uoff[k], ws + b->wsoff[k], b->pr[k]->ws_need);
    if (st != CEM_OK) return st;
  }
  b->ws = ws;
  b->u = u;
  b->u0 = u_base;
  b->plan_dt = b->plan_cfl = -1.0;
  b->bound = true;
  return CEM_OK;
}

cem_status cem_batch_upload_state(cem_batch* b, const double* host_u) {
  if (!b || !b->bound || !host_u) return fail(CEM_EINVAL, "batch not bound / null");
  for (int k = 0; k < b->count; ++k) {
    cem_status st = cem_upload_state(b->pr[k], host_u + b->uoff[k]);
    if (st != CEM_OK) return st;
  }
  return CEM_OK;
}

cem_status cem_batch_download_state(cem_batch* b, double* host_u) {
  if (!b || !b->bound || !host_u) return fail(CEM_EINVAL, "batch not bound / null");
  for (int k = 0; k < b->count; ++k) {
    cem_status st = cem_download_state(b->pr[k], host_u + b->uoff[k]);
    if (st != CEM_OK) return st;
  }
  return CEM_OK;
}

cem_status cem_batch_set_bounds(cem_batch* b, int from_state, double u_min, double u_max) {
  if (!b || !b->bound) return fail(CEM_EINVAL, "batch not bound");
  for (int k = 0; k < b->count; ++k) {
    cem_status st = cem_set_bounds(b->pr[k], from_state, u_min, u_max);
    if (st != CEM_OK) return st;
  }
  batch_drop_graph(b);
  b->plan_dt = b->plan_cfl = -1.0;   // the stage arguments carry the bounds
  return CEM_OK;
}

cem_status cem_batch_set_graphs(cem_batch* b, int enable) {
  if (!b) return fail(CEM_EINVAL, "null batch");
  b->use_graphs = enable != 0;
  return CEM_OK;
}

cem_status cem_batch_step(cem_batch* b, double dt, double cfl, int nsteps) {
  if (!b || !b->bound) return fail(CEM_EINVAL, "batch not bound");
  if (!(dt > 0.0) && !(cfl > 0.0)) return fail(CEM_EINVAL, "need dt > 0 or cfl > 0");
  if (nsteps < 0) return fail(CEM_EINVAL, "nsteps < 0");
  for (cem_ctx* c : b->pr) {
    if (c->kind != CEM_EULER && !c->bounds_set) return fail(CEM_EINVAL, "scalar bounds not set");
    if (c->kind == CEM_KPP && !c->fnode_valid) {
      // nodal fluxes of the uploaded state (refreshed by every update after)
      StageArgs a = make_args(c);
      hipLaunchKernelGGL((k_nodal_flux<2, KPP>), dim3(nblocks(c->N, 256)), dim3(256), 0, c->stream, a);
      HIPCHK(hipGetLastError());
      c->fnode_valid = true;
    }
  }
  const BatchFns fn = pick_batch(b->d, b->p, b->kind, b->mixed);
  if (b->plan_dt != dt || b->plan_cfl != cfl) {
    batch_drop_graph(b);
    cem_status st = fn.plan(b, dt, cfl);
    if (st != CEM_OK) return st;
  }
  if (!b->use_graphs || b->pr[0]->timing_mask) {
    for (int n = 0; n < nsteps; ++n)
      for (int s = 0; s < 3; ++s) {
        cem_status st = fn.stage(b, s, b->stream);
        if (st != CEM_OK) return st;
      }
    return CEM_OK;
  }
  if (!b->graph) {
    if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    cem_status st = CEM_OK;
    for (int s = 0; s < 3 && st == CEM_OK; ++s) st = fn.stage(b, s, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st != CEM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(CEM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->graph = nullptr;
      return fail(CEM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
  }
  for (int n = 0; n < nsteps; ++n) HIPCHK(hipGraphLaunch(b->graph, b->stream));
  return CEM_OK;
}

cem_status cem_batch_reset_counters(cem_batch* b) {
  if (!b || !b->bound) return fail(CEM_EINVAL, "batch not bound");
  for (cem_ctx* c : b->pr) {
    cem_status st = cem_reset_counters(c);
    if (st != CEM_OK) return st;
  }
  return CEM_OK;
}

cem_status cem_batch_set_plan(cem_batch* b, int order, int xlines_cap, int ytile_lds_bytes, int elem1_kernel) {
  if (!b) return fail(CEM_EINVAL, "null batch");
  if (order < 0 || order > 1) return fail(CEM_EINVAL, "order must be 0 (input) or 1 (largest first)");
  if (xlines_cap < 256 || xlines_cap > 65536) return fail(CEM_EINVAL, "xlines_cap out of [256, 65536]");
  if (ytile_lds_bytes < 8192 || ytile_lds_bytes > 65536) return fail(CEM_EINVAL, "ytile_lds_bytes out of [8192, 65536]");
  if (elem1_kernel < 0 || elem1_kernel > 1) return fail(CEM_EINVAL, "elem1_kernel must be 0 (tile) or 1 (system)");
  if (elem1_kernel == 1 && !(b->kind == CEM_EULER && b->d >= 2))
    return fail(CEM_EINVAL, "the system element kernels serve the Euler equations in 2D and 3D");
  b->order = order;
  b->xlines_cap = xlines_cap;
  b->ytile_cap = ytile_lds_bytes;
  b->elem1_sys = elem1_kernel;
  batch_drop_graph(b);
  b->plan_dt = b->plan_cfl = -1.0;     // the next step rebuilds the plan
  return CEM_OK;
}

cem_status cem_batch_set_line_kernels(cem_batch* b, int matrix) {
  if (!b) return fail(CEM_EINVAL, "null batch");
  if (matrix < 0 || matrix > 1) return fail(CEM_EINVAL, "line kernels must be 0 (vector) or 1 (matrix)");
  b->line_mfma = matrix;
  batch_drop_graph(b);
  b->plan_dt = b->plan_cfl = -1.0;
  return CEM_OK;
}

cem_status cem_batch_set_fused_update(cem_batch* b, int enable) {
  if (!b) return fail(CEM_EINVAL, "null batch");
  b->fuse_update = enable != 0;
  batch_drop_graph(b);
  b->plan_dt = b->plan_cfl = -1.0;
  return CEM_OK;
}

cem_status cem_batch_set_timing(cem_batch* b, unsigned mask) {
  if (!b || b->pr.empty()) return fail(CEM_EINVAL, "null batch");
  return cem_set_timing(b->pr[0], mask);
}

cem_status cem_batch_kernel_times(cem_batch* b, double* total_ms, long long* launches, int n) {
  if (!b || b->pr.empty()) return fail(CEM_EINVAL, "null batch");
  HIPCHK(hipStreamSynchronize(b->stream));
  return cem_kernel_times(b->pr[0], total_ms, launches, n);
}

cem_status cem_batch_check_invariants(cem_batch* b, cem_invariants* out, int n) {
  if (!b || !b->bound || !out || n != b->count) return fail(CEM_EINVAL, "need one record per problem");
  cem_status worst = CEM_OK;
  for (int k = 0; k < b->count; ++k) {
    cem_status st = cem_check_invariants(b->pr[k], &out[k]);
    if (st == CEM_EHIP || st == CEM_EINVAL) return st;
    if (st == CEM_EIDP || (st == CEM_ECFL && worst == CEM_OK)) worst = st;
  }
  return worst;
}

cem_status cem_batch_autotune(cem_batch* b, double dt, double cfl, int steps, void* scratch, size_t scratch_bytes,
                              char* report, size_t report_cap) {
  if (!b || !b->bound || !scratch) return fail(CEM_EINVAL, "batch not bound / null scratch");
  if (steps < 1) return fail(CEM_EINVAL, "steps < 1");
  const size_t bytes = (size_t)b->uoff.back() * sizeof(double);
  if (scratch_bytes < bytes) return fail(CEM_ENOMEM, "scratch smaller than the batch state");
  auto restore = [&]() -> cem_status {
    HIPCHK(hipMemcpyAsync(b->u, scratch, bytes, hipMemcpyDeviceToDevice, b->stream));
    for (cem_ctx* c : b->pr) c->fnode_valid = false;   // derived nodal fluxes follow the state
    return CEM_OK;
  };
  HIPCHK(hipMemcpyAsync(scratch, b->u, bytes, hipMemcpyDeviceToDevice, b->stream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // the knobs of a plan and the values tried: problem order, values staged
  // per block of the x-line kernels, LDS bytes of a strided line tile (runs
  // per thread ky = 1, 2, 4 of the vector kernels; row groups of the
  // matrix-core tiles), for 2D Euler the element pass-1 kernel (16 x 8
  // element LDS tile with one thread per element, or blocks of 32/64
  // elements with one thread per element and component), and
  // the line kernels (matrix-core tiles or vector runs)
  struct Knobs { int order, xcap, ycap, sys, mfma; };
  struct Trial { Knobs k; float ms; };
  const bool sys_choice = b->d == 2 && b->kind == CEM_EULER;
  const std::vector<int> orders = {0, 1}, xcaps = {512, 1024, 2048, 4096}, ycaps = {20480, 40960, 57344};
  const std::vector<int> syss = sys_choice ? std::vector<int>{0, 1} : std::vector<int>{b->elem1_sys};
  // line passes: matrix-core tiles or the vector kernels
  const std::vector<int> mfmas = {0, 1};
  std::vector<Trial> trials;
  cem_status st = CEM_OK;
  auto run_trial = [&](const Knobs& k, float* ms_out) -> cem_status {
    b->order = k.order;
    b->xlines_cap = k.xcap;
    b->ytile_cap = k.ycap;
    b->elem1_sys = k.sys;
    b->line_mfma = k.mfma;
    batch_drop_graph(b);
    b->plan_dt = b->plan_cfl = -1.0;
    cem_status s2;
    if ((s2 = restore()) != CEM_OK) return s2;
    if ((s2 = cem_batch_step(b, dt, cfl, 1)) != CEM_OK) return s2;      // plan, capture, warm
    if ((s2 = restore()) != CEM_OK) return s2;
    if ((s2 = cem_batch_step(b, dt, cfl, 1)) != CEM_OK) return s2;      // nodal fluxes outside the timing
    if ((s2 = restore()) != CEM_OK) return s2;
    for (cem_ctx* c : b->pr) c->fnode_valid = c->kind != CEM_KPP;
    if (b->kind == CEM_KPP) {
      // KPP: the restored state needs its nodal fluxes before timing
      for (cem_ctx* c : b->pr) {
        StageArgs a = make_args(c);
        hipLaunchKernelGGL((k_nodal_flux<2, KPP>), dim3(nblocks(c->N, 256)), dim3(256), 0, c->stream, a);
        c->fnode_valid = true;
      }
    }
    HIPCHK(hipEventRecord(e0, b->stream));
    if ((s2 = cem_batch_step(b, dt, cfl, steps)) != CEM_OK) return s2;
    HIPCHK(hipEventRecord(e1, b->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    *ms_out = ms / steps;
    return CEM_OK;
  };
  // coordinate search from the current plan: each knob in turn over its
  // values, the others at their best so far
  Knobs best_k{b->order, b->xlines_cap, b->ytile_cap, b->elem1_sys, b->line_mfma};
  float best_ms = 0.0f;
  if ((st = run_trial(best_k, &best_ms)) == CEM_OK) trials.push_back({best_k, best_ms});
  for (int knob = 0; knob < 5 && st == CEM_OK; ++knob) {
    const std::vector<int>& vals =
        knob == 0 ? orders : knob == 1 ? xcaps : knob == 2 ? ycaps : knob == 3 ? syss : mfmas;
    for (int v : vals) {
      Knobs k = best_k;
      int* slot = knob == 0 ? &k.order : knob == 1 ? &k.xcap : knob == 2 ? &k.ycap : knob == 3 ? &k.sys : &k.mfma;
      *slot = v;
      bool seen = false;       // each plan is timed once
      for (const Trial& t : trials)
        seen = seen || (t.k.order == k.order && t.k.xcap == k.xcap && t.k.ycap == k.ycap && t.k.sys == k.sys &&
                        t.k.mfma == k.mfma);
      if (seen) continue;
      float ms = 0.0f;
      if ((st = run_trial(k, &ms)) != CEM_OK) break;
      trials.push_back({k, ms});
      if (ms < best_ms) {
        best_ms = ms;
        best_k = k;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != CEM_OK) return st;
  b->order = best_k.order;
  b->xlines_cap = best_k.xcap;
  b->ytile_cap = best_k.ycap;
  b->elem1_sys = best_k.sys;
  b->line_mfma = best_k.mfma;
  batch_drop_graph(b);
  b->plan_dt = b->plan_cfl = -1.0;
  st = restore();
  if (st != CEM_OK) return st;
  HIPCHK(hipStreamSynchronize(b->stream));
  st = cem_batch_reset_counters(b);
  if (st != CEM_OK) return st;
  if (report && report_cap) {
    auto rec = [&](const Knobs& k, float ms) {
      char buf[256];
      std::snprintf(buf, sizeof(buf),
                    "{\"order\": \"%s\", \"xlines_cap\": %d, \"ytile_lds_bytes\": %d, \"elem1\": \"%s\", "
                    "\"lines\": \"%s\", \"ms_per_step\": %.4f}",
                    k.order ? "largest_first" : "input", k.xcap, k.ycap, k.sys ? "system" : "tile",
                    k.mfma ? "matrix" : "vector", ms);
      return std::string(buf);
    };
    std::string r = "{\"trials\": [";
    for (size_t k = 0; k < trials.size(); ++k) r += (k ? ", " : "") + rec(trials[k].k, trials[k].ms);
    r += "], \"best\": " + rec(best_k, best_ms) + "}";
    std::snprintf(report, report_cap, "%s", r.c_str());
  }
  return CEM_OK;
}

// ---------------------------------------------------------------------------
// No-allocation variant of cem_step: the workspace is a static device array
// (one copy per GPU, held until the process ends) instead of the bound one.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

__device__ __align__(256) char scratch[CEM_STATIC_WORKSPACE_BYTES];

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the static array on the current device: looked up once
// per device (the host-side name of the array is not a device address).
cem_status static_workspace(char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CEM_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CEM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return CEM_OK;
}

}  // namespace

extern "C" {

cem_status cem_step_static(cem_ctx* c, double* u, double* u_base, double dt, double cfl, int nsteps) {
  if (!c || !u || !u_base) return fail(CEM_EINVAL, "null argument");
  if (u == u_base) return fail(CEM_EINVAL, "u and u_base must differ");
  if (nsteps < 0) return fail(CEM_EINVAL, "nsteps < 0");
  if (!(dt > 0.0) && !(cfl > 0.0)) return fail(CEM_EINVAL, "need dt > 0 or cfl > 0");
  if (c->kind != CEM_EULER && !c->bounds_set && !(std::isfinite(c->prm.u_min) && std::isfinite(c->prm.u_max)))
    return fail(CEM_EINVAL, "scalar bounds not set (cem_params u_min/u_max or cem_set_bounds)");
  if (c->ws_need > (size_t)CEM_STATIC_WORKSPACE_BYTES)
    return fail(CEM_ENOMEM, "problem needs " + std::to_string(c->ws_need) + " workspace bytes; the static "
                "workspace holds " + std::to_string((size_t)CEM_STATIC_WORKSPACE_BYTES));
  char* ws = nullptr;
  cem_status st = static_workspace(&ws);
  if (st != CEM_OK) return st;
  // the context's own binding is set aside for the call and restored after
  struct Saved {
    double *u, *u0;
    char* ws;
    bool bound, bounds_set, fnode_valid;
    int lds_max;
  } sv{c->u, c->u0, c->ws, c->bound, c->bounds_set, c->fnode_valid, c->lds_max};
  auto restore = [&]() {
    c->u = sv.u;
    c->u0 = sv.u0;
    c->ws = sv.ws;
    c->bound = sv.bound;
    c->bounds_set = sv.bounds_set;
    c->fnode_valid = sv.fnode_valid;
    c->lds_max = sv.lds_max;
  };
  c->u = u;
  c->u0 = u_base;
  c->ws = ws;
  c->bound = true;
  c->bounds_set = true;
  {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
      restore();
      return fail(CEM_EHIP, "device query failed");
    }
    c->lds_max = v;
  }
  // tables into the array; counters and the dt / CFL words start at zero
  // (fill kernels, not memset nodes, so that a caller may capture the call)
  hipError_t e = hipMemcpyAsync(c->ws + c->o_tab, c->tabblob.data(), c->tabblob.size() * 8,
                                hipMemcpyHostToDevice, c->stream);
  const int64_t ncnt = (int64_t)c->cnt_slots * 2;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_zero_words, dim3(nblocks(ncnt, 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<unsigned*>(c->ws + c->o_counts), ncnt);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, c->stream, reinterpret_cast<unsigned*>(c->ws + c->o_dtbuf),
                       (int64_t)16);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    restore();
    return fail(CEM_EHIP, std::string("static workspace set-up: ") + hipGetErrorString(e));
  }
  if (c->kind == CEM_KPP) {
    // nodal fluxes of the given state
    StageArgs a = make_args(c);
    hipLaunchKernelGGL((k_nodal_flux<2, KPP>), dim3(nblocks(c->N, 256)), dim3(256), 0, c->stream, a);
    if ((e = hipGetLastError()) != hipSuccess) {
      restore();
      return fail(CEM_EHIP, std::string("k_nodal_flux: ") + hipGetErrorString(e));
    }
  }
  c->fnode_valid = true;
  for (int n = 0; n < nsteps && st == CEM_OK; ++n) st = step_direct(c, dt, cfl);
  restore();
  return st;
}

}  // extern "C"
