// gfx950 kernels of one explicit SSP-RK stage of the limited CG-WENO scheme
// (Kuzmin, Hajduk & Vedral, arXiv:2509.04673, the five-step algorithm of
// Sec. 4.3), on a uniform periodic box of cube cells, Bernstein Q_p.
//
// Data layout (HBM): nodal arrays are structure-of-arrays, component-major,
// u[c * N + node], node = i_0 + L_0 (i_1 + L_1 i_2) with i_k in [0, p n_k).
// Per-element arrays are component-major with the element index fastest,
// x[(c * NL + local) * E + e], so one-thread-per-element stores coalesce.
// Assembly into shared nodes is a node-centric gather in a fixed order (no
// float atomics): results are bitwise reproducible run to run.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace cem {

constexpr int ADV = 0, KPP = 1, EUL = 2, NCV = 3;

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
// k-th base-(p+1) digit of a local id (axis 0 fastest)
__host__ __device__ constexpr int dig(int loc, int k, int P1) {
  return k == 0 ? loc % P1 : dig(loc / P1, k - 1, P1);
}

struct PhysParams {
  double vel[3];
  double vnorm;     // |v| (advection)
  double gam;       // ratio of specific heats (Euler)
  int rn;           // 2 gamma / (gamma - 1) when an integer in [2, 32] (7 for 1.4, 5 for 5/3), else 0
};

struct DevTabs {
  const double* sf;     // compact tables of the sum-factorised kernels (SFLayout)
  const float* sf32;    // the same tables rounded to float (mixed precision)
};

// Compact tables of the sum-factorised element operators: 1D P1 x P1
// matrices (Gauss values, derivatives, weights, mass, stiffness,
// int B_a' B_b, the two extension maps) and the packed semi-norm form.
template <int D, int P> struct SFLayout {
  static constexpr int P1 = P + 1, PP = P1 * P1, NL = ipow(P1, D);
  static constexpr int vq = 0, dq = PP, wq = 2 * PP, g = 3 * PP, k1 = 4 * PP, ct = 5 * PP;
  static constexpr int ext = 6 * PP, qp = 8 * PP;
  static constexpr int total = qp + NL * (NL + 1) / 2;
};

extern __shared__ double cem_smem[];

// read-only element tables (scalar loads: every lane reads the same entry)
// The tables are read through the constant address space: they are not
// written while a kernel runs, so uniform reads become scalar loads into
// SGPRs instead of vector loads that occupy VGPRs.  V: double, or float for
// the contractions of the mixed-precision form.
template <class V> struct TabRef {
  typedef const V __attribute__((address_space(4))) cv;
  const V* g;
  __device__ __forceinline__ V operator()(int i) const { return ((const cv*)g)[i]; }
};

template <class V> struct TabSel;
template <> struct TabSel<double> {
  __device__ static const double* of(const DevTabs& t) { return t.sf; }
};
template <> struct TabSel<float> {
  __device__ static const float* of(const DevTabs& t) { return t.sf32; }
};

struct MeshArgs {
  int n[3];         // elements per axis (1 for unused axes)
  int L[3];         // nodes per axis (1 for unused axes)
  int64_t N, E;
  double h;
  int bnd1d;        // 1: a non-periodic 1D line (L[0] = p n + 1, boundary facets at both ends)
};

// boundary conditions of a non-periodic line (the values of cem_bc_kind)
constexpr int kBcState = 1, kBcOutflow = 2, kBcWall = 3;

struct StageArgs {
  MeshArgs mesh;
  DevTabs tab;
  PhysParams ph;
  double q, rexp, eps, w_lin, eps_pos;
  int gamma_mode, alpha_mode, beta_mode;   // 0 method, 1 force 0, 2 force 1
  int flux_mode;        // 0 flux limiter, dt_e of (40); 1 f = f^H, dt_e of (37); 2 f = f^H, reduced (40)
  double umin, umax, clamp_tol;
  int bounds_local;     // scalar limiters: 0 the global [umin, umax], 1 per-element bounds in bnd
  double* bnd;          // [2][E] per-element lower, upper bounds (bounds_local)
  int contrib_q1;       // scalar Q1: element contributions of Sec. 5.3 (low-order derivative in udot)
  int store_r;          // the assembly fused with the first mass pass also stores r (a debug tap only)
  int fuse_upd;         // 2D systems: 0, or log2 of pass 2's elements per block when pass 2 updates
                        // the nodes whose elements all lie in its block
  int cnt_off;          // first counter slot of the pass-2 blocks (fuse_upd)
  double* fdiv;         // [E] int_dK f_h . n of each element (contrib_q1)
  int bc_kind[2];       // non-periodic line: kBc* of the low and high end
  double bc_u[2][5];    // kBcState: the prescribed conserved state of each end
  double* fbnd;         // non-periodic line: [2 ends][2][M], [.][1] the boundary
                        // facet's boundary flux F(u_end, u_hat; n) (outward)
  const double* u;      // stage input u^(s)   [M][N]
  double* u0;           // step base u^n       [M][N]
  double* uout;         // stage output (may alias u: per-node read-then-write)
  double* g;            // [D][M][N] projected gradient
  double* fnode;        // [D][M][N] nodal fluxes f_k(u_j) of the stage input (kNodal physics)
  double* r;            // [M][N] residual
  double* udot;         // [M][N]
  double* relem;        // [M][NL][E] element vectors (residual, then update)
  double* ue;           // [M][E] cell averages
  double* ubarL;        // [M][E] low-order intermediate averages
  double* ubar;         // [M][E] flux-limited intermediate averages
  double* fahi;         // [D][M][E] raw antidiffusive flux of the +e_k facet
  double* dte;          // [E] pseudo time steps
  double* gam;          // [E] WENO sensor
  double* nu;           // [E] viscosity
  double* beta;         // [E] slope-limiter factor
  // float intermediates of the mixed-precision form (null in float64 runs)
  float* g32;           // [D][M][N]
  float* r32;           // [M][N]
  float* udot32;        // [M][N]
  double* dtbuf;        // [4]: dt, min dt_e, cfl flag, (spare)
  double* dtpart;       // per-block minima of dt_e from the element pass
  int* counts;          // per-block [2]: clamped, violations
  double rk_a, rk_b;    // u_out = a u0 + b u^FE
  int stage;            // 0, 1, 2
  int copy_base;        // stage 0 of a step: write u_base = u before updating
  int ndtpart;          // number of per-block dt_e minima
  int dt_ready;         // 1: k_stage_dt has reduced them into dtbuf
  double dt_fixed, cfl; // stage 0: dt = dt_fixed > 0 ? dt_fixed : cfl min_e dt_e
};

// ---------------------------------------------------------------------------
// physics
// ---------------------------------------------------------------------------
template <int D, int PH> struct Phys;

// flux_all(u, f): all d directional fluxes f[k * M + c] at one state.
// kNodal: the flux is expensive enough (transcendental) that its nodal
// values f(u_j) are computed once per node and stage and stored.
__device__ __forceinline__ void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sin_cos(float x, float* s, float* c) { sincosf(x, s, c); }

template <int D> struct Phys<D, ADV> {
  static constexpr int M = 1;
  static constexpr bool kNodal = false;
  template <class T>
  __device__ static inline void flux_all(const T* u, T* f, const PhysParams& pp) {
#pragma unroll
    for (int k = 0; k < D; ++k) f[k] = (T)pp.vel[k] * u[0];
  }
  template <class T>
  __device__ static inline void flux(int k, const T* u, T* f, const PhysParams& pp) {
    f[0] = (T)pp.vel[k] * u[0];
  }
  __device__ static inline double node_speed(const double*, const PhysParams& pp) { return pp.vnorm; }
  __device__ static inline double riemann_speed(const double*, const double*, int k, const PhysParams& pp) {
    return fabs(pp.vel[k]);
  }
  __device__ static inline double riemann_speed_n(const double*, const double*, const double* n,
                                                  const PhysParams& pp) {
    double vn = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) vn += pp.vel[k] * n[k];
    return fabs(vn);
  }
};

template <int D> struct Phys<D, KPP> {
  static constexpr int M = 1;
  static constexpr bool kNodal = true;
  template <class T>
  __device__ static inline void flux_all(const T* u, T* f, const PhysParams&) {
    T s, c;
    sin_cos(u[0], &s, &c);
    f[0] = s;
    f[1] = c;
  }
  template <class T>
  __device__ static inline void flux(int k, const T* u, T* f, const PhysParams&) {
    T s, c;
    sin_cos(u[0], &s, &c);
    f[0] = (k == 0) ? s : c;
  }
  // |f'(u)| = |(cos u, -sin u)| = 1
  __device__ static inline double node_speed(const double*, const PhysParams&) { return 1.0; }
  __device__ static inline double riemann_speed(const double*, const double*, int, const PhysParams&) {
    return 1.0;
  }
  __device__ static inline double riemann_speed_n(const double*, const double*, const double*, const PhysParams&) {
    return 1.0;
  }
};

// The nonconvex flux of Sec. 5.1.2 on a line: u (1 - u) / 4 for u <= 1/2
// (concave), u (u - 1) / 2 + 3/16 above (convex), C^1 at 1/2.  |f'| is
// piecewise linear with its only minimum (0) at 1/2, so the largest |f'|
// between two states is at one of them.
template <int D> struct Phys<D, NCV> {
  // (instantiated with D = 1 only: the dispatch offers it on lines)
  static constexpr int M = 1;
  static constexpr bool kNodal = false;
  template <class T>
  __device__ static inline T f1(T u) {
    return u <= (T)0.5 ? (T)0.25 * u * ((T)1 - u) : (T)0.5 * u * (u - (T)1) + (T)0.1875;
  }
  __device__ static inline double df(double u) { return u <= 0.5 ? 0.25 - 0.5 * u : u - 0.5; }
  template <class T>
  __device__ static inline void flux_all(const T* u, T* f, const PhysParams&) { f[0] = f1(u[0]); }
  template <class T>
  __device__ static inline void flux(int, const T* u, T* f, const PhysParams&) { f[0] = f1(u[0]); }
  __device__ static inline double node_speed(const double* u, const PhysParams&) { return fabs(df(u[0])); }
  __device__ static inline double riemann_speed(const double* uL, const double* uR, int, const PhysParams&) {
    return fmax(fabs(df(uL[0])), fabs(df(uR[0])));
  }
  __device__ static inline double riemann_speed_n(const double* uL, const double* uR, const double*,
                                                  const PhysParams&) {
    return fmax(fabs(df(uL[0])), fabs(df(uR[0])));
  }
};

// pow kept out of the callers' register allocation (a rarely taken path)
__device__ __attribute__((noinline)) double pow_out_of_line(double x, double y) { return pow(x, y); }

template <int D> struct Phys<D, EUL> {
  static constexpr int M = D + 2;
  static constexpr bool kNodal = false;
  // every quotient by the density is a product with 1 / rho, which the
  // compiler computes once per state however many fluxes, pressures and
  // speeds of that state are formed (one division instead of up to five)
  template <class T>
  __device__ static inline T pressure(const T* u, const PhysParams& pp) {
    T m2 = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) m2 += u[1 + k] * u[1 + k];
    const T ir = (T)1 / u[0];
    return ((T)pp.gam - (T)1) * (u[D + 1] - (T)0.5 * m2 * ir);
  }
  template <class T>
  __device__ static inline void flux(int k, const T* u, T* f, const PhysParams& pp) {
    const T p = pressure(u, pp);
    const T ir = (T)1 / u[0];
    const T vk = u[1 + k] * ir;
    f[0] = u[1 + k];
#pragma unroll
    for (int j = 0; j < D; ++j) f[1 + j] = u[1 + j] * vk + (j == k ? p : (T)0);
    f[D + 1] = vk * (u[D + 1] + p);
  }
  template <class T>
  __device__ static inline void flux_all(const T* u, T* f, const PhysParams& pp) {
#pragma unroll
    for (int k = 0; k < D; ++k) flux(k, u, f + k * M, pp);
  }
  __device__ static inline double node_speed(const double* u, const PhysParams& pp) {
    double v2 = 0.0;
    const double ir = 1.0 / u[0];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double v = u[1 + k] * ir;
      v2 += v * v;
    }
    const double c = sqrt(fmax(0.0, pp.gam * pressure(u, pp) * ir));
    return sqrt(v2) + c;
  }
  // x^n for an integer n >= 1 (repeated squaring)
  __device__ static inline double int_pow(double x, int n) {
    double r = 1.0, b = x;
    for (;;) {
      if (n & 1) r *= b;
      n >>= 1;
      if (!n) return r;
      b *= b;
    }
  }
  // p^(-ex), ex = (gamma - 1) / (2 gamma).  With the integer n = 1 / ex of
  // common gases: p = m 2^e with e = n q + r, 0 <= r < n, so p^(-1/n) =
  // 2^(-q) (m 2^r)^(-1/n); the root of p' = m 2^r in [0.5, 2^31) is Newton's
  // method on p' y^n = 1 from a float seed (hardware log2 / exp2), y <- y
  // (n + 1 - p' y^n) / n, whose relative error (~1e-7) squares to ~1e-12 and
  // then to float64 rounding in the second step.  pow's special values are
  // kept (0 -> inf, inf -> 0, negative or NaN -> NaN).  A double pow costs
  // ~230 instructions here, this ~30; other gases call pow out of line (it
  // would otherwise raise the register pressure of every caller).
  __device__ static inline double p_pow_mex(double p, double ex, const PhysParams& pp) {
    if (!pp.rn) return pow_out_of_line(p, -ex);
    if (!(p > 0.0)) return p == 0.0 ? (double)INFINITY : (double)NAN;
    if (p == (double)INFINITY) return 0.0;
    const int n = pp.rn;
    int e;
    const double m = frexp(p, &e);
    const int q = (int)floorf((float)e / (float)n);
    const double pr = ldexp(m, e - q * n);
    const double inv_n = 1.0 / n;
    double y = (double)exp2f(-log2f((float)pr) / (float)n);
    y *= ((double)(n + 1) - pr * int_pow(y, n)) * inv_n;
    y *= ((double)(n + 1) - pr * int_pow(y, n)) * inv_n;
    return ldexp(y, -q);
  }
  // x^(1 / ex): x^n with the integer n, else pow out of line
  __device__ static inline double pow_inv_ex(double x, double ex, const PhysParams& pp) {
    return pp.rn ? int_pow(x, pp.rn) : pow_out_of_line(x, 1.0 / ex);
  }
  // Guaranteed upper bound of the largest wave speed of the 1D Riemann
  // problem along +e_k: two-rarefaction estimate of the star pressure
  // (Guermond & Popov 2016), an upper bound for 1 < gamma <= 5/3.
  __device__ static inline double riemann_speed(const double* uL, const double* uR, int k,
                                                const PhysParams& pp) {
    const double g = pp.gam;
    const double irL = 1.0 / uL[0], irR = 1.0 / uR[0];
    const double vL = uL[1 + k] * irL, vR = uR[1 + k] * irR;
    const double pL = pressure(uL, pp), pR = pressure(uR, pp);
    const double cL = sqrt(fmax(0.0, g * pL * irL));
    const double cR = sqrt(fmax(0.0, g * pR * irR));
    const double ex = (g - 1.0) / (2.0 * g);
    const double num = fmax(cL + cR - 0.5 * (g - 1.0) * (vR - vL), 0.0);
    const double den = cL * p_pow_mex(pL, ex, pp) + cR * p_pow_mex(pR, ex, pp);
    const double ps = pow_inv_ex(num / den, ex, pp);
    const double kap = (g + 1.0) / (2.0 * g);
    const double l1 = vL - cL * sqrt(1.0 + kap * fmax(0.0, (ps - pL) / pL));
    const double l3 = vR + cR * sqrt(1.0 + kap * fmax(0.0, (ps - pR) / pR));
    return fmax(fmax(-l1, 0.0), fmax(l3, 0.0));
  }
  // the same bound along a unit normal n (the 1D problem sees v . n)
  __device__ static inline double riemann_speed_n(const double* uL, const double* uR, const double* n,
                                                  const PhysParams& pp) {
    const double g = pp.gam;
    double mL = 0.0, mR = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      mL += n[k] * uL[1 + k];
      mR += n[k] * uR[1 + k];
    }
    const double irL = 1.0 / uL[0], irR = 1.0 / uR[0];
    const double vL = mL * irL, vR = mR * irR;
    const double pL = pressure(uL, pp), pR = pressure(uR, pp);
    const double cL = sqrt(fmax(0.0, g * pL * irL));
    const double cR = sqrt(fmax(0.0, g * pR * irR));
    const double ex = (g - 1.0) / (2.0 * g);
    const double num = fmax(cL + cR - 0.5 * (g - 1.0) * (vR - vL), 0.0);
    const double den = cL * p_pow_mex(pL, ex, pp) + cR * p_pow_mex(pR, ex, pp);
    const double ps = pow_inv_ex(num / den, ex, pp);
    const double kap = (g + 1.0) / (2.0 * g);
    const double l1 = vL - cL * sqrt(1.0 + kap * fmax(0.0, (ps - pL) / pL));
    const double l3 = vR + cR * sqrt(1.0 + kap * fmax(0.0, (ps - pR) / pR));
    return fmax(fmax(-l1, 0.0), fmax(l3, 0.0));
  }
};

// Appendix A: largest alpha in [0,1] with ubar + alpha f / mi admissible
// (density, then pressure through P(alpha) >= alpha R), strict margin eps.
template <int D>
__device__ inline double euler_alpha(const double* ub, const double* f, double mi, double eps) {
  const double rho = ub[0], en = ub[D + 1], fr = f[0], fe = f[D + 1];
  double a = 1.0;
  if (mi * rho * (1.0 - eps) + fr < 0.0) a = (1.0 - eps) * (-mi * rho / fr);
  double m2 = 0.0, mf = 0.0, f2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    m2 += ub[1 + k] * ub[1 + k];
    mf += ub[1 + k] * f[1 + k];
    f2 += f[1 + k] * f[1 + k];
  }
  const double Q = mi * (0.5 * m2 - rho * en);
  const double R = rho * fe + en * fr - mf + fmin(0.0, fe * fr - 0.5 * f2) / mi;
  if (R < (1.0 - eps) * Q) a = fmin(a, (1.0 - eps) * Q / R);
  return fmin(a, 1.0);
}

// Boundary data u_hat of end `side` (0 low, 1 high) of a non-periodic line
// for the interior state u: the prescribed state, u itself (outflow) or,
// for Euler, u with reversed momentum (reflecting wall)
template <int M>
__device__ __forceinline__ void bc_ghost(const StageArgs& a, int side, const double* u, double* uh) {
  // (selects with constant indices: the kernel argument is not indexed by a
  // runtime value)
  const int kind = side ? a.bc_kind[1] : a.bc_kind[0];
#pragma unroll
  for (int c = 0; c < M; ++c) uh[c] = kind == kBcState ? (side ? a.bc_u[1][c] : a.bc_u[0][c]) : u[c];
  if (M > 1 && kind == kBcWall) uh[1] = -u[1];
}

// XCD-aware block order: the hardware hands workgroup b to XCD b mod 8, and
// each XCD has its own L2.  Giving XCD x the contiguous range of logical
// blocks [x q + min(x, r), ... + q + (x < r)), q = nb / 8, r = nb mod 8, puts
// neighbouring elements (which share nodes) on the same L2.  A bijection of
// [0, nb).
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / kNumXcd, r = nb - q * kNumXcd;
  const int x = b % kNumXcd, k = b / kNumXcd;
  return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------------------
// index helpers
// ---------------------------------------------------------------------------
// element and node ids are below 2^31 (checked at create): 32-bit division
__device__ inline void elem_coords(int64_t e, const MeshArgs& m, int* ei) {
  const unsigned n0 = (unsigned)m.n[0], n1 = (unsigned)m.n[1];
  unsigned r = (unsigned)e;
  ei[0] = (int)(r % n0);
  r /= n0;
  ei[1] = (int)(r % n1);
  ei[2] = (int)(r / n1);
}

__device__ inline int64_t elem_id(const int* ei, const MeshArgs& m) {
  return ei[0] + (int64_t)m.n[0] * (ei[1] + (int64_t)m.n[1] * ei[2]);
}

__device__ inline int64_t node_stride(int k, const MeshArgs& m) {
  return k == 0 ? 1 : (k == 1 ? (int64_t)m.L[0] : (int64_t)m.L[0] * m.L[1]);
}

// global node offsets along axis k of the local indices a = 0..P of the
// element with periodic coordinate ek in [-n, 2n) (a neighbour's at most one
// period out of range)
template <int P>
__device__ inline void axis_offsets(int ek, int k, const MeshArgs& m, int* off) {
  const int n = m.n[k], L = m.L[k];
  if (ek < 0) ek += n;
  else if (ek >= n) ek -= n;
  const int s = (int)node_stride(k, m);      // node ids are below 2^31
#pragma unroll
  for (int a = 0; a <= P; ++a) {
    int i = P * ek + a;
    if (i >= L) i -= L;
    off[a] = i * s;
  }
}

template <int D, int P>
__device__ inline int local_node(int loc, const int (*off)[P + 1]) {
  int s = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) s += off[k][dig(loc, k, P + 1)];
  return s;
}


// ---------------------------------------------------------------------------
// line operators: out = scale * (M_1D^{-1} or M_1D^{-1} C_1D) applied along
// axis k; one thread per output value; exact periodic rows for short lines,
// rows truncated far below rounding for long ones
// ---------------------------------------------------------------------------
// TI / TO: value types of the input and output arrays; the operator is
// applied in TO (double, or float in the mixed-precision form) with weights
// of that type
struct LineArgs {
  const void* in;
  void* out;
  const void* w;       // [P][taps]
  int taps, first, L, P;
  int64_t stride, total, N;
  double scale;
};

template <class TI, class TO>
__device__ __forceinline__ void k_line_body(const LineArgs& a, int bx) {
  const int64_t t = (int64_t)bx * blockDim.x + threadIdx.x;
  if (t >= a.total) return;
  const TI* in = static_cast<const TI*>(a.in);
  const int64_t c = t / a.N, i = t - c * a.N;
  const int64_t ik = (i / a.stride) % a.L;
  const int64_t base = c * a.N + i - ik * a.stride;
  const int cls = (int)(ik % a.P);
  const TO* w = static_cast<const TO*>(a.w) + (int64_t)cls * a.taps;
  int j = (int)((ik + a.first) % a.L);
  if (j < 0) j += a.L;
  TO acc = 0;
  for (int tt = 0; tt < a.taps; ++tt) {
    acc += w[tt] * (TO)in[base + j * a.stride];
    if (++j == a.L) j = 0;
  }
  static_cast<TO*>(a.out)[t] = (TO)a.scale * acc;
}

template <class TI, class TO>
__global__ void __launch_bounds__(256) k_line(LineArgs a) {
  k_line_body<TI, TO>(a, blockIdx.x);
}

// Register-blocked line operator for long lines (L >= R + TAPS): the rows of
// the periodic inverse decay exponentially, so 2W+1 taps of the infinite-line
// rows reproduce them to 1e-17 of the row peak.  Lanes of a wave take different
// transverse lines at the same run of R consecutive outputs along the axis,
// so every output of a lane shares its node class with the other lanes and
// the weights are wave-uniform (scalar loads); each thread keeps R
// accumulators and streams R + TAPS - 1 inputs once.
// W: half-width; runs of R = P * RE outputs, RE in {1, 2, 4} chosen per
// launch so that small meshes still fill the chip
template <int P> struct LineTaps;
constexpr int kLineMaxRE = 4;
// S: per-class weight stride, 2W+1 taps zero padded to a multiple of every
// run length P * RE
template <int P_, int W_> struct LineTapsBase {
  static constexpr int W = W_;
  static constexpr int S = (2 * W_ + 1 + kLineMaxRE * P_ - 1) / (kLineMaxRE * P_) * (kLineMaxRE * P_);
};
template <> struct LineTaps<1> : LineTapsBase<1, 30> {};
template <> struct LineTaps<2> : LineTapsBase<2, 44> {};
template <> struct LineTaps<3> : LineTapsBase<3, 57> {};
// float operators (mixed precision): rows cut below 1e-9 of their peak
template <int P> struct LineTaps32;
template <> struct LineTaps32<1> : LineTapsBase<1, 18> {};
template <> struct LineTaps32<2> : LineTapsBase<2, 26> {};
template <> struct LineTaps32<3> : LineTapsBase<3, 32> {};
template <int P, class V> struct LineTapsV : LineTaps<P> {};
template <int P> struct LineTapsV<P, float> : LineTaps32<P> {};

struct LineFastArgs {
  const void* in;      // TI
  void* out;           // TO
  const void* w;       // TO [P][S] (taps zero padded), tap t at offset t - W
  int L, axis;
  int L0, L1;
  int64_t N, NT, ntrans;   // NT = N / L lines per component
  int nlb;                 // lines per block (axis 0 LDS kernel)
  int gx;                  // blocks across lines of a 2D grid (batched launches)
  int ky;                  // runs per thread of the strided kernel (tile length 8 R ky)
  int re;                  // run length R = P re of the strided kernel (1 or 2)
};

template <int P, int RE, class TI, class TO>
__global__ void __launch_bounds__(256) k_line_fast(LineFastArgs a) {
  constexpr int W = LineTapsV<P, TO>::W, R = P * RE, S = LineTapsV<P, TO>::S;
  const TI* in = static_cast<const TI*>(a.in);
  TO* out = static_cast<TO*>(a.out);
  const TO* w = static_cast<const TO*>(a.w);
  constexpr int NB = S / R;                       // tap blocks of R (zero padded)
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.ntrans) return;
  const int64_t comp = t / a.NT, rr = t - comp * a.NT;
  int64_t base, sl;
  if (a.axis == 0) {
    base = comp * a.N + rr * a.L0;
    sl = 1;
  } else if (a.axis == 1) {
    const int64_t x = rr % a.L0, z = rr / a.L0;
    base = comp * a.N + x + z * (int64_t)a.L0 * a.L1;
    sl = a.L0;
  } else {
    base = comp * a.N + rr;
    sl = (int64_t)a.L0 * a.L1;
  }
  const int s = blockIdx.y * R;            // first output of the run (uniform)
  int pos = s - W;                         // input feeding tap 0 of output 0
  if (pos < 0) pos += a.L;
  // acc[r] = sum_t w[r % P][t] in[s + r + t - W]; taps are walked in blocks
  // of R with a window of 2R inputs held in registers
  TO acc[R], win[2 * R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    win[r] = (TO)in[base + (int64_t)pos * sl];
    if (++pos == a.L) pos = 0;
  }
  // unrolled so that the loads of several tap blocks are in flight at once
#pragma unroll 8
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      win[R + r] = (TO)in[base + (int64_t)pos * sl];
      if (++pos == a.L) pos = 0;
    }
    const TO* wb = w + b * R;          // weights of taps b*R .. b*R+R-1
#pragma unroll
    for (int tt = 0; tt < R; ++tt) {
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const TO wv = wb[c * S + tt];
#pragma unroll
        for (int r = c; r < R; r += P) acc[r] += wv * win[r + tt];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) win[r] = win[R + r];
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (s + r < a.L) out[base + (int64_t)(s + r) * sl] = acc[r];
}

// One run of R = P * RE outputs of a line operator: acc[r] = sum_t
// w[r % P][t] x(s + r + t - W), with x read through ld(j) for the inputs
// j = 0, 1, ... of the run's window (x(s - W + j)).  Taps are walked in blocks
// of R with a 2R-input register window; weights are wave-uniform.
template <int P, int RE, class LD, class V>
__device__ __forceinline__ void line_run(const V* __restrict__ wg, const LD& ld, V* acc) {
  constexpr int R = P * RE, S = LineTapsV<P, V>::S, NB = S / R;
  // the weights are block-uniform: read through the constant address space
  // (scalar loads, SGPR operands of the FMAs; staging them in LDS instead
  // measured slower)
  typedef const V __attribute__((address_space(4))) CV;
  const CV* w = (const CV*)wg;
  V win[2 * R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) win[r] = ld(r);
#pragma unroll 4
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) win[R + r] = ld((b + 1) * R + r);
    const CV* wb = w + b * R;
#pragma unroll
    for (int tt = 0; tt < R; ++tt) {
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const V wv = wb[c * S + tt];
#pragma unroll
        for (int r = c; r < R; r += P) acc[r] += wv * win[r + tt];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) win[r] = win[R + r];
  }
}

// LDS rows of the axis-0 kernels hold a periodic line padded on both sides,
// row[k] = x((k - W) mod L) for k < line_row_len(L), so that the window of
// every run is a plain slice: run s reads row[s + j], j < S + R.
template <int P, class V>
__host__ __device__ constexpr int line_row_len(int L) {
  return L + LineTapsV<P, V>::S + kLineMaxRE * P;
}

// LDS slot of row position k when the row is read in runs of R: one unused
// slot after every R values when R is even, so that lanes reading runs R
// apart have an odd stride and fall in different LDS banks.  For s a
// multiple of R, lds_slot(s + j) = lds_slot(s) + lds_slot(j).
template <int R>
__host__ __device__ constexpr int lds_slot(int k) {
  return (R % 2 == 0) ? k + k / R : k;
}

// row pitch in LDS slots: enough for every run length the axis-0 kernels use
// (R = P or 2P)
template <int P, class V>
__host__ __device__ constexpr int line_row_pitch(int L) {
  return line_row_len<P, V>(L) + line_row_len<P, V>(L) / (P % 2 == 0 ? P : 2 * P) + 1;
}

// lines per block of the axis-0 kernels (runs of R outputs): enough lines
// for a run per thread of a 256-thread block, up to cap LDS slots per block
template <int P, class V>
__host__ __device__ inline int line_rows_per_block(int L, int64_t nlines, int cap, int R) {
  const int per = cap / line_row_pitch<P, V>(L);
  const int64_t runs = (L + R - 1) / R;
  int64_t want = (256 + runs - 1) / runs;
  if (want > nlines) want = nlines;
  return per < 1 ? 1 : (int)(want < per ? (want < 1 ? 1 : want) : per);
}

// Line operators of a non-periodic 1D line (Mb^{-1} or Mb^{-1} Cb), one
// thread per output value: the first blo and last bhi rows are exact rows
// over the first / last cw nodes, the rows between them the infinite-line
// rows of their node class (i mod p) at offsets -W..W.  Every access stays
// inside the line: blo, bhi >= W, or blo = N with cw = N (short lines).
struct BndLineArgs {
  const double* in;     // [M][N]
  double* out;          // [M][N]
  const double* wf;     // [P][S] the interior rows zero padded to the stride of the
                        // register-blocked runs (k_line_bnd_runs), offsets -W..
  const double* wi;     // [P][2W + 1]
  const double* lo;     // [cw][blo] (by column: consecutive rows, consecutive weights)
  const double* hi;     // [cw][bhi]
  int64_t N, total;     // nodes of the line, M N
  int P, W, blo, bhi, cw;
};

// sum_j w[j ld] x[j], j < n, in four interleaved partial sums (independent
// loads and FMAs in flight: the end-block rows are long serial loops)
__device__ __forceinline__ double dot4(const double* w, int64_t ld, const double* x, int n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = 0;
  for (; j + 4 <= n; j += 4) {
    s0 = fma(w[j * ld], x[j], s0);
    s1 = fma(w[(j + 1) * ld], x[j + 1], s1);
    s2 = fma(w[(j + 2) * ld], x[j + 2], s2);
    s3 = fma(w[(j + 3) * ld], x[j + 3], s3);
  }
  for (; j < n; ++j) s0 = fma(w[j * ld], x[j], s0);
  return (s0 + s1) + (s2 + s3);
}

// output i of component c by its row (end block or interior row); the end
// blocks are stored by column, so the rows of consecutive threads read
// consecutive weights while x[j] is the same address for all of them
__device__ __forceinline__ double line_bnd_row(const BndLineArgs& a, const double* x, int64_t i) {
  if (i < a.blo) return dot4(a.lo + i, a.blo, x, a.cw);
  if (i >= a.N - a.bhi) return dot4(a.hi + (i - (a.N - a.bhi)), a.bhi, x + (a.N - a.cw), a.cw);
  return dot4(a.wi + (int)(i % a.P) * (2 * a.W + 1), 1, x + (i - a.W), 2 * a.W + 1);
}

__device__ __forceinline__ void k_line_bnd_body(const BndLineArgs& a, int bx) {
  const int64_t q = (int64_t)bx * blockDim.x + threadIdx.x;
  if (q >= a.total) return;
  const int64_t c = q / a.N, i = q - c * a.N;
  a.out[q] = line_bnd_row(a, a.in + c * a.N, i);
}

__global__ void __launch_bounds__(256) k_line_bnd(BndLineArgs a) { k_line_bnd_body(a, blockIdx.x); }

// Long lines: a block stages 256 R + S inputs of component blockIdx.y in LDS
// (zero outside the line) and each thread computes a run of R = P RE
// outputs starting at a multiple of R (so output r has class r mod P).  Runs
// that lie inside the interior rows take the register-blocked taps
// (line_run, weights wf); the rows of runs that touch an end block are then
// spread over the block, one row per thread, from global memory.  Every LDS
// slot read lies in the staged window, every global read inside the line.
template <int P, int RE>
__device__ __forceinline__ void k_line_bnd_runs_body(const BndLineArgs& a, int bx, int by) {
  constexpr int W = LineTaps<P>::W, R = P * RE, S = LineTaps<P>::S;
  constexpr int LW = 256 * R + S;                  // staged window
  double* sm = reinterpret_cast<double*>(cem_smem);
  const int64_t N = a.N;
  const int64_t c = by;
  const int64_t s0 = (int64_t)bx * (256 * R);
  const double* x = a.in + c * N;
  const int64_t ws = s0 - W;                      // input of window slot 0
  for (int k = threadIdx.x; k < LW; k += 256) {
    const int64_t g = ws + k;
    sm[lds_slot<R>(k)] = (g >= 0 && g < N) ? x[g] : 0.0;
  }
  __syncthreads();
  const int64_t s = s0 + (int64_t)threadIdx.x * R;
  double* y = a.out + c * N;
  auto interior_run = [&](int64_t rs) { return rs >= a.blo && rs + R <= N - a.bhi; };
  if (s < N && interior_run(s)) {
    // interior: x(s - W + j) = window slot threadIdx.x R + j
    const int off = threadIdx.x * R;
    auto ld = [&](int j) { return sm[lds_slot<R>(off + j)]; };
    double acc[R];
    line_run<P, RE>(a.wf, ld, acc);
#pragma unroll
    for (int r = 0; r < R; ++r) y[s + r] = acc[r];
  }
  // the rows of the other runs of the tile: those of the runs starting
  // below blo, [s0, e1), and of the runs reaching past N - bhi, [s2, te),
  // two lanes per row (each half of the taps, summed by a lane shuffle: the
  // end rows are the block's longest serial chains).  The trip count is the
  // same for the whole block, so every lane reaches the shuffle.
  const int64_t te = s0 + 256 * R < N ? s0 + 256 * R : N;
  auto run_up = [&](int64_t v) { return v <= s0 ? s0 : s0 + (v - s0 + R - 1) / R * R; };
  const int64_t e1 = min(run_up(a.blo), te);
  const int64_t s2 = min(max(run_up(N - a.bhi - R + 1), e1), te);
  const int n1 = (int)(e1 - s0), nend = n1 + (int)(te - s2);
  const int half = threadIdx.x & 1;
  for (int base = 0; base < nend; base += 128) {
    const int r = base + (int)(threadIdx.x >> 1);
    double part = 0.0;
    int64_t i = 0;
    if (r < nend) {
      i = r < n1 ? s0 + r : s2 + (r - n1);
      const double* w;
      const double* xs;
      int64_t ld;
      int n;
      if (i < a.blo) {
        w = a.lo + i, ld = a.blo, xs = x, n = a.cw;
      } else if (i >= N - a.bhi) {
        w = a.hi + (i - (N - a.bhi)), ld = a.bhi, xs = x + (N - a.cw), n = a.cw;
      } else {
        w = a.wi + (int)(i % a.P) * (2 * a.W + 1), ld = 1, xs = x + (i - a.W), n = 2 * a.W + 1;
      }
      const int h0 = n / 2;
      part = half ? dot4(w + h0 * ld, ld, xs + h0, n - h0) : dot4(w, ld, xs, h0);
    }
    const double sum = part + __shfl_xor(part, 1);
    if (r < nend && half == 0) y[i] = sum;
  }
}

template <int P, int RE>
__global__ void __launch_bounds__(256) k_line_bnd_runs(BndLineArgs a) {
  k_line_bnd_runs_body<P, RE>(a, blockIdx.x, blockIdx.y);
}

// x((k - W) mod L) of the padded row position k
__device__ __forceinline__ int line_wrap(int k, int W, int L) {
  int x = k - W;
  while (x < 0) x += L;
  while (x >= L) x -= L;
  return x;
}

// Integer division by a block-uniform divisor d >= 1 without a division
// per use: q = floor(n / d) = umulhi(n, ceil(2^32 / d)) for d >= 2, exact
// whenever n d < 2^32 (the error of the rounded reciprocal, below n / 2^32,
// stays under 1 / d).  The staging and run loops of the line kernels index
// a block's lines with n < 2^17 and d < 2^13.
struct DivMagic {
  unsigned d, m;
  __device__ __forceinline__ explicit DivMagic(unsigned d_) : d(d_), m(d_ > 1u ? 0xFFFFFFFFu / d_ + 1u : 0u) {}
  __device__ __forceinline__ unsigned div(unsigned n) const { return d > 1u ? __umulhi(n, m) : n; }
};

// Axis 0 (contiguous lines): a block stages nlb whole lines in LDS (one
// coalesced copy, periodic wrap inside LDS) and each thread computes runs of
// R outputs.  Consecutive lanes take consecutive runs.
template <int P, int RE, class TI, class TO>
__device__ __forceinline__ void k_line_x_body(const LineFastArgs& a, int bx) {
  constexpr int W = LineTapsV<P, TO>::W, R = P * RE;
  static_assert(R % 2 == 1 || R >= (P % 2 == 0 ? P : 2 * P), "row pitch too short for this run length");
  const int L = a.L;
  TO* sm = reinterpret_cast<TO*>(cem_smem);
  const int64_t t0 = (int64_t)bx * a.nlb;
  const int nl = (int)min((int64_t)a.nlb, a.ntrans - t0);
  const TI* src = static_cast<const TI*>(a.in) + t0 * L;   // lines of axis 0 are contiguous
  const int LS = line_row_len<P, TO>(L), LP = line_row_pitch<P, TO>(L);
  // four values per thread and pass: the loads are issued before the stores
  // (block indices by magic-number division: an integer division per value
  // made the staging cost as much as the taps of the short lines)
  const int nv = nl * LS, nt = (int)blockDim.x;
  const DivMagic dls((unsigned)LS);
  for (int i0 = threadIdx.x; i0 < nv; i0 += 4 * nt) {
    TO v[4];
    int slot[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = i0 + k * nt, line = (int)dls.div((unsigned)i), pos = i - line * LS;
      slot[k] = line * LP + lds_slot<R>(pos);
      v[k] = i < nv ? (TO)src[line * L + line_wrap(pos, W, L)] : (TO)0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i0 + k * nt < nv) sm[slot[k]] = v[k];
  }
  __syncthreads();
  const int runs = (L + R - 1) / R;
  const DivMagic drun((unsigned)runs);
  for (int g = threadIdx.x; g < nl * runs; g += blockDim.x) {
    const int line = (int)drun.div((unsigned)g), s = (g - line * runs) * R;
    const TO* row = sm + line * LP + lds_slot<R>(s);
    auto ld = [&](int j) { return row[lds_slot<R>(j)]; };
    TO acc[R];
    line_run<P, RE>(static_cast<const TO*>(a.w), ld, acc);
    TO* dst = static_cast<TO*>(a.out) + (t0 + line) * L;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (s + r < L) dst[s + r] = acc[r];
  }
}

template <int P, int RE, class TI, class TO>
__global__ void __launch_bounds__(256) k_line_x(LineFastArgs a) {
  k_line_x_body<P, RE, TI, TO>(a, xcd_block(blockIdx.x, gridDim.x));
}

// Axes 1 and 2 (strided lines): a block stages a tile of 32 consecutive
// transverse lines x (TY + S) line positions in LDS (coalesced rows) and
// computes TY = 8R outputs per line; a wave is 32 lines x 2 runs.
constexpr int kTileX = 32;
// Longer tiles re-read less of the 2W halo: a thread computes ky runs
// (rows rg + 8 q, q < ky), the tile covers TY = 8 R ky outputs per line.
// ky: the longest tile that still leaves >= 2048 blocks for one problem.
inline int64_t line_y_blocks(int64_t ntrans, int L, int R, int ky) {
  return (ntrans + kTileX - 1) / kTileX * ((L + 8 * R * ky - 1) / (8 * R * ky));
}

// (and whose tile fits 40 KB of LDS, four blocks per CU)
inline int line_y_runs(int64_t ntrans, int L, int R, int S, int vbytes) {
  for (int ky = 4; ky > 1; ky /= 2)
    if (line_y_blocks(ntrans, L, R, ky) >= 2048 && (8 * R * ky + S) * kTileX * vbytes <= 40960) return ky;
  return 1;
}

// Run length re P of the axis-0 kernels: the longest (re <= rmax) that keeps
// 2^19 threads (longer runs read fewer LDS values per output), at least rmin
inline int line_x_re(int64_t ntrans, int L, int P, int W, int rmin, int rmax) {
  for (int re = rmax; re > rmin; re /= 2)
    if (L >= re * P + 2 * W && ntrans * ((L + re * P - 1) / (re * P)) >= ((int64_t)1 << 19)) return re;
  return rmin;
}

// Run length of the strided kernel: runs of 2P outputs halve the LDS reads
// per output (the window of a run is R + S inputs), at half the threads, so
// they are taken only where 2048 blocks remain
inline int line_y_re(int64_t ntrans, int L, int P, int W) {
  return (L >= 2 * P + 2 * W && line_y_blocks(ntrans, L, 2 * P, 1) >= 2048) ? 2 : 1;
}

template <int P, int RE, class TI, class TO>
__device__ __forceinline__ void k_line_y_body(const LineFastArgs& a, int bx, int by) {
  // rows: the window of the last run reads up to TY + S - 1 (zero-weight tail)
  constexpr int W = LineTapsV<P, TO>::W, R = P * RE;
  const int TY = 8 * R * a.ky, ROWS = TY + LineTapsV<P, TO>::S;
  const int L = a.L;
  TO* sm = reinterpret_cast<TO*>(cem_smem);
  const TI* in = static_cast<const TI*>(a.in);
  const int t0 = bx * kTileX;
  const int s0 = by * TY;
  const int tx = threadIdx.x % kTileX, rg = threadIdx.x / kTileX;   // rg = 0..7
  // base of transverse line t and the stride along the line; 32-bit: every
  // offset is below m N < 2^31 (checked at create)
  auto base_of = [&](int t) -> int {
    const int NT = (int)a.NT, comp = t / NT, rr = t - comp * NT;
    if (a.axis == 1) {
      const int x = rr % a.L0, z = rr / a.L0;
      return comp * (int)a.N + x + z * a.L0 * a.L1;
    }
    return comp * (int)a.N + rr;
  };
  const int sl = (a.axis == 1) ? a.L0 : a.L0 * a.L1;
  const bool have = t0 + tx < a.ntrans;
  const int b = have ? base_of(t0 + tx) : 0;
  int p = s0 - W;
  if (p < 0) p += L;
  p += rg;
  if (p >= L) p -= L;
  // eight rows per pass: the loads are issued before the first LDS store
  int row = rg;
  for (; row + 56 < ROWS; row += 64) {
    TO v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[k] = have ? (TO)in[b + p * sl] : (TO)0;
      p += 8;
      if (p >= L) p -= L;
      if (p >= L) p -= L;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) sm[(row + 8 * k) * kTileX + tx] = v[k];
  }
  for (; row < ROWS; row += 8) {
    sm[row * kTileX + tx] = have ? (TO)in[b + p * sl] : (TO)0;
    p += 8;
    if (p >= L) p -= L;
    if (p >= L) p -= L;
  }
  __syncthreads();
  if (!have) return;
  TO* out = static_cast<TO*>(a.out);
#pragma unroll 1
  for (int q = 0; q < a.ky; ++q) {
    const int row0 = (rg + 8 * q) * R, s = s0 + row0;
    if (s >= L) return;
    const TO* col = sm + row0 * kTileX + tx;
    auto ld = [&](int j) { return col[j * kTileX]; };
    TO acc[R];
    line_run<P, RE>(static_cast<const TO*>(a.w), ld, acc);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (s + r < L) out[b + (s + r) * sl] = acc[r];
  }
}

template <int P, int RE, class TI, class TO>
__global__ void __launch_bounds__(256) k_line_y(LineFastArgs a) {
  k_line_y_body<P, RE, TI, TO>(a, blockIdx.x, blockIdx.y);
}

// The independent projected-gradient passes of all axes in one launch:
// blocks [0, nb[0]) run the axis-0 LDS kernel, the following nb[k] blocks
// the strided kernel of axis k (its 2D grid flattened with gx blocks across
// lines).  Each block runs exactly one body.
struct MultiLineArgs {
  LineFastArgs a[3];
  int nb[3];
  int naxes;
};

template <int P, int REX, int REY, class TI, class TO>
__global__ void __launch_bounds__(256) k_line_multi(MultiLineArgs m) {
  int b = blockIdx.x;
  if (b < m.nb[0]) {
    k_line_x_body<P, REX, TI, TO>(m.a[0], b);
    return;
  }
  b -= m.nb[0];
  for (int k = 1; k < m.naxes; ++k) {
    if (b < m.nb[k]) {
      k_line_y_body<P, REY, TI, TO>(m.a[k], b % m.a[k].gx, b / m.a[k].gx);
      return;
    }
    b -= m.nb[k];
  }
}

// ---------------------------------------------------------------------------
// step 1 of the algorithm: element loop (WENO sensor, viscosity, residual)
// plus the facet data of step 3 (f^H, f^L, lambda, dt_e, low-order average)
// ---------------------------------------------------------------------------
// Reductions over a wave (64 lanes, every lane gets the result) and over a
// block (one LDS slot per wave, one barrier); min and integer sums are exact,
// so the order of the combination does not matter
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// minimum of v over the NT threads of a block, returned to every thread;
// every thread of the block must call it, once per kernel
template <int NT>
__device__ __forceinline__ double block_min(double v) {
  constexpr int NW = NT / 64;
  static_assert(NT % 64 == 0 && NW >= 1, "block of whole waves");
  __shared__ double red[NW];
  v = wave_min(v);
  if constexpr (NW == 1) {
    return v;
  } else {
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = red[0];
#pragma unroll
    for (int k = 1; k < NW; ++k) m = fmin(m, red[k]);
    return m;
  }
}

// minimum of dt_e over the NT threads of a block (threads past the last
// element contribute +inf) written to part[bx] (bx: the block's index)
template <int NT>
__device__ inline void block_min_dt_n(double* part, double v, int bx) {
  const double m = block_min<NT>(v);
  if (threadIdx.x == 0) part[bx] = m;
}

__device__ inline void block_min_dt(double* part, double v, int bx) { block_min_dt_n<128>(part, v, bx); }


// f(integral constant K) for K = 0 .. N-1: a loop whose index is a
// compile-time constant in the body (an axis or a component as a template
// argument)
template <int K> struct IC {
  static constexpr int value = K;
};
template <int N, int K = 0, class F>
__device__ __forceinline__ void static_for(const F& f) {
  if constexpr (K < N) {
    f(IC<K>{});
    static_for<N, K + 1>(f);
  }
}

// component c of a value array computed for all components, as a sum of
// masked terms (exact: one term is v[c], the others are +0).  Where a whole
// flux array is computed only to pick one entry, a select chain was folded
// by the compiler into a dynamically indexed stack array (scratch stores and
// loads); this form stays in registers.
template <int M, class V>
__device__ __forceinline__ V pick_m(const V* v, int c) {
  V r = 0;
#pragma unroll
  for (int k = 0; k < M; ++k) r += (c == k) ? v[k] : (V)0;
  return r;
}

// ---------------------------------------------------------------------------
// Line operators on the matrix cores (float64).  16 lines x TY = 128
// outputs of a line operator are a block-Toeplitz product out[i][j] =
// sum_x K[i][x] in[x][j], K[i][x] = w[i mod P][x - i + W] inside the band
// and 0 outside: eight row groups of 16 outputs, each a chain of NQ =
// ceil((16 + 2W) / 4) V_MFMA_F64_16X16X4_F64 steps along its band.  The
// matrix cores have the vector units' FP64 peak, but the vector kernels read
// S + R staged inputs per R outputs from LDS and were bound by LDS bandwidth
// on the strided axes; here one 512-byte LDS read feeds 1024 multiply-adds.
// Lane layout of the instructions (checked with one-wave probes on gfx950):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// D[4 r + l / 16][l % 16] in result r for float64, D[4 (l / 16) + r][l % 16]
// for float (the mixed form's line passes, V_MFMA_F32_16X16X4_F32).  The strided axes multiply K (A) by
// the staged inputs (B), so a result row is one output position across 16
// consecutive lines (a 128-byte store); axis 0 multiplies the transposed
// product, inputs as A and K as B, so a result row is 16 consecutive
// outputs of one line.
//
// A block walks a segment of its 16 lines in chunks of TY outputs.  The
// staged rows live in an LDS ring of 256 rows: chunk c reads rows base ..
// base + TY + HALO - 1 (mod 256), base = c TY; the TY new rows of chunk c+1
// are loaded into registers before chunk c's products and stored after
// them, over rows the next chunk no longer needs (TY + HALO <= 256), so the
// halo is read from HBM once per segment and the loads overlap the matrix
// work.
// ---------------------------------------------------------------------------
typedef double cem_v4d __attribute__((ext_vector_type(4)));
typedef float cem_v4f __attribute__((ext_vector_type(4)));
constexpr int kMfmaLines = 16;     // lines per block
constexpr int kMfmaTY = 128;       // outputs per chunk (8 row groups of 16)
constexpr int kMfmaRing = 256;     // LDS ring rows
template <class V> struct MfmaV;
template <> struct MfmaV<double> {
  typedef cem_v4d acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // result row of register r in lane l (kk = l / 16): 4 r + kk
  static __device__ __forceinline__ int row(int r, int kk) { return 4 * r + kk; }
};
template <> struct MfmaV<float> {
  typedef cem_v4f acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // the float instruction groups its result rows by lane: 4 kk + r (probed)
  static __device__ __forceinline__ int row(int r, int kk) { return 4 * kk + r; }
};
template <int P, class V = double> struct MfmaLine {
  static constexpr int W = LineTapsV<P, V>::W, S = LineTapsV<P, V>::S;
  static constexpr int NQ = (16 + 2 * W + 3) / 4;   // band steps of 4 inputs
  static constexpr int HALO = 4 * NQ - 16;          // staged rows beyond the TY outputs
  static_assert(kMfmaTY + HALO <= kMfmaRing, "chunk and halo must fit the ring");
  // K's row groups are alike when P divides 16 (chunk starts are multiples
  // of 16): the K operand of every step stays in registers; for P = 3 it is
  // read from the weights staged in LDS
  static constexpr bool KREG = 16 % P == 0;
};

// LDS bytes of a block
template <int P, class V = double>
__host__ __device__ constexpr size_t line_mfma_lds() {
  return (size_t)kMfmaRing * kMfmaLines * sizeof(V) +
         (MfmaLine<P, V>::KREG ? 0 : (size_t)P * MfmaLine<P, V>::S * sizeof(V));
}

// block (bx, by): lines bx*16 .. +15, outputs [by a.ky TY, (by + 1) a.ky TY)
// of them (a.ky chunks per segment).  TI: input values (converted to TO as
// they are staged); TO: the operator's type (float64 or float, the mixed
// form), with float accumulation in the float case as in the vector kernels
template <int P, bool AX0, class TI, class TO>
__device__ __forceinline__ void k_line_mfma_body(const LineFastArgs& a, int bx, int by) {
  using ML = MfmaLine<P, TO>;
  using MV = MfmaV<TO>;
  constexpr int W = ML::W, S = ML::S, NQ = ML::NQ, LW = kMfmaLines, TY = kMfmaTY, RB = kMfmaRing;
  constexpr int ROWS = TY + ML::HALO, NV = TY / 16;
  const int L = a.L;
  TO* sm = reinterpret_cast<TO*>(cem_smem);
  TO* wsm = sm + RB * LW;
  const TI* in = static_cast<const TI*>(a.in);
  TO* out = static_cast<TO*>(a.out);
  const TO* w = static_cast<const TO*>(a.w);
  const int t0 = bx * LW, seg0 = by * a.ky * TY;
  const int nch = min(a.ky, (L - seg0 + TY - 1) / TY);
  const int ntrans = (int)a.ntrans;
  // offset of line t (32-bit: every offset is below m N < 2^31) and the
  // stride along it; the lines of axis 0 are contiguous
  auto base_of = [&](int t) -> int {
    if constexpr (AX0) return t * L;
    const int NT = (int)a.NT, comp = t / NT, rr = t - comp * NT;
    if (a.axis == 1) {
      const int x = rr % a.L0, z = rr / a.L0;
      return comp * (int)a.N + x + z * a.L0 * a.L1;
    }
    return comp * (int)a.N + rr;
  };
  const int sl = AX0 ? 1 : (a.axis == 1 ? a.L0 : a.L0 * a.L1);
  // staging: thread (j, r0) = (tid % 16, tid / 16) takes rows r0 + 16 k of
  // line j.  A row of the strided axes is one contiguous segment of 16
  // values; on axis 0 four lanes read four contiguous values of one line.
  const int j = threadIdx.x & (LW - 1), r0 = threadIdx.x >> 4;
  const bool have = t0 + j < ntrans;
  const int lb = have ? base_of(t0 + j) : 0;
  auto wrap = [&](int p) {
    while (p < 0) p += L;
    while (p >= L) p -= L;
    return p;
  };
  // chunk 0: ring rows 0 .. ROWS-1 = positions seg0 - W + row
  {
    int p = wrap(seg0 - W + r0);
    int row = r0;
    for (; row + 112 < ROWS; row += 128) {
      TO v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        v[k] = have ? (TO)in[lb + p * sl] : (TO)0;
        p += 16;
        if (p >= L) p -= L;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) sm[(row + 16 * k) * LW + j] = v[k];
    }
    for (; row < ROWS; row += 16) {
      sm[row * LW + j] = have ? (TO)in[lb + p * sl] : (TO)0;
      p += 16;
      if (p >= L) p -= L;
    }
    if constexpr (!ML::KREG)
      for (int i = threadIdx.x; i < P * S; i += blockDim.x) wsm[i] = w[i];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ii = lane & 15, kk = lane >> 4;
  // K operand of band step q: K[ii][kk] of the step = w[class][4 q + kk - ii]
  TO kreg[ML::KREG ? NQ : 1];
  if constexpr (ML::KREG) {
    const int cls = ii % P;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int t = 4 * q + kk - ii;
      kreg[q] = (t >= 0 && t < S) ? w[cls * S + t] : (TO)0;
    }
  }
  __syncthreads();
  const int oline = t0 + ii;                 // strided axes: this lane's output line
  const int ob = oline < ntrans ? base_of(oline) : 0;
  for (int c = 0; c < nch; ++c) {
    const int s = seg0 + c * TY, base = (c * TY) & (RB - 1);
    // the next chunk's new rows (positions s + TY - W + HALO + r0 + 16 k)
    const bool more = c + 1 < nch;
    TO v[NV];
    if (more) {
      int p = wrap(s + TY - W + ML::HALO + r0);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        v[k] = have ? (TO)in[lb + p * sl] : (TO)0;
        p += 16;
        if (p >= L) p -= L;
      }
    }
    // wave wv: row groups wv and wv + 4, two independent chains
    typename MV::acc acc[2];
    int cls[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      acc[h] = typename MV::acc{0, 0, 0, 0};
      cls[h] = (s + 16 * (wv + 4 * h) + ii) % P;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        TO kv;
        if constexpr (ML::KREG) {
          kv = kreg[q];
        } else {
          const int t = 4 * q + kk - ii;
          kv = (t >= 0 && t < S) ? wsm[cls[h] * S + t] : (TO)0;
        }
        const int row = (base + 16 * (wv + 4 * h) + 4 * q + kk) & (RB - 1);
        const TO xv = sm[row * LW + ii];
        acc[h] = AX0 ? MV::mma(xv, kv, acc[h]) : MV::mma(kv, xv, acc[h]);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = wv + 4 * h;
      if constexpr (AX0) {
        const int pos = s + 16 * g + ii;
        if (pos < L) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int line = t0 + MV::row(r, kk);
            if (line < ntrans) out[line * L + pos] = acc[h][r];
          }
        }
      } else if (oline < ntrans) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int pos = s + 16 * g + MV::row(r, kk);
          if (pos < L) out[ob + pos * sl] = acc[h][r];
        }
      }
    }
    if (!more) break;
    __syncthreads();     // every wave is done with chunk c's rows
#pragma unroll
    for (int k = 0; k < NV; ++k) sm[((base + ROWS + r0 + 16 * k) & (RB - 1)) * LW + j] = v[k];
    __syncthreads();
  }
}

template <int P, bool AX0, class TI, class TO>
__global__ void __launch_bounds__(256) k_line_mfma(LineFastArgs a) {
  k_line_mfma_body<P, AX0, TI, TO>(a, blockIdx.x, blockIdx.y);
}

// chunks per segment of an MFMA line block: whole lines unless fewer than
// min_blocks blocks would result, then segments of ceil(chunks / k) chunks
inline int line_mfma_chunks(int64_t ntrans, int L, int64_t min_blocks) {
  const int64_t gx = (ntrans + kMfmaLines - 1) / kMfmaLines;
  const int chunks = (L + kMfmaTY - 1) / kMfmaTY;
  int nseg = 1;
  while (nseg < chunks && gx * nseg < min_blocks) ++nseg;
  return (chunks + nseg - 1) / nseg;
}

// ---------------------------------------------------------------------------
// sum-factorised element operators
// ---------------------------------------------------------------------------
// y = (A along axis K) x with the P1 x P1 table A at offset ao:
// y[i] = sum_b A[i_K][b] x[i | i_K = b]  (TRN: A[b][i_K])
template <int D, int P, int K, class TB, class V>
__device__ __forceinline__ void ax1(const TB& T, int ao, bool trn, const V* x, V* y) {
  constexpr int P1 = P + 1, NL = ipow(P1, D), ST = ipow(P1, K);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int ai = (i / ST) % P1, i0 = i - ai * ST;
    V s = 0;
#pragma unroll
    for (int b = 0; b < P1; ++b) s += T(ao + (trn ? b * P1 + ai : ai * P1 + b)) * x[i0 + b * ST];
    y[i] = s;
  }
}

template <int D, int P, class TB, class V>
__device__ __forceinline__ void ax(int k, const TB& T, int ao, bool trn, const V* x, V* y) {
  if (k == 0) ax1<D, P, 0>(T, ao, trn, x, y);
  else if constexpr (D > 1) {
    if (k == 1) ax1<D, P, 1>(T, ao, trn, x, y);
    else if constexpr (D > 2) ax1<D, P, 2>(T, ao, trn, x, y);
  }
}

// y = (A_{D-1} (x) ... (x) A_0) x with table offsets mo[j] along axis j
template <int D, int P, class TB, class V>
__device__ __forceinline__ void tensor_apply(const TB& T, const int* mo, bool trn, const V* x, V* y) {
  constexpr int NL = ipow(P + 1, D);
  if constexpr (D == 0) {
    y[0] = x[0];
  } else {
    V t[NL];
    ax<D, P>(0, T, mo[0], trn, x, D == 1 ? y : t);
    if constexpr (D == 2) ax<D, P>(1, T, mo[1], trn, t, y);
    if constexpr (D == 3) {
      V t2[NL];
      ax<D, P>(1, T, mo[1], trn, t, t2);
      ax<D, P>(2, T, mo[2], trn, t2, y);
    }
  }
}

// x^T Q x with Q packed as upper-triangle rows (off-diagonals doubled)
template <int NL, class TB, class V>
__device__ __forceinline__ V qsym(const TB& T0, int off, const V* x) {
  // The coefficients are block-uniform scalar loads.  Issued all at once
  // (NL (NL+1)/2 of them) they overflow the SGPRs and get parked in VGPR
  // lanes, one v_readlane per use; tying the pointer of every third row to
  // the running sum makes the loads stream row group by row group.
  TB T = T0;
  V s = 0;
  int p = off;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    if (i % 3 == 0) asm volatile("" : "+s"(T.g) : "v"(s));
    V t = T(p++) * x[i];
#pragma unroll
    for (int j = i + 1; j < NL; ++j) t += T(p++) * x[j];
    s += x[i] * t;
  }
  return s;
}

// int over the reference cell of d/dt_k B_i: +-1/(p+1)^(d-1) on the two
// facets normal to axis k, 0 elsewhere (exact, used by the mixed form to
// move the flux of the cell average between element and assembled terms)
template <int D, int P>
__device__ __forceinline__ double ref_grad_int(int i, int k) {
  constexpr double w = 1.0 / ipow(P + 1, D - 1);
  const int ik = dig(i, k, P + 1);
  return ik == P ? w : (ik == 0 ? -w : 0.0);
}

// Node access of the element passes.  GlobalNodes gathers straight from the
// nodal arrays; TileNodes2 reads a block's LDS tile (2D): u with a
// one-element halo (the WENO candidates and facet neighbours) and, when it
// fits, g on the block's own nodes.
template <int D, int P, int M> struct GlobalNodes {
  const StageArgs* a;
  int ei[3];
  int off[D][P + 1];
  __device__ __forceinline__ GlobalNodes(const StageArgs& a_, int64_t e) : a(&a_) {
    elem_coords(e, a_.mesh, ei);
#pragma unroll
    for (int k = 0; k < D; ++k) axis_offsets<P>(ei[k], k, a_.mesh, off[k]);
  }
  __device__ __forceinline__ void load_own(double (*U)[ipow(P + 1, D)]) const {
    constexpr int NL = ipow(P + 1, D);
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int64_t nd = local_node<D, P>(j, off);
#pragma unroll
      for (int c = 0; c < M; ++c) U[c][j] = a->u[c * a->mesh.N + nd];
    }
  }
  // neighbour l = 2k + (s > 0) across the facet normal to axis k
  __device__ __forceinline__ void load_nbr(int c, int l, double* cn) const {
    constexpr int NL = ipow(P + 1, D);
    const int k = l / 2, s = (l % 2) ? 1 : -1;
    int offn[D][P + 1];
#pragma unroll
    for (int kk = 0; kk < D; ++kk) axis_offsets<P>(ei[kk] + (kk == k ? s : 0), kk, a->mesh, offn[kk]);
#pragma unroll
    for (int j = 0; j < NL; ++j) cn[j] = a->u[c * a->mesh.N + local_node<D, P>(j, offn)];
  }
  __device__ __forceinline__ int own_node(int j) const { return local_node<D, P>(j, off); }
  // coefficient j of component c, re-read (not merged with earlier reads of
  // the same value: the offset passes through an empty asm)
  __device__ __forceinline__ double own(int c, int j) const {
    int nd = local_node<D, P>(j, off);
    asm volatile("" : "+v"(nd));
    return a->u[c * a->mesh.N + nd];
  }
  // direction k of the projected gradient of component c
  template <class V>
  __device__ __forceinline__ void load_grad_k(int c, int k, V* gk) const {
    constexpr int NL = ipow(P + 1, D);
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int64_t q = ((int64_t)k * M + c) * a->mesh.N + local_node<D, P>(j, off);
      if constexpr (sizeof(V) == 4) gk[j] = a->g32[q];
      else gk[j] = a->g[q];
    }
  }
  // projected gradient: g (float64) or g32 (mixed precision)
  template <class V>
  __device__ __forceinline__ void load_grad(int c, V (*gk)[ipow(P + 1, D)]) const {
    constexpr int NL = ipow(P + 1, D);
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int64_t nd = local_node<D, P>(j, off);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const int64_t q = ((int64_t)k * M + c) * a->mesh.N + nd;
        if constexpr (sizeof(V) == 4) gk[k][j] = a->g32[q];
        else gk[k][j] = a->g[q];
      }
    }
  }
};

template <int P, int M> struct Tile2 {
  static constexpr int TEX = 16, TEY = 8;                       // elements per block
  static constexpr int NX = P * (TEX + 2) + 1, NY = P * (TEY + 2) + 1, NXY = NX * NY;
  static constexpr int GX = P * TEX + 1, GY = P * TEY + 1, GXY = GX * GY;
  static constexpr bool stage_g = M * NXY + 2 * M * GXY <= 4096;
  static constexpr int words = M * NXY + (stage_g ? 2 * M * GXY : 0);
};

template <int P, int M> struct TileNodes2 {
  using TT = Tile2<P, M>;
  static constexpr int NL = (P + 1) * (P + 1);
  const StageArgs* a;
  int base, gbase;          // tile offsets of local node (0, 0)
  GlobalNodes<2, P, M> gl;  // fallback for g when it is not staged
  __device__ __forceinline__ TileNodes2(const StageArgs& a_, int64_t e, int tx, int ty)
      : a(&a_), gl(a_, e) {
    base = P * (ty + 1) * TT::NX + P * (tx + 1);
    gbase = P * ty * TT::GX + P * tx;
  }
  __device__ __forceinline__ int64_t own_node(int j) const { return gl.own_node(j); }
  __device__ __forceinline__ void load_own(double (*U)[NL]) const {
#pragma unroll
    for (int j = 0; j < NL; ++j)
#pragma unroll
      for (int c = 0; c < M; ++c) U[c][j] = cem_smem[c * TT::NXY + base + (j / (P + 1)) * TT::NX + j % (P + 1)];
  }
  // coefficient j of component c, re-read from the tile (see GlobalNodes)
  __device__ __forceinline__ double own(int c, int j) const {
    int o = base;
    asm volatile("" : "+v"(o));
    return cem_smem[c * TT::NXY + o + (j / (P + 1)) * TT::NX + j % (P + 1)];
  }
  __device__ __forceinline__ void load_nbr(int c, int l, double* cn) const {
    const int k = l / 2, s = (l % 2) ? 1 : -1;
    const int b = base + s * P * (k == 0 ? 1 : TT::NX);
#pragma unroll
    for (int j = 0; j < NL; ++j) cn[j] = cem_smem[c * TT::NXY + b + (j / (P + 1)) * TT::NX + j % (P + 1)];
  }
  template <class V>
  __device__ __forceinline__ void load_grad_k(int c, int k, V* gk) const {
    if constexpr (TT::stage_g) {
      const double* gs = cem_smem + M * TT::NXY;
#pragma unroll
      for (int j = 0; j < NL; ++j)
        gk[j] = (V)gs[(k * M + c) * TT::GXY + gbase + (j / (P + 1)) * TT::GX + j % (P + 1)];
    } else {
      gl.load_grad_k(c, k, gk);
    }
  }
  template <class V>
  __device__ __forceinline__ void load_grad(int c, V (*gk)[NL]) const {
    if constexpr (TT::stage_g) {
      const double* gs = cem_smem + M * TT::NXY;
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < NL; ++j)
          gk[k][j] = (V)gs[(k * M + c) * TT::GXY + gbase + (j / (P + 1)) * TT::GX + j % (P + 1)];
    } else {
      gl.load_grad(c, gk);
    }
  }
};

// Subcell bound dt_e^max of Lemma 1 (eq. 37): over the boundary nodes i,
// c_i = int_dK phi_i n = h^{d-1}/(p+1)^{d-1} sum over the facets holding i of
// their outward normals, lambda_0i the Riemann speed of (u_0, u_i) along
// c_i / |c_i|, m_i = h^d / (p+1)^d; u_0 the mean of the interior nodes and
// s = 1, or for Q1 u_0 = u^e, m_0 = |K| and s = 2.
//
// |c_j| lambda_0j of local node j (0 for an interior node)
template <int D, int P, class PHY>
__device__ inline double subcell_node(int j, const double* u0, const double* uj, double h, const PhysParams& ph) {
  constexpr int P1 = P + 1;
  double cf = 1.0;
#pragma unroll
  for (int k = 0; k < D - 1; ++k) cf *= h * (1.0 / P1);
  double cv[3] = {0.0, 0.0, 0.0};
  int nf = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int dk = dig(j, k, P1);
    if (dk == P) { cv[k] = 1.0; ++nf; }
    else if (dk == 0) { cv[k] = -1.0; ++nf; }
  }
  if (nf == 0) return 0.0;
  const double nrm = sqrt((double)nf);
  double n[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) n[k] = cv[k] / nrm;
  return cf * nrm * PHY::riemann_speed_n(u0, uj, n, ph);
}

// the bound from min_j m_j / (|c_j| lambda_0j) over the boundary nodes and
// the sum of |c_j| lambda_0j
template <int D, int P>
__device__ inline double subcell_combine(double tnode, double csum, double h) {
  constexpr int NL = ipow(P + 1, D), NI = ipow(P - 1, D);
  double hd = 1.0;
#pragma unroll
  for (int k = 0; k < D; ++k) hd *= h;
  const double m0 = NI > 0 ? NI * hd * (1.0 / NL) : hd;
  const double t = fmin(tnode, csum > 0.0 ? m0 / csum : 1.0e300);
  return NI > 0 ? t : 0.5 * t;
}

template <int D, int P>
__device__ inline bool interior_node(int j) {
  bool in = true;
#pragma unroll
  for (int k = 0; k < D; ++k) in = in && dig(j, k, P + 1) != 0 && dig(j, k, P + 1) != P;
  return in;
}

// U(c, j): coefficient j of component c
template <int D, int P, class PHY, class UA>
__device__ inline double subcell_dt(const UA& U, const double* ue, double h, const PhysParams& ph) {
  constexpr int NL = ipow(P + 1, D), M = PHY::M, NI = ipow(P - 1, D);
  double hd = 1.0;
#pragma unroll
  for (int k = 0; k < D; ++k) hd *= h;
  const double mi = hd * (1.0 / NL);
  double u0[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NL; ++j)
      if (interior_node<D, P>(j)) s += U(c, j);
    u0[c] = NI > 0 ? s * (1.0 / (NI > 0 ? NI : 1)) : ue[c];
  }
  double tnode = 1.0e300, csum = 0.0;
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    double uj[M];
#pragma unroll
    for (int c = 0; c < M; ++c) uj[c] = U(c, j);
    const double cl = subcell_node<D, P, PHY>(j, u0, uj, h, ph);
    if (cl > 0.0) tnode = fmin(tnode, mi / cl);
    csum += cl;
  }
  return subcell_combine<D, P>(tnode, csum, h);
}

// Exchange of gamma_e and nu_e between the two roles of a split element
// pass: ROLE 1 computes the sensor, the viscosity and the facet data, ROLE 2
// the element residual of the same element, each in its own thread; ROLE 0
// does everything.  Each role passes the exchange barrier exactly once.
struct NoXchg {
  __device__ void put(double, double) const {}
  __device__ void sync() const {}
  __device__ void get(double&, double&) const {}
};
struct LdsXchg {
  double* slot;    // gamma at slot[0], nu at slot[stride] (LDS)
  int stride;
  __device__ void put(double gam, double nu) const {
    slot[0] = gam;
    slot[stride] = nu;
  }
  __device__ void sync() const { __syncthreads(); }
  __device__ void get(double& gam, double& nu) const {
    gam = slot[0];
    nu = slot[stride];
  }
};

// RT: value type of the sensor and residual contractions (double, or float
// in the mixed-precision form); cell averages, facet data and dt_e are
// always float64.  ROLE: 0 the whole pass; two threads per element: 1 the
// sensor, viscosity and facets, 2 the residual; three threads per element:
// 3 the sensor and viscosity, 2 the residual, 4 the facets.  Roles 1 and 3
// hand gamma_e and nu_e to role 2 through xc; every role passes xc's one
// barrier once.
template <int D, int P, int PH, bool WS, class RT, class NS, int ROLE = 0, class XC = NoXchg>
__device__ __forceinline__ double elem1_body(const StageArgs& a, int64_t e, const NS& ns, const XC& xc = XC()) {
  using PHY = Phys<D, PH>;
  using SF = SFLayout<D, P>;
  constexpr int P1 = P + 1, NL = ipow(P1, D), M = PHY::M, NF = NL / P1;
  constexpr bool MIX = sizeof(RT) == 4;
  const TabRef<RT> T{TabSel<RT>::of(a.tab)};
  const MeshArgs& ms = a.mesh;
  const int64_t E = ms.E;
  const double h = ms.h;
  // systems keep no register copy of the element's coefficients: they are
  // read from the tile (or memory) where they are needed (with the one
  // thread per element of the 2D Euler tile, the copy, the candidate
  // extensions and the facet section's temporaries took more than 256
  // registers and spilled)
  constexpr bool KEEPU = M == 1;
  double U[KEEPU ? M : 1][KEEPU ? NL : 1];
  if constexpr (KEEPU) ns.load_own(U);
  auto Uc = [&](int c, int j) -> double {
    if constexpr (KEEPU) return U[c][j];
    else return ns.own(c, j);
  };
  double ue[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NL; ++j) s += Uc(c, j);
    ue[c] = s * (1.0 / NL);
  }

  // nodal fluxes of the facet nodes (stored by the previous update), read
  // before the sensor's arithmetic: the facet section uses them last
  constexpr bool kPre = PHY::kNodal && (ROLE == 0 || ROLE == 1 || ROLE == 4);
  double fpre[kPre ? D : 1][2][kPre ? NL : 1][M];
  if constexpr (kPre) {
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int j = 0; j < NL; ++j) {
          if (dig(j, k, P1) != (side ? P : 0)) continue;
          const int64_t nd = ns.own_node(j);
#pragma unroll
          for (int c = 0; c < M; ++c) fpre[k][side][j][c] = a.fnode[((int64_t)k * M + c) * ms.N + nd];
        }
  }

  // ---- WENO sensor (Sec. 2.2, eqs. 7-8), per component; systems take the
  // minimum.  Candidates are extended into K_e by the blossom maps; every
  // semi-norm is the same packed quadratic form on coefficients shifted by
  // their first entry (exactly zero for constant polynomials).  The
  // nonlinear weights share one denominator, so sum_l w_l (u - u_l) builds
  // up with unnormalised weights as each candidate is formed and is scaled
  // once at the end: every candidate is extended once.
  double nbr_mean[2 * D][M];
  double gam = 0.0, nu = 0.0;
  if constexpr (ROLE == 4) {
    // the facets need the neighbours' cell averages (as the sensor takes them)
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
      for (int l = 0; l < 2 * D; ++l) {
        double cn[NL], sum = 0.0;
        ns.load_nbr(c, l, cn);
#pragma unroll
        for (int j = 0; j < NL; ++j) sum += cn[j];
        nbr_mean[l][c] = sum * (1.0 / NL);
      }
  }
  if constexpr (ROLE != 2 && ROLE != 4) {
  double gmin = 1.0;
  const bool sense = a.gamma_mode == 0;
  const RT wl0 = (RT)(1.0 - 2 * D * a.w_lin), wlin = (RT)a.w_lin, eps = (RT)a.eps;
  auto nrm = [&](RT b) { return (a.rexp == 2.0) ? b : (RT)pow((double)b, 0.5 * a.rexp); };
  for (int c = 0; c < M; ++c) {
    RT ct[NL];
    // systems: the component is a runtime value here, so the coefficients
    // are re-read (U[c][j] would index a register array dynamically)
    const double u00 = M > 1 ? ns.own(c, 0) : Uc(0, 0);
#pragma unroll
    for (int j = 0; j < NL; ++j) ct[j] = (RT)((M > 1 ? ns.own(c, j) : Uc(0, j)) - u00);
    const RT beta0 = qsym<NL>(T, SF::qp, ct);
    RT wsum = wl0 / (nrm(beta0) + eps);
    RT w[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) w[j] = 0;
#pragma unroll
    for (int l = 0; l < 2 * D; ++l) {
      double cn[NL], sum = 0.0;
      RT cr[NL], xe[NL];
      ns.load_nbr(c, l, cn);
      if constexpr (M == 1) {
        // systems recompute the neighbour means in the facet section (a
        // register array indexed by the runtime component would sit in
        // scratch, and these values would stay live through the residual)
#pragma unroll
        for (int j = 0; j < NL; ++j) sum += cn[j];
        nbr_mean[l][c] = sum * (1.0 / NL);
      }
      if (!sense) continue;
#pragma unroll
      for (int j = 0; j < NL; ++j) cr[j] = (RT)(cn[j] - cn[0]);
      ax<D, P>(l / 2, T, SF::ext + (l % 2) * P1 * P1, false, cr, xe);
      RT wt = wlin / (nrm(qsym<NL>(T, SF::qp, xe)) + eps);
      if constexpr (D == 1) {
        // a boundary facet of a non-periodic line has no neighbour: its
        // candidate is absent
        if (ms.bnd1d && ((l == 0 && e == 0) || (l == 1 && e == E - 1))) wt = 0;
      }
      wsum += wt;
#pragma unroll
      for (int i = 0; i < NL; ++i) w[i] += wt * (ct[i] - xe[i]);
    }
    if (!sense) continue;
    const RT iws = (RT)1 / wsum;
#pragma unroll
    for (int i = 0; i < NL; ++i) w[i] *= iws;
    // the ratio of eq. (7) is 0/0 on constant elements; it is regularised
    // with the weights' epsilon: ||u - u*|| / (||u||^2 + eps)^(1/2)
    const RT q2 = qsym<NL>(T, SF::qp, w);
    const RT dev = sqrt(q2 > (RT)0 ? q2 : (RT)0);
    const RT b0 = beta0 > (RT)0 ? beta0 : (RT)0;
    RT ratio = dev / sqrt(b0 + eps);
    ratio = ratio < (RT)1 ? ratio : (RT)1;
    const double gc = 1.0 - (a.q == 1.0 ? (double)ratio : pow((double)ratio, a.q));
    gmin = fmin(gmin, gc);
  }
  gam = a.gamma_mode == 0 ? gmin : (a.gamma_mode == 1 ? 0.0 : 1.0);

  // ---- viscosity nu_e = lambda_e h / (2p), lambda_e the largest nodal speed
  double lam = 0.0;
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    double uj[M];
#pragma unroll
    for (int c = 0; c < M; ++c) uj[c] = Uc(c, j);
    lam = fmax(lam, PHY::node_speed(uj, a.ph));
  }
  nu = lam * h / (2.0 * P);
  }   // roles 0, 1 and 3
  if constexpr (ROLE == 1 || ROLE == 3) {
    xc.put(gam, nu);
    xc.sync();
  }
  if constexpr (ROLE == 3) {
    a.gam[e] = gam;
    a.nu[e] = nu;
    return 1.0e300;
  }

  // ---- element residual R_i = int grad phi_i . f(u_h) - s_h^e(phi_i, u_h),
  // sum-factorised: interpolate to the Gauss points, evaluate the flux, test
  // with the gradients (transposed 1D tables)
  double hpow = 1.0;
#pragma unroll
  for (int k = 0; k < D - 1; ++k) hpow *= h;   // h^{D-1}
  // Mixed form (deviation form): the float contractions act on U - ubar and
  // on f(u_h) - f(ubar) (fluxes evaluated in float64); a constant flux
  // contributes exactly zero to the element residual minus the boundary
  // integral, so float rounding scales with the variation inside the
  // element, not with the size of u or f.
  double foa[D * M];
  PHY::flux_all(ue, foa, a.ph);          // fluxes of the own average
  // systems: the residual one component at a time (SEQ): the Gauss-point
  // states of all components stay in registers, the nodal coefficients are
  // re-read where needed, and each component's element vector is stored as
  // soon as it is complete (fewer live registers than all components' R, U
  // and fluxes at once)
  constexpr bool SEQ = M > 1 && ROLE == 0 && WS;
  auto store_rc = [&](int c, int i, RT v) {
    const int64_t q = ((int64_t)c * NL + i) * E + e;
    if constexpr (MIX) {
      double fb = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) fb += foa[k * M + c] * ref_grad_int<D, P>(i, k);
      a.relem[q] = (double)v + hpow * fb;
    } else {
      a.relem[q] = v;
    }
  };
  if constexpr (SEQ) {
    RT uq[M][NL];
    {
      const int mv[3] = {SF::vq, SF::vq, SF::vq};
#pragma unroll
      for (int c = 0; c < M; ++c) {
        RT uc[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) uc[j] = MIX ? (RT)(Uc(c, j) - ue[c]) : (RT)Uc(c, j);
        tensor_apply<D, P>(T, mv, false, uc, uq[c]);
      }
    }
    RT wq[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      RT wv = 1;
#pragma unroll
      for (int j = 0; j < D; ++j) wv *= T(SF::wq + dig(q, j, P1));
      wq[q] = wv;
    }
    const RT sa = (RT)(nu * hpow / h), sg = (RT)(nu * gam * hpow);
    static_for<M>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const TabRef<RT>& Tc = T;
      // the stabilisation first, one gradient direction at a time (fewer
      // live registers than both directions of g with the flux sums)
      RT st[NL];
      {
        RT s1[NL], s2[NL];
#pragma unroll
        for (int i = 0; i < NL; ++i) s1[i] = s2[i] = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          int ms1[3] = {SF::g, SF::g, SF::g}, ms2[3] = {SF::g, SF::g, SF::g};
          ms1[k] = SF::k1;
          ms2[k] = SF::ct;
          RT t[NL], v[NL];
#pragma unroll
          for (int i = 0; i < NL; ++i) v[i] = MIX ? (RT)(ns.own(c, i) - ue[c]) : (RT)ns.own(c, i);
          tensor_apply<D, P>(Tc, ms1, false, v, t);
#pragma unroll
          for (int i = 0; i < NL; ++i) s1[i] += t[i];
          ns.load_grad_k(c, k, v);
          tensor_apply<D, P>(Tc, ms2, false, v, t);
#pragma unroll
          for (int i = 0; i < NL; ++i) s2[i] += t[i];
        }
#pragma unroll
        for (int i = 0; i < NL; ++i) st[i] = sa * s1[i] - sg * s2[i];
      }
      RT Rc[NL];
#pragma unroll
      for (int i = 0; i < NL; ++i) Rc[i] = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        RT Fc[NL];
#pragma unroll
        for (int q = 0; q < NL; ++q) {
          if constexpr (MIX) {
            double uv[M], fv[M];
#pragma unroll
            for (int c2 = 0; c2 < M; ++c2) uv[c2] = ue[c2] + (double)uq[c2][q];
            PHY::flux(k, uv, fv, a.ph);
            Fc[q] = wq[q] * (RT)(pick_m<M>(fv, c) - pick_m<M>(foa + k * M, c));
          } else {
            RT uv[M], fv[M];
#pragma unroll
            for (int c2 = 0; c2 < M; ++c2) uv[c2] = uq[c2][q];
            PHY::flux(k, uv, fv, a.ph);
            Fc[q] = wq[q] * pick_m<M>(fv, c);
          }
        }
        int mt[3] = {SF::vq, SF::vq, SF::vq};
        mt[k] = SF::dq;
        RT t[NL];
        tensor_apply<D, P>(Tc, mt, true, Fc, t);
#pragma unroll
        for (int i = 0; i < NL; ++i) Rc[i] += t[i];
      }
#pragma unroll
      for (int i = 0; i < NL; ++i) store_rc(c, i, (RT)hpow * Rc[i] - st[i]);
    });
  }
  if constexpr ((ROLE == 0 || ROLE == 2) && !SEQ) {
  RT R[M][NL];
  {
    RT uq[M][NL];
    int mv[3] = {SF::vq, SF::vq, SF::vq};
#pragma unroll
    for (int c = 0; c < M; ++c) {
      RT uc[NL];
#pragma unroll
      for (int j = 0; j < NL; ++j) uc[j] = MIX ? (RT)(Uc(c, j) - ue[c]) : (RT)Uc(c, j);
      tensor_apply<D, P>(T, mv, false, uc, uq[c]);
    }
    RT wq[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      RT wv = 1;
#pragma unroll
      for (int j = 0; j < D; ++j) wv *= T(SF::wq + dig(q, j, P1));
      wq[q] = wv;
    }
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
      for (int i = 0; i < NL; ++i) R[c][i] = 0;
    // all directional fluxes at once when they are cheap to keep (scalar
    // problems; one sincos per point for KPP), else one direction at a time
    constexpr bool allk = (M == 1);
    RT FA[allk ? D : 1][NL];
    if constexpr (allk) {
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        if constexpr (MIX) {
          double uv = ue[0] + (double)uq[0][q], fv[D];
          PHY::flux_all(&uv, fv, a.ph);
#pragma unroll
          for (int kk = 0; kk < D; ++kk) FA[kk][q] = wq[q] * (RT)(fv[kk] - foa[kk]);
        } else {
          RT fv[D];
          PHY::flux_all(&uq[0][q], fv, a.ph);
#pragma unroll
          for (int kk = 0; kk < D; ++kk) FA[kk][q] = wq[q] * fv[kk];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      RT F[M][NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        if constexpr (allk) {
          F[0][q] = FA[k][q];
        } else if constexpr (MIX) {
          double uv[M], fv[M];
#pragma unroll
          for (int c = 0; c < M; ++c) uv[c] = ue[c] + (double)uq[c][q];
          PHY::flux(k, uv, fv, a.ph);
#pragma unroll
          for (int c = 0; c < M; ++c) F[c][q] = wq[q] * (RT)(fv[c] - foa[k * M + c]);
        } else {
          RT uv[M], fv[M];
#pragma unroll
          for (int c = 0; c < M; ++c) uv[c] = uq[c][q];
          PHY::flux(k, uv, fv, a.ph);
#pragma unroll
          for (int c = 0; c < M; ++c) F[c][q] = wq[q] * fv[c];
        }
      }
      int mt[3] = {SF::vq, SF::vq, SF::vq};
      mt[k] = SF::dq;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        RT t[NL];
        tensor_apply<D, P>(T, mt, true, F[c], t);
#pragma unroll
        for (int i = 0; i < NL; ++i) R[c][i] += t[i];
      }
    }
  }
  // element vectors are float64; in the mixed form the flux of the cell
  // average (removed from the float contraction) is added back exactly
  auto store_r = [&](int c, int i, RT v) {
    const int64_t q = ((int64_t)c * NL + i) * E + e;
    if constexpr (MIX) {
      double fb = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) fb += foa[k * M + c] * ref_grad_int<D, P>(i, k);
      a.relem[q] = (double)v + hpow * fb;
    } else {
      a.relem[q] = v;
    }
  };
  if constexpr (!WS) {
    // residual without the stabilisation term
    if constexpr (ROLE == 2) xc.sync();
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
      for (int i = 0; i < NL; ++i) store_r(c, i, (RT)hpow * R[c][i]);
  } else if constexpr (ROLE == 2) {
    // the stabilisation sums first; gamma_e and nu_e from the other role
    RT s1[M][NL], s2[M][NL];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      RT gk[D][NL], uc[NL];
      ns.load_grad(c, gk);
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        s1[c][i] = s2[c][i] = 0;
        uc[i] = MIX ? (RT)(Uc(c, i) - ue[c]) : (RT)Uc(c, i);
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        int ms1[3] = {SF::g, SF::g, SF::g}, ms2[3] = {SF::g, SF::g, SF::g};
        ms1[k] = SF::k1;
        ms2[k] = SF::ct;
        RT t[NL];
        tensor_apply<D, P>(T, ms1, false, uc, t);
#pragma unroll
        for (int i = 0; i < NL; ++i) s1[c][i] += t[i];
        tensor_apply<D, P>(T, ms2, false, gk[k], t);
#pragma unroll
        for (int i = 0; i < NL; ++i) s2[c][i] += t[i];
      }
    }
    xc.sync();
    xc.get(gam, nu);
    const RT sa = (RT)(nu * hpow / h), sg = (RT)(nu * gam * hpow);
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
      for (int i = 0; i < NL; ++i) store_r(c, i, (RT)hpow * R[c][i] - (sa * s1[c][i] - sg * s2[c][i]));
  }
  const RT sa = (RT)(nu * hpow / h), sg = (RT)(nu * gam * hpow);   // nu h^{D-2}, nu gamma h^{D-1}
#pragma unroll
  for (int c = 0; c < (WS && ROLE == 0 ? M : 0); ++c) {
    RT gk[D][NL];
    ns.load_grad(c, gk);
    RT s1[NL], s2[NL], uc[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      s1[i] = s2[i] = 0;
      uc[i] = MIX ? (RT)(Uc(c, i) - ue[c]) : (RT)Uc(c, i);   // the stiffness annihilates constants
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      int ms1[3] = {SF::g, SF::g, SF::g}, ms2[3] = {SF::g, SF::g, SF::g};
      ms1[k] = SF::k1;
      ms2[k] = SF::ct;
      RT t[NL];
      tensor_apply<D, P>(T, ms1, false, uc, t);
#pragma unroll
      for (int i = 0; i < NL; ++i) s1[i] += t[i];
      tensor_apply<D, P>(T, ms2, false, gk[k], t);
#pragma unroll
      for (int i = 0; i < NL; ++i) s2[i] += t[i];
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) store_r(c, i, (RT)hpow * R[c][i] - (sa * s1[i] - sg * s2[i]));
  }
  }   // roles 0 and 2
  if constexpr (ROLE == 2) return 1.0e300;

  // ---- facets (Sec. 4, eqs. 18, 40, 42, 51): canonical orientation is from
  // the lower to the upper element along +e_k; both sides evaluate it alike.
  // The ends of a non-periodic line are boundary facets: the neighbour's
  // average becomes the boundary data of u^e (low-order flux, local bounds)
  // and f^H the boundary flux of the end node.
  bool bfac[2] = {false, false};
  if constexpr (D == 1) {
    bfac[0] = ms.bnd1d && e == 0;
    bfac[1] = ms.bnd1d && e == E - 1;
    if constexpr (M == 1) {
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
        if (bfac[sd]) {
          double gh[M];
          bc_ghost<M>(a, sd, ue, gh);
          nbr_mean[sd][0] = gh[0];
        }
    }
  }
  double lamsum = 0.0, fLsum[M], fHout[M];
#pragma unroll
  for (int c = 0; c < M; ++c) fLsum[c] = fHout[c] = 0.0;
  // one facet at a time: the axis a compile-time constant (the facet-node
  // indices stay constants), and for systems the two sides a rolled loop,
  // so that the Riemann speeds (three pow each) and facet sums of all facets
  // are not in flight at once (in the one-thread 2D Euler tile that alone
  // took more than 256 registers)
  static_for<D>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const double* fo = foa + k * M;
    auto facet = [&](int side) {
      double unb[M];
      if constexpr (M > 1 && ROLE != 4) {
        if (D == 1 && bfac[side]) {
          bc_ghost<M>(a, side, ue, unb);
        } else {
#pragma unroll
          for (int c = 0; c < M; ++c) {
            double cn[NL], sum = 0.0;
            ns.load_nbr(c, 2 * k + side, cn);
#pragma unroll
            for (int j = 0; j < NL; ++j) sum += cn[j];
            unb[c] = sum * (1.0 / NL);
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) unb[c] = nbr_mean[2 * k + side][c];
      }
      const double* un = unb;
      double fn[M];
      PHY::flux(k, un, fn, a.ph);
      const double* uL = side ? ue : un;
      const double* uR = side ? un : ue;
      const double* fl = side ? fo : fn;
      const double* fr = side ? fn : fo;
      double fH[M];
#pragma unroll
      for (int c = 0; c < M; ++c) fH[c] = 0.0;
      if (D == 1 && bfac[side]) {
        // boundary facet: f^H = f^partial = F(u_j, u_hat_j; n) of the end
        // node j (eq. fluxLLF; |S| = |c_j| = 1 on a line), in the +x
        // orientation of the canonical facets
        const int j = side ? P : 0;
        double uj[M], gj[M], fa[M], fz[M];
#pragma unroll
        for (int c = 0; c < M; ++c) uj[c] = SEQ ? ns.own(c, j) : Uc(c, j);
        bc_ghost<M>(a, side, uj, gj);
        const double* pL = side ? uj : gj;
        const double* pR = side ? gj : uj;
        PHY::flux(k, pL, fa, a.ph);
        PHY::flux(k, pR, fz, a.ph);
        const double lb = PHY::riemann_speed(pL, pR, k, a.ph);
#pragma unroll
        for (int c = 0; c < M; ++c) {
          fH[c] = 0.5 * (fa[c] + fz[c]) - 0.5 * lb * (pR[c] - pL[c]);
          // the outward boundary flux: -a(phi_j, u_h) - b(phi_j, u_h, u_hat)
          // leaves -F(u_j, u_hat; n) at the end node (eqs. weak:stab2,
          // bidef); pass 2 takes it for the element's boundary integral
          const double Fb = side ? fH[c] : -fH[c];
          a.fbnd[(side * 2 + 1) * M + c] = Fb;
          a.relem[((int64_t)c * NL + j) * E + e] -= Fb;
        }
      } else {
#pragma unroll
        for (int j = 0; j < NL; ++j) {
          if (dig(j, k, P1) != (side ? P : 0)) continue;
          double fj[M];
          if constexpr (PHY::kNodal) {
#pragma unroll
            for (int c = 0; c < M; ++c) fj[c] = fpre[k][side][j][c];
          } else {
            double uj[M];
#pragma unroll
            for (int c = 0; c < M; ++c) uj[c] = SEQ ? ns.own(c, j) : Uc(c, j);
            PHY::flux(k, uj, fj, a.ph);
          }
#pragma unroll
          for (int c = 0; c < M; ++c) fH[c] += fj[c];
        }
      }
      const double lm = PHY::riemann_speed(uL, uR, k, a.ph);
      lamsum += lm;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const double fLc = 0.5 * (fl[c] + fr[c]) - 0.5 * lm * (uR[c] - uL[c]);
        fLsum[c] += side ? fLc : -fLc;
        fHout[c] += side ? fH[c] * (1.0 / NF) : -(fH[c] * (1.0 / NF));
        if (side) a.fahi[((int64_t)k * M + c) * E + e] = fLc - fH[c] * (1.0 / NF);
      }
    };
    if constexpr (M == 1) {
      facet(0);
      facet(1);
    } else {
#pragma unroll 1
      for (int side = 0; side < 2; ++side) facet(side);
    }
  });
  double dt_e = h / lamsum;                                   // eq. (40)
  if (a.flux_mode != 0) {
    // flux limiter off (Sec. 4.3, steps 3-4): f_ee' = f^H and ubar^e =
    // u^e - dt_e / h sum_facets f^H . n, with dt_e of Lemma 1 (eq. 37) or
    // eq. (40) reduced until ubar^e is admissible
    if (a.flux_mode == 1) {
      if constexpr (SEQ)
        dt_e = subcell_dt<D, P, PHY>([&](int c, int j) { return ns.own(c, j); }, ue, h, a.ph);
      else
        dt_e = subcell_dt<D, P, PHY>([&](int c, int j) { return Uc(c, j); }, ue, h, a.ph);
    } else if constexpr (PH == EUL) {
      double dl[M];
#pragma unroll
      for (int c = 0; c < M; ++c) dl[c] = -dt_e / h * fHout[c];
      dt_e *= euler_alpha<D>(ue, dl, 1.0, a.eps_pos);
    } else {
      const double Dr = fHout[0] / h;
      const double lim = Dr > 0.0 ? (ue[0] - a.umin) / Dr : (Dr < 0.0 ? (a.umax - ue[0]) / -Dr : 1.0e300);
      dt_e = fmin(dt_e, fmax(lim, 0.0));
    }
#pragma unroll
    for (int c = 0; c < M; ++c) a.ubar[c * E + e] = ue[c] - dt_e / h * fHout[c];
  }
  a.dte[e] = dt_e;
  if constexpr (ROLE != 4) {
    a.gam[e] = gam;
    a.nu[e] = nu;
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    a.ue[c * E + e] = ue[c];
    a.ubarL[c * E + e] = ue[c] - dt_e / h * fLsum[c];
  }
  if constexpr (M == 1) {
    // Q1 contributions: int_dK f_h . n = |S| sum over facets of the outward
    // facet means of f(u_j) . n (the low-order scheme's a_i, Sec. 3)
    if (a.contrib_q1) {
      double area = 1.0;
#pragma unroll
      for (int k = 0; k < D - 1; ++k) area *= h;
      a.fdiv[e] = area * fHout[0];
    }
    // local bounds of the scalar limiters (Sec. 4.1, 4.2): the range of the
    // cell averages of K_e and its 2d facet neighbours; it holds ubar^{e,L}
    // (a convex combination of u^e and the facets' bar states).  NaN
    // propagates, as it does through the global bounds' tests.
    if (a.bounds_local) {
      double lo = ue[0], hi = ue[0];
#pragma unroll
      for (int l = 0; l < 2 * D; ++l) {
        const double v = nbr_mean[l][0];
        lo = (v < lo || v != v) ? v : lo;
        hi = (v > hi || v != v) ? v : hi;
      }
      a.bnd[e] = lo;
      a.bnd[E + e] = hi;
    }
  }
  if constexpr (ROLE == 4) xc.sync();
  return dt_e;
}

template <int D, int P, int PH, bool WS, class RT>
__device__ __forceinline__ void k_elem1_body(const StageArgs& a, int bx) {
  const int64_t e = (int64_t)bx * blockDim.x + threadIdx.x;
  double dt_e = 1.0e300;
  if (e < a.mesh.E) dt_e = elem1_body<D, P, PH, WS, RT>(a, e, GlobalNodes<D, P, Phys<D, PH>::M>(a, e));
  block_min_dt(a.dtpart, dt_e, bx);     // every thread of the block reaches this
}

template <int D, int P, int PH, bool WS, class RT>
__global__ void __launch_bounds__(128) k_elem1(StageArgs a) {
  k_elem1_body<D, P, PH, WS, RT>(a, blockIdx.x);
}

// 2D element pass on a 16 x 8 element tile: the block first stages the
// tile's nodes (one-element halo) and, when it fits, g in LDS.
template <int P, int PH, class RT>
__device__ __forceinline__ void tile_stage(const StageArgs& a, int ex0, int ey0) {
  constexpr int M = Phys<2, PH>::M;
  using TT = Tile2<P, M>;
  const MeshArgs& ms = a.mesh;
  const int L0 = ms.L[0], L1 = ms.L[1];
  int X0 = P * (ex0 - 1), Y0 = P * (ey0 - 1);
  if (X0 < 0) X0 += L0;
  if (Y0 < 0) Y0 += L1;
  // four values per thread and pass, loads issued before the LDS stores;
  // periodic wrap by subtraction (tile offsets are below 2 L on all but the
  // smallest meshes)
  const int nt = (int)blockDim.x;
  auto wrap = [](int x, int L) {
    while (x >= L) x -= L;
    return x;
  };
  for (int q0 = threadIdx.x; q0 < M * TT::NXY; q0 += 4 * nt) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = q0 + k * nt;
      if (q < M * TT::NXY) {
        const int c = q / TT::NXY, r = q - c * TT::NXY, iy = r / TT::NX, ix = r - iy * TT::NX;
        const int gx = wrap(X0 + ix, L0), gy = wrap(Y0 + iy, L1);
        v[k] = a.u[c * ms.N + gx + (int64_t)L0 * gy];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (q0 + k * nt < M * TT::NXY) cem_smem[q0 + k * nt] = v[k];
  }
  if constexpr (TT::stage_g) {
    double* gs = cem_smem + M * TT::NXY;
    for (int q0 = threadIdx.x; q0 < 2 * M * TT::GXY; q0 += 4 * nt) {
      double v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = q0 + k * nt;
        if (q < 2 * M * TT::GXY) {
          const int kc = q / TT::GXY, r = q - kc * TT::GXY, iy = r / TT::GX, ix = r - iy * TT::GX;
          const int gx = wrap(P * ex0 + ix, L0), gy = wrap(P * ey0 + iy, L1);
          const int64_t gi = (int64_t)kc * ms.N + gx + (int64_t)L0 * gy;
          if constexpr (sizeof(RT) == 4) v[k] = a.g32[gi];
          else v[k] = a.g[gi];
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (q0 + k * nt < 2 * M * TT::GXY) gs[q0 + k * nt] = v[k];
    }
  }
  __syncthreads();
}

template <int P, int PH, bool WS, class RT>
__device__ __forceinline__ void k_elem1_tile_body(const StageArgs& a, int bx) {
  constexpr int M = Phys<2, PH>::M;
  using TT = Tile2<P, M>;
  const MeshArgs& ms = a.mesh;
  const int nbx = (ms.n[0] + TT::TEX - 1) / TT::TEX;
  const int ex0 = (bx % nbx) * TT::TEX, ey0 = (bx / nbx) * TT::TEY;
  tile_stage<P, PH, RT>(a, ex0, ey0);
  const int tx = threadIdx.x % TT::TEX, ty = threadIdx.x / TT::TEX;
  const int ex = ex0 + tx, ey = ey0 + ty;
  double dt_e = 1.0e300;
  if (ex < ms.n[0] && ey < ms.n[1]) {
    const int64_t e = ex + (int64_t)ms.n[0] * ey;
    dt_e = elem1_body<2, P, PH, WS, RT>(a, e, TileNodes2<P, M>(a, e, tx, ty));
  }
  block_min_dt(a.dtpart, dt_e, bx);     // every thread of the block reaches this
}

// two waves per SIMD up to Q2 (the 512-problem Q2 Euler batch: 8.3 -> 7.8 ms
// per launch); Q3 keeps one (at two it spills: 512^2 Euler 0.34 -> 0.67 ms)
#define CEM_TILE_BOUNDS __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(P <= 2 ? 2 : 1)))

template <int P, int PH, bool WS, class RT>
__global__ void CEM_TILE_BOUNDS k_elem1_tile(StageArgs a) {
  k_elem1_tile_body<P, PH, WS, RT>(a, xcd_block(blockIdx.x, gridDim.x));
}

// The same pass with two threads per element (256 threads): role 1 the
// sensor, the viscosity and the facet data, role 2 the element residual;
// they meet once in LDS (gamma_e, nu_e).  Twice the waves of the one-thread
// form, each with about half the work and fewer live registers.
template <int P, int PH, bool WS, class RT>
__device__ __forceinline__ void k_elem1_tile2_body(const StageArgs& a, int bx) {
  constexpr int M = Phys<2, PH>::M;
  using TT = Tile2<P, M>;
  using TN = TileNodes2<P, M>;
  constexpr int NE = TT::TEX * TT::TEY;
  const MeshArgs& ms = a.mesh;
  const int nbx = (ms.n[0] + TT::TEX - 1) / TT::TEX;
  const int ex0 = (bx % nbx) * TT::TEX, ey0 = (bx / nbx) * TT::TEY;
  tile_stage<P, PH, RT>(a, ex0, ey0);
  const int role2 = (int)threadIdx.x >= NE, li = (int)threadIdx.x - (role2 ? NE : 0);
  const int tx = li % TT::TEX, ty = li / TT::TEX;
  const int ex = ex0 + tx, ey = ey0 + ty;
  const LdsXchg xc{cem_smem + TT::words + li, NE};
  // Lanes past the mesh edge run the body of the last element of their row
  // or column (which lies in this tile): every lane of the block then
  // reaches the exchange barrier inside the body once, in uniform control
  // flow.  Their stores repeat the owner's bitwise-equal values; their dt_e
  // repeats a value of the block.
  const int tx1 = min(ex, ms.n[0] - 1) - ex0, ty1 = min(ey, ms.n[1] - 1) - ey0;
  const int64_t e = (ex0 + tx1) + (int64_t)ms.n[0] * (ey0 + ty1);
  const TN ns(a, e, tx1, ty1);
  double dt_e = 1.0e300;
  if (role2) elem1_body<2, P, PH, WS, RT, TN, 2>(a, e, ns, xc);
  else dt_e = elem1_body<2, P, PH, WS, RT, TN, 1>(a, e, ns, xc);
  block_min_dt_n<2 * NE>(a.dtpart, dt_e, bx);
}

template <int P, int PH, bool WS, class RT>
__global__ void __launch_bounds__(256) k_elem1_tile2(StageArgs a) {
  k_elem1_tile2_body<P, PH, WS, RT>(a, xcd_block(blockIdx.x, gridDim.x));
}

// Three threads per element (384 threads): role 3 the sensor and the
// viscosity, role 2 the residual, role 4 the facet data and dt_e.  Only the
// residual waits for gamma_e and nu_e (the block's one barrier).
template <int P, int PH, bool WS, class RT>
__device__ __forceinline__ void k_elem1_tile3_body(const StageArgs& a, int bx) {
  constexpr int M = Phys<2, PH>::M;
  using TT = Tile2<P, M>;
  using TN = TileNodes2<P, M>;
  constexpr int NE = TT::TEX * TT::TEY;
  const MeshArgs& ms = a.mesh;
  const int nbx = (ms.n[0] + TT::TEX - 1) / TT::TEX;
  const int ex0 = (bx % nbx) * TT::TEX, ey0 = (bx / nbx) * TT::TEY;
  tile_stage<P, PH, RT>(a, ex0, ey0);
  const int role = (int)threadIdx.x / NE, li = (int)threadIdx.x - role * NE;
  const int tx = li % TT::TEX, ty = li / TT::TEX;
  const int ex = ex0 + tx, ey = ey0 + ty;
  const LdsXchg xc{cem_smem + TT::words + li, NE};
  // lanes past the mesh edge repeat the last element of their row or column
  // (see k_elem1_tile2_body): the exchange barrier stays in uniform control
  // flow
  const int tx1 = min(ex, ms.n[0] - 1) - ex0, ty1 = min(ey, ms.n[1] - 1) - ey0;
  const int64_t e = (ex0 + tx1) + (int64_t)ms.n[0] * (ey0 + ty1);
  const TN ns(a, e, tx1, ty1);
  double dt_e = 1.0e300;
  if (role == 0) elem1_body<2, P, PH, WS, RT, TN, 3>(a, e, ns, xc);
  else if (role == 1) elem1_body<2, P, PH, WS, RT, TN, 2>(a, e, ns, xc);
  else dt_e = elem1_body<2, P, PH, WS, RT, TN, 4>(a, e, ns, xc);
  block_min_dt_n<3 * NE>(a.dtpart, dt_e, bx);
}

template <int P, int PH, bool WS, class RT>
__global__ void __launch_bounds__(384) k_elem1_tile3(StageArgs a) {
  k_elem1_tile3_body<P, PH, WS, RT>(a, xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// steps 3-4: flux limiter (eq. 53 / Appendix A), element contributions
// (eq. 45), slope limiter (eqs. 54-55 / Appendix A); stores the element
// update vector [m_i^e (ubar - u_i) + beta f_i^e] / dt_e
// ---------------------------------------------------------------------------
// limited flux fb of the facet between eL (lower) and eR (upper): fA its raw
// antidiffusive flux, uLs / uRs the two low-order averages, dtL / dtR the
// two pseudo time steps
// and, for scalar problems, bL / bR the two elements' bounds {lower, upper};
// ghost 1 or 2: the lower or upper side is a boundary facet's exterior,
// whose (absent) element imposes nothing (eq. 53, e' > E_h)
template <int D, int PH>
__device__ inline void limit_facet(const StageArgs& a, const double* fA, const double* uLs, const double* uRs,
                                   double dtL, double dtR, const double* bL, const double* bR, double* fb,
                                   int ghost = 0) {
  using PHY = Phys<D, PH>;
  constexpr int M = PHY::M;
  const double phi = a.mesh.h / (2.0 * D);     // |K| / |dK|
  if (a.alpha_mode == 2) {
#pragma unroll
    for (int c = 0; c < M; ++c) fb[c] = fA[c];
    return;
  }
  if (a.alpha_mode == 1) {
#pragma unroll
    for (int c = 0; c < M; ++c) fb[c] = 0.0;
    return;
  }
  if constexpr (PH == EUL) {
    double dL[M], dR[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      dL[c] = fA[c] / phi * dtL;
      dR[c] = -fA[c] / phi * dtR;
    }
    const double al = fmin(ghost == 1 ? 1.0 : euler_alpha<D>(uLs, dL, 1.0, a.eps_pos),
                           ghost == 2 ? 1.0 : euler_alpha<D>(uRs, dR, 1.0, a.eps_pos));
#pragma unroll
    for (int c = 0; c < M; ++c) fb[c] = al * fA[c];
  } else {
    // eL keeps ubar^{eL} within its upper bound and eR within its lower
    // one (and the mirror for f^min)
    const double inf = (double)INFINITY;
    const double fmx = fmin(ghost == 1 ? inf : phi * (bL[1] - uLs[0]) / dtL,
                            ghost == 2 ? inf : phi * (uRs[0] - bR[0]) / dtR);
    const double fmn = fmax(ghost == 1 ? -inf : phi * (bL[0] - uLs[0]) / dtL,
                            ghost == 2 ? -inf : phi * (uRs[0] - bR[1]) / dtR);
    fb[0] = fA[0] >= 0.0 ? fmin(fA[0], fmx) : fmax(fA[0], fmn);
  }
}

template <int D, int P, int PH, class RT>
__device__ __forceinline__ void k_elem2_body(const StageArgs& a, int bx) {
  using PHY = Phys<D, PH>;
  constexpr int P1 = P + 1, NL = ipow(P1, D), M = PHY::M, NF = NL / P1;
  constexpr bool MIX = sizeof(RT) == 4;
  const TabRef<RT> T{TabSel<RT>::of(a.tab)};
  const int64_t e = (int64_t)bx * blockDim.x + threadIdx.x;
  const MeshArgs& ms = a.mesh;
  if (e >= ms.E) return;
  const int64_t N = ms.N, E = ms.E;
  const double h = ms.h;
  int ei[3];
  elem_coords(e, ms, ei);
  int off[D][P1];
#pragma unroll
  for (int k = 0; k < D; ++k) axis_offsets<P>(ei[k], k, ms, off[k]);

  // ---- flux-limited intermediate average (eq. 44).  The data of all 2D
  // facets and the element's nodes are loaded first, in straight-line code:
  // behind the limiter's (uniform) branches each facet's loads waited for
  // the previous facet's arithmetic.
  const double dt_e = a.dte[e];
  double fAl[D][M], fAh[D][M], ubl[D][M], ubh[D][M], ubc[M], uec[M], dtl[D], dth[D], bl[D][2], bh[D][2];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int en[3] = {ei[0], ei[1], ei[2]};
    en[k] = ei[k] == 0 ? ms.n[k] - 1 : ei[k] - 1;
    const int64_t elo = elem_id(en, ms);
    en[k] = ei[k] + 1 == ms.n[k] ? 0 : ei[k] + 1;
    const int64_t ehi = elem_id(en, ms);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      fAl[k][c] = a.fahi[((int64_t)k * M + c) * E + elo];    // facet (elo, e)
      fAh[k][c] = a.fahi[((int64_t)k * M + c) * E + e];      // facet (e, ehi)
      ubl[k][c] = a.ubarL[c * E + elo];
      ubh[k][c] = a.ubarL[c * E + ehi];
    }
    dtl[k] = a.dte[elo];
    dth[k] = a.dte[ehi];
    if (M == 1 && a.bounds_local) {
      bl[k][0] = a.bnd[elo];
      bl[k][1] = a.bnd[E + elo];
      bh[k][0] = a.bnd[ehi];
      bh[k][1] = a.bnd[E + ehi];
    } else {
      bl[k][0] = bh[k][0] = a.umin;
      bl[k][1] = bh[k][1] = a.umax;
    }
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    ubc[c] = a.ubarL[c * E + e];
    uec[c] = a.ue[c * E + e];
  }
  // the ends of a non-periodic line: element 0's low facet and the last
  // element's high facet are boundary facets.  The high one's raw flux is in
  // fahi like any +x facet; the low one's is formed here as pass 1 formed
  // it, f^L = F(u_hat^e', u^e) along +x minus f^H = -F(u_end, u_hat; -1)
  bool glo = false, ghi = false;
  if constexpr (D == 1) {
    glo = ms.bnd1d && e == 0;
    ghi = ms.bnd1d && e == E - 1;
    if (glo) {
      double gh[M], fa[M], fz[M];
      bc_ghost<M>(a, 0, uec, gh);
      PHY::flux(0, gh, fa, a.ph);
      PHY::flux(0, uec, fz, a.ph);
      const double lm = PHY::riemann_speed(gh, uec, 0, a.ph);
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const double fLc = 0.5 * (fa[c] + fz[c]) - 0.5 * lm * (uec[c] - gh[c]);
        fAl[0][c] = fLc + a.fbnd[M + c];
      }
    }
  }
  // the element's own bounds (scalar limiters: flux and slope)
  double bc[2] = {a.umin, a.umax};
  if (M == 1 && a.bounds_local) {
    bc[0] = a.bnd[e];
    bc[1] = a.bnd[E + e];
  }
  double U[M][NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const int64_t nd = local_node<D, P>(j, off);
#pragma unroll
    for (int c = 0; c < M; ++c) U[c][j] = a.u[c * N + nd];
  }
  double ub[M];
  if (a.flux_mode != 0) {
#pragma unroll
    for (int c = 0; c < M; ++c) ub[c] = a.ubar[c * E + e];   // f = f^H, written by element pass 1
  } else {
    double fbs[M];
#pragma unroll
    for (int c = 0; c < M; ++c) fbs[c] = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double fb[M];
      limit_facet<D, PH>(a, fAl[k], ubl[k], ubc, dtl[k], dt_e, bl[k], bc, fb, glo ? 1 : 0);
#pragma unroll
      for (int c = 0; c < M; ++c) fbs[c] -= fb[c];
      limit_facet<D, PH>(a, fAh[k], ubc, ubh[k], dt_e, dth[k], bc, bh[k], fb, ghi ? 2 : 0);
#pragma unroll
      for (int c = 0; c < M; ++c) fbs[c] += fb[c];
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
      ub[c] = ubc[c] + dt_e / h * fbs[c];
      a.ubar[c * E + e] = ub[c];
    }
  }

  // ---- boundary integral B_i = int_{dK} phi_i f_h . n (so that
  // int grad phi_i . f_h + int phi_i div f_h = B_i) and F^e = sum_i B_i:
  // on each facet the (D-1)-dimensional Gram of the facet nodes
  using SF = SFLayout<D, P>;
  double hpow = 1.0;
#pragma unroll
  for (int k = 0; k < D - 1; ++k) hpow *= h;
  // On a boundary facet of a non-periodic line f_h . n is replaced by the
  // boundary flux F(u_end, u_hat; n) of pass 1, whose phi_i-part element
  // pass 1 already put into the residual vector: with g_i^e of eq. (aecb),
  // int grad phi_i . (f(u_h) - f_h) - int (phi_i - m_i/|K|) div f_h - g_i^e
  // = R_i - B_i + F^e / NL with B_i without that facet's term and F^e
  // taking F(u_end, u_hat; n) for it (a point value in 1D)
  RT fb[M][NL];
  double feb[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    feb[c] = 0.0;
#pragma unroll
    for (int i = 0; i < NL; ++i) fb[c][i] = 0;
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (D == 1 && (side ? ghi : glo)) {
#pragma unroll
        for (int c = 0; c < M; ++c) feb[c] += a.fbnd[(side * 2 + 1) * M + c];
        continue;
      }
      const int av = side ? P : 0;
      const RT sg = (RT)(side ? hpow : -hpow);
      double fbar[M];                  // mixed form: flux of the cell average
      if constexpr (MIX) PHY::flux(k, uec, fbar, a.ph);
      RT fn[M][NF > 0 ? NF : 1];
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        if (dig(j, k, P1) != av) continue;
        const int fj = j % ipow(P1, k) + (j / ipow(P1, k + 1)) * ipow(P1, k);   // drop digit k
        double fv[M];
        if constexpr (PHY::kNodal) {
          const int64_t nd = local_node<D, P>(j, off);
#pragma unroll
          for (int c = 0; c < M; ++c) fv[c] = a.fnode[((int64_t)k * M + c) * N + nd];
        } else {
          double uj[M];
#pragma unroll
          for (int c = 0; c < M; ++c) uj[c] = U[c][j];
          PHY::flux(k, uj, fv, a.ph);
        }
#pragma unroll
        for (int c = 0; c < M; ++c) fn[c][fj] = MIX ? (RT)(fv[c] - fbar[c]) : (RT)fv[c];
      }
      const int mg[3] = {SF::g, SF::g, SF::g};
#pragma unroll
      for (int c = 0; c < M; ++c) {
        RT t[NF > 0 ? NF : 1];
        tensor_apply<D - 1, P>(T, mg, false, fn[c], t);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
          if (dig(i, k, P1) != av) continue;
          const int fi = i % ipow(P1, k) + (i / ipow(P1, k + 1)) * ipow(P1, k);
          fb[c][i] += sg * t[fi];
        }
      }
    }
  }
  double hd = hpow * h;
  const double mloc = hd * (1.0 / NL);
  // f_i^e of eq. (45): the contraction terms in RT, their sum promoted.  In
  // the mixed form the terms' element sum (zero in exact arithmetic, eq. 47)
  // is removed in float64 so that the update stays conservative to float64
  // round-off.
  double f[M][NL];
  // Q1 form of Sec. 5.3 (scalar, p = 1, float64): gamma_e (m_i^e (u_i - u^e)
  // - dt_e [int (phi_i - m_i^e/|K|) div f_h + int phi_i (udot_h^L -
  // udot_i^L)]), udot holding the low-order derivative; with int phi_i div
  // f_h = B_i - int grad phi_i . f_h, the bracket is B_i - G_i - F^e / NL +
  // the mass term, G_i = sum_j f_k(u_j) int d_k phi_i phi_j by the 1D Q1
  // integrals (int B_a' B_b = -1/2 or 1/2 as a = 0 or 1; int B_a B_b = 1/3,
  // 1/6)
  constexpr bool Q1F = P == 1 && M == 1 && !MIX;
  const bool q1 = Q1F && a.contrib_q1;
  double q1g[Q1F ? NL : 1];
  if constexpr (Q1F) {
    if (q1) {
      double fall[D][NL];
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        if constexpr (PHY::kNodal) {
          const int64_t nd = local_node<D, P>(j, off);
#pragma unroll
          for (int k = 0; k < D; ++k) fall[k][j] = a.fnode[(int64_t)k * N + nd];
        } else {
#pragma unroll
          for (int k = 0; k < D; ++k) {
            double fv[1];
            PHY::flux(k, &U[0][j], fv, a.ph);
            fall[k][j] = fv[0];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        double gi = 0.0;
#pragma unroll
        for (int j = 0; j < NL; ++j)
#pragma unroll
          for (int k = 0; k < D; ++k) {
            double cf = dig(i, k, 2) ? 0.5 : -0.5;
#pragma unroll
            for (int l = 0; l < D; ++l)
              if (l != k) cf *= dig(i, l, 2) == dig(j, l, 2) ? (1.0 / 3.0) : (1.0 / 6.0);
            gi += cf * fall[k][j];
          }
        q1g[i] = hpow * gi;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    RT Fe = (RT)feb[c];
#pragma unroll
    for (int i = 0; i < NL; ++i) Fe += fb[c][i];
    RT ud[NL], mu[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int64_t q = c * N + local_node<D, P>(j, off);
      if constexpr (MIX) ud[j] = a.udot32[q];
      else ud[j] = a.udot[q];
    }
    const int mg[3] = {SF::g, SF::g, SF::g};
    tensor_apply<D, P>(T, mg, false, ud, mu);
    double fbar[D];                 // mixed form: fluxes of the cell average
    if constexpr (MIX) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double fk[M];
        PHY::flux(k, uec, fk, a.ph);
        fbar[k] = fk[c];
      }
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const RT Tc = (RT)hd * mu[i] - (RT)mloc * ud[i];
      const double R = a.relem[((int64_t)c * NL + i) * E + e];
      if constexpr (MIX) {
        double rb = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) rb += fbar[k] * ref_grad_int<D, P>(i, k);
        f[c][i] = (R - hpow * rb) + (double)(-fb[c][i] + Fe * (RT)(1.0 / NL) - Tc);
      } else if constexpr (Q1F) {
        f[c][i] = q1 ? (double)(q1g[i] - fb[c][i] + Fe * (RT)(1.0 / NL) - Tc)
                     : (double)(R - fb[c][i] + Fe * (RT)(1.0 / NL) - Tc);
      } else {
        f[c][i] = (double)(R - fb[c][i] + Fe * (RT)(1.0 / NL) - Tc);
      }
    }
    double zs = 0.0;
    if constexpr (MIX) {
#pragma unroll
      for (int i = 0; i < NL; ++i) zs += f[c][i];
      zs *= 1.0 / NL;
    }
    const double gsc = q1 ? a.gam[e] : 1.0;
#pragma unroll
    for (int i = 0; i < NL; ++i) f[c][i] = gsc * (mloc * (U[c][i] - uec[c]) + dt_e * (f[c][i] - zs));
  }

  // ---- slope limiter
  double beta = 1.0;
  if (a.beta_mode == 1) {
    beta = 0.0;
  } else if (a.beta_mode == 0) {
    if constexpr (PH == EUL) {
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        double fi[M];
#pragma unroll
        for (int c = 0; c < M; ++c) fi[c] = f[c][i];
        beta = fmin(beta, euler_alpha<D>(ub, fi, mloc, a.eps_pos));
      }
    } else {
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const double fi = f[0][i];
        double bi = 1.0;
        // ubar is in bounds up to rounding: a ratio made negative by a
        // rounding excess counts as 0
        if (fi > 0.0) bi = fmax(0.0, fmin(1.0, mloc * (bc[1] - ub[0]) / fi));
        else if (fi < 0.0) bi = fmax(0.0, fmin(1.0, mloc * (bc[0] - ub[0]) / fi));
        beta = fmin(beta, bi);
      }
    }
  }
  a.beta[e] = beta;
  const double idt = 1.0 / dt_e;
#pragma unroll
  for (int c = 0; c < M; ++c)
#pragma unroll
    for (int i = 0; i < NL; ++i)
      a.relem[((int64_t)c * NL + i) * E + e] = (mloc * (ub[c] - U[c][i]) + beta * f[c][i]) * idt;
}

template <int D, int P, int PH, class RT>
__global__ void __launch_bounds__(128) k_elem2(StageArgs a) {
  k_elem2_body<D, P, PH, RT>(a, xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// node-centric gathers of element vectors (fixed element order per node)
// ---------------------------------------------------------------------------
template <int D, int P>
__device__ inline int node_elements(int64_t i, const MeshArgs& m, int64_t* eids, int* locs) {
  if constexpr (D == 1) {
    // the two end nodes of a non-periodic line belong to one element each
    if (m.bnd1d && (i == 0 || i == m.L[0] - 1)) {
      eids[0] = i == 0 ? 0 : m.n[0] - 1;
      locs[0] = i == 0 ? 0 : P;
      return 1;
    }
  }
  int ik[3] = {0, 0, 0};
  unsigned r = (unsigned)i;                 // node ids are below 2^31
  ik[0] = (int)(r % (unsigned)m.L[0]);
  r /= (unsigned)m.L[0];
  if (D > 1) {
    ik[1] = (int)(r % (unsigned)m.L[1]);
    r /= (unsigned)m.L[1];
  }
  if (D > 2) ik[2] = (int)r;
  int cnt[3], ek[3][2], ak[3][2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    cnt[k] = 1;
    ek[k][0] = 0;
    ak[k][0] = 0;
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int e0 = ik[k] / P, a0 = ik[k] % P;
    if (a0 == 0) {
      cnt[k] = 2;
      ek[k][0] = e0 == 0 ? m.n[k] - 1 : e0 - 1;   // lower element sees it at a = P
      ak[k][0] = P;
      ek[k][1] = e0;
      ak[k][1] = 0;
    } else {
      ek[k][0] = e0;
      ak[k][0] = a0;
    }
  }
  int nrec = 0;
  for (int z = 0; z < cnt[2]; ++z)
    for (int y = 0; y < cnt[1]; ++y)
      for (int x = 0; x < cnt[0]; ++x) {
        const int ee[3] = {ek[0][x], ek[1][y], ek[2][z]};
        eids[nrec] = elem_id(ee, m);
        locs[nrec] = ak[0][x] + (P + 1) * (ak[1][y] + (P + 1) * ak[2][z]);
        ++nrec;
      }
  return nrec;
}

// RT: value type of the assembled residual r (float in the mixed form); the
// element vectors are float64 and summed in float64
template <class RT> struct ResPtr;
template <> struct ResPtr<double> {
  __device__ static double* r(const StageArgs& a) { return a.r; }
};
template <> struct ResPtr<float> {
  __device__ static float* r(const StageArgs& a) { return a.r32; }
};

template <int D, int P, int M, class RT>
__device__ __forceinline__ void k_gather_r_body(const StageArgs& a, int bx) {
  constexpr int NL = ipow(P + 1, D);
  const int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  if (i >= a.mesh.N) return;
  int64_t eids[8];
  int locs[8];
  const int nrec = node_elements<D, P>(i, a.mesh, eids, locs);
  const int64_t E = a.mesh.E, N = a.mesh.N;
  RT* r = ResPtr<RT>::r(a);
#pragma unroll
  for (int c = 0; c < M; ++c) {
    double s = 0.0;
    #pragma unroll
    for (int t = 0; t < (1 << D); ++t)    // constant indices into eids / locs
      if (t < nrec) s += a.relem[((int64_t)c * NL + locs[t]) * E + eids[t]];
    r[c * N + i] = (RT)s;
  }
}

template <int D, int P, int M, class RT>
__global__ void __launch_bounds__(256) k_gather_r(StageArgs a) {
  k_gather_r_body<D, P, M, RT>(a, xcd_block(blockIdx.x, gridDim.x));
}

// u^FE_i = u_i + dt / m_i sum_e [m_i^e (ubar^e - u_i) + beta_e f_i^e] / dt_e
// (eq. 49), then the Shu-Osher combination u_out = a u0 + b u^FE and, for
// scalar problems, the round-off clamp to the global bounds.
// global time step of the stage from the per-block minima of dt_e (every
// block reduces them itself; block 0 records dt, the running minimum and the
// CFL flag of eq. (23))
__device__ inline void stage_dt_record(const StageArgs& a, double mn) {
  const double dt = a.stage == 0 ? (a.dt_fixed > 0.0 ? a.dt_fixed : a.cfl * mn) : a.dtbuf[0];
  if (a.stage == 0) a.dtbuf[0] = dt;
  a.dtbuf[1] = a.stage == 0 ? mn : fmin(a.dtbuf[1], mn);
  if (dt > mn) a.dtbuf[2] = 1.0;
}

__device__ inline double stage_dt(const StageArgs& a, int bx) {
  if (a.dt_ready) return a.dtbuf[0];       // reduced by k_stage_dt (uniform branch)
  double m = 1.0e300;
  for (int j = threadIdx.x; j < a.ndtpart; j += 256) m = fmin(m, a.dtpart[j]);
  const double mn = block_min<256>(m);
  if (bx == 0 && threadIdx.x == 0) stage_dt_record(a, mn);
  return a.stage == 0 ? (a.dt_fixed > 0.0 ? a.dt_fixed : a.cfl * mn) : a.dtbuf[0];
}

// the stage update of one nodal value: u^FE = u_i + dt / m_i sum (eq. 49),
// then the SSP-RK combination a u^n + b u^FE.  Explicit fused multiply-adds,
// so that every kernel that updates nodes rounds alike (contraction left to
// the compiler may pick different products in different callers).
__device__ __forceinline__ double stage_value(double ui, double ub, double sum, double dt_over_m, const StageArgs& a) {
  const double ufe = fma(dt_over_m, sum, ui);
  return (a.rk_a == 0.0) ? ufe : fma(a.rk_a, ub, a.rk_b * ufe);
}

template <int D, int P, int PH>
__device__ __forceinline__ void k_update_body(const StageArgs& a, int bx) {
  constexpr int M = Phys<D, PH>::M;
  constexpr bool SCALAR = PH != EUL;
  constexpr int NL = ipow(P + 1, D);
  __shared__ int red[2][4];
  const int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  bool live = i < a.mesh.N;
  const int64_t E = a.mesh.E, N = a.mesh.N;
  // the node's data is read first, so that its loads overlap the reduction
  // of the time step
  double ssum[M], uin[M], ubase[M];
  int nrec = 0;
  int64_t eids[8];
  int locs[8];
  if (live) {
    nrec = node_elements<D, P>(i, a.mesh, eids, locs);
    if constexpr (D == 2 && PH == EUL) {
      // nodes whose elements all lie in one block of the system pass 2 were
      // updated there (fuse_upd: the blocks hold 2^fuse_upd consecutive
      // elements)
      if (a.fuse_upd) {
        bool same = true;
        for (int t = 1; t < nrec; ++t) same = same && ((eids[t] >> a.fuse_upd) == (eids[0] >> a.fuse_upd));
        live = !same;
      }
    }
  }
  if (live) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      double s = 0.0;
      #pragma unroll
      for (int t = 0; t < (1 << D); ++t)    // constant indices into eids / locs
        if (t < nrec) s += a.relem[((int64_t)c * NL + locs[t]) * E + eids[t]];
      ssum[c] = s;
      uin[c] = a.u[c * N + i];
      ubase[c] = (a.rk_a == 0.0) ? 0.0 : a.u0[c * N + i];
    }
  }
  const double dt = stage_dt(a, bx);      // every thread of the block (256)
  int nclamp = 0, nbad = 0;
  if (live) {
    double hd = 1.0;
#pragma unroll
    for (int k = 0; k < D; ++k) hd *= a.mesh.h;
    const double mi = nrec * (hd * (1.0 / NL));
    double vout[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const double s = ssum[c];
      const double ui = uin[c];
      if (a.copy_base) a.u0[c * N + i] = ui;
      double v = stage_value(ui, ubase[c], s, dt / mi, a);
      if (SCALAR) {
        // round-off excess is clamped and counted; larger excursions (only
        // possible with a limiter switched off) and non-finite values are
        // kept and counted (the test is written so that NaN fails it)
        if (!(v >= a.umin && v <= a.umax)) {
          if (v > a.umax && v - a.umax <= a.clamp_tol) { ++nclamp; v = a.umax; }
          else if (v < a.umin && a.umin - v <= a.clamp_tol) { ++nclamp; v = a.umin; }
          else ++nbad;
        }
      }
      a.uout[c * N + i] = v;
      vout[c] = v;
    }
    if constexpr (!SCALAR) {
      // invariant domain of the Euler equations: rho > 0 and p > 0 at every
      // node (Theorem 1); each failed condition counts once, NaN included
      const double pr = Phys<D, PH>::pressure(vout, a.ph);
      nbad += !(vout[0] > 0.0);
      nbad += !(pr > 0.0);
    }
    if constexpr (Phys<D, PH>::kNodal) {
      // nodal fluxes of the new state, read by the next stage's element passes
      double f[D * M];
      Phys<D, PH>::flux_all(vout, f, a.ph);
#pragma unroll
      for (int q = 0; q < D * M; ++q) a.fnode[q * N + i] = f[q];
    }
  }
  // per-block counters, touched only when this stage counted something
  nclamp = wave_sum(nclamp);
  nbad = wave_sum(nbad);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = nclamp;
    red[1][threadIdx.x >> 6] = nbad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int c0 = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const int c1 = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    if (c0 != 0) a.counts[2 * bx] += c0;
    if (c1 != 0) a.counts[2 * bx + 1] += c1;
  }
}

template <int D, int P, int PH>
__global__ void __launch_bounds__(256) k_update(StageArgs a) {
  k_update_body<D, P, PH>(a, xcd_block(blockIdx.x, gridDim.x));
}

// nodal fluxes f_k(u_j) of the bound state (kNodal physics), used when the
// state did not come from a stage update (upload, bind, direct stage calls)
template <int D, int PH>
__global__ void __launch_bounds__(256) k_nodal_flux(StageArgs a) {
  constexpr int M = Phys<D, PH>::M;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.mesh.N) return;
  double v[M], f[D * M];
#pragma unroll
  for (int c = 0; c < M; ++c) v[c] = a.u[c * a.mesh.N + i];
  Phys<D, PH>::flux_all(v, f, a.ph);
#pragma unroll
  for (int q = 0; q < D * M; ++q) a.fnode[q * a.mesh.N + i] = f[q];
}

// The same reduction in one block of 1024 threads, ahead of the node update,
// when there are many per-block minima (k_update then reads dtbuf[0] instead
// of every block reducing all of them itself)
__device__ __forceinline__ void k_stage_dt_body(const StageArgs& a) {
  double m = 1.0e300;
  for (int j = threadIdx.x; j < a.ndtpart; j += 1024) m = fmin(m, a.dtpart[j]);
  const double mn = block_min<1024>(m);
  if (threadIdx.x == 0) stage_dt_record(a, mn);
}

__global__ void __launch_bounds__(1024) k_stage_dt(StageArgs a) { k_stage_dt_body(a); }

// LDS words of the fused gather's per-line slot table (ints per line)
constexpr int kGatherLineInts = 10;

// Residual assembly fused with the first mass-solve pass (axis 0): a block
// gathers r = sum_e (element residual vectors) for nlb whole x-lines into LDS
// (fixed element order per node, as k_gather_r), stores r, then applies the
// axis-0 line operator.
template <int D, int P, int M, int RE, class RT>
__device__ __forceinline__ void k_gather_line_x_body(const StageArgs& sa, const LineFastArgs& a, int bx) {
  constexpr int W = LineTapsV<P, RT>::W, R = P * RE, NL = ipow(P + 1, D);
  const int L = a.L;
  RT* sm = reinterpret_cast<RT*>(cem_smem);
  RT* rr = ResPtr<RT>::r(sa);
  const int64_t t0 = (int64_t)bx * a.nlb;
  const int nl = (int)min((int64_t)a.nlb, a.ntrans - t0);
  const int64_t E = sa.mesh.E, N = sa.mesh.N;
  const int lpc = (int)(N / L);                  // lines per component
  const int LS = line_row_len<P, RT>(L), LP = line_row_pitch<P, RT>(L);
  static_assert(R % 2 == 1 || R >= (P % 2 == 0 ? P : 2 * P), "row pitch too short for this run length");
  // Per line of the block: its component and the transverse element slots
  // of its nodes (one or two per axis > 0, lower element first), so that a
  // node's elements follow from its x position alone.  32-bit offsets: the
  // element vectors hold m (p+1)^d E < 2^31 values (checked at create).
  // ln[ql]: [0] component, [1] slots, [2..5] element offset n0 (ey + n1 ez),
  // [6..9] local offset (p+1) (ay + (p+1) az), in the order of k_gather_r
  int* ln = reinterpret_cast<int*>(sm + (size_t)a.nlb * LP);
  for (int ql = threadIdx.x; ql < nl; ql += blockDim.x) {
    const int line = (int)t0 + ql, c = line / lpc;
    unsigned r = (unsigned)(line - c * lpc);
    int ik[3] = {0, 0, 0};
    if (D > 1) {
      ik[1] = (int)(r % (unsigned)sa.mesh.L[1]);
      r /= (unsigned)sa.mesh.L[1];
    }
    if (D > 2) ik[2] = (int)r;
    int cnt[3] = {1, 1, 1}, ek[3][2] = {{0, 0}, {0, 0}, {0, 0}}, ak[3][2] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
    for (int k = 1; k < D; ++k) {
      const int e0 = ik[k] / P, a0 = ik[k] % P;
      if (a0 == 0) {
        cnt[k] = 2;
        ek[k][0] = e0 == 0 ? sa.mesh.n[k] - 1 : e0 - 1;
        ak[k][0] = P;
        ek[k][1] = e0;
      } else {
        ek[k][0] = e0;
        ak[k][0] = a0;
      }
    }
    int ns = 0;
    for (int z = 0; z < cnt[2]; ++z)
      for (int y = 0; y < cnt[1]; ++y) {
        ln[ql * kGatherLineInts + 2 + ns] = sa.mesh.n[0] * (ek[1][y] + sa.mesh.n[1] * ek[2][z]);
        ln[ql * kGatherLineInts + 6 + ns] = (P + 1) * (ak[1][y] + (P + 1) * ak[2][z]);
        ++ns;
      }
    ln[ql * kGatherLineInts] = c;
    ln[ql * kGatherLineInts + 1] = ns;
  }
  __syncthreads();
  const DivMagic dl((unsigned)L);
  const int Ei = (int)E;
  for (int q = threadIdx.x; q < nl * L; q += blockDim.x) {
    const int ql = (int)dl.div((unsigned)q), x = q - ql * L;
    const int* li = ln + ql * kGatherLineInts;
    const int c = li[0], nyz = li[1];
    // x slots: the lower element (local a = P) first where x is a vertex
    const int e0 = x / P, a0 = x - e0 * P;
    const int nx = a0 == 0 ? 2 : 1;
    const int ex0 = a0 == 0 ? (e0 == 0 ? sa.mesh.n[0] - 1 : e0 - 1) : e0;
    const int ax0 = a0 == 0 ? P : a0;
    const int cb = c * NL;
    double s = 0.0;
#pragma unroll
    for (int yz = 0; yz < (D == 3 ? 4 : (D == 2 ? 2 : 1)); ++yz) {
      if (yz < nyz) {
        const int eb = li[2 + yz], lb = cb + li[6 + yz];
        s += sa.relem[(int64_t)((lb + ax0) * Ei + eb + ex0)];
        if (nx == 2) s += sa.relem[(int64_t)(lb * Ei + eb + e0)];
      }
    }
    sm[ql * LP + lds_slot<R>(W + x)] = (RT)s;
    if (sa.store_r) rr[(t0 + ql) * L + x] = (RT)s;   // component-major: line t0 + ql starts at c N + ...
  }
  __syncthreads();
  // periodic padding of the rows from their interiors
  const int pad = LS - L;
  const DivMagic dpad((unsigned)pad);
  for (int q = threadIdx.x; q < nl * pad; q += blockDim.x) {
    const int ql = (int)dpad.div((unsigned)q), h = q - ql * pad;
    const int k = h < W ? h : L + h;
    sm[ql * LP + lds_slot<R>(k)] = sm[ql * LP + lds_slot<R>(W + line_wrap(k, W, L))];
  }
  __syncthreads();
  const int runs = (L + R - 1) / R;
  const DivMagic drun((unsigned)runs);
  for (int g = threadIdx.x; g < nl * runs; g += blockDim.x) {
    const int line = (int)drun.div((unsigned)g), s = (g - line * runs) * R;
    const RT* row = sm + line * LP + lds_slot<R>(s);
    auto ld = [&](int j) { return row[lds_slot<R>(j)]; };
    RT acc[R];
    line_run<P, RE>(static_cast<const RT*>(a.w), ld, acc);
    RT* dst = static_cast<RT*>(a.out) + (t0 + line) * L;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (s + r < L) dst[s + r] = acc[r];
  }
}

template <int D, int P, int M, int RE, class RT>
__global__ void __launch_bounds__(256) k_gather_line_x(StageArgs sa, LineFastArgs a) {
  k_gather_line_x_body<D, P, M, RE, RT>(sa, a, xcd_block(blockIdx.x, gridDim.x));
}

// zero fill of n 32-bit words (counters and flags that must start at zero,
// in code a caller may capture into a graph: a kernel, not a memset node)
// Low-order time derivative for the Q1 contributions (Sec. 3, the
// low-order scheme with its Rusanov term; periodic, b_i = 0):
// udot_i^L = -(1 / |E_i|) sum over the elements e around node i of
// F^e / |K| + (u_i - u^e) / dt_e, F^e = int_dK f_h . n from element pass 1;
// m_i^e / m_i = 1 / |E_i| for Bernstein elements.  Elements in
// node_elements' fixed order.  Scalar problems.
template <int D, int P>
__global__ void __launch_bounds__(256) k_udot_lo(StageArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.mesh.N) return;
  int64_t eids[8];
  int locs[8];
  const int ne = node_elements<D, P>(i, a.mesh, eids, locs);
  double vol = 1.0;
#pragma unroll
  for (int k = 0; k < D; ++k) vol *= a.mesh.h;
  const double ui = a.u[i];
  double s = 0.0;
  for (int r = 0; r < ne; ++r) {
    const int64_t e = eids[r];
    s += a.fdiv[e] / vol + (ui - a.ue[e]) / a.dte[e];
  }
  a.udot[i] = -s / ne;
}

__global__ void __launch_bounds__(256) k_zero_words(unsigned* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// float -> double copy (debug taps of the mixed-precision intermediates)
__global__ void __launch_bounds__(256) k_widen(const float* in, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

// ---------------------------------------------------------------------------
// reductions for invariant checks: per-block partials, then one block
// ---------------------------------------------------------------------------
struct InvArgs {
  const double* u;
  int64_t N;
  int M, D, euler;
  double gam, mnode;      // lumped-mass unit h^D / NL
  int P;
  int Lx, Ly;
  double umin, umax, tol; // scalar bounds and round-off clamp width
  double* part;           // [blocks][M*3 + 4]
};

// number of partial values per block: per component min, max, mass; then
// rho_min, p_min (Euler), the count of non-finite values and the count of
// failed invariant-domain conditions of the state
__host__ __device__ inline int inv_nvals(int M) { return M * 3 + 4; }

__device__ inline int node_mult(int64_t i, int D, int P, int Lx, int Ly) {
  int ik[3] = {(int)(i % Lx), 0, 0};
  if (D > 1) ik[1] = (int)((i / Lx) % Ly);
  if (D > 2) ik[2] = (int)(i / ((int64_t)Lx * Ly));
  int m = 1;
  for (int k = 0; k < D; ++k)
    if (ik[k] % P == 0) m *= 2;
  return m;
}

// min / max that return NaN when either argument is NaN (fmin / fmax drop
// it, which would hide a diverged state from the checks)
__device__ __forceinline__ double nan_min(double x, double y) { return (x < y || x != x) ? x : y; }
__device__ __forceinline__ double nan_max(double x, double y) { return (x > y || x != x) ? x : y; }

__global__ void __launch_bounds__(256) k_inv_partial(InvArgs a) {
  __shared__ double red[256];
  const int nv = inv_nvals(a.M);
  const int64_t per = (a.N + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * per, hi = min(a.N, lo + per);
  for (int v = 0; v < nv; ++v) {
    const int c = v / 3, kind = v < a.M * 3 ? v % 3 : 3 + (v - a.M * 3);
    // kinds: 0 min, 1 max, 2 mass, 3 rho_min, 4 p_min, 5 non-finite, 6 violations
    const bool is_min = kind == 0 || kind == 3 || kind == 4, is_sum = kind == 2 || kind >= 5;
    double acc = is_min ? 1.0e300 : (kind == 1 ? -1.0e300 : 0.0);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      if (kind <= 2) {
        const double x = a.u[c * a.N + i];
        if (kind == 0) acc = nan_min(acc, x);
        else if (kind == 1) acc = nan_max(acc, x);
        else acc += a.mnode * node_mult(i, a.D, a.P, a.Lx, a.Ly) * x;
      } else if (kind == 5) {
        for (int q = 0; q < a.M; ++q) acc += !isfinite(a.u[q * a.N + i]);
      } else if (a.euler) {
        const double rho = a.u[i];
        double m2 = 0.0;
        for (int k = 0; k < a.D; ++k) m2 += a.u[(1 + k) * a.N + i] * a.u[(1 + k) * a.N + i];
        const double pr = (a.gam - 1.0) * (a.u[(a.D + 1) * a.N + i] - 0.5 * m2 / rho);
        if (kind == 3) acc = nan_min(acc, rho);
        else if (kind == 4) acc = nan_min(acc, pr);
        else acc += (double)(!(rho > 0.0)) + (double)(!(pr > 0.0));
      } else if (kind == 6) {
        // a scalar value outside the bounds by more than the clamp width,
        // or not a number
        const double x = a.u[i];
        acc += !(x >= a.umin - a.tol && x <= a.umax + a.tol);
      }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        const double x = red[threadIdx.x], y = red[threadIdx.x + s];
        red[threadIdx.x] = is_sum ? x + y : (is_min ? nan_min(x, y) : nan_max(x, y));
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) a.part[(int64_t)blockIdx.x * nv + v] = red[0];
    __syncthreads();
  }
}

}  // namespace cem
