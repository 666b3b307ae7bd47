// Element passes of systems (the Euler equations, m = d + 2 components) on
// gfx950: one thread per (element, component).  A block holds EB elements
// and m groups of EB threads, group c working on component c.  Everything
// that acts on one component at a time (the WENO sensor of eqs. (7)-(8), the
// interpolation to the Gauss points, the test-function contractions, the
// stabilisation, the consistent-mass term) runs in the component's thread;
// what couples the components (fluxes at Gauss points and facet nodes, node
// and facet wave speeds, the positivity factors of Appendix A) reads the full
// states from one LDS buffer S[point][component][element].
//
// Register budget: a thread holds at most three arrays of (p+1)^d doubles.
// The element's own coefficients are read from S (LDS addresses are a base
// register plus an immediate), not re-gathered from HBM: held 64-bit gather
// addresses were what exhausted the registers of the 3D Q2 pass.
#pragma once
#include "kernels.hpp"

namespace cem {

template <int D, int P, int PH, int EB_> struct SysLayout {
  static constexpr int EB = EB_;
  static constexpr int M = Phys<D, PH>::M, P1 = P + 1, NL = ipow(P1, D);
  static constexpr int NS = NL * M * EB;         // nodal states, later Gauss-point states
  static constexpr int oUe = NS;                 // [M][EB] cell averages (pass 1)
  static constexpr int oNm = oUe + M * EB;       // [2D][M][EB] neighbour averages (pass 1)
  static constexpr int oPart = oNm + 2 * D * M * EB;   // [M][EB] per-group maxima / minima
  static constexpr int oGam = oPart + M * EB;    // [M][EB] per-component sensor values
  static constexpr int oFac = oGam + M * EB;     // [2D][EB] facet wave speeds or facet alphas
  static constexpr int oUb = oFac + 2 * D * EB;  // [M][EB] flux-limited averages (pass 2)
  static constexpr int oRed = oUb + M * EB;      // [EB] dt_e of the block
  static constexpr int words = oRed + EB;
  static constexpr size_t bytes = (size_t)words * sizeof(double);
};

// elements per block: 64 when the block's LDS stays within 64 KiB, else 32;
// block bx holds elements bx EB .. bx EB + EB - 1 (consecutive lanes store
// consecutive elements of the [c][E] arrays).  Bricks of 8 x 2 x 2 elements
// (facet neighbours along y and z in the same block) measured slower on the
// 128^3 Q2 blast: 78.0 against 76.0 ms per step, the per-element stores
// coalescing in runs of 8.
template <int D, int P, int PH> struct SysTile {
  static constexpr int EB = SysLayout<D, P, PH, 64>::bytes <= 65536 ? 64 : 32;
  using LY = SysLayout<D, P, PH, EB>;
  // blocks over a mesh of n[0] x n[1] x n[2] elements
  __host__ __device__ static int64_t blocks(const int* n) {
    int64_t E = 1;
    for (int k = 0; k < D; ++k) E *= n[k];
    return (E + EB - 1) / EB;
  }
  // element of lane le in block bx; false for lanes past the mesh (they redo
  // the last element and store nothing)
  __device__ static bool element(const MeshArgs& m, int bx, int le, int64_t* e) {
    const int64_t e0 = (int64_t)bx * EB;
    const bool live = e0 + le < m.E;
    *e = live ? e0 + le : m.E - 1;
    return live;
  }
};

// component c of a value array computed for all components (a select chain:
// no dynamically indexed register array)
template <int M, class V>
__device__ __forceinline__ V pick_c(const V* v, int c) {
  V r = v[0];
#pragma unroll
  for (int k = 1; k < M; ++k)
    if (c == k) r = v[k];
  return r;
}


// v[i] for a runtime i < K, and v[i] = x, without a dynamically indexed
// register array (which would live in scratch)
template <int K, class V>
__device__ __forceinline__ V get_sel(const V* v, int i) {
  V r = v[0];
#pragma unroll
  for (int k = 1; k < K; ++k)
    if (i == k) r = v[k];
  return r;
}
template <int K, class V>
__device__ __forceinline__ void set_sel(V* v, int i, V x) {
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (i == k) v[k] = x;
}

// x <- (A along axis K) x in place, one line of P+1 values at a time (the
// same sums as ax1 with a (P+1)-value temporary instead of a second array)
template <int D, int P, int K, class TB, class V>
__device__ __forceinline__ void ax_ip1(const TB& T, int ao, bool trn, V* x) {
  constexpr int P1 = P + 1, NL = ipow(P1, D), ST = ipow(P1, K);
#pragma unroll
  for (int i0 = 0; i0 < NL; ++i0) {
    if ((i0 / ST) % P1 != 0) continue;   // i0 starts a line along axis K
    V v[P1];
#pragma unroll
    for (int b = 0; b < P1; ++b) v[b] = x[i0 + b * ST];
#pragma unroll
    for (int ai = 0; ai < P1; ++ai) {
      V s = 0;
#pragma unroll
      for (int b = 0; b < P1; ++b) s += T(ao + (trn ? b * P1 + ai : ai * P1 + b)) * v[b];
      x[i0 + ai * ST] = s;
    }
  }
}

template <int D, int P, class TB, class V>
__device__ __forceinline__ void ax_ip(int k, const TB& T, int ao, bool trn, V* x) {
  if (k == 0) ax_ip1<D, P, 0>(T, ao, trn, x);
  else if constexpr (D > 1) {
    if (k == 1) ax_ip1<D, P, 1>(T, ao, trn, x);
    else if constexpr (D > 2) ax_ip1<D, P, 2>(T, ao, trn, x);
  }
}

// x <- (A_{D-1} (x) ... (x) A_0) x in place, axis 0 first (as tensor_apply)
template <int D, int P, class TB, class V>
__device__ __forceinline__ void tensor_ip(const TB& T, const int* mo, bool trn, V* x) {
  if constexpr (D >= 1) ax_ip1<D, P, 0>(T, mo[0], trn, x);
  if constexpr (D >= 2) ax_ip1<D, P, 1>(T, mo[1], trn, x);
  if constexpr (D >= 3) ax_ip1<D, P, 2>(T, mo[2], trn, x);
}

// component c of the Euler flux along axis k (both may be runtime values):
// the same operations as Phys<D, EUL>::flux, written with selects so that
// no register array is indexed dynamically
template <int D, class V>
__device__ __forceinline__ V euler_flux_comp(int k, int c, const V* u, double gam) {
  V mk = u[1];
  if (D > 1 && k == 1) mk = u[2];
  if (D > 2 && k == 2) mk = u[3];
  V m2 = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) m2 += u[1 + j] * u[1 + j];
  const V ir = (V)1 / u[0];
  const V p = ((V)gam - (V)1) * (u[D + 1] - (V)0.5 * m2 * ir);
  const V vk = mk * ir;
  V r = pick_c<D + 2>(u, c) * vk + (c - 1 == k ? p : (V)0);
  if (c == 0) r = mk;
  if (c == D + 1) r = vk * (u[D + 1] + p);
  return r;
}

// full state of point q from S (component-major inside a point)
template <int M, int EB>
__device__ __forceinline__ void state_at(const double* S, int q, int le, double* u) {
#pragma unroll
  for (int k = 0; k < M; ++k) u[k] = S[(q * M + k) * EB + le];
}

// minimum of dt_e over the block's elements (group 0 holds them)
template <int EB>
__device__ __forceinline__ void block_min_dt_sys(double* red, double* part, int c, int le, double v, int bx) {
  if (c == 0) red[le] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int i = 1; i < EB; ++i) m = fmin(m, red[i]);
    part[bx] = m;
  }
}

// Element pass 1 of systems in two launches, each with fewer live registers
// than the whole (so that two waves per SIMD fit without more spilling):
// PART 1 the sensor, viscosity and facet data; PART 2 the element residual,
// from the cell averages, gamma_e and nu_e that PART 1 stored.
template <int D, int P, int PH, class RT, int PART>
__device__ __forceinline__ void k_elem1_sys_body(const StageArgs& a, int bx) {
  static_assert(PH == EUL, "system element pass 1 is written for the Euler equations");
  static_assert(PART == 1 || PART == 2, "PART 1: sensor and facets, PART 2: residual");
  using PHY = Phys<D, PH>;
  using SF = SFLayout<D, P>;
  using LY = typename SysTile<D, P, PH>::LY;
  constexpr int EB = LY::EB, P1 = P + 1, NL = LY::NL, M = LY::M, NF = NL / P1, CS = M * EB;
  constexpr bool MIX = sizeof(RT) == 4;
  const TabRef<RT> T{TabSel<RT>::of(a.tab)};
  const MeshArgs& ms = a.mesh;
  const int64_t E = ms.E, N = ms.N;
  const double h = ms.h;
  const int c = threadIdx.x / EB, le = threadIdx.x - c * EB;
  int64_t e;                                   // idle lanes redo the last element, store nothing
  const bool live = SysTile<D, P, PH>::element(ms, bx, le, &e);
  double* S = cem_smem;
  double* Us = S + c * EB + le;               // own coefficients / Gauss values: Us[j * CS]
  const GlobalNodes<D, P, M> ns(a, e);

  // ---- own coefficients into S, cell average
  double ue_c = 0.0;
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const double v = a.u[c * N + ns.own_node(j)];
    ue_c += v;
    Us[j * CS] = v;
  }
  ue_c *= (1.0 / NL);
  double uo[M], gam, nu;
  if constexpr (PART == 2) {
    // stored by PART 1 (the same sums)
    ue_c = a.ue[c * E + e];
#pragma unroll
    for (int k = 0; k < M; ++k) uo[k] = a.ue[k * E + e];
    gam = a.gam[e];
    nu = a.nu[e];
  } else {

  // ---- WENO sensor of component c (Sec. 2.2, eqs. 7-8): candidates are
  // the facet neighbours extended into K_e by the blossom maps; semi-norms
  // are the packed quadratic form on coefficients shifted by their first
  // entry.  The neighbour averages go to S for the facet fluxes.  The
  // neighbour loops are not unrolled: unrolled, the compiler issues all 2d
  // candidates' loads together and runs out of registers.
  // The nonlinear weights share one denominator: sum_l w_l (u - u_l)
  // builds up with unnormalised weights as each candidate is formed and is
  // scaled once at the end, so every candidate is extended once.
  double gc = 1.0;
  {
    const bool sense = a.gamma_mode == 0;
    auto nrm = [&](RT b) { return (a.rexp == 2.0) ? b : (RT)pow((double)b, 0.5 * a.rexp); };
    const RT eps = (RT)a.eps, wlin = (RT)a.w_lin;
    const double u0 = Us[0];
    RT beta0;
    {
      RT x[NL];
#pragma unroll
      for (int j = 0; j < NL; ++j) x[j] = (RT)(Us[j * CS] - u0);
      beta0 = qsym<NL>(T, SF::qp, x);
    }
    RT wsum = (RT)(1.0 - 2 * D * a.w_lin) / (nrm(beta0) + eps);
    RT w[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) w[j] = 0;
    // the axis is a compile-time constant in the body, so the candidate
    // arrays stay in registers; the two sides of an axis form a rolled loop
    static_for<D>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
#pragma unroll 1
      for (int side = 0; side < 2; ++side) {
        const int l = 2 * k + side;
        double cn[NL], sum = 0.0;
        ns.load_nbr(c, l, cn);
#pragma unroll
        for (int j = 0; j < NL; ++j) sum += cn[j];
        S[LY::oNm + (l * M + c) * EB + le] = sum * (1.0 / NL);
        if (!sense) continue;
        RT cr[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) cr[j] = (RT)(cn[j] - cn[0]);
        ax_ip1<D, P, k>(T, SF::ext + side * P1 * P1, false, cr);
        const RT wt = wlin / (nrm(qsym<NL>(T, SF::qp, cr)) + eps);
        wsum += wt;
#pragma unroll
        for (int i = 0; i < NL; ++i) w[i] += wt * ((RT)(Us[i * CS] - u0) - cr[i]);
      }
    });
    if (sense) {
      const RT iws = (RT)1 / wsum;
#pragma unroll
      for (int i = 0; i < NL; ++i) w[i] *= iws;
      // 0/0 on constant elements, regularised with the weights' epsilon
      const RT q2 = qsym<NL>(T, SF::qp, w);
      const RT dev = sqrt(q2 > (RT)0 ? q2 : (RT)0);
      RT ratio = dev / sqrt((beta0 > (RT)0 ? beta0 : (RT)0) + eps);
      ratio = ratio < (RT)1 ? ratio : (RT)1;
      gc = 1.0 - (a.q == 1.0 ? (double)ratio : pow((double)ratio, a.q));
    }
  }
  S[LY::oUe + c * EB + le] = ue_c;
  S[LY::oGam + c * EB + le] = gc;
  __syncthreads();

  // ---- facet wave speeds (eq. 18), facet l handled by group l mod m;
  // node speeds (viscosity), nodes j = c, c + m, ...
#pragma unroll
  for (int k = 0; k < M; ++k) uo[k] = S[LY::oUe + k * EB + le];
#pragma unroll
  for (int l = 0; l < 2 * D; ++l) {
    if (l % M != c) continue;
    double un[M];
#pragma unroll
    for (int k = 0; k < M; ++k) un[k] = S[LY::oNm + (l * M + k) * EB + le];
    const int k = l / 2;
    const double lm = (l % 2) ? PHY::riemann_speed(uo, un, k, a.ph) : PHY::riemann_speed(un, uo, k, a.ph);
    S[LY::oFac + l * EB + le] = lm;
  }
  {
    double lam = 0.0;
    for (int j = c; j < NL; j += M) {
      double uj[M];
      state_at<M, EB>(S, j, le, uj);
      lam = fmax(lam, PHY::node_speed(uj, a.ph));
    }
    S[LY::oPart + c * EB + le] = lam;
  }
  __syncthreads();
  double gmin = 1.0, lam = 0.0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    gmin = fmin(gmin, S[LY::oGam + k * EB + le]);
    lam = fmax(lam, S[LY::oPart + k * EB + le]);
  }
  gam = a.gamma_mode == 0 ? gmin : (a.gamma_mode == 1 ? 0.0 : 1.0);
  nu = lam * h / (2.0 * P);

  // ---- facet fluxes of component c (eqs. 18, 40, 42, 51): f^L against the
  // neighbour averages, f^H = mean of f(u_j) n over the facet's nodes
  double lamsum = 0.0, fLsum = 0.0, fHout = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double fo[M];
    PHY::flux(k, uo, fo, a.ph);
    const double foc = pick_m<M>(fo, c);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int l = 2 * k + side;
      double un[M], fn[M];
#pragma unroll
      for (int kk = 0; kk < M; ++kk) un[kk] = S[LY::oNm + (l * M + kk) * EB + le];
      PHY::flux(k, un, fn, a.ph);
      const double fnc = pick_m<M>(fn, c), unc = pick_m<M>(un, c);
      const double lm = S[LY::oFac + l * EB + le];
      lamsum += lm;
      const double fl = side ? foc : fnc, fr = side ? fnc : foc;
      const double uL = side ? ue_c : unc, uR = side ? unc : ue_c;
      const double fLc = 0.5 * (fl + fr) - 0.5 * lm * (uR - uL);
      fLsum += side ? fLc : -fLc;
      if (side || a.flux_mode != 0) {
        double fH = 0.0;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
          if (dig(j, k, P1) != (side ? P : 0)) continue;
          double uj[M], fj[M];
          state_at<M, EB>(S, j, le, uj);
          PHY::flux(k, uj, fj, a.ph);
          fH += pick_m<M>(fj, c);
        }
        fHout += side ? fH * (1.0 / NF) : -(fH * (1.0 / NF));
        if (side && live) a.fahi[((int64_t)k * M + c) * E + e] = fLc - fH * (1.0 / NF);
      }
    }
  }
  double dt_e = h / lamsum;                                   // eq. (40)
  if (a.flux_mode != 0) {
    // flux limiter off (Sec. 4.3, steps 3-4): ubar^e = u^e - dt_e / h sum
    // f^H . n, dt_e of Lemma 1 (eq. 37) or eq. (40) reduced until ubar^e is
    // admissible.  The groups share the work through S (oGam, oPart, oUb
    // are free here once every thread has read gamma and the node speeds).
    __syncthreads();
    if (a.flux_mode == 1) {
      constexpr int NI = ipow(P - 1, D);
      double u0[M];
#pragma unroll
      for (int k = 0; k < M; ++k) u0[k] = uo[k];
      if constexpr (NI > 0) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
          double sum = 0.0;
#pragma unroll
          for (int j = 0; j < NL; ++j)
            if (interior_node<D, P>(j)) sum += S[(j * M + k) * EB + le];
          u0[k] = sum * (1.0 / (NI > 0 ? NI : 1));
        }
      }
      double hd = 1.0;
#pragma unroll
      for (int k = 0; k < D; ++k) hd *= h;
      const double mi = hd * (1.0 / NL);
      double tnode = 1.0e300, csum = 0.0;
      for (int j = c; j < NL; j += M) {        // boundary nodes split over the groups
        double uj[M];
        state_at<M, EB>(S, j, le, uj);
        const double cl = subcell_node<D, P, PHY>(j, u0, uj, h, a.ph);
        if (cl > 0.0) tnode = fmin(tnode, mi / cl);
        csum += cl;
      }
      S[LY::oGam + c * EB + le] = tnode;
      S[LY::oPart + c * EB + le] = csum;
      __syncthreads();
      tnode = 1.0e300;
      csum = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        tnode = fmin(tnode, S[LY::oGam + k * EB + le]);
        csum += S[LY::oPart + k * EB + le];
      }
      dt_e = subcell_combine<D, P>(tnode, csum, h);
    } else {
      S[LY::oUb + c * EB + le] = fHout;
      __syncthreads();
      double dl[M];
#pragma unroll
      for (int k = 0; k < M; ++k) dl[k] = -dt_e / h * S[LY::oUb + k * EB + le];
      dt_e *= euler_alpha<D>(uo, dl, 1.0, a.eps_pos);
    }
    if (live) a.ubar[c * E + e] = ue_c - dt_e / h * fHout;
  }
  if (live) {
    a.ue[c * E + e] = ue_c;
    a.ubarL[c * E + e] = ue_c - dt_e / h * fLsum;
    if (c == 0) {
      a.dte[e] = dt_e;
      a.gam[e] = gam;
      a.nu[e] = nu;
    }
  }
  block_min_dt_sys<EB>(S + LY::oRed, a.dtpart, c, le, live ? dt_e : 1.0e300, bx);
  return;
  }   // PART 1

  // ---- element residual R_i = int grad phi_i . f(u_h) - s_h^e(phi_i, u_h):
  // the stabilisation first (from the nodal coefficients), then the Gauss-
  // point states replace the nodal ones in S for the flux term
  double hpow = 1.0;
#pragma unroll
  for (int k = 0; k < D - 1; ++k) hpow *= h;   // h^{D-1}
  RT R[NL];
  {
    const RT sa = (RT)(nu * hpow / h), sg = (RT)(nu * gam * hpow);
#pragma unroll
    for (int i = 0; i < NL; ++i) R[i] = 0;
    // not unrolled: unrolled, all D (p+1)^d gradient loads are issued up
    // front and spilled
#pragma unroll 1
    for (int k = 0; k < D; ++k) {
      const int ms1[3] = {k == 0 ? SF::k1 : SF::g, k == 1 ? SF::k1 : SF::g, k == 2 ? SF::k1 : SF::g};
      const int ms2[3] = {k == 0 ? SF::ct : SF::g, k == 1 ? SF::ct : SF::g, k == 2 ? SF::ct : SF::g};
      RT t[NL];
#pragma unroll
      for (int j = 0; j < NL; ++j) t[j] = MIX ? (RT)(Us[j * CS] - ue_c) : (RT)Us[j * CS];
      tensor_ip<D, P>(T, ms1, false, t);
#pragma unroll
      for (int i = 0; i < NL; ++i) R[i] -= sa * t[i];
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        const int64_t q = ((int64_t)k * M + c) * N + ns.own_node(j);
        if constexpr (MIX) t[j] = a.g32[q];
        else t[j] = a.g[q];
      }
      tensor_ip<D, P>(T, ms2, false, t);
#pragma unroll
      for (int i = 0; i < NL; ++i) R[i] += sg * t[i];
    }
  }
  {
    // mixed form: interpolate U - ubar in float, keep the states in float64
    RT uq[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) uq[j] = MIX ? (RT)(Us[j * CS] - ue_c) : (RT)Us[j * CS];
    const int mv[3] = {SF::vq, SF::vq, SF::vq};
    tensor_ip<D, P>(T, mv, false, uq);
    __syncthreads();    // every thread is done with the nodal states
#pragma unroll
    for (int q = 0; q < NL; ++q) Us[q * CS] = MIX ? ue_c + (double)uq[q] : (double)uq[q];
  }
  __syncthreads();
  // flux term, one axis at a time (a rolled loop: unrolled, the axes'
  // Gauss-point work is interleaved and runs out of registers)
#pragma unroll 1
  for (int k = 0; k < D; ++k) {
    RT F[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      RT wv = 1;
#pragma unroll
      for (int j = 0; j < D; ++j) wv *= T(SF::wq + dig(q, j, P1));
      if constexpr (MIX) {
        // flux deviation from the cell average's flux, evaluated in float64
        double uv[M];
#pragma unroll
        for (int kk = 0; kk < M; ++kk) uv[kk] = S[(q * M + kk) * EB + le];
        F[q] = wv * (RT)(euler_flux_comp<D>(k, c, uv, a.ph.gam) - euler_flux_comp<D>(k, c, uo, a.ph.gam));
      } else {
        RT uv[M];
#pragma unroll
        for (int kk = 0; kk < M; ++kk) uv[kk] = (RT)S[(q * M + kk) * EB + le];
        F[q] = wv * euler_flux_comp<D>(k, c, uv, a.ph.gam);
      }
    }
    const int mt[3] = {k == 0 ? SF::dq : SF::vq, k == 1 ? SF::dq : SF::vq, k == 2 ? SF::dq : SF::vq};
    tensor_ip<D, P>(T, mt, true, F);
#pragma unroll
    for (int i = 0; i < NL; ++i) R[i] += (RT)hpow * F[i];
  }
  if (live) {
    // element vectors are float64; the mixed form adds back the flux of the
    // cell average removed from the float contraction
    double fbk[D];
#pragma unroll
    for (int k = 0; k < D; ++k) fbk[k] = MIX ? euler_flux_comp<D>(k, c, uo, a.ph.gam) : 0.0;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      double v = (double)R[i];
      if constexpr (MIX) {
        double fb = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) fb += fbk[k] * ref_grad_int<D, P>(i, k);
        v += hpow * fb;
      }
      a.relem[((int64_t)c * NL + i) * E + e] = v;
    }
  }
}

// pass 2: at least two waves per SIMD in float64 (the 2D pass fits three),
// three in the 3D mixed form (23.6 -> 20.9 ms per six launches; float64 at
// three spills and slows, 22.7 -> 25.4); the 2D mixed form as float64 (held
// at three it spilled: Q2 batch 4.4 -> 3.9 ms per launch without)
#define CEM_SYS2_BOUNDS __launch_bounds__((Phys<D, PH>::M * SysTile<D, P, PH>::EB)) \
  __attribute__((amdgpu_waves_per_eu(sizeof(RT) == 4 && D == 3 ? 3 : 2, sizeof(RT) == 4 && D == 3 ? 3 : 8)))

// both halves of pass 1 (the whole pass in one kernel needed 256 VGPRs plus
// AGPRs, one wave per SIMD, 22.4 ms per launch on the 128^3 Q2 blast; the
// halves at two waves 6.9 + 7.6 ms): two waves per SIMD in float64, three in
// the mixed form, whose float contractions need fewer registers (ms per six
// launches: sensor half 37.4 -> 31.7, residual half 44.7 -> 40.5; float64 at
// three waves spills and slows, residual 45.4 -> 61.6)
#define CEM_SYS1_BOUNDS __launch_bounds__((Phys<D, PH>::M * SysTile<D, P, PH>::EB)) \
  __attribute__((amdgpu_waves_per_eu(sizeof(RT) == 4 ? 3 : 2, sizeof(RT) == 4 ? 3 : 2)))

template <int D, int P, int PH, class RT>
__global__ void CEM_SYS1_BOUNDS k_elem1_sys(StageArgs a) {
  k_elem1_sys_body<D, P, PH, RT, 1>(a, xcd_block(blockIdx.x, gridDim.x));
}

template <int D, int P, int PH, class RT>
__global__ void CEM_SYS1_BOUNDS k_resid_sys(StageArgs a) {
  k_elem1_sys_body<D, P, PH, RT, 2>(a, xcd_block(blockIdx.x, gridDim.x));
}

// flux-pair factor of Appendix A for the facet between eL and eR normal to
// axis k (states ubar^{e,L} of both sides, increments of the raw f^A)
template <int D>
__device__ inline double euler_facet_alpha(const StageArgs& a, int k, int64_t eL, int64_t eR) {
  constexpr int M = D + 2;
  if (a.alpha_mode == 2) return 1.0;
  if (a.alpha_mode == 1) return 0.0;
  const int64_t E = a.mesh.E;
  const double dtL = a.dte[eL], dtR = a.dte[eR];
  const double phi = a.mesh.h / (2.0 * D);
  double uLs[M], uRs[M], dL[M], dR[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const double fA = a.fahi[((int64_t)k * M + q) * E + eL];
    uLs[q] = a.ubarL[q * E + eL];
    uRs[q] = a.ubarL[q * E + eR];
    dL[q] = fA / phi * dtL;
    dR[q] = -fA / phi * dtR;
  }
  return fmin(euler_alpha<D>(uLs, dL, 1.0, a.eps_pos), euler_alpha<D>(uRs, dR, 1.0, a.eps_pos));
}

template <int D, int P, int PH, class RT>
__device__ __forceinline__ void k_elem2_sys_body(const StageArgs& a, int bx) {
  static_assert(PH == EUL, "system element pass 2 is written for the Euler equations");
  using PHY = Phys<D, PH>;
  using SF = SFLayout<D, P>;
  using LY = typename SysTile<D, P, PH>::LY;
  constexpr int EB = LY::EB, P1 = P + 1, NL = LY::NL, M = LY::M, NF = NL / P1, CS = M * EB;
  constexpr bool MIX = sizeof(RT) == 4;
  const TabRef<RT> T{TabSel<RT>::of(a.tab)};
  const MeshArgs& ms = a.mesh;
  const int64_t E = ms.E, N = ms.N;
  const double h = ms.h;
  const int c = threadIdx.x / EB, le = threadIdx.x - c * EB;
  int64_t e;
  const bool live = SysTile<D, P, PH>::element(ms, bx, le, &e);
  double* S = cem_smem;
  double* Us = S + c * EB + le;
  const GlobalNodes<D, P, M> ns(a, e);
  int64_t enb[2 * D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int en[3] = {ns.ei[0], ns.ei[1], ns.ei[2]};
    en[k] = ns.ei[k] == 0 ? ms.n[k] - 1 : ns.ei[k] - 1;
    enb[2 * k] = elem_id(en, ms);
    en[k] = ns.ei[k] + 1 == ms.n[k] ? 0 : ns.ei[k] + 1;
    enb[2 * k + 1] = elem_id(en, ms);
  }

  // ---- facet factors (Appendix A), facet l handled by group l mod m;
  // own coefficients into S
#pragma unroll
  for (int l = 0; l < 2 * D; ++l) {
    if (l % M != c || a.flux_mode != 0) continue;
    const int k = l / 2;
    S[LY::oFac + l * EB + le] =
        (l % 2) ? euler_facet_alpha<D>(a, k, e, enb[l]) : euler_facet_alpha<D>(a, k, enb[l], e);
  }
#pragma unroll
  for (int j = 0; j < NL; ++j) Us[j * CS] = a.u[c * N + ns.own_node(j)];
  __syncthreads();

  // ---- flux-limited average (eq. 44)
  const double dt_e = a.dte[e];
  double fbs = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (a.flux_mode != 0) break;
    fbs -= S[LY::oFac + (2 * k) * EB + le] * a.fahi[((int64_t)k * M + c) * E + enb[2 * k]];
    fbs += S[LY::oFac + (2 * k + 1) * EB + le] * a.fahi[((int64_t)k * M + c) * E + e];
  }
  const double ub_c = a.flux_mode != 0 ? a.ubar[c * E + e]      // f = f^H, from element pass 1
                                       : a.ubarL[c * E + e] + dt_e / h * fbs;
  const double ue_c = a.ue[c * E + e];
  S[LY::oUb + c * EB + le] = ub_c;
  if (live && a.flux_mode == 0) a.ubar[c * E + e] = ub_c;

  // ---- boundary integral B_i = int_{dK} phi_i f_h . n of component c (the
  // mixed form integrates f_h - f(ubar), its contraction partner)
  double ueall[M];
#pragma unroll
  for (int k = 0; k < M; ++k) ueall[k] = a.ue[k * E + e];
  double hpow = 1.0;
#pragma unroll
  for (int k = 0; k < D - 1; ++k) hpow *= h;
  RT fb[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) fb[i] = 0;
  // the axis as a compile-time constant: left to "#pragma unroll" the
  // compiler kept the axis loop rolled, and the facet-node index arithmetic
  // became runtime divisions and dynamically indexed registers; the two
  // sides stay a rolled loop (fewer live registers)
  static_for<D>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {
      const int av = side ? P : 0;
      const RT sg = (RT)(side ? hpow : -hpow);
      const double fbar = MIX ? euler_flux_comp<D>(k, c, ueall, a.ph.gam) : 0.0;
      RT fn[NF];
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        if (dig(j, k, P1) != av) continue;
        const int fj = j % ipow(P1, k) + (j / ipow(P1, k + 1)) * ipow(P1, k);
        double uj[M], fv[M];
        state_at<M, EB>(S, j, le, uj);
        PHY::flux(k, uj, fv, a.ph);
        fn[fj] = (RT)(pick_m<M>(fv, c) - fbar);
      }
      const int mg[3] = {SF::g, SF::g, SF::g};
      tensor_ip<D - 1, P>(T, mg, false, fn);
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        if (dig(i, k, P1) != av) continue;
        const int fi = i % ipow(P1, k) + (i / ipow(P1, k + 1)) * ipow(P1, k);
        fb[i] += sg * fn[fi];
      }
    }
  });
  // ---- element contributions f_i^e of eq. (45); dU_i = m_i^e (ubar - u_i)
  const double hd = hpow * h, mloc = hd * (1.0 / NL);
  double dU[NL], f[NL];
  {
    RT Fe = 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) Fe += fb[i];
    auto udot_at = [&](int j) -> RT {
      const int64_t q = c * N + ns.own_node(j);
      if constexpr (MIX) return a.udot32[q];
      else return a.udot[q];
    };
    RT mu[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) mu[j] = udot_at(j);
    const int mg[3] = {SF::g, SF::g, SF::g};
    tensor_ip<D, P>(T, mg, false, mu);
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const RT Tc = (RT)hd * mu[i] - (RT)mloc * udot_at(i);
      const double R = a.relem[((int64_t)c * NL + i) * E + e];
      if constexpr (MIX) {
        double rb = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) rb += euler_flux_comp<D>(k, c, ueall, a.ph.gam) * ref_grad_int<D, P>(i, k);
        f[i] = (R - hpow * rb) + (double)(-fb[i] + Fe * (RT)(1.0 / NL) - Tc);
      } else {
        f[i] = (double)(R - fb[i] + Fe * (RT)(1.0 / NL) - Tc);
      }
    }
    // mixed form: remove the float rounding of the element sum of the
    // contraction terms (zero in exact arithmetic, eq. 47)
    double zs = 0.0;
    if constexpr (MIX) {
#pragma unroll
      for (int i = 0; i < NL; ++i) zs += f[i];
      zs *= 1.0 / NL;
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const double Ui = Us[i * CS];
      f[i] = mloc * (Ui - ue_c) + dt_e * (f[i] - zs);
      dU[i] = mloc * (ub_c - Ui);
    }
  }
  __syncthreads();    // all reads of the nodal states are done

  // ---- slope limiter (Appendix A on every node, ubar_i = ubar^e)
#pragma unroll
  for (int i = 0; i < NL; ++i) Us[i * CS] = f[i];
  __syncthreads();
  {
    double ub[M];
#pragma unroll
    for (int k = 0; k < M; ++k) ub[k] = S[LY::oUb + k * EB + le];
    double bp = 1.0;
    for (int i = c; i < NL; i += M) {
      double fi[M];
      state_at<M, EB>(S, i, le, fi);
      bp = fmin(bp, euler_alpha<D>(ub, fi, mloc, a.eps_pos));
    }
    S[LY::oPart + c * EB + le] = bp;
  }
  __syncthreads();
  double beta = 1.0;
#pragma unroll
  for (int k = 0; k < M; ++k) beta = fmin(beta, S[LY::oPart + k * EB + le]);
  if (a.beta_mode == 1) beta = 0.0;
  else if (a.beta_mode == 2) beta = 1.0;
  const double idt = 1.0 / dt_e;
  if constexpr (D == 2) {
    if (a.fuse_upd) {
      // ---- fused update (eq. 49 and the SSP-RK combination) of the nodes
      // whose elements all lie in this block (its EB consecutive elements):
      // their update vectors meet in LDS instead of HBM.  The other nodes'
      // vectors are stored for k_update as before.  Each node is updated by
      // the component threads of its first element in node_elements' order
      // (the lower one along each axis: the element holding it at local
      // indices >= 1), summing in that order, as k_update does; the stage
      // dt was reduced by k_stage_dt ahead of this launch.
      const int64_t e0 = (int64_t)bx * EB;
      const int n0 = ms.n[0], n1 = ms.n[1], ex = ns.ei[0], ey = ns.ei[1];
      const int exm = ex == 0 ? n0 - 1 : ex - 1, exq = ex + 1 == n0 ? 0 : ex + 1;
      const int eym = ey == 0 ? n1 - 1 : ey - 1, eyq = ey + 1 == n1 ? 0 : ey + 1;
      auto id_of = [&](int x, int y) { return (int64_t)x + (int64_t)y * n0; };
      auto inb = [&](int x, int y) {
        const int64_t q = id_of(x, y);
        return q >= e0 && q < e0 + EB;
      };
      const bool bl = inb(exm, ey), br = inb(exq, ey), bd = inb(ex, eym), bu = inb(ex, eyq);
      const bool bdl = inb(exm, eym), bdr = inb(exq, eym), bul = inb(exm, eyq), bur = inb(exq, eyq);
      auto interior = [&](int ax, int ay) {
        bool in = true;
        if (ax == 0) in = in && bl;
        if (ax == P) in = in && br;
        if (ay == 0) in = in && bd;
        if (ay == P) in = in && bu;
        if (ax == 0 && ay == 0) in = in && bdl;
        if (ax == P && ay == 0) in = in && bdr;
        if (ax == 0 && ay == P) in = in && bul;
        if (ax == P && ay == P) in = in && bur;
        return in;
      };
      double vv[NL];
#pragma unroll
      for (int i = 0; i < NL; ++i) vv[i] = (dU[i] + beta * f[i]) * idt;
      if (live) {
        if (c == 0) a.beta[e] = beta;
#pragma unroll
        for (int i = 0; i < NL; ++i)
          if (!interior(i % P1, i / P1)) a.relem[((int64_t)c * NL + i) * E + e] = vv[i];
      }
      // every read of the nodal states and of f from S is behind the
      // barrier of the slope limiter: S now takes the update vectors
#pragma unroll
      for (int i = 0; i < NL; ++i) Us[i * CS] = vv[i];
      __syncthreads();
      const double dt = a.dtbuf[0];
      const double hd = h * h;
      constexpr int NO = P * P;              // owned local nodes (indices >= 1)
      double nv[NO];
      bool own[NO];
#pragma unroll
      for (int ay = 1; ay <= P; ++ay)
#pragma unroll
        for (int ax = 1; ax <= P; ++ax) {
          const int o = (ax - 1) + P * (ay - 1), j = ax + P1 * ay;
          own[o] = live && interior(ax, ay);
          nv[o] = 0.0;
          if (own[o]) {
            const int nx = ax == P ? 2 : 1, ny = ay == P ? 2 : 1;
            double sum = 0.0;
            for (int yy = 0; yy < ny; ++yy)
              for (int xx = 0; xx < nx; ++xx) {
                const int lane = (int)(id_of(xx ? exq : ex, yy ? eyq : ey) - e0);
                const int jj = (xx ? 0 : ax) + P1 * (yy ? 0 : ay);
                sum += S[(jj * M + c) * EB + lane];
              }
            const double mi = (nx * ny) * (hd * (1.0 / NL));
            const int64_t nd = ns.own_node(j);
            const double ui = a.u[c * N + nd];
            const double ub = (a.rk_a == 0.0) ? 0.0 : a.u0[c * N + nd];
            if (a.copy_base) a.u0[c * N + nd] = ui;
            const double v = stage_value(ui, ub, sum, dt / mi, a);
            a.uout[c * N + nd] = v;
            nv[o] = v;
          }
        }
      // invariant domain at the updated nodes (rho > 0, p > 0; each failed
      // condition counts once, NaN included), counted by component 0
      __syncthreads();                       // every read of the update vectors is done
#pragma unroll
      for (int o = 0; o < NO; ++o) S[(o * M + c) * EB + le] = nv[o];
      __syncthreads();
      int nbad = 0;
      if (c == 0) {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          if (!own[o]) continue;
          double st[M];
          state_at<M, EB>(S, o, le, st);
          nbad += !(st[0] > 0.0);
          nbad += !(PHY::pressure(st, a.ph) > 0.0);
        }
      }
      nbad = wave_sum(nbad);
      __syncthreads();                       // S is rewritten below
      if ((threadIdx.x & 63) == 0) S[threadIdx.x >> 6] = (double)nbad;
      __syncthreads();
      if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < (M * EB) / 64; ++w) tot += (int)S[w];
        if (tot != 0) a.counts[2 * (a.cnt_off + bx) + 1] += tot;
      }
      return;
    }
  }
  if (live) {
    if (c == 0) a.beta[e] = beta;
#pragma unroll
    for (int i = 0; i < NL; ++i) a.relem[((int64_t)c * NL + i) * E + e] = (dU[i] + beta * f[i]) * idt;
  }
}

template <int D, int P, int PH, class RT>
__global__ void CEM_SYS2_BOUNDS k_elem2_sys(StageArgs a) {
  k_elem2_sys_body<D, P, PH, RT>(a, xcd_block(blockIdx.x, gridDim.x));
}

}  // namespace cem
