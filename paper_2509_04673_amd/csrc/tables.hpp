// Host-side constant tables of the Bernstein Q_p element for the HIP path.
//
// Everything is derived here from closed forms in long double and rounded to
// double once:
//   * mixed-degree Bernstein Gram integrals
//       int_0^1 B^p_a B^q_b = C(p,a) C(q,b) / ((p+q+1) C(p+q, a+b)),
//   * derivatives through d^m/dt^m B^p_a = p!/(p-m)! sum_i (-1)^i C(m,i)
//     B^{p-m}_{a-m+i},
//   * Gauss-Legendre points by Newton iteration on the Legendre recurrence,
//   * the neighbour-extension maps by blossoming (de Casteljau with a
//     different parameter per level),
//   * the periodic line operators M_1D^{-1} and M_1D^{-1} C_1D by Gaussian
//     elimination with partial pivoting.
// Element geometry: cube cells of side h; the reference cell is [0,1]^d with
// local node ids lexicographic, axis 0 fastest.
#pragma once
#include <vector>

namespace cem {

struct LineKernel {
  int taps = 0;       // number of taps per output
  int first = 0;      // offset of tap 0 relative to the output node
  std::vector<double> w;   // [P classes][taps]
  // infinite-line rows padded to the fixed width 2*wfast+1 of the
  // register-blocked kernel (empty when the line is too short for it)
  int wfast = 0;
  std::vector<double> wf;  // [P][sfast]: 2*wfast+1 taps, zero padded
  // the same rows cut below 1e-9 of their peak (float kernels), width wfast32
  int wfast32 = 0;
  std::vector<double> wf32;  // [P][sfast32]
};

// Line operators Mb^{-1} and Mb^{-1} Cb of a non-periodic line of
// Nb = p n + 1 nodes (consistent 1D mass matrix and int psi_i psi_j').
// Rows blo <= i < Nb - bhi are the infinite-line rows of node class i mod p
// at offsets -W..W: the ends change them by less than 1e-17 of the peak.
// The first blo rows span columns [0, cw) and the last bhi rows columns
// [Nb - cw, Nb), exact to long-double rounding (entries dropped beyond cw
// are below 1e-17 of the peak).  A short line keeps every row exact:
// blo = Nb, bhi = 0, cw = Nb.  The end blocks are stored by column, so that
// threads computing consecutive rows read consecutive weights.
struct BoundedLine {
  int W = 0, blo = 0, bhi = 0, cw = 0;
  std::vector<double> wi;       // [p][2W + 1]
  std::vector<double> lo, hi;   // [cw][blo], [cw][bhi]
};

struct HostTables {
  int d = 0, p = 0, nl = 0, nlf = 0;
  std::vector<double> vq, dq, wq;   // [P1][P1] B_a(t_q), B_a'(t_q); [P1] weights
  std::vector<double> ext;          // [2][P1][P1] extension maps (low, high neighbour)
  std::vector<double> g1, k1, ct1;  // [P1][P1] 1D mass, stiffness, int B_a' B_b
  std::vector<double> qp;           // packed upper triangle of the semi-norm form,
                                    // row i: Q_ii, 2 Q_i,i+1, ..., 2 Q_i,NL-1
  LineKernel kgrad[3], kmass[3];    // per axis line operators (physical h)
  BoundedLine bgrad, bmass;         // axis 0 of a non-periodic line (1D)
};

// Build all tables for dimension d, degree p, cell size h and L_k nodes per
// axis.  Returns false on an unsupported (d, p).
// wfast[p]: half-width of the register-blocked line kernel, rfast[p]: its
// shortest run of outputs, sfast[p]: its per-class weight stride (all must
// match the device templates)
// wfast32[p], sfast32[p]: width and stride of the float kernels (rows cut
// below 1e-9 of their peak)
bool build_tables(int d, int p, double h, const int L[3], const int wfast[5], const int rfast[5],
                  const int sfast[5], const int wfast32[5], const int sfast32[5], HostTables& out);

// The line operators of a non-periodic line of n cells (into T.bgrad,
// T.bmass).  Returns false on an unsupported degree.
bool build_bounded_line(int p, int n, double h, HostTables& T);

}  // namespace cem
