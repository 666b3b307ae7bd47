// Host-side constant tables of the Bernstein Q_p element (see tables.hpp).
#include "tables.hpp"

#include <cmath>
#include <cstdlib>
#include <vector>

namespace cem {
namespace {

using LD = long double;

LD binom(int n, int k) {
  if (k < 0 || k > n) return 0.0L;
  LD r = 1.0L;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// int_0^1 B^p_a B^q_b dt (zero when an index is out of range)
LD gram(int p, int a, int q, int b) {
  if (a < 0 || a > p || b < 0 || b > q) return 0.0L;
  return binom(p, a) * binom(q, b) / ((p + q + 1) * binom(p + q, a + b));
}

LD falling(int p, int m) {   // p! / (p-m)!
  LD r = 1.0L;
  for (int i = 0; i < m; ++i) r *= (p - i);
  return r;
}

// int_0^1 B^{p(m)}_a B^{p(n)}_b : derivative orders m (test) and n (trial)
LD gram_deriv(int p, int a, int m, int b, int n) {
  LD s = 0.0L;
  for (int i = 0; i <= m; ++i)
    for (int j = 0; j <= n; ++j) {
      LD sg = ((i + j) % 2) ? -1.0L : 1.0L;
      s += sg * binom(m, i) * binom(n, j) * gram(p - m, a - m + i, p - n, b - n + j);
    }
  return falling(p, m) * falling(p, n) * s;
}

LD bern(int p, int a, LD t) {
  return binom(p, a) * std::pow(t, (LD)a) * std::pow(1.0L - t, (LD)(p - a));
}

LD bern_deriv(int p, int a, LD t) {
  if (p == 0) return 0.0L;
  LD l = (a - 1 >= 0) ? bern(p - 1, a - 1, t) : 0.0L;
  LD r = (a <= p - 1) ? bern(p - 1, a, t) : 0.0L;
  return p * (l - r);
}

void gauss_legendre(int n, std::vector<LD>& t, std::vector<LD>& w) {
  t.assign(n, 0.0L);
  w.assign(n, 0.0L);
  const LD pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    LD x = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    LD dp = 0.0L;
    for (int it = 0; it < 100; ++it) {
      LD p0 = 1.0L, p1 = x;
      for (int j = 1; j < n; ++j) {
        LD p2 = ((2 * j + 1) * x * p1 - j * p0) / (j + 1);
        p0 = p1;
        p1 = p2;
      }
      const LD pn = p1, pm = p0;   // P_n(x), P_{n-1}(x)
      dp = n * (x * pn - pm) / (x * x - 1.0L);
      LD dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-19L) break;
    }
    // ascending order on [0,1]
    t[n - 1 - i] = 0.5L * (1.0L + x);
    w[n - 1 - i] = 1.0L / ((1.0L - x * x) * dp * dp);
  }
}

// Blossom of the degree-p Bernstein polynomial with coefficient vector c at
// parameters par[0..p-1] (de Casteljau, one parameter per level).
LD blossom(int p, const std::vector<LD>& c, const std::vector<LD>& par) {
  std::vector<LD> b = c;
  for (int r = 0; r < p; ++r)
    for (int i = 0; i < p - r; ++i) b[i] = (1.0L - par[r]) * b[i] + par[r] * b[i + 1];
  return b[0];
}

// Dense Gaussian elimination with partial pivoting: solves A X = B in place.
void dense_solve(int n, std::vector<LD> A, std::vector<LD>& B, int nrhs) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + k]) > std::fabs(A[(size_t)piv * n + k])) piv = i;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)piv * n + j]);
      for (int j = 0; j < nrhs; ++j) std::swap(B[(size_t)k * nrhs + j], B[(size_t)piv * nrhs + j]);
    }
    for (int i = k + 1; i < n; ++i) {
      LD f = A[(size_t)i * n + k] / A[(size_t)k * n + k];
      if (f == 0.0L) continue;
      for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
      for (int j = 0; j < nrhs; ++j) B[(size_t)i * nrhs + j] -= f * B[(size_t)k * nrhs + j];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    for (int j = 0; j < nrhs; ++j) {
      LD s = B[(size_t)k * nrhs + j];
      for (int i = k + 1; i < n; ++i) s -= A[(size_t)k * n + i] * B[(size_t)i * nrhs + j];
      B[(size_t)k * nrhs + j] = s / A[(size_t)k * n + k];
    }
  }
}

// Rows of M^{-1} and M^{-1} C for the P node classes of a periodic line of
// Lp nodes (degree p, cell h): out_m[c][j], out_g[c][j], j = 0..Lp-1.
void periodic_line_rows(int p, int Lp, LD h, std::vector<LD>& out_m, std::vector<LD>& out_g) {
  const int ne = Lp / p;
  std::vector<LD> M((size_t)Lp * Lp, 0.0L), C((size_t)Lp * Lp, 0.0L);
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a <= p; ++a)
      for (int b = 0; b <= p; ++b) {
        int i = (p * e + a) % Lp, j = (p * e + b) % Lp;
        M[(size_t)i * Lp + j] += h * gram(p, a, p, b);
        C[(size_t)i * Lp + j] += gram_deriv(p, a, 0, b, 1);   // int psi_i psi_j'
      }
  // M symmetric: row c of M^{-1} is the solution of M z = e_c
  std::vector<LD> B((size_t)Lp * p, 0.0L);
  for (int c = 0; c < p; ++c) B[(size_t)c * p + c] = 1.0L;
  dense_solve(Lp, M, B, p);
  out_m.assign((size_t)p * Lp, 0.0L);
  out_g.assign((size_t)p * Lp, 0.0L);
  for (int c = 0; c < p; ++c) {
    for (int j = 0; j < Lp; ++j) out_m[(size_t)c * Lp + j] = B[(size_t)j * p + c];
    // row c of M^{-1} C = z^T C
    for (int j = 0; j < Lp; ++j) {
      LD s = 0.0L;
      for (int i = 0; i < Lp; ++i) s += out_m[(size_t)c * Lp + i] * C[(size_t)i * Lp + j];
      out_g[(size_t)c * Lp + j] = s;
    }
  }
}

constexpr int kExactMax = 480;   // lines up to this length use the exact inverse

// rows of the periodic operators on a line of Lp nodes, cut to taps
void fill_kernel(int p, int Lp, const std::vector<LD>& rows, int taps, int first, std::vector<double>& w) {
  w.assign((size_t)p * taps, 0.0);
  for (int c = 0; c < p; ++c)
    for (int t = 0; t < taps; ++t) {
      int j = ((c + first + t) % Lp + Lp) % Lp;
      w[(size_t)c * taps + t] = (double)rows[(size_t)c * Lp + j];
    }
}

// half-width beyond which the rows fall below thresh of their peak (1e-17:
// the dropped taps then sum to a few 1e-17 of the peak, below float64
// rounding of the kept ones)
int decay_width(int p, int Lp, const std::vector<LD>& rows, LD thresh = 1e-17L) {
  LD peak = 0.0L;
  for (LD v : rows) peak = std::max(peak, std::fabs(v));
  int W = 0;
  for (int c = 0; c < p; ++c)
    for (int j = 0; j < Lp; ++j) {
      int dist = j - c;
      if (dist > Lp / 2) dist -= Lp;
      if (dist < -Lp / 2) dist += Lp;
      if (std::fabs(rows[(size_t)c * Lp + j]) > thresh * peak) W = std::max(W, std::abs(dist));
    }
  return W;
}

void line_kernels(int p, int L, LD h, int wfast, int rfast, int sfast, int wfast32, int sfast32, LineKernel& km,
                  LineKernel& kg) {
  // infinite-line rows from a periodic auxiliary line long enough for the
  // periodic images to vanish below 1e-20
  const int Laux = ((4 * wfast + 64 + p - 1) / p) * p;
  std::vector<LD> am, ag;
  periodic_line_rows(p, Laux, h, am, ag);
  const bool fast = L >= rfast + 2 * wfast && decay_width(p, Laux, am) <= wfast &&
                    decay_width(p, Laux, ag) <= wfast && decay_width(p, Laux, am, 1e-9L) <= wfast32 &&
                    decay_width(p, Laux, ag, 1e-9L) <= wfast32;
  for (LineKernel* k : {&km, &kg}) {
    const std::vector<LD>& rows = (k == &km) ? am : ag;
    k->wfast = 0;
    k->wf.clear();
    k->wfast32 = 0;
    k->wf32.clear();
    if (fast) {
      // taps 0..2W at offsets -W..W, each class row zero padded to the
      // stride sfast of the device kernel
      k->wfast = wfast;
      std::vector<double> tmp;
      fill_kernel(p, Laux, rows, 2 * wfast + 1, -wfast, tmp);
      k->wf.assign((size_t)p * sfast, 0.0);
      for (int cc = 0; cc < p; ++cc)
        for (int t = 0; t < 2 * wfast + 1; ++t) k->wf[(size_t)cc * sfast + t] = tmp[(size_t)cc * (2 * wfast + 1) + t];
      k->wfast32 = wfast32;
      fill_kernel(p, Laux, rows, 2 * wfast32 + 1, -wfast32, tmp);
      k->wf32.assign((size_t)p * sfast32, 0.0);
      for (int cc = 0; cc < p; ++cc)
        for (int t = 0; t < 2 * wfast32 + 1; ++t)
          k->wf32[(size_t)cc * sfast32 + t] = tmp[(size_t)cc * (2 * wfast32 + 1) + t];
    }
  }
  // generic kernel: the exact periodic rows of this line
  std::vector<LD> rm, rg;
  if (L <= kExactMax) {
    periodic_line_rows(p, L, h, rm, rg);
    km.taps = kg.taps = L;
    km.first = kg.first = -(L / 2);
    fill_kernel(p, L, rm, L, -(L / 2), km.w);
    fill_kernel(p, L, rg, L, -(L / 2), kg.w);
  } else {
    const int Wm = decay_width(p, Laux, am), Wg = decay_width(p, Laux, ag);
    km.taps = 2 * Wm + 1;
    km.first = -Wm;
    kg.taps = 2 * Wg + 1;
    kg.first = -Wg;
    fill_kernel(p, Laux, am, km.taps, km.first, km.w);
    fill_kernel(p, Laux, ag, kg.taps, kg.first, kg.w);
  }
}

// Rows of Mb^{-1} and Mb^{-1} Cb of a non-periodic line of nb = p ne + 1
// nodes for the requested row indices (dense storage, band-limited LU
// without pivoting: Mb is symmetric positive definite with half-bandwidth p).
void bounded_line_rows(int p, int ne, LD h, const std::vector<int>& rows, std::vector<LD>& out_m,
                       std::vector<LD>& out_g) {
  const int nb = p * ne + 1;
  std::vector<LD> M((size_t)nb * nb, 0.0L), C((size_t)nb * nb, 0.0L);
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a <= p; ++a)
      for (int b = 0; b <= p; ++b) {
        const int i = p * e + a, j = p * e + b;
        M[(size_t)i * nb + j] += h * gram(p, a, p, b);
        C[(size_t)i * nb + j] += gram_deriv(p, a, 0, b, 1);   // int psi_i psi_j'
      }
  // LU in place (L unit lower, U upper), both within the band
  for (int k = 0; k < nb; ++k)
    for (int i = k + 1; i <= std::min(nb - 1, k + p); ++i) {
      const LD f = M[(size_t)i * nb + k] / M[(size_t)k * nb + k];
      M[(size_t)i * nb + k] = f;
      for (int j = k + 1; j <= std::min(nb - 1, k + p); ++j) M[(size_t)i * nb + j] -= f * M[(size_t)k * nb + j];
    }
  const size_t nr = rows.size();
  out_m.assign(nr * nb, 0.0L);
  out_g.assign(nr * nb, 0.0L);
  std::vector<LD> z(nb);
  for (size_t r = 0; r < nr; ++r) {
    // row i of the symmetric Mb^{-1} is the solution of Mb z = e_i
    std::fill(z.begin(), z.end(), 0.0L);
    z[rows[r]] = 1.0L;
    for (int i = 1; i < nb; ++i)
      for (int k = std::max(0, i - p); k < i; ++k) z[i] -= M[(size_t)i * nb + k] * z[k];
    for (int i = nb - 1; i >= 0; --i) {
      for (int k = i + 1; k <= std::min(nb - 1, i + p); ++k) z[i] -= M[(size_t)i * nb + k] * z[k];
      z[i] /= M[(size_t)i * nb + i];
    }
    for (int j = 0; j < nb; ++j) {
      out_m[r * nb + j] = z[j];
      LD s = 0.0L;
      for (int k = std::max(0, j - p); k <= std::min(nb - 1, j + p); ++k) s += z[k] * C[(size_t)k * nb + j];
      out_g[r * nb + j] = s;
    }
  }
}

}  // namespace

bool build_bounded_line(int p, int n, double h, HostTables& T) {
  if (p < 1 || p > 4 || n < 2) return false;
  const LD hl = (LD)h;
  const int nb = p * n + 1;
  // infinite-line rows: a periodic auxiliary line long enough for the
  // periodic images to vanish, cut where both operators fall below 1e-17
  // of their peak
  const int Laux = ((4 * 64 + 64 + p - 1) / p) * p;
  std::vector<LD> am, ag;
  periodic_line_rows(p, Laux, hl, am, ag);
  const int W = std::max(decay_width(p, Laux, am), decay_width(p, Laux, ag));
  LD pk_m = 0.0L, pk_g = 0.0L;
  for (LD v : am) pk_m = std::max(pk_m, std::fabs(v));
  for (LD v : ag) pk_g = std::max(pk_g, std::fabs(v));
  auto inf_row = [&](const std::vector<LD>& rows, int cls, int off) -> LD {
    if (off < -W || off > W) return 0.0L;
    return rows[(size_t)cls * Laux + ((cls + off) % Laux + Laux) % Laux];
  };
  // exact rows near the low end on a line of at most nx cells (the far
  // end's influence on them is then far below rounding); the high end
  // mirrors it but is computed directly on the same line
  const int nx = std::min(n, (8 * W + 64) / p + 2);
  const int nbx = p * nx + 1;
  const int want = std::min(nbx, 3 * W + 2 * p);
  std::vector<int> rws;
  for (int i = 0; i < want; ++i) rws.push_back(i);
  for (int i = 0; i < want; ++i) rws.push_back(nbx - want + i);
  std::vector<LD> rm, rg;
  bounded_line_rows(p, nx, hl, rws, rm, rg);
  BoundedLine* outs[2] = {&T.bmass, &T.bgrad};
  // the first row index from which the exact rows match the infinite ones
  // (checked for all classes, both ends, both operators)
  const LD tol = 4e-17L;
  int B = W;
  auto dev = [&](int i, bool hi_end, bool grad) {
    const std::vector<LD>& R = grad ? rg : rm;
    const std::vector<LD>& I = grad ? ag : am;
    const LD pk = grad ? pk_g : pk_m;
    const int r = hi_end ? 2 * want - 1 - i : i;    // row index in rws
    const int row = rws[r];
    LD mx = 0.0L;
    for (int j = 0; j < nbx; ++j) mx = std::max(mx, std::fabs(R[(size_t)r * nbx + j] - inf_row(I, row % p, j - row)));
    return mx / pk;
  };
  // The banded layout (exact end blocks of B rows, the infinite-line rows
  // between them) wherever both end blocks fit on the line and their rows
  // meet the infinite ones: on lines shorter than the auxiliary line the
  // exact rows are those of the line itself (nx = n), so the checks below
  // see both ends.  Otherwise every row is exact (a dense operator over the
  // whole line).  Long lines must take the banded layout.
  const bool must_band = nb > 2 * want;
  bool banded = nb >= 2 * W + 2 * p + 1;
  if (banded) {
    for (; B + p <= want; ++B) {
      bool ok = true;
      for (int i = B; i < B + p && ok; ++i)
        for (int e = 0; e < 2 && ok; ++e)
          for (int g = 0; g < 2 && ok; ++g) ok = dev(i, e == 1, g == 1) <= tol;
      if (ok) break;
    }
    banded = B + p <= want && 2 * B <= nb && B + W + 1 <= nb;
    // the dropped entries of the end rows must be negligible too
    for (int g = 0; g < 2 && banded; ++g) {
      const std::vector<LD>& R = g ? rg : rm;
      const LD pk = g ? pk_g : pk_m;
      for (int i = 0; i < B && banded; ++i)
        for (int j = B + W + 1; j < nbx; ++j)
          if (std::fabs(R[(size_t)i * nbx + j]) > tol * pk) {
            banded = false;
            break;
          }
    }
  }
  if (must_band && !banded) return false;
  const bool short_line = !banded;
  for (int g = 0; g < 2; ++g) {
    BoundedLine& K = *outs[g];
    const std::vector<LD>& I = g ? ag : am;
    K.W = W;
    K.wi.assign((size_t)p * (2 * W + 1), 0.0);
    for (int cls = 0; cls < p; ++cls)
      for (int t = 0; t <= 2 * W; ++t) K.wi[(size_t)cls * (2 * W + 1) + t] = (double)inf_row(I, cls, t - W);
    if (short_line) {
      // every row exact, on the line itself
      std::vector<int> all(nb);
      for (int i = 0; i < nb; ++i) all[i] = i;
      std::vector<LD> em, eg;
      bounded_line_rows(p, n, hl, all, em, eg);
      const std::vector<LD>& R = g ? eg : em;
      K.blo = nb;
      K.bhi = 0;
      K.cw = nb;
      K.lo.assign((size_t)nb * nb, 0.0);
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) K.lo[(size_t)j * nb + i] = (double)R[(size_t)i * nb + j];
      K.hi.clear();
      continue;
    }
    const std::vector<LD>& R = g ? rg : rm;
    K.blo = K.bhi = B;
    K.cw = B + W + 1;
    K.lo.assign((size_t)B * K.cw, 0.0);
    K.hi.assign((size_t)B * K.cw, 0.0);
    for (int i = 0; i < B; ++i)
      for (int j = 0; j < K.cw; ++j) {
        K.lo[(size_t)j * B + i] = (double)R[(size_t)i * nbx + j];
        // high block row i is line row nb - B + i; its columns nb - cw + j
        const int r = 2 * want - B + i;          // rws[r] = nbx - B + i
        K.hi[(size_t)j * B + i] = (double)R[(size_t)r * nbx + (nbx - K.cw + j)];
      }
  }
  return true;
}

bool build_tables(int d, int p, double h, const int L[3], const int wfast[5], const int rfast[5],
                  const int sfast[5], const int wfast32[5], const int sfast32[5], HostTables& T) {
  if (d < 1 || d > 3 || p < 1 || p > 4) return false;
  const int P1 = p + 1;
  int nl = 1;
  for (int k = 0; k < d; ++k) nl *= P1;
  int nlf = nl / P1;
  T.d = d;
  T.p = p;
  T.nl = nl;
  T.nlf = nlf;

  std::vector<LD> tq, wq;
  gauss_legendre(P1, tq, wq);
  T.vq.resize(P1 * P1);
  T.dq.resize(P1 * P1);
  T.wq.resize(P1);
  for (int q = 0; q < P1; ++q) {
    T.wq[q] = (double)wq[q];
    for (int a = 0; a < P1; ++a) {
      T.vq[q * P1 + a] = (double)bern(p, a, tq[q]);
      T.dq[q * P1 + a] = (double)bern_deriv(p, a, tq[q]);
    }
  }

  // 1D building blocks (long double)
  auto G1 = [&](int a, int b) { return gram(p, a, p, b); };
  auto K1 = [&](int a, int b) { return gram_deriv(p, a, 1, b, 1); };
  auto CT1 = [&](int a, int b) { return gram_deriv(p, a, 1, b, 0); };   // int B_a' B_b
  auto digit = [&](int loc, int k) {
    for (int i = 0; i < k; ++i) loc /= P1;
    return loc % P1;
  };

  // semi-norm form: sum over 1 <= |k| <= p of tensor products of the 1D
  // m-th derivative Grams (scale-free on cube cells)
  std::vector<LD> Q((size_t)nl * nl, 0.0L);
  int nk = 1;
  for (int k = 0; k < d; ++k) nk *= P1;
  for (int mi = 0; mi < nk; ++mi) {
    int ord[3] = {0, 0, 0}, tot = 0;
    for (int k = 0; k < d; ++k) {
      ord[k] = digit(mi, k);
      tot += ord[k];
    }
    if (tot < 1 || tot > p) continue;
    for (int i = 0; i < nl; ++i)
      for (int j = 0; j < nl; ++j) {
        LD v = 1.0L;
        for (int k = 0; k < d; ++k) v *= gram_deriv(p, digit(i, k), ord[k], digit(j, k), ord[k]);
        Q[(size_t)i * nl + j] += v;
      }
  }

  // neighbour-extension maps: the polynomial of the low neighbour seen on
  // K_e lives on t in [1,2] of its own cell, the high neighbour's on [-1,0]
  std::vector<LD> E1[2];
  const LD lims[2][2] = {{1.0L, 2.0L}, {-1.0L, 0.0L}};
  T.ext.assign(2 * P1 * P1, 0.0);
  for (int s = 0; s < 2; ++s) {
    E1[s].assign(P1 * P1, 0.0L);
    for (int r = 0; r < P1; ++r) {
      std::vector<LD> par(p);
      for (int i = 0; i < p; ++i) par[i] = (i < p - r) ? lims[s][0] : lims[s][1];
      for (int a = 0; a < P1; ++a) {
        std::vector<LD> unit(P1, 0.0L);
        unit[a] = 1.0L;
        E1[s][r * P1 + a] = blossom(p, unit, par);
        T.ext[(s * P1 + r) * P1 + a] = (double)E1[s][r * P1 + a];
      }
    }
  }
  // 1D tables of the sum-factorised element operators
  T.g1.assign(P1 * P1, 0.0);
  T.k1.assign(P1 * P1, 0.0);
  T.ct1.assign(P1 * P1, 0.0);
  for (int a = 0; a < P1; ++a)
    for (int b = 0; b < P1; ++b) {
      T.g1[a * P1 + b] = (double)G1(a, b);
      T.k1[a * P1 + b] = (double)K1(a, b);
      T.ct1[a * P1 + b] = (double)CT1(a, b);
    }
  T.qp.clear();
  for (int i = 0; i < nl; ++i)
    for (int j = i; j < nl; ++j) T.qp.push_back((double)((j == i ? 1.0L : 2.0L) * Q[(size_t)i * nl + j]));

  for (int k = 0; k < d; ++k)
    line_kernels(p, L[k], (LD)h, wfast[p], rfast[p], sfast[p], wfast32[p], sfast32[p], T.kmass[k], T.kgrad[k]);
  return true;
}

}  // namespace cem
