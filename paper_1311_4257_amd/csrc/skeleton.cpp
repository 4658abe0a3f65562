// Directional skeletons of Eq. 2 (Section 2.1), computed on the host in float64.
//
// For a box of width w centred at 0 and a far region X, the skeleton is
// (b, a, D): equivalent points b in the box, check points a in X and an
// r x r matrix D such that G(x, y) ~= sum_q G(x, b_q) sum_p D_qp G(a_p, y).
// The paper points to a random sampling method built on pivoted QR; the
// steps taken here:
//   1. draw sample sets Y (uniform in the box) and X (the far region);
//   2. column-pivoted Householder QR of a Gaussian sketch of M = G(X, Y),
//      stopped at the first rank r whose trailing Frobenius norm is <= tau of
//      the total; b = Y at the first r pivots;
//   3. column-pivoted QR of a Gaussian sketch of M^T for r steps; a = X at
//      those pivots;
//   4. D = G(X, b)^+ M G(a, Y)^+ (least squares through Householder QR), the
//      middle factor that best reproduces M from the chosen rows and columns.
// Far regions: at HF width w and wedge l, the boxes of the offsets that can
// occur in an interaction list at width w and fall in wedge l, plus the check
// points of every wedge l' of width 2w with l' -> l, shifted into each child's
// frame (the hierarchical wedges of Figure 2); at the LF width 1/2 the V-list
// boxes plus the shifted check points of the six width-1 wedges.  Widths are
// built from w_hi downwards.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "geometry.hpp"
#include "internal.hpp"

namespace dfmm {

namespace {

// Sample sizes: wider boxes (more wavelengths across, wider far regions) and
// tighter tolerances need denser samples for the skeleton to hold between them.
constexpr double kNY = 900.0;      // candidate equivalent points, box width <= 1
constexpr double kNOwn = 1200.0;   // far-region samples per unit width
constexpr int kMinPerBox = 6;

void sample_sizes(double w, double tau, int* n_own, int* n_y) {
  double ww = w < 1.0 ? 1.0 : w;
  double o = kNOwn * ww, y = kNY * (1.0 + 0.35 * std::log2(ww));
  if (tau < 1e-6) {
    o *= 2.5;
    y *= 16.0 / 9.0;
  }
  *n_own = int(std::lround(o));
  *n_y = int(std::lround(y));
}
constexpr uint64_t kSeed = 0x5eed0fd1f3a11ULL;

// SplitMix64 (Steele, Lea, Flood 2014) -> uniform double in [0, 1).
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
  }
  double uniform() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// G(x, y) in float64: (cos 2 pi r, sin 2 pi r) / r, zero at r = 0.
inline void green64(const double* x, const double* y, double* re, double* im) {
  double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
  double r = std::sqrt(dx * dx + dy * dy + dz * dz);
  if (r == 0.0) {
    *re = *im = 0.0;
    return;
  }
  double s = std::sin(2.0 * M_PI * r), c = std::cos(2.0 * M_PI * r);
  *re = c / r;
  *im = s / r;
}

// Complex matrix, column-major, interleaved (re, im).
struct CMat {
  int m = 0, n = 0;
  std::vector<double> d;
  CMat() = default;
  CMat(int m_, int n_) : m(m_), n(n_), d(size_t(2) * m_ * n_, 0.0) {}
  double* col(int j) { return d.data() + size_t(2) * m * j; }
  const double* col(int j) const { return d.data() + size_t(2) * m * j; }
};

CMat kernel_matrix(const std::vector<double>& X, const std::vector<double>& Y) {
  int m = int(X.size() / 3), n = int(Y.size() / 3);
  CMat M(m, n);
  for (int j = 0; j < n; ++j) {
    double* c = M.col(j);
    for (int i = 0; i < m; ++i) green64(&X[3 * i], &Y[3 * j], c + 2 * i, c + 2 * i + 1);
  }
  return M;
}

CMat transpose(const CMat& A) {
  CMat T(A.n, A.m);
  for (int j = 0; j < A.n; ++j)
    for (int i = 0; i < A.m; ++i) {
      T.d[2 * (size_t(i) * A.n + j)] = A.d[2 * (size_t(j) * A.m + i)];
      T.d[2 * (size_t(i) * A.n + j) + 1] = A.d[2 * (size_t(j) * A.m + i) + 1];
    }
  return T;
}

// Householder reflector on x[0..L) (interleaved complex), in place: x becomes
// v with H = I - beta v v^H and H x = alpha e1.  Returns beta; *ar,*ai = alpha.
double householder(double* x, int L, double* ar, double* ai) {
  double nrm2 = 0.0;
  for (int i = 0; i < L; ++i) nrm2 += x[2 * i] * x[2 * i] + x[2 * i + 1] * x[2 * i + 1];
  double nrm = std::sqrt(nrm2);
  if (nrm == 0.0) {
    *ar = *ai = 0.0;
    return 0.0;
  }
  double a0 = std::hypot(x[0], x[1]);
  double pr = 1.0, pi = 0.0;
  if (a0 > 0.0) {
    pr = x[0] / a0;
    pi = x[1] / a0;
  }
  // v = x + phase * nrm * e1 ; alpha = -phase * nrm
  x[0] += pr * nrm;
  x[1] += pi * nrm;
  *ar = -pr * nrm;
  *ai = -pi * nrm;
  return 1.0 / (nrm * (nrm + a0));
}

// y[0..L) -= beta * v * (v^H y)
inline void apply_reflector(const double* v, int L, double beta, double* y) {
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < L; ++i) {
    double vr = v[2 * i], vi = v[2 * i + 1], yr = y[2 * i], yi = y[2 * i + 1];
    sr += vr * yr + vi * yi;  // conj(v) * y
    si += vr * yi - vi * yr;
  }
  sr *= beta;
  si *= beta;
  for (int i = 0; i < L; ++i) {
    double vr = v[2 * i], vi = v[2 * i + 1];
    y[2 * i] -= vr * sr - vi * si;
    y[2 * i + 1] -= vr * si + vi * sr;
  }
}

// Column-pivoted QR of A (destroyed).  Stops after max_steps steps or when the
// trailing Frobenius norm is <= tol * ||A||_F (tol < 0 disables that test).
// Returns the pivot order of the first `rank` columns.
std::vector<int> pivoted_qr(CMat& A, double tol, int max_steps) {
  int m = A.m, n = A.n;
  std::vector<double> nrm(n), orig(n);
  std::vector<int> piv(n);
  double total = 0.0;
  for (int j = 0; j < n; ++j) {
    const double* c = A.col(j);
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += c[2 * i] * c[2 * i] + c[2 * i + 1] * c[2 * i + 1];
    nrm[j] = orig[j] = s;
    total += s;
    piv[j] = j;
  }
  int kmax = std::min({m, n, max_steps});
  int k = 0;
  std::vector<double> tmp(size_t(2) * m);
  for (; k < kmax; ++k) {
    if (tol >= 0.0) {
      double rest = 0.0;
      for (int j = k; j < n; ++j) rest += nrm[j];
      if (rest <= tol * tol * total) break;
    }
    int p = k;
    for (int j = k + 1; j < n; ++j)
      if (nrm[j] > nrm[p]) p = j;
    if (p != k) {
      std::swap(piv[k], piv[p]);
      std::swap(nrm[k], nrm[p]);
      std::swap(orig[k], orig[p]);
      std::memcpy(tmp.data(), A.col(k), sizeof(double) * 2 * m);
      std::memcpy(A.col(k), A.col(p), sizeof(double) * 2 * m);
      std::memcpy(A.col(p), tmp.data(), sizeof(double) * 2 * m);
    }
    double* v = A.col(k) + 2 * k;
    int L = m - k;
    double ar, ai;
    double beta = householder(v, L, &ar, &ai);
    for (int j = k + 1; j < n; ++j) {
      double* y = A.col(j) + 2 * k;
      if (beta != 0.0) apply_reflector(v, L, beta, y);
      double t = y[0] * y[0] + y[1] * y[1];
      nrm[j] -= t;
      if (nrm[j] < 1e-6 * orig[j]) {  // downdate lost accuracy: recompute
        double s = 0.0;
        for (int i = 1; i < L; ++i) s += y[2 * i] * y[2 * i] + y[2 * i + 1] * y[2 * i + 1];
        nrm[j] = orig[j] = s;
      }
    }
    nrm[k] = 0.0;
  }
  piv.resize(k);
  return piv;
}

// Least squares X = A^+ B for tall A (m x r, full column rank): Householder
// QR of A, Q^H B, then back substitution.  A and B are destroyed.
CMat lstsq(CMat& A, CMat& B) {
  int m = A.m, r = A.n, k = B.n;
  std::vector<double> beta(r), diag(2 * r);
  for (int j = 0; j < r; ++j) {
    double* v = A.col(j) + 2 * j;
    int L = m - j;
    double ar, ai;
    beta[j] = householder(v, L, &ar, &ai);
    diag[2 * j] = ar;
    diag[2 * j + 1] = ai;
    for (int c = j + 1; c < r; ++c)
      if (beta[j] != 0.0) apply_reflector(v, L, beta[j], A.col(c) + 2 * j);
    for (int c = 0; c < k; ++c)
      if (beta[j] != 0.0) apply_reflector(v, L, beta[j], B.col(c) + 2 * j);
  }
  CMat X(r, k);
  for (int c = 0; c < k; ++c) {
    const double* b = B.col(c);
    double* x = X.col(c);
    for (int i = r - 1; i >= 0; --i) {
      double sr = b[2 * i], si = b[2 * i + 1];
      for (int j = i + 1; j < r; ++j) {
        double ar = A.col(j)[2 * i], ai = A.col(j)[2 * i + 1];
        sr -= ar * x[2 * j] - ai * x[2 * j + 1];
        si -= ar * x[2 * j + 1] + ai * x[2 * j];
      }
      double dr = diag[2 * i], di = diag[2 * i + 1];
      double den = dr * dr + di * di;
      x[2 * i] = (sr * dr + si * di) / den;
      x[2 * i + 1] = (si * dr - sr * di) / den;
    }
  }
  return X;
}

CMat conj_transpose(const CMat& A) {
  CMat T = transpose(A);
  for (size_t i = 1; i < T.d.size(); i += 2) T.d[i] = -T.d[i];
  return T;
}

std::vector<double> pick(const std::vector<double>& P, const std::vector<int>& idx) {
  std::vector<double> out(3 * idx.size());
  for (size_t i = 0; i < idx.size(); ++i)
    for (int k = 0; k < 3; ++k) out[3 * i + k] = P[3 * size_t(idx[i]) + k];
  return out;
}

// C = A^H B for column-major complex A (m x p) and B (m x n); cache-blocked,
// four independent partial sums per dot product.
CMat gemm_hn(const CMat& A, const CMat& B) {
  const int m = A.m, p = A.n, n = B.n;
  CMat C(p, n);
  constexpr int BI = 8, BJ = 8, BL = 512;
  for (int j0 = 0; j0 < n; j0 += BJ)
    for (int i0 = 0; i0 < p; i0 += BI)
      for (int l0 = 0; l0 < m; l0 += BL) {
        const int l1 = std::min(m, l0 + BL);
        for (int j = j0; j < std::min(n, j0 + BJ); ++j) {
          const double* bc = B.col(j);
          for (int i = i0; i < std::min(p, i0 + BI); ++i) {
            const double* ac = A.col(i);
            double sr[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
            int l = l0;
            for (; l + 4 <= l1; l += 4)
              for (int u = 0; u < 4; ++u) {
                const double ar = ac[2 * (l + u)], ai = ac[2 * (l + u) + 1];
                const double br = bc[2 * (l + u)], bi = bc[2 * (l + u) + 1];
                sr[u] += ar * br + ai * bi;
                si[u] += ar * bi - ai * br;
              }
            for (; l < l1; ++l) {
              const double ar = ac[2 * l], ai = ac[2 * l + 1], br = bc[2 * l], bi = bc[2 * l + 1];
              sr[0] += ar * br + ai * bi;
              si[0] += ar * bi - ai * br;
            }
            C.col(j)[2 * i] += (sr[0] + sr[1]) + (sr[2] + sr[3]);
            C.col(j)[2 * i + 1] += (si[0] + si[1]) + (si[2] + si[3]);
          }
        }
      }
  return C;
}

// Thin Householder QR of A (m x r, full column rank): returns the explicit
// orthonormal factor Q (m x r); R (upper, r x r) is left in A's upper part with
// its diagonal in rdiag.
CMat thin_q(CMat& A, std::vector<double>& rdiag) {
  const int m = A.m, r = A.n;
  std::vector<double> beta(r);
  rdiag.assign(2 * size_t(r), 0.0);
  for (int j = 0; j < r; ++j) {
    double* v = A.col(j) + 2 * j;
    double ar, ai;
    beta[j] = householder(v, m - j, &ar, &ai);
    rdiag[2 * j] = ar;
    rdiag[2 * j + 1] = ai;
    for (int c = j + 1; c < r; ++c)
      if (beta[j] != 0.0) apply_reflector(v, m - j, beta[j], A.col(c) + 2 * j);
  }
  CMat Q(m, r);
  for (int c = 0; c < r; ++c) {
    Q.col(c)[2 * c] = 1.0;
    for (int j = std::min(c, r - 1); j >= 0; --j)
      if (beta[j] != 0.0) apply_reflector(A.col(j) + 2 * j, m - j, beta[j], Q.col(c) + 2 * j);
  }
  return Q;
}

// Solve R X = B in place (R upper r x r stored in A's upper part, diagonal rdiag).
void back_substitute(const CMat& A, const std::vector<double>& rdiag, CMat& B) {
  const int r = A.n;
  for (int c = 0; c < B.n; ++c) {
    double* x = B.col(c);
    for (int i = r - 1; i >= 0; --i) {
      double sr = x[2 * i], si = x[2 * i + 1];
      for (int j = i + 1; j < r; ++j) {
        const double ar = A.col(j)[2 * i], ai = A.col(j)[2 * i + 1];
        sr -= ar * x[2 * j] - ai * x[2 * j + 1];
        si -= ar * x[2 * j + 1] + ai * x[2 * j];
      }
      const double dr = rdiag[2 * i], di = rdiag[2 * i + 1], den = dr * dr + di * di;
      x[2 * i] = (sr * dr + si * di) / den;
      x[2 * i + 1] = (si * dr - sr * di) / den;
    }
  }
}

// C^+ B for tall C (m x r) through its explicit thin Q: R^{-1} (Q^H B).
CMat lstsq_q(CMat C, const CMat& B) {
  std::vector<double> rdiag;
  CMat Q = thin_q(C, rdiag);
  CMat Z = gemm_hn(Q, B);
  back_substitute(C, rdiag, Z);
  return Z;
}

// Skeleton of Eq. 2 from the samples X (far) and Y (box):
//   column selection: a Gaussian sketch Omega M (k x nY) of M = G(X, Y) is
//   pivoted-QR factored (randomized column-pivoted QR: the sketch preserves
//   column norms and angles of M up to small distortion); the rank r is the
//   first with trailing Frobenius norm <= tau of the total;
//   row selection: the same on a Gaussian sketch of M^T (r steps);
//   D = G(X, b)^+ M G(a, Y)^+.
Skel make_skeleton(const std::vector<double>& X, const std::vector<double>& Y, double tau, uint64_t seed) {
  CMat M = kernel_matrix(X, Y);
  const int m = M.m, n = M.n;
  const int ks = std::min(n, tau < 1e-6 ? 384 : 256);
  CMat Om(m, ks);
  Rng rng(seed);
  for (int c = 0; c < ks; ++c)
    for (int i = 0; i < m; ++i) {  // Box-Muller, real Gaussian entries
      double u1 = rng.uniform(), u2 = rng.uniform();
      if (u1 < 1e-300) u1 = 1e-300;
      Om.col(c)[2 * i] = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    }
  CMat Zs = gemm_hn(Om, M);  // ks x n
  std::vector<int> pc = pivoted_qr(Zs, tau, ks - 8);
  int r = int(pc.size());
  Skel s;
  s.r = r;
  s.b = pick(Y, pc);
  // rows: column-pivoted QR of a Gaussian sketch of M^T (k x m), r steps
  CMat Om2(n, ks);
  for (int c = 0; c < ks; ++c)
    for (int i = 0; i < n; ++i) {
      double u1 = rng.uniform(), u2 = rng.uniform();
      if (u1 < 1e-300) u1 = 1e-300;
      Om2.col(c)[2 * i] = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    }
  CMat Zr = gemm_hn(Om2, transpose(M));  // ks x m
  std::vector<int> pr = pivoted_qr(Zr, -1.0, r);
  s.a = pick(X, pr);
  CMat C = kernel_matrix(X, s.b);  // m x r
  // Z = G(X,b)^+ M  (r x nY);  D^H = (G(a,Y)^H)^+ Z^H
  CMat Z = lstsq_q(C, M);
  CMat Ra = conj_transpose(kernel_matrix(s.a, Y));  // nY x r
  CMat Zh = conj_transpose(Z);                       // nY x r
  CMat Dh = lstsq(Ra, Zh);                           // r x r = D^H
  s.D.assign(size_t(2) * r * r, 0.0);
  for (int q = 0; q < r; ++q)
    for (int p = 0; p < r; ++p) {  // D[q][p] = conj(Dh[p][q])
      s.D[2 * (size_t(q) * r + p)] = Dh.col(q)[2 * p];
      s.D[2 * (size_t(q) * r + p) + 1] = -Dh.col(q)[2 * p + 1];
    }
  (void)m;
  return s;
}

void sample_boxes(Rng& rng, const std::vector<double>& centres, double w, int n_total, std::vector<double>& out) {
  size_t nb = centres.size() / 3;
  if (nb == 0) return;
  size_t k = std::max<size_t>(kMinPerBox, (size_t(n_total) + nb - 1) / nb);
  for (size_t b = 0; b < nb; ++b)
    for (size_t i = 0; i < k; ++i)
      for (int t = 0; t < 3; ++t) out.push_back(centres[3 * b + t] + w * (rng.uniform() - 0.5));
}

void add_inherited(const Skel& parent, double w, std::vector<double>& out) {
  for (int o = 0; o < 8; ++o) {
    double d[3] = {((o & 1) - 0.5) * w, (((o >> 1) & 1) - 0.5) * w, (((o >> 2) & 1) - 0.5) * w};
    for (int p = 0; p < parent.r; ++p)
      for (int t = 0; t < 3; ++t) out.push_back(parent.a[3 * p + t] - d[t]);
  }
}

template <class F>
void parallel_for(int n, F&& fn) {
  unsigned hc = std::thread::hardware_concurrency();
  int nt = int(std::max(1u, std::min(hc ? hc : 1u, 16u)));
  nt = std::min(nt, n);
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int i = next++; i < n; i = next++) fn(i);
    });
  for (auto& x : th) x.join();
}

}  // namespace

void build_opset(OpSetImpl& set) {
  const double tau = set.tau;
  int emax = 0;
  while ((1 << emax) < set.w_hi) ++emax;
  set.hf.assign(emax + 1, {});
  for (int e = emax; e >= 0; --e) {
    int64_t w = int64_t(1) << e;
    std::vector<int64_t> offs = list_offsets_e2(e + 1);
    int ndir = int(6 * w * w);
    std::vector<std::vector<double>> own(ndir);
    for (size_t i = 0; i < offs.size(); i += 3) {
      int l = direction(offs[i], offs[i + 1], offs[i + 2], w);
      for (int t = 0; t < 3; ++t) own[l].push_back(double(offs[i + t]) * double(w));
    }
    std::vector<Skel>& out = set.hf[e];
    out.assign(ndir, Skel());
    parallel_for(ndir, [&](int l) {
      Rng rng(kSeed ^ (uint64_t(e + 1) << 40) ^ (uint64_t(l) << 8));
      int n_own, n_y;
      sample_sizes(double(w), tau, &n_own, &n_y);
      std::vector<double> X;
      sample_boxes(rng, own[l], double(w), n_own, X);
      if (e < emax)
        for (int lp = 0; lp < int(6 * 4 * w * w); ++lp)
          if (direction_down(lp, 2 * w) == l) add_inherited(set.hf[e + 1][lp], double(w), X);
      std::vector<double> Y(3 * size_t(n_y));
      for (auto& v : Y) v = (rng.uniform() - 0.5) * double(w);
      out[l] = make_skeleton(X, Y, tau, kSeed ^ (uint64_t(e + 7) << 48) ^ (uint64_t(l) << 16) ^ 0x9e37ULL);
    });
  }
  // low-frequency width 1/2
  Rng rng(kSeed);
  std::vector<int64_t> offs = list_offsets_e2(0);
  std::vector<double> cen;
  for (int64_t v : offs) cen.push_back(0.5 * double(v));
  int n_own, n_y;
  sample_sizes(0.5, tau, &n_own, &n_y);
  std::vector<double> X;
  sample_boxes(rng, cen, 0.5, n_own, X);
  for (const Skel& p : set.hf[0]) add_inherited(p, 0.5, X);
  std::vector<double> Y(3 * size_t(n_y));
  for (auto& v : Y) v = (rng.uniform() - 0.5) * 0.5;
  set.lf = make_skeleton(X, Y, tau, kSeed ^ 0x1f1f1f1fULL);
}

// Deeper low-frequency widths (adaptive trees, Section 2.2).  The kernel is not
// scale invariant, so each width w = 1/4, 1/8, ... has its own non-directional
// skeleton, sampled like the width-1/2 one: the boxes at the interaction-list
// offsets of width w, plus the check points of the width-2w skeleton seen from
// the 8 child positions (where LF-M2M and LF-L2L evaluate the child's
// skeleton).
void build_lf_deep(OpSetImpl& set, int n) {
  const double tau = set.tau;
  const std::vector<int64_t> offs = list_offsets_e2(0);
  while (int(set.lf_deep.size()) < n) {
    const int k = int(set.lf_deep.size()) + 1;  // width 2^-(1 + k)
    const double w = std::ldexp(0.5, -k);
    const Skel& parent = k == 1 ? set.lf : set.lf_deep[size_t(k) - 2];
    Rng rng(kSeed ^ (uint64_t(0x5a5a) << 32) ^ uint64_t(k));
    std::vector<double> cen;
    for (int64_t v : offs) cen.push_back(w * double(v));
    int n_own, n_y;
    sample_sizes(w, tau, &n_own, &n_y);
    std::vector<double> X;
    sample_boxes(rng, cen, w, n_own, X);
    add_inherited(parent, w, X);
    std::vector<double> Y(3 * size_t(n_y));
    for (auto& v : Y) v = (rng.uniform() - 0.5) * w;
    set.lf_deep.push_back(make_skeleton(X, Y, tau, kSeed ^ (uint64_t(0x3c3c) << 40) ^ uint64_t(k)));
  }
}

// ---- file format ----------------------------------------------------------
// "DFMMOPS2", float64 tau, int32 w_hi, int32 count, then `count` skeletons in
// the order w = 1 (dirs 0..5), w = 2 (0..23), ..., w_hi, then the LF skeleton;
// each: int32 r, float64 a[3r], float64 b[3r], float64 D[2 r r] (row-major
// complex).  Little-endian.

bool save_opset(const OpSetImpl& set, const std::string& path) {
  std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  bool ok = true;
  auto W = [&](const void* p, size_t n) { ok = ok && std::fwrite(p, 1, n, f) == n; };
  W("DFMMOPS2", 8);
  W(&set.tau, 8);
  int32_t whi = set.w_hi, cnt = 1;
  for (auto& v : set.hf) cnt += int32_t(v.size());
  W(&whi, 4);
  W(&cnt, 4);
  auto put = [&](const Skel& s) {
    int32_t r = s.r;
    W(&r, 4);
    W(s.a.data(), 8 * s.a.size());
    W(s.b.data(), 8 * s.b.size());
    W(s.D.data(), 8 * s.D.size());
  };
  for (auto& v : set.hf)
    for (auto& s : v) put(s);
  put(set.lf);
  ok = (std::fclose(f) == 0) && ok;
  if (ok) ok = std::rename(tmp.c_str(), path.c_str()) == 0;
  if (!ok) std::remove(tmp.c_str());
  return ok;
}

bool load_opset(OpSetImpl& set, const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  bool ok = true;
  auto R = [&](void* p, size_t n) { ok = ok && std::fread(p, 1, n, f) == n; };
  char magic[8];
  R(magic, 8);
  ok = ok && std::memcmp(magic, "DFMMOPS2", 8) == 0;
  int32_t whi = 0, cnt = 0;
  R(&set.tau, 8);
  R(&whi, 4);
  R(&cnt, 4);
  if (ok && (whi < 1 || (whi & (whi - 1)) || whi > 64)) ok = false;
  if (ok) {
    set.w_hi = whi;
    int emax = 0;
    while ((1 << emax) < whi) ++emax;
    int expect = 1;
    for (int e = 0; e <= emax; ++e) expect += 6 << (2 * e);
    ok = cnt == expect;
    set.hf.assign(emax + 1, {});
    auto get = [&](Skel& s) {
      int32_t r = 0;
      R(&r, 4);
      if (!ok || r < 1 || r > 4096) {
        ok = false;
        return;
      }
      s.r = r;
      s.a.resize(3 * size_t(r));
      s.b.resize(3 * size_t(r));
      s.D.resize(2 * size_t(r) * r);
      R(s.a.data(), 8 * s.a.size());
      R(s.b.data(), 8 * s.b.size());
      R(s.D.data(), 8 * s.D.size());
    };
    for (int e = 0; ok && e <= emax; ++e) {
      set.hf[e].assign(size_t(6) << (2 * e), Skel());
      for (auto& s : set.hf[e])
        if (ok) get(s);
    }
    if (ok) get(set.lf);
  }
  std::fclose(f);
  return ok;
}

}  // namespace dfmm

namespace dfmm {

// "DFMMLFD1", float64 tau, int32 n, then n skeletons (widths 1/4, 1/8, ...) as
// in the operator-set file.
bool save_lf_deep(const OpSetImpl& set, const std::string& path) {
  std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  bool ok = true;
  auto W = [&](const void* p, size_t n) { ok = ok && std::fwrite(p, 1, n, f) == n; };
  W("DFMMLFD1", 8);
  W(&set.tau, 8);
  int32_t cnt = int32_t(set.lf_deep.size());
  W(&cnt, 4);
  for (const Skel& s : set.lf_deep) {
    int32_t r = s.r;
    W(&r, 4);
    W(s.a.data(), 8 * s.a.size());
    W(s.b.data(), 8 * s.b.size());
    W(s.D.data(), 8 * s.D.size());
  }
  ok = (std::fclose(f) == 0) && ok;
  if (ok) ok = std::rename(tmp.c_str(), path.c_str()) == 0;
  if (!ok) std::remove(tmp.c_str());
  return ok;
}

bool load_lf_deep(OpSetImpl& set, const std::string& path, int n) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  bool ok = true;
  auto R = [&](void* p, size_t k) { ok = ok && std::fread(p, 1, k, f) == k; };
  char magic[8];
  R(magic, 8);
  ok = ok && std::memcmp(magic, "DFMMLFD1", 8) == 0;
  double tau = 0.0;
  int32_t cnt = 0;
  R(&tau, 8);
  R(&cnt, 4);
  ok = ok && tau == set.tau && cnt >= n && cnt <= kMaxLfLevels;
  std::vector<Skel> out;
  for (int i = 0; ok && i < n; ++i) {
    Skel s;
    int32_t r = 0;
    R(&r, 4);
    if (!ok || r < 1 || r > 4096) {
      ok = false;
      break;
    }
    s.r = r;
    s.a.resize(3 * size_t(r));
    s.b.resize(3 * size_t(r));
    s.D.resize(2 * size_t(r) * r);
    R(s.a.data(), 8 * s.a.size());
    R(s.b.data(), 8 * s.b.size());
    R(s.D.data(), 8 * s.D.size());
    out.push_back(std::move(s));
  }
  std::fclose(f);
  if (ok) set.lf_deep = std::move(out);
  return ok;
}

}  // namespace dfmm
