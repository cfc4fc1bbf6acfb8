// Host-side lattice algebra: the 3x3 Bloch blocks of the kagome kinetic
// matrix (Eqs. (3)-(4)) and their exponentials, tabulated per momentum.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "common.h"

namespace kdqmc {

namespace {

using cd = std::complex<double>;

// One directed hopping term of Eq. (3): row sublattice `to`, column
// sublattice `from`, cell displacement (row cell - column cell) = (d1, d2).
struct Hop {
  int to, from, d1, d2;
};

// Eq. (3) term by term (s = 0, 1, 2 for A, B, C; K_s maps cell x to x+1):
//   I (x) (I + K_s) (x) delta_a : B <- A, displacements (0,0), (0,+1)
//   (I + K_s) (x) I (x) delta_b : C <- A, displacements (0,0), (+1,0)
//   (I (x) I + K_s (x) K_s^T) (x) delta_c : C <- B, displacements (0,0), (+1,-1)
// plus the Hermitian conjugate of each (from <-> to, d -> -d).
constexpr Hop kHops[6] = {
    {1, 0, 0, 0}, {1, 0, 0, 1}, {2, 0, 0, 0}, {2, 0, 1, 0}, {2, 1, 0, 0}, {2, 1, 1, -1},
};

// App. A1, triangular lattice (one site per cell):
//   I (x) K_s + K_s (x) I + K_s (x) K_s : displacements (0,+1), (+1,0), (+1,+1)
constexpr Hop kTriHops[3] = {{0, 0, 0, 1}, {0, 0, 1, 0}, {0, 0, 1, 1}};
// App. A2, honeycomb lattice (sublattices 0, 1):
//   (I (x) I + I (x) K_s + K_s (x) I) (x) delta : 1 <- 0 at (0,0), (0,+1), (+1,0)
constexpr Hop kHonHops[3] = {{1, 0, 0, 0}, {1, 0, 0, 1}, {1, 0, 1, 0}};

// H(k)_{s s'} = sum over hops (s <- s', d) of -t exp(-i k.d), for the forward
// transform v^(k) = sum_x exp(-i k.x) v(x) (so (K v)^ = H(k) v^); the S x S
// block of the lattice in the top-left corner, zeros elsewhere.
void bloch_H_lattice(int lattice, double t, double k1, double k2, cd h[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) h[a][b] = 0.0;
  const Hop* hops = lattice == KDQMC_TRIANGULAR ? kTriHops : lattice == KDQMC_HONEYCOMB ? kHonHops : kHops;
  const int nh = lattice == KDQMC_KAGOME ? 6 : 3;
  for (int q = 0; q < nh; ++q) {
    const Hop& hp = hops[q];
    const double ph = -(k1 * hp.d1 + k2 * hp.d2);
    const cd v = -t * std::polar(1.0, ph);
    h[hp.to][hp.from] += v;
    h[hp.from][hp.to] += std::conj(v);
  }
}

void bloch_H(double t, double k1, double k2, cd h[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) h[a][b] = 0.0;
  for (const Hop& hp : kHops) {
    const double ph = -(k1 * hp.d1 + k2 * hp.d2);
    const cd v = -t * std::polar(1.0, ph);
    h[hp.to][hp.from] += v;
    h[hp.from][hp.to] += std::conj(v);
  }
}

void matmul3(const cd a[3][3], const cd b[3][3], cd out[3][3]) {
  cd r[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cd s = 0.0;
      for (int k = 0; k < 3; ++k) s += a[i][k] * b[k][j];
      r[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[i][j] = r[i][j];
}

// exp(A) for a 3x3 complex matrix: scaling and squaring with a Taylor
// series of 30 terms on ||A / 2^s|| <= 1/2.
void expm3(const cd a[3][3], cd out[3][3]) {
  double nrm = 0.0;
  for (int i = 0; i < 3; ++i) {
    double row = 0.0;
    for (int j = 0; j < 3; ++j) row += std::abs(a[i][j]);
    nrm = std::max(nrm, row);
  }
  int s = 0;
  while (nrm > 0.5) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = std::ldexp(1.0, -s);
  cd x[3][3], term[3][3], sum[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      x[i][j] = a[i][j] * sc;
      term[i][j] = (i == j) ? 1.0 : 0.0;
      sum[i][j] = term[i][j];
    }
  for (int n = 1; n <= 30; ++n) {
    matmul3(term, x, term);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        term[i][j] /= double(n);
        sum[i][j] += term[i][j];
      }
  }
  for (int q = 0; q < s; ++q) matmul3(sum, sum, sum);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[i][j] = sum[i][j];
}

// Real eigenvalues of a 3x3 Hermitian matrix (trigonometric solution of the
// characteristic cubic), ascending.
void eig3_hermitian(const cd h[3][3], double ev[3]) {
  const double a = h[0][0].real(), b = h[1][1].real(), c = h[2][2].real();
  const double tr = a + b + c;
  const double m = tr / 3.0;
  // shifted matrix B = H - m I
  cd s[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s[i][j] = h[i][j] - ((i == j) ? m : 0.0);
  double p2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) p2 += std::norm(s[i][j]);
  const double p = std::sqrt(p2 / 6.0);
  if (p == 0.0) {
    ev[0] = ev[1] = ev[2] = m;
    return;
  }
  cd bm[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) bm[i][j] = s[i][j] / p;
  const cd det = bm[0][0] * (bm[1][1] * bm[2][2] - bm[1][2] * bm[2][1]) -
                 bm[0][1] * (bm[1][0] * bm[2][2] - bm[1][2] * bm[2][0]) +
                 bm[0][2] * (bm[1][0] * bm[2][1] - bm[1][1] * bm[2][0]);
  double r = det.real() / 2.0;
  r = std::max(-1.0, std::min(1.0, r));
  const double phi = std::acos(r) / 3.0;
  const double e0 = m + 2.0 * p * std::cos(phi);
  const double e2 = m + 2.0 * p * std::cos(phi + 2.0 * kPi / 3.0);
  const double e1 = tr - e0 - e2;
  ev[0] = e2;
  ev[1] = e1;
  ev[2] = e0;
}

// Eigen-decomposition of a 3x3 Hermitian matrix by cyclic complex Jacobi
// rotations: h = V diag(w) V^+, w ascending, V unitary (columns = vectors).
// Each rotation first turns h_pq real by a diagonal phase, then zeroes it by
// a real plane rotation of angle 0.5 atan2(2 |h_pq|, h_qq - h_pp).
void jacobi3(const cd h_in[3][3], double w[3], cd V[3][3]) {
  cd a[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      a[i][j] = h_in[i][j];
      V[i][j] = (i == j) ? 1.0 : 0.0;
    }
  double scale = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) scale += std::norm(a[i][j]);
  for (int sweep = 0; sweep < 60; ++sweep) {
    const double off = std::norm(a[0][1]) + std::norm(a[0][2]) + std::norm(a[1][2]);
    if (off <= 1e-34 * (scale + 1e-300)) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double r = std::abs(a[p][q]);
      if (r == 0.0) continue;
      const cd ph = a[p][q] / r;  // exp(i phi)
      const double th = 0.5 * std::atan2(2.0 * r, a[q][q].real() - a[p][p].real());
      const double c = std::cos(th), sn = std::sin(th);
      // G = identity except the (p, q) block diag(1, e^{-i phi}) [[c, s], [-s, c]]
      cd G[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G[i][j] = (i == j) ? 1.0 : 0.0;
      const cd e = std::conj(ph);
      G[p][p] = c;
      G[p][q] = sn;
      G[q][p] = -sn * e;
      G[q][q] = c * e;
      cd t1[3][3], Gh[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Gh[i][j] = std::conj(G[j][i]);
      matmul3(a, G, t1);
      matmul3(Gh, t1, a);
      matmul3(V, G, t1);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = t1[i][j];
      a[q][p] = 0.0;
      a[p][q] = 0.0;
    }
  }
  int ord[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (a[ord[j]][ord[j]].real() < a[ord[i]][ord[i]].real()) std::swap(ord[i], ord[j]);
  cd Vs[3][3];
  for (int k = 0; k < 3; ++k) {
    w[k] = a[ord[k]][ord[k]].real();
    for (int i = 0; i < 3; ++i) Vs[i][k] = V[i][ord[k]];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = Vs[i][j];
}

}  // namespace

// The trial orbitals of the projector form: the lowest n_occ eigenvectors of
// K_T = K + eps (n_A - n_C) (per cell), real and orthonormal, from the 3x3
// Bloch blocks H(k) + diag(eps, 0, -eps) (the potential is translation
// invariant).  A state of momentum k is psi(x, s) = e^{i k.x} v_s / L; the
// pair k, -k (equal levels, H(-k) = H(k)*) gives sqrt(2) Re psi and
// sqrt(2) Im psi, a self-conjugate k (2k on the grid's origin) the real psi.
int trial_orbitals(int L, double t, int n_occ, double eps, double* P) {
  const int N = 3 * L * L;
  if (n_occ < 1 || n_occ > N) return set_error(KDQMC_EINVAL, "n_occ must be in 1..N");
  struct Lev {
    double e;
    int m1, m2, b;
  };
  std::vector<Lev> lev;
  std::vector<cd> vec((size_t)L * L * 9);
  for (int m1 = 0; m1 < L; ++m1)
    for (int m2 = 0; m2 < L; ++m2) {
      cd h[3][3], V[3][3];
      bloch_H(t, 2.0 * kPi * m1 / L, 2.0 * kPi * m2 / L, h);
      h[0][0] += eps;
      h[2][2] -= eps;
      double w[3];
      jacobi3(h, w, V);
      for (int b = 0; b < 3; ++b) {
        lev.push_back({w[b], m1, m2, b});
        for (int sidx = 0; sidx < 3; ++sidx) vec[((size_t)(m1 * L + m2) * 3 + b) * 3 + sidx] = V[sidx][b];
      }
    }
  std::stable_sort(lev.begin(), lev.end(), [](const Lev& x, const Lev& y) { return x.e < y.e; });
  if (n_occ < N && lev[n_occ].e - lev[n_occ - 1].e < 1e-8)
    return set_error(KDQMC_EINVAL, "open shell: trial levels n_occ and n_occ+1 are degenerate (choose eps or n_occ)");
  std::vector<char> sel((size_t)L * L * 3, 0);
  for (int i = 0; i < n_occ; ++i) sel[(size_t)(lev[i].m1 * L + lev[i].m2) * 3 + lev[i].b] = 1;
  const double inv = 1.0 / L, r2 = std::sqrt(2.0) / L;
  int col = 0;
  for (int m1 = 0; m1 < L; ++m1)
    for (int m2 = 0; m2 < L; ++m2)
      for (int b = 0; b < 3; ++b) {
        const size_t kb = (size_t)(m1 * L + m2) * 3 + b;
        if (!sel[kb]) continue;
        const int n1 = (L - m1) % L, n2 = (L - m2) % L;
        const bool self = (n1 == m1 && n2 == m2);
        if (!self && m1 * L + m2 > n1 * L + n2) continue;  // emitted with its partner
        if (!self && !sel[(size_t)(n1 * L + n2) * 3 + b])
          return set_error(KDQMC_EINVAL, "open shell: a level of k is selected without that of -k");
        cd v[3];
        for (int sidx = 0; sidx < 3; ++sidx) v[sidx] = vec[kb * 3 + sidx];
        if (self) {  // a real vector up to a phase: make the largest component real
          int im = 0;
          for (int sidx = 1; sidx < 3; ++sidx)
            if (std::abs(v[sidx]) > std::abs(v[im])) im = sidx;
          const cd ph = std::conj(v[im]) / std::abs(v[im]);
          for (int sidx = 0; sidx < 3; ++sidx) v[sidx] *= ph;
        }
        const int ncols = self ? 1 : 2;
        if (col + ncols > n_occ) return set_error(KDQMC_EINVAL, "trial orbitals: inconsistent level count");
        for (int x1 = 0; x1 < L; ++x1)
          for (int x2 = 0; x2 < L; ++x2) {
            const cd ex = std::polar(1.0, 2.0 * kPi * double(m1 * x1 + m2 * x2) / L);
            for (int sidx = 0; sidx < 3; ++sidx) {
              const cd psi = ex * v[sidx];
              const size_t row = (size_t)((x1 * L + x2) * 3 + sidx);
              if (self) {
                P[row * n_occ + col] = psi.real() * inv;
              } else {
                P[row * n_occ + col] = psi.real() * r2;
                P[row * n_occ + col + 1] = psi.imag() * r2;
              }
            }
          }
        col += ncols;
      }
  if (col != n_occ) return set_error(KDQMC_EINVAL, "trial orbitals: inconsistent level count");
  return KDQMC_OK;
}

bool lattice_supported(int L) {
  switch (L) {
    case 3: case 6: case 9: case 12: case 15: case 18: case 24:
      return true;
    default:
      return false;
  }
}

int lattice_nsub(int lattice) {
  return lattice == KDQMC_TRIANGULAR ? 1 : lattice == KDQMC_HONEYCOMB ? 2 : 3;
}

void bloch_table(int lattice, int L, double t, double scale, double shift, double* tab) {
  const int S = lattice_nsub(lattice);
  const double norm = 1.0 / double(L * L);
  for (int m1 = 0; m1 < L; ++m1)
    for (int m2 = 0; m2 < L; ++m2) {
      const double k1 = 2.0 * kPi * m1 / L, k2 = 2.0 * kPi * m2 / L;
      cd h[3][3], e[3][3];
      bloch_H_lattice(lattice, t, k1, k2, h);
      // the S x S block (the zero padding exponentiates to the identity)
      for (int i = 0; i < S; ++i) {
        h[i][i] -= shift;
        for (int j = 0; j < S; ++j) h[i][j] *= scale;
      }
      expm3(h, e);
      double* out = tab + 2 * S * S * (m1 * L + m2);
      for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j) {
          out[2 * (S * i + j)] = e[i][j].real() * norm;
          out[2 * (S * i + j) + 1] = e[i][j].imag() * norm;
        }
    }
}

double dirac_mu(int /*L*/, double t) {
  // The Dirac point of the kagome bands sits at k = (2 pi/3, -2 pi/3) in the
  // reciprocal basis of the cell coordinates; there the two dispersive
  // bands are degenerate.  Return that doubly degenerate eigenvalue.
  cd h[3][3];
  bloch_H(t, 2.0 * kPi / 3.0, -2.0 * kPi / 3.0, h);
  double ev[3];
  eig3_hermitian(h, ev);
  return (std::abs(ev[0] - ev[1]) < std::abs(ev[1] - ev[2])) ? 0.5 * (ev[0] + ev[1])
                                                              : 0.5 * (ev[1] + ev[2]);
}

}  // namespace kdqmc
