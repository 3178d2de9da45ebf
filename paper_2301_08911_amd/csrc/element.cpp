// Host-side element constants of the 8-node trilinear brick (unit cube, E = 1).
//
// K0 is built from exact one-dimensional integrals of the linear shape
// functions (mass, stiffness and mixed 2x2 matrices) combined by tensor
// product, with the isotropic tensor C_piqj = lambda d_pi d_qj +
// mu (d_pq d_ij + d_pj d_iq).  From K0 the library derives:
//   * its Walsh-Hadamard mode form (the level-0 operator, C^H, sensitivities),
//   * the macro-strain load templates K0 chi^i (Sec. 4.2, Eq. macro-strain),
//   * the diagonal blocks K0[a,a] used by block-Jacobi (Sec. 4.2, Eq.
//     st-assemb-gs: S_v = sum_e s_e K0[7-e, 7-e]),
//   * the sub-element Galerkin matrices W_s^T K0 W_s used to assemble the
//     first coarse level from densities (Sec. 4.2, Eq. st-level-2).
#include <cmath>
#include <cstdio>
#include <cstring>

#include "hmg_internal.hpp"

namespace hmg {
namespace {

inline int bit(int a, int k) { return (a >> k) & 1; }

// int over [0,1] of (d/dx if di) N_a * (d/dx if dj) N_b, N_0 = 1 - x, N_1 = x.
double integral_1d(int a, int b, bool da, bool db) {
  static const double M[2][2] = {{1.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 1.0 / 3.0}};
  static const double S[2][2] = {{1.0, -1.0}, {-1.0, 1.0}};
  static const double Dm[2][2] = {{-0.5, -0.5}, {0.5, 0.5}};  // int N_a' N_b
  if (da && db) return S[a][b];
  if (da) return Dm[a][b];
  if (db) return Dm[b][a];
  return M[a][b];
}

// int over the unit cube of d_i N_a d_j N_b
double grad_integral(int a, int i, int b, int j) {
  double v = 1.0;
  for (int k = 0; k < 3; ++k) v *= integral_1d(bit(a, k), bit(b, k), k == i, k == j);
  return v;
}

}  // namespace

int build_element_consts(double nu, ElementConsts* out, char* err, size_t errlen) {
  std::memset(out, 0, sizeof(*out));
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));

  // ---- K0
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
          double tr = 0.0;
          for (int i = 0; i < 3; ++i) tr += grad_integral(a, i, b, i);
          out->K0[3 * a + p][3 * b + q] = lam * grad_integral(a, p, b, q) +
                                          mu * ((p == q ? tr : 0.0) + grad_integral(a, q, b, p));
        }

  // ---- the ten distinct magnitudes of K0 (k0_sel), checked against K0
  {
    const double M[2] = {1.0 / 6.0, 1.0 / 3.0}, G[2] = {-1.0, 1.0};
    for (int ei = 0; ei < 2; ++ei)
      for (int c = 0; c < 3; ++c) {
        const int ej = c >= 1 ? 1 : 0, em = c >= 2 ? 1 : 0;
        out->kv[3 * ei + c] = (lam + 2 * mu) * G[ei] * M[ej] * M[em] +
                              mu * M[ei] * (G[ej] * M[em] + G[em] * M[ej]);
      }
    for (int em = 0; em < 2; ++em) {
      out->kv[6 + 2 * em] = (lam - mu) * M[em] / 4.0;
      out->kv[6 + 2 * em + 1] = (lam + mu) * M[em] / 4.0;
    }
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b)
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) {
            const int sel = k0_sel(a, p, b, q);
            const double v = (sel & 1) ? -out->kv[sel >> 1] : out->kv[sel >> 1];
            if (std::fabs(v - out->K0[3 * a + p][3 * b + q]) > 1e-14) {
              std::snprintf(err, errlen, "K0 entry (%d,%d) does not follow its selector",
                            3 * a + p, 3 * b + q);
              return 1;
            }
          }
  }

  // ---- mode form Kt = H K0 H / 64
  double Kt[24][24];
  auto H = [](int a, int m) { return (__builtin_popcount(a & m) & 1) ? -1.0 : 1.0; };
  for (int m = 0; m < 8; ++m)
    for (int k = 0; k < 3; ++k)
      for (int m2 = 0; m2 < 8; ++m2)
        for (int k2 = 0; k2 < 3; ++k2) {
          double acc = 0.0;
          for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) acc += H(a, m) * out->K0[3 * a + k][3 * b + k2] * H(b, m2);
          Kt[3 * m + k][3 * m2 + k2] = acc / 64.0;
        }
  ModeK<double>& mk = out->mk;
  mk.b = Kt[3][7];
  mk.ab = Kt[3][3] - mk.b;
  mk.cs = Kt[4][4];
  mk.p = Kt[9][9];
  mk.q = Kt[9][20];
  mk.g = Kt[11][16];
  mk.fg = Kt[11][11] - mk.g;
  mk.z = Kt[21][21];
  // Rebuild Kt from the block pattern and require an exact match.
  double R[24][24];
  std::memset(R, 0, sizeof(R));
  auto I = [](int m, int k) { return 3 * m + k; };
  const int normal[3] = {I(1, 0), I(2, 1), I(4, 2)};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[normal[i]][normal[j]] = (i == j) ? mk.ab + mk.b : mk.b;
  const int shear[3][2] = {{I(1, 1), I(2, 0)}, {I(1, 2), I(4, 0)}, {I(2, 2), I(4, 1)}};
  for (auto& s : shear)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) R[s[i]][s[j]] = mk.cs;
  const int pairs[3][2] = {{I(3, 0), I(6, 2)}, {I(3, 1), I(5, 2)}, {I(5, 0), I(6, 1)}};
  for (auto& s : pairs)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) R[s[i]][s[j]] = (i == j) ? mk.p : mk.q;
  const int triple[3] = {I(3, 2), I(5, 1), I(6, 0)};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[triple[i]][triple[j]] = (i == j) ? mk.fg + mk.g : mk.g;
  for (int k = 0; k < 3; ++k) R[I(7, k)][I(7, k)] = mk.z;
  double scale = 0.0, dev = 0.0;
  for (int i = 0; i < 24; ++i)
    for (int j = 0; j < 24; ++j) {
      scale = std::fmax(scale, std::fabs(Kt[i][j]));
      dev = std::fmax(dev, std::fabs(Kt[i][j] - R[i][j]));
    }
  if (!(dev <= 1e-13 * scale)) {
    std::snprintf(err, errlen, "element stiffness does not have the expected mode pattern (dev %g)",
                  dev);
    return 1;
  }

  // ---- unit-strain displacements (element-relative coordinates) and loads
  double chi[NCASE][24];
  std::memset(chi, 0, sizeof(chi));
  for (int b = 0; b < 8; ++b) {
    const double x0 = bit(b, 0), x1 = bit(b, 1), x2 = bit(b, 2);
    chi[0][3 * b + 0] = x0;
    chi[1][3 * b + 1] = x1;
    chi[2][3 * b + 2] = x2;
    chi[3][3 * b + 0] = 0.5 * x1;
    chi[3][3 * b + 1] = 0.5 * x0;
    chi[4][3 * b + 1] = 0.5 * x2;
    chi[4][3 * b + 2] = 0.5 * x1;
    chi[5][3 * b + 0] = 0.5 * x2;
    chi[5][3 * b + 2] = 0.5 * x0;
  }
  for (int c = 0; c < NCASE; ++c)
    for (int i = 0; i < 24; ++i) {
      double acc = 0.0;
      for (int j = 0; j < 24; ++j) acc += out->K0[i][j] * chi[c][j];
      out->load[c][i / 3][i % 3] = acc;
    }
  for (int c = 0; c < NCASE; ++c)
    for (int m = 0; m < 8; ++m)
      for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int a = 0; a < 8; ++a) acc += H(a, m) * chi[c][3 * a + k];
        out->chihat[c][m][k] = acc;
      }

  // ---- diagonal blocks: K0[a,a] = dd I + oo sg(a,p) sg(a,q) off the diagonal
  out->dd = out->K0[0][0];
  out->oo = out->K0[0][1];
  for (int a = 0; a < 8; ++a)
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        const double sp = bit(a, p) ? 1.0 : -1.0, sq = bit(a, q) ? 1.0 : -1.0;
        const double want = (p == q) ? out->dd : out->oo * sp * sq;
        if (std::fabs(out->K0[3 * a + p][3 * a + q] - want) > 1e-14) {
          std::snprintf(err, errlen, "unexpected diagonal block pattern of K0");
          return 1;
        }
      }

  // ---- spectral bound of block Jacobi on one element: largest eigenvalue of
  // blockdiag(K0)^-1 K0, by power iteration (24 unknowns, run to convergence).
  // Since K = sum_e s_e Q_e^T K0 Q_e and D = sum_e s_e blockdiag(K0 placed at e),
  // lambda_max(D^-1 K) <= lam0 for every density field.
  {
    double Dinv[8][3][3];
    for (int a = 0; a < 8; ++a) {
      double m[3][3];
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) m[p][q] = out->K0[3 * a + p][3 * a + q];
      const double c00 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
      const double c01 = m[0][2] * m[2][1] - m[0][1] * m[2][2];
      const double c02 = m[0][1] * m[1][2] - m[0][2] * m[1][1];
      const double c10 = m[1][2] * m[2][0] - m[1][0] * m[2][2];
      const double c11 = m[0][0] * m[2][2] - m[0][2] * m[2][0];
      const double c12 = m[0][2] * m[1][0] - m[0][0] * m[1][2];
      const double c20 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
      const double c21 = m[0][1] * m[2][0] - m[0][0] * m[2][1];
      const double c22 = m[0][0] * m[1][1] - m[0][1] * m[1][0];
      const double det = m[0][0] * c00 + m[0][1] * c10 + m[0][2] * c20;
      const double inv[3][3] = {{c00, c01, c02}, {c10, c11, c12}, {c20, c21, c22}};
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) Dinv[a][p][q] = inv[p][q] / det;
    }
    double x[24], y[24];
    for (int i = 0; i < 24; ++i) x[i] = 1.0 + 0.37 * i - 0.011 * i * i;
    double lam = 0.0;
    for (int it = 0; it < 20000; ++it) {
      for (int i = 0; i < 24; ++i) {
        y[i] = 0.0;
        for (int j = 0; j < 24; ++j) y[i] += out->K0[i][j] * x[j];
      }
      double num = 0.0, den = 0.0;  // Rayleigh quotient x^T K0 x / x^T D x
      for (int i = 0; i < 24; ++i) num += x[i] * y[i];
      double z[24];
      for (int a = 0; a < 8; ++a)
        for (int p = 0; p < 3; ++p) {
          z[3 * a + p] = 0.0;
          for (int q = 0; q < 3; ++q) z[3 * a + p] += Dinv[a][p][q] * y[3 * a + q];
        }
      for (int a = 0; a < 8; ++a)
        for (int p = 0; p < 3; ++p) {
          double dx = 0.0;
          for (int q = 0; q < 3; ++q) dx += out->K0[3 * a + p][3 * a + q] * x[3 * a + q];
          den += x[3 * a + p] * dx;
        }
      lam = num / den;
      double nrm = 0.0;
      for (int i = 0; i < 24; ++i) nrm += z[i] * z[i];
      nrm = std::sqrt(nrm);
      for (int i = 0; i < 24; ++i) x[i] = z[i] / nrm;
    }
    out->lam0 = lam;
  }

  // ---- sub-element Galerkin matrices of the dyadic first coarse level
  subelement_matrices(out->K0, 2, &out->msig[0][0][0]);
  return 0;
}

// Fine element at sub-position sigma = (sx, sy, sz) in 0..F-1 of a coarse
// element F fine cells long; its node b sits at xi = (sigma + b) / F in
// coarse-element coordinates and takes the trilinear weights of the coarse
// nodes A (Eq. st-assemb-w).  Matrix sigma = sx + F (sy + F sz) is
// W_sigma^T K0 W_sigma, 24 x 24 row-major.
void subelement_matrices(const double K0[24][24], int F, double* out) {
  for (int sg = 0; sg < F * F * F; ++sg) {
    const int sub[3] = {sg % F, (sg / F) % F, sg / (F * F)};
    double w[8][8];
    for (int b = 0; b < 8; ++b)
      for (int A = 0; A < 8; ++A) {
        double v = 1.0;
        for (int t = 0; t < 3; ++t) {
          const double xi = (double)(sub[t] + bit(b, t)) / F;
          v *= bit(A, t) ? xi : 1.0 - xi;
        }
        w[b][A] = v;
      }
    double* M = out + (size_t)sg * 576;
    for (int A = 0; A < 8; ++A)
      for (int Bn = 0; Bn < 8; ++Bn)
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) {
            double acc = 0.0;
            for (int a = 0; a < 8; ++a)
              for (int b = 0; b < 8; ++b) acc += w[a][A] * K0[3 * a + p][3 * b + q] * w[b][Bn];
            M[(3 * A + p) * 24 + 3 * Bn + q] = acc;
          }
  }
}

}  // namespace hmg
