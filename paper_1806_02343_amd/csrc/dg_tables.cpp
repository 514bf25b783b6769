// Reference-element tables: Gauss-Legendre rules (Sec. 3.5), the Legendre
// basis (Sec. 3.2) and the locally divergence-free basis (Sec. 3.3, App. A),
// evaluated at volume, face and projection points.
#include "dg_tables.h"

#include <algorithm>
#include <array>
#include <cmath>

namespace dgmhd {

namespace {

// Legendre polynomial and derivative by the three-term recurrence and the
// derivative recurrence l'_{k+1} = l'_{k-1} + (2k+1) l_k.
void leg(int k, double x, double& p, double& dp) {
  double pm = 1.0, pc = x, dm = 0.0, dc = 1.0;
  if (k == 0) { p = 1.0; dp = 0.0; return; }
  for (int j = 1; j < k; ++j) {
    double pn = ((2 * j + 1) * x * pc - j * pm) / (j + 1);
    double dn = dm + (2 * j + 1) * pc;
    pm = pc; pc = pn; dm = dc; dc = dn;
  }
  p = pc; dp = dc;
}

double legv(int k, double x) { double p, dp; leg(k, x, p, dp); return p; }
double legd(int k, double x) { double p, dp; leg(k, x, p, dp); return dp; }

// Dense polynomial in three variables, exponents up to DM each.
struct Poly {
  int DM = 0;
  std::vector<double> c;  // index i + (DM+1)(j + (DM+1) k)
  explicit Poly(int dm = 0) : DM(dm), c((dm + 1) * (dm + 1) * (dm + 1), 0.0) {}
  double& at(int i, int j, int k) { return c[i + (DM + 1) * (j + (DM + 1) * k)]; }
  double at(int i, int j, int k) const { return c[i + (DM + 1) * (j + (DM + 1) * k)]; }
  bool zero() const { for (double v : c) if (v != 0.0) return false; return true; }
  int degree() const {
    int g = -1;
    for (int k = 0; k <= DM; ++k) for (int j = 0; j <= DM; ++j) for (int i = 0; i <= DM; ++i)
      if (at(i, j, k) != 0.0) g = std::max(g, i + j + k);
    return g;
  }
  Poly deriv(int a) const {
    Poly r(DM);
    for (int k = 0; k <= DM; ++k) for (int j = 0; j <= DM; ++j) for (int i = 0; i <= DM; ++i) {
      double v = at(i, j, k);
      if (v == 0.0) continue;
      int e[3] = {i, j, k};
      if (e[a] == 0) continue;
      double f = v * e[a];
      e[a] -= 1;
      r.at(e[0], e[1], e[2]) += f;
    }
    return r;
  }
  double eval(const double* xi, int D) const {
    double s = 0.0;
    for (int k = 0; k <= DM; ++k) for (int j = 0; j <= DM; ++j) for (int i = 0; i <= DM; ++i) {
      double v = at(i, j, k);
      if (v == 0.0) continue;
      double t = v * std::pow(xi[0], i) * std::pow(xi[1], j);
      if (D == 3) t *= std::pow(xi[2], k);
      s += t;
    }
    return s;
  }
};

// Monomial coefficients of l_k, from l_k = 2^-k sum_m (-1)^m C(k,m) C(2k-2m,k) x^(k-2m).
std::vector<double> leg_coeffs(int k) {
  std::vector<double> c(k + 1, 0.0);
  auto binom = [](int n, int r) { double b = 1; for (int i = 1; i <= r; ++i) b = b * (n - r + i) / i; return b; };
  for (int m = 0; 2 * m <= k; ++m)
    c[k - 2 * m] = ((m % 2) ? -1.0 : 1.0) * binom(k, m) * binom(2 * k - 2 * m, k) / std::ldexp(1.0, k);
  return c;
}

Poly legendre_product(const int* e, int DM) {
  Poly p(DM);
  auto c0 = leg_coeffs(e[0]), c1 = leg_coeffs(e[1]), c2 = leg_coeffs(e[2]);
  for (size_t i = 0; i < c0.size(); ++i) for (size_t j = 0; j < c1.size(); ++j) for (size_t k = 0; k < c2.size(); ++k)
    p.at((int)i, (int)j, (int)k) += c0[i] * c1[j] * c2[k];
  return p;
}

// integral of xi^e over [-1,1]^D
double mono_int(int i, int j, int k, int D) {
  auto one = [](int e) { return (e % 2) ? 0.0 : 2.0 / (e + 1); };
  double r = one(i) * one(j);
  if (D == 3) r *= one(k); else if (k != 0) return 0.0;
  return r;
}

double pinner(const Poly& a, const Poly& b, int D) {
  double s = 0.0;
  int M = a.DM;
  for (int k1 = 0; k1 <= M; ++k1) for (int j1 = 0; j1 <= M; ++j1) for (int i1 = 0; i1 <= M; ++i1) {
    double x = a.at(i1, j1, k1);
    if (x == 0.0) continue;
    for (int k2 = 0; k2 <= M; ++k2) for (int j2 = 0; j2 <= M; ++j2) for (int i2 = 0; i2 <= M; ++i2) {
      double y = b.at(i2, j2, k2);
      if (y == 0.0) continue;
      s += x * y * mono_int(i1 + i2, j1 + j2, k1 + k2, D);
    }
  }
  return s;
}

using Vec = std::vector<Poly>;  // D components

double vinner(const Vec& a, const Vec& b, int D) {
  double s = 0.0;
  for (int c = 0; c < D; ++c) s += pinner(a[c], b[c], D);
  return s;
}

void axpy(Vec& y, double a, const Vec& x) {
  for (size_t c = 0; c < y.size(); ++c)
    for (size_t i = 0; i < y[c].c.size(); ++i) y[c].c[i] += a * x[c].c[i];
}

Poly psub(const Poly& a, const Poly& b) {
  Poly r = a;
  for (size_t i = 0; i < r.c.size(); ++i) r.c[i] -= b.c[i];
  return r;
}

// Locally divergence-free basis of App. A in double precision (modified
// Gram-Schmidt with one re-orthogonalisation pass).
bool build_ldf(int D, int d, std::vector<Vec>& basis, std::vector<int>& degs, std::string& err) {
  int DM = d + 1;
  // pool polynomials: Legendre products of degree <= d+1 in the mode order
  std::vector<std::array<int, 3>> ex;
  for (int g = 0; g <= DM; ++g) {
    if (D == 2) {
      for (int k1 = g; k1 >= 0; --k1) ex.push_back({k1, g - k1, 0});
    } else {
      for (int k1 = g; k1 >= 0; --k1)
        for (int k2 = g - k1; k2 >= 0; --k2) ex.push_back({k1, k2, g - k1 - k2});
    }
  }
  std::vector<Vec> cand;
  std::vector<int> cdeg;
  auto push = [&](const Vec& v) {
    int g = -1;
    for (auto& p : v) g = std::max(g, p.degree());
    if (g < 0) return;
    cand.push_back(v);
    cdeg.push_back(g);
  };
  for (int comp = 0; comp < (D == 3 ? 3 : 1); ++comp) {
    for (auto& e : ex) {
      Poly Q = legendre_product(e.data(), DM);
      // V has Q in component `comp` (3-D) or in the z component (2-D)
      Poly zero(DM);
      Poly Vx = zero, Vy = zero, Vz = zero;
      if (D == 3) { if (comp == 0) Vx = Q; else if (comp == 1) Vy = Q; else Vz = Q; }
      else Vz = Q;
      // curl V = (dy Vz - dz Vy, dz Vx - dx Vz, dx Vy - dy Vx)
      Vec cv;
      cv.push_back(psub(Vz.deriv(1), Vy.deriv(2)));
      cv.push_back(psub(Vx.deriv(2), Vz.deriv(0)));
      if (D == 3) cv.push_back(psub(Vy.deriv(0), Vx.deriv(1)));
      push(cv);
    }
  }
  std::vector<int> order(cand.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cdeg[a] < cdeg[b]; });
  int target = ndiv(D, d);
  std::vector<double> norms;
  for (int idx : order) {
    const Vec& c = cand[idx];
    Vec r = c;
    double cn = vinner(c, c, D);
    for (int pass = 0; pass < 2; ++pass)
      for (size_t j = 0; j < basis.size(); ++j) {
        double pr = vinner(r, basis[j], D) / norms[j];
        if (pr != 0.0) axpy(r, -pr, basis[j]);
      }
    double rn = vinner(r, r, D);
    if (rn <= 1e-20 * cn) continue;
    // clean round-off below the exact-arithmetic scale
    for (auto& p : r) for (auto& v : p.c) if (std::fabs(v) < 1e-14 * std::sqrt(cn)) v = 0.0;
    basis.push_back(r);
    norms.push_back(vinner(r, r, D));
    degs.push_back(cdeg[idx]);
    if ((int)basis.size() == target) break;
  }
  if ((int)basis.size() != target) { err = "LDF generator did not reach N_div"; return false; }
  return true;
}

}  // namespace

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    // Tricomi's asymptotic first guess, then Newton
    double t = pi * (4.0 * (i + 1) - 1.0) / (4.0 * n + 2.0);
    double z = (1.0 - 1.0 / (8.0 * n * n) + 1.0 / (8.0 * n * n * n)) * std::cos(t);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      leg(n, z, p, dp);
      double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p, dp;
    leg(n, z, p, dp);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  for (int i = 0; i < n / 2; ++i) {  // exact symmetry
    double a = 0.5 * (x[n - 1 - i] - x[i]);
    double b = 0.5 * (w[n - 1 - i] + w[i]);
    x[i] = -a; x[n - 1 - i] = a; w[i] = b; w[n - 1 - i] = b;
  }
  if (n % 2) x[n / 2] = 0.0;
}

namespace {

double poly1(const std::vector<double>& c, double x) {
  double s = 0.0;
  for (size_t i = c.size(); i-- > 0;) s = s * x + c[i];
  return s;
}

std::vector<double> deriv1(const std::vector<double>& c) {
  std::vector<double> r(c.size() > 1 ? c.size() - 1 : 1, 0.0);
  for (size_t i = 1; i < c.size(); ++i) r[i - 1] = (double)i * c[i];
  return r;
}

// Tables of the dynamic refinement (Sec. 4.4) on the Legendre product basis
// phi_n = prod_a l_{e_a}(xi_a), from exact 1-D integrals (Gauss rules with
// d + 1 points, exact for the degrees involved):
//  SQ_a[n][m] = sum_{k=1..d} 2^(2k-1) int d^k phi_n/dxi_a^k d^k phi_m/dxi_a^k
//  PRO_o[m][n] = <phi_m(eta), phi_n((eta + s_o)/2)> / <phi_m, phi_m>
//  RES_o[m][n] = 2^-D <phi_n(eta), phi_m((eta + s_o)/2)> / <phi_m, phi_m>
// (s_o = +-1 per axis from the bits of the octant o).
void amr_tables(Tables& t) {
  const int D = t.D, d = t.d, N = t.N, NO = 1 << D;
  std::vector<double> x, w;
  gauss_legendre(d + 1, x, w);
  std::vector<std::vector<double>> lc(d + 1);
  for (int k = 0; k <= d; ++k) lc[k] = leg_coeffs(k);
  // 1-D factors
  auto mass1 = [&](int e) { return 2.0 / (2.0 * e + 1.0); };
  // derivative products: I[k][e][f] = int l_e^(k) l_f^(k)
  std::vector<double> Id((size_t)(d + 1) * (d + 1) * (d + 1), 0.0);
  for (int e = 0; e <= d; ++e)
    for (int f = 0; f <= d; ++f) {
      std::vector<double> ce = lc[e], cf = lc[f];
      for (int k = 1; k <= d; ++k) {
        ce = deriv1(ce);
        cf = deriv1(cf);
        double sacc = 0.0;
        for (size_t q = 0; q < x.size(); ++q) sacc += w[q] * poly1(ce, x[q]) * poly1(cf, x[q]);
        Id[((size_t)k * (d + 1) + e) * (d + 1) + f] = sacc;
      }
    }
  // half-interval products: H[s][f][e] = int l_f(eta) l_e((eta + s)/2), s = -1 (0) or +1 (1)
  std::vector<double> H((size_t)2 * (d + 1) * (d + 1), 0.0);
  for (int sd = 0; sd < 2; ++sd)
    for (int f = 0; f <= d; ++f)
      for (int e = 0; e <= d; ++e) {
        double sacc = 0.0;
        for (size_t q = 0; q < x.size(); ++q)
          sacc += w[q] * poly1(lc[f], x[q]) * poly1(lc[e], 0.5 * (x[q] + (sd ? 1.0 : -1.0)));
        H[((size_t)sd * (d + 1) + f) * (d + 1) + e] = sacc;
      }
  const int* ex = t.expo.data();
  t.SQ.assign((size_t)D * N * N, 0.0);
  for (int a = 0; a < D; ++a)
    for (int n = 0; n < N; ++n)
      for (int m = 0; m < N; ++m) {
        bool same = true;
        double other = 1.0;
        for (int b = 0; b < D; ++b) {
          if (b == a) continue;
          if (ex[3 * n + b] != ex[3 * m + b]) same = false;
          else other *= mass1(ex[3 * n + b]);
        }
        if (!same) continue;
        double sacc = 0.0;
        for (int k = 1; k <= d; ++k)
          sacc += std::ldexp(1.0, 2 * k - 1) * Id[((size_t)k * (d + 1) + ex[3 * n + a]) * (d + 1) + ex[3 * m + a]];
        t.SQ[((size_t)a * N + n) * N + m] = sacc * other;
      }
  t.PRO.assign((size_t)NO * N * N, 0.0);
  t.RES.assign((size_t)NO * N * N, 0.0);
  for (int o = 0; o < NO; ++o)
    for (int m = 0; m < N; ++m)
      for (int n = 0; n < N; ++n) {
        double pr = 1.0, rs = 1.0;
        for (int b = 0; b < D; ++b) {
          const int sd = (o >> b) & 1, em = ex[3 * m + b], en = ex[3 * n + b];
          pr *= H[((size_t)sd * (d + 1) + em) * (d + 1) + en] / mass1(em);
          rs *= 0.5 * H[((size_t)sd * (d + 1) + en) * (d + 1) + em] / mass1(em);
        }
        t.PRO[((size_t)o * N + m) * N + n] = pr;
        t.RES[((size_t)o * N + m) * N + n] = rs;
      }
}

}  // namespace

bool build_tables(int D, int d, int divb, Tables& t, std::string& err) {
  if (D != 2 && D != 3) { err = "dim must be 2 or 3"; return false; }
  if (d < 1 || d > 3) { err = "degree must be 1..3"; return false; }
  t.D = D; t.d = d; t.divb = divb;
  t.P = d + 1;
  t.N = nmodes_scalar(D, d);
  t.Q = (D == 2) ? t.P * t.P : t.P * t.P * t.P;
  t.FP = (D == 2) ? t.P : t.P * t.P;
  if (divb == GLM) {
    t.NV = 9; t.NLEG = 9; t.NLDF = 0;
    for (int v = 0; v < 9; ++v) t.leg_var.push_back(v);
  } else {
    t.NV = 8;
    for (int v = 0; v < 5; ++v) t.leg_var.push_back(v);
    for (int c = D; c < 3; ++c) t.leg_var.push_back(5 + c);
    t.NLEG = (int)t.leg_var.size();
    t.NLDF = ndiv(D, d);
  }
  t.NMODES = t.NLEG * t.N + t.NLDF;
  const int P = t.P, N = t.N, Q = t.Q, FP = t.FP;
  gauss_legendre(P, t.xg, t.wg);
  // mode exponents: total degree, then k1 descending, then k2 descending
  for (int g = 0; g <= d; ++g) {
    if (D == 2) {
      for (int k1 = g; k1 >= 0; --k1) { t.expo.push_back(k1); t.expo.push_back(g - k1); t.expo.push_back(0); }
    } else {
      for (int k1 = g; k1 >= 0; --k1)
        for (int k2 = g - k1; k2 >= 0; --k2) { t.expo.push_back(k1); t.expo.push_back(k2); t.expo.push_back(g - k1 - k2); }
    }
  }
  auto Pl = [&](int l, const double* xi) {
    double v = 1.0;
    for (int a = 0; a < D; ++a) v *= legv(t.expo[3 * l + a], xi[a]);
    return v;
  };
  auto dPl = [&](int l, int a, const double* xi) {
    double v = 1.0;
    for (int b = 0; b < D; ++b) v *= (b == a) ? legd(t.expo[3 * l + b], xi[b]) : legv(t.expo[3 * l + b], xi[b]);
    return v;
  };
  // volume points
  std::vector<double> xq(Q * D), wq(Q);
  for (int q = 0; q < Q; ++q) {
    int q0 = q % P, q1 = (q / P) % P, q2 = q / (P * P);
    xq[q * D + 0] = t.xg[q0]; xq[q * D + 1] = t.xg[q1];
    wq[q] = t.wg[q0] * t.wg[q1];
    if (D == 3) { xq[q * D + 2] = t.xg[q2]; wq[q] *= t.wg[q2]; }
  }
  // face points: [a][s][r] -> xi
  std::vector<double> xf(D * 2 * FP * D), wf(FP);
  for (int r = 0; r < FP; ++r) wf[r] = (D == 2) ? t.wg[r] : t.wg[r % P] * t.wg[r / P];
  for (int a = 0; a < D; ++a)
    for (int s = 0; s < 2; ++s)
      for (int r = 0; r < FP; ++r) {
        double* xi = &xf[((a * 2 + s) * FP + r) * D];
        xi[a] = s ? 1.0 : -1.0;
        int j = 0;
        for (int b = 0; b < D; ++b) {
          if (b == a) continue;
          xi[b] = t.xg[j == 0 ? r % P : r / P];
          ++j;
        }
      }
  t.V.assign(Q * N, 0.0);
  t.GW.assign(D * Q * N, 0.0);
  for (int q = 0; q < Q; ++q)
    for (int l = 0; l < N; ++l) {
      t.V[q * N + l] = Pl(l, &xq[q * D]);
      for (int a = 0; a < D; ++a) t.GW[(a * Q + q) * N + l] = wq[q] * dPl(l, a, &xq[q * D]);
    }
  t.TF.assign(D * 2 * FP * N, 0.0);
  t.LF.assign(D * 2 * FP * N, 0.0);
  for (int a = 0; a < D; ++a)
    for (int s = 0; s < 2; ++s)
      for (int r = 0; r < FP; ++r)
        for (int l = 0; l < N; ++l) {
          double v = Pl(l, &xf[((a * 2 + s) * FP + r) * D]);
          t.TF[((a * 2 + s) * FP + r) * N + l] = v;
          t.LF[((a * 2 + s) * FP + r) * N + l] = wf[r] * v;
        }
  // sub-face tables for 2:1 hanging faces: the points of quarter j of a face
  // are xi_t = (xi_t^GL + o)/2 with o = -1 / +1 by bit t of j (tangential
  // axes in increasing order); index 0 is the full face
  const int NSUB = 1 + (1 << (D - 1));
  t.TFS.assign(D * 2 * NSUB * FP * N, 0.0);
  t.LFS.assign(D * 2 * NSUB * FP * N, 0.0);
  for (int a = 0; a < D; ++a)
    for (int sd = 0; sd < 2; ++sd)
      for (int sb = 0; sb < NSUB; ++sb)
        for (int r = 0; r < FP; ++r) {
          double xi[3] = {0, 0, 0};
          xi[a] = sd ? 1.0 : -1.0;
          int j = 0;
          for (int b = 0; b < D; ++b) {
            if (b == a) continue;
            double x = t.xg[j == 0 ? r % P : r / P];
            if (sb > 0) x = 0.5 * (x + (((sb - 1) >> j) & 1 ? 1.0 : -1.0));
            xi[b] = x;
            ++j;
          }
          const double scale = sb > 0 ? std::ldexp(1.0, -(D - 1)) : 1.0;
          for (int l = 0; l < N; ++l) {
            const double v = Pl(l, xi);
            const size_t o = ((((size_t)a * 2 + sd) * NSUB + sb) * FP + r) * N + l;
            t.TFS[o] = v;
            t.LFS[o] = scale * wf[r] * v;
          }
        }
  // mass
  t.Mass.assign(t.NMODES, 0.0);
  t.Minv.assign(t.NMODES, 0.0);
  for (int j = 0; j < t.NLEG; ++j)
    for (int l = 0; l < N; ++l) {
      double m = 1.0;
      for (int a = 0; a < D; ++a) m *= 2.0 / (2 * t.expo[3 * l + a] + 1);
      t.Mass[j * N + l] = m;
    }
  // projection rule with d+3 points
  std::vector<double> xp, wp;
  gauss_legendre(d + 3, xp, wp);
  const int PP = d + 3;
  t.NPROJ = (D == 2) ? PP * PP : PP * PP * PP;
  t.xproj.assign(t.NPROJ * D, 0.0);
  std::vector<double> wpj(t.NPROJ);
  for (int p = 0; p < t.NPROJ; ++p) {
    int p0 = p % PP, p1 = (p / PP) % PP, p2 = p / (PP * PP);
    t.xproj[p * D + 0] = xp[p0]; t.xproj[p * D + 1] = xp[p1];
    wpj[p] = wp[p0] * wp[p1];
    if (D == 3) { t.xproj[p * D + 2] = xp[p2]; wpj[p] *= wp[p2]; }
  }
  t.wproj = wpj;
  t.VPW.assign(t.NPROJ * N, 0.0);
  t.VP.assign(t.NPROJ * N, 0.0);
  for (int p = 0; p < t.NPROJ; ++p)
    for (int l = 0; l < N; ++l) {
      t.VP[p * N + l] = Pl(l, &t.xproj[p * D]);
      t.VPW[p * N + l] = wpj[p] * t.VP[p * N + l];
    }
  if (t.NLDF) {
    std::vector<Vec> basis;
    if (!build_ldf(D, d, basis, t.ldf_deg, err)) return false;
    const int L = t.NLDF;
    t.PV.assign(D * Q * L, 0.0);
    t.PGW.assign(D * D * Q * L, 0.0);
    t.PTF.assign(D * 2 * D * FP * L, 0.0);
    t.PLF.assign(D * 2 * D * FP * L, 0.0);
    t.Pmean.assign(D * L, 0.0);
    t.Plin.assign(D * D * L, 0.0);
    t.PVPW.assign(D * t.NPROJ * L, 0.0);
    t.PVP.assign(D * t.NPROJ * L, 0.0);
    for (int l = 0; l < L; ++l) {
      double nrm = vinner(basis[l], basis[l], D);
      t.Mass[t.NLEG * N + l] = nrm;
      for (int c = 0; c < D; ++c) {
        const Poly& pc = basis[l][c];
        for (int q = 0; q < Q; ++q) {
          t.PV[(c * Q + q) * L + l] = pc.eval(&xq[q * D], D);
          for (int a = 0; a < D; ++a)
            t.PGW[((a * D + c) * Q + q) * L + l] = wq[q] * pc.deriv(a).eval(&xq[q * D], D);
        }
        for (int a = 0; a < D; ++a)
          for (int s = 0; s < 2; ++s)
            for (int r = 0; r < FP; ++r) {
              double v = pc.eval(&xf[((a * 2 + s) * FP + r) * D], D);
              t.PTF[(((a * 2 + s) * D + c) * FP + r) * L + l] = v;
              t.PLF[(((a * 2 + s) * D + c) * FP + r) * L + l] = wf[r] * v;
            }
        // mean: integral / 2^D
        t.Pmean[c * L + l] = pinner(pc, [&] { Poly one(pc.DM); one.at(0, 0, 0) = 1.0; return one; }(), D) /
                             std::ldexp(1.0, D);
        for (int b = 0; b < D; ++b) {
          Poly xb(pc.DM);
          if (b == 0) xb.at(1, 0, 0) = 1.0; else if (b == 1) xb.at(0, 1, 0) = 1.0; else xb.at(0, 0, 1) = 1.0;
          t.Plin[(c * D + b) * L + l] = pinner(pc, xb, D) / pinner(xb, xb, D);
        }
        for (int p = 0; p < t.NPROJ; ++p) {
          t.PVP[(c * t.NPROJ + p) * L + l] = pc.eval(&t.xproj[p * D], D);
          t.PVPW[(c * t.NPROJ + p) * L + l] = wpj[p] * t.PVP[(c * t.NPROJ + p) * L + l];
        }
      }
    }
  }
  for (int m = 0; m < t.NMODES; ++m) t.Minv[m] = 1.0 / t.Mass[m];
  amr_tables(t);
  return true;
}

}  // namespace dgmhd
