// Host-side reference-element tables of the DG scheme (built once per handle).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace dgmhd {

enum { GLM = 0, POWELL = 1 };

inline int nmodes_scalar(int D, int d) {
  if (d < 0) return 0;
  return D == 2 ? (d + 1) * (d + 2) / 2 : (d + 1) * (d + 2) * (d + 3) / 6;
}
inline int ndiv(int D, int d) { return D * nmodes_scalar(D, d) - nmodes_scalar(D, d - 1); }

// Reference-element data.  Point orderings: volume q = q0 + P (q1 + P q2);
// face of axis a: tangential axes b0 < b1 in increasing order, r = r0 + P r1.
// Face side index s: 0 is the face at xi_a = -1, 1 the face at xi_a = +1.
struct Tables {
  int D = 0, d = 0, divb = 0, P = 0, N = 0, Q = 0, FP = 0;
  int NV = 0, NLEG = 0, NLDF = 0, NMODES = 0, NPROJ = 0;
  std::vector<int> leg_var;            // [NLEG] conserved variable of each Legendre block
  std::vector<int> expo;               // [N][3] exponents of the Legendre modes
  std::vector<double> xg, wg;          // 1-D Gauss-Legendre rule, P points
  std::vector<double> V;               // [Q][N]         P_l(xi_q)
  std::vector<double> GW;              // [D][Q][N]      w_q dP_l/dxi_a (xi_q)
  std::vector<double> TF;              // [D][2][FP][N]  P_l at face points
  std::vector<double> LF;              // [D][2][FP][N]  w_r P_l at face points
  std::vector<double> TFS;             // [D][2][1+2^(D-1)][FP][N]  P_l at (sub-)face points; sub+1
  std::vector<double> LFS;             // [D][2][1+2^(D-1)][FP][N]  w_r P_l, times 2^-(D-1) on quarters
  std::vector<double> Minv;            // [NMODES]
  std::vector<double> Mass;            // [NMODES]
  // locally divergence-free basis (Powell)
  std::vector<int> ldf_deg;            // [NLDF]
  std::vector<double> PV;              // [D(c)][Q][NLDF]
  std::vector<double> PGW;             // [D(a)][D(c)][Q][NLDF]  w_q dPhi_c/dxi_a
  std::vector<double> PTF;             // [D(a)][2][D(c)][FP][NLDF]
  std::vector<double> PLF;             // [D(a)][2][D(c)][FP][NLDF]  w_r Phi_c
  std::vector<double> Pmean;           // [D(c)][NLDF] cell average of Phi_c
  std::vector<double> Plin;            // [D(c)][D(b)][NLDF] <Phi_c, xi_b>/<xi_b, xi_b>
  // (d+3)-point projection rule
  std::vector<double> xproj;           // [NPROJ][D]
  std::vector<double> VPW;             // [NPROJ][N]         w_p P_l(xi_p)
  std::vector<double> PVPW;            // [D(c)][NPROJ][NLDF] w_p Phi_c(xi_p)
  std::vector<double> wproj;           // [NPROJ] weights of the rule (sum 2^D)
  // dynamic refinement (Sec. 4.4), Legendre basis
  std::vector<double> SQ;              // [D][N][N] smoothness quadratic forms: S_a(u) = w^T SQ_a w
  std::vector<double> PRO;             // [2^D][N][N] child o weights = PRO_o . parent weights
  std::vector<double> RES;             // [2^D][N][N] parent weights = sum_o RES_o . child o weights
  std::vector<double> VP;              // [NPROJ][N]         P_l(xi_p)
  std::vector<double> PVP;             // [D(c)][NPROJ][NLDF] Phi_c(xi_p)
};

// Gauss-Legendre nodes (ascending) and weights on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// Build all tables; returns false with a message on failure.
bool build_tables(int D, int d, int divb, Tables& t, std::string& err);

}  // namespace dgmhd
