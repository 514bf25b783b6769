// Pointwise ideal-MHD physics on the device: equation of state, analytic flux
// (eq. mhd-flux), signal speed (eq. cfl), face normal field
// (eq. bxface-average-alfven), HLLD (Miyoshi & Kusano 2005) and the GLM
// upwind fluxes (Sec. 4.1.5).  T is the arithmetic type of the path; the
// thermal pressure is always recovered from the total energy in FP64.
#pragma once
#include <hip/hip_runtime.h>

namespace dgmhd {

enum { V_RHO = 0, V_M1 = 1, V_E = 4, V_B1 = 5, V_PSI = 8 };

// p = (gamma-1)(E - m^2/(2 rho) - B^2/2), evaluated in FP64.
template <typename T>
__device__ __forceinline__ double pressure64(const T* u, double gamma) {
  double r = (double)u[0];
  double m2 = (double)u[1] * (double)u[1] + (double)u[2] * (double)u[2] + (double)u[3] * (double)u[3];
  double b2 = (double)u[5] * (double)u[5] + (double)u[6] * (double)u[6] + (double)u[7] * (double)u[7];
  return (gamma - 1.0) * ((double)u[4] - 0.5 * m2 / r - 0.5 * b2);
}

// The same with 1/rho given in FP64 (a product instead of a division).
template <typename T>
__device__ __forceinline__ double pressure64_ir(const T* u, double gamma, double ir) {
  double m2 = (double)u[1] * (double)u[1] + (double)u[2] * (double)u[2] + (double)u[3] * (double)u[3];
  double b2 = (double)u[5] * (double)u[5] + (double)u[6] * (double)u[6] + (double)u[7] * (double)u[7];
  return (gamma - 1.0) * ((double)u[4] - 0.5 * m2 * ir - 0.5 * b2);
}

// Reciprocal used by the flux and Riemann-solver arithmetic: the hardware
// estimate refined by Newton steps (FP64: two steps, relative error at the
// level of the last bit; FP32: one step).  Not correctly rounded, and 1/0
// gives NaN rather than inf (both mark a broken state).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  r = fmaf(fmaf(-x, r, 1.0f), r, r);
  return r;
}

// 1/sqrt(x) the same way: the hardware estimate and Newton steps
// r <- r (3/2 - x r^2 / 2) (FP64: two, FP32: one).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = fma(r, fma(-h * r, r, 0.5), r);
  r = fma(r, fma(-h * r, r, 0.5), r);
  return r;
}
__device__ __forceinline__ float rsqrt_nr(float x) {
  float r = __builtin_amdgcn_rsqf(x);
  r = fmaf(r, fmaf(-0.5f * x * r, r, 0.5f), r);
  return r;
}

// sqrt(x) as x / sqrt(x) from the refined reciprocal square root: a few ulp,
// 0 at 0, NaN for x < 0 or NaN (as sqrt would).
template <typename T>
__device__ __forceinline__ T sqrt_nr(T x) {
  const T r = x * rsqrt_nr(x);
  return x == T(0) ? T(0) : r;
}

// Thermal pressure in FP64 for a state whose 1/rho the caller holds in type T:
// reused in FP64, recomputed by an FP64 division otherwise.
template <typename T>
__device__ __forceinline__ double pressure_of(const T* u, double gamma, T ir) {
  if constexpr (sizeof(T) == sizeof(double)) return pressure64_ir(u, gamma, (double)ir);
  else return pressure64(u, gamma);
}

// Analytic flux along axis a of the NV-component state u (NV = 9: GLM).
template <typename T, int NV>
__device__ __forceinline__ void mhd_flux(const T* u, int a, double gamma, T ch2, T* f) {
  const T r = u[0];
  const T ir = recip(r);
  const T v0 = u[1] * ir, v1 = u[2] * ir, v2 = u[3] * ir;
  const T b0 = u[5], b1 = u[6], b2 = u[7];
  const T p = (T)pressure_of(u, gamma, ir);
  const T pt = p + T(0.5) * (b0 * b0 + b1 * b1 + b2 * b2);
  const T vb = v0 * b0 + v1 * b1 + v2 * b2;
  const T va = a == 0 ? v0 : (a == 1 ? v1 : v2);
  const T ba = a == 0 ? b0 : (a == 1 ? b1 : b2);
  f[0] = r * va;
  f[1] = u[1] * va - b0 * ba;
  f[2] = u[2] * va - b1 * ba;
  f[3] = u[3] * va - b2 * ba;
  f[1 + a] += pt;
  f[4] = (u[4] + pt) * va - vb * ba;
  f[5] = b0 * va - v0 * ba;
  f[6] = b1 * va - v1 * ba;
  f[7] = b2 * va - v2 * ba;
  if (NV == 9) {
    f[5 + a] += u[8];
    f[8] = ch2 * ba;
  }
}

// Flux deviation f_a(ubar + du) - f_a(ubar) of a state given as a cell-mean
// reference plus a deviation, written as an exact rearrangement of
// eq. mhd-flux into products that carry a deviation factor (with
// v = vbar + dv: m_b v_a - mbar_b vbar_a = mbar_b dv_a + dm_b v_a, and so on),
// so that FP32 rounding stays relative to the deviation instead of to the
// background flux.  The thermal-pressure deviation is recovered in FP64:
//   dp = (gamma-1) (dE - (dm.v + mbar.dv)/2 - (Bbar.dB + |dB|^2/2)).
// vbar may carry rounding: dv = (dm - vbar drho)/rho keeps the rearrangement
// exact up to terms proportional to the deviation.
struct MeanRef {
  float u[9];  // conserved mean state (GLM: 9 components)
  float v[3];  // mean velocity
  float ept;   // Ebar + pbar + |Bbar|^2 / 2
  float vb;    // vbar . Bbar
  __device__ __forceinline__ void init(const float* ub, double gamma) {
    double ud[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      u[k] = ub[k];
      ud[k] = (double)ub[k];
    }
    const double ir = 1.0 / ud[0];
    double vd[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      vd[b] = ud[1 + b] * ir;
      v[b] = (float)vd[b];
    }
    const double b2 = ud[5] * ud[5] + ud[6] * ud[6] + ud[7] * ud[7];
    ept = (float)(ud[4] + pressure64_ir(ud, gamma, ir) + 0.5 * b2);
    vb = (float)(vd[0] * ud[5] + vd[1] * ud[6] + vd[2] * ud[7]);
  }
};

// Per-point quantities shared by the D axes.
struct DevPoint {
  float dv[3], v[3], B[3];
  float dpt;   // deviation of p + |B|^2/2
  float dEpt;  // deviation of E + p + |B|^2/2
  float dvB;   // deviation of v . B
};

__device__ __forceinline__ void dev_point(const MeanRef& m, const float* du, double gamma, DevPoint& q) {
  const float ir = recip(m.u[0] + du[0]);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    q.dv[b] = (du[1 + b] - m.v[b] * du[0]) * ir;
    q.v[b] = m.v[b] + q.dv[b];
    q.B[b] = m.u[5 + b] + du[5 + b];
  }
  double dke = 0.0, dme = 0.0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    dke += (double)du[1 + b] * (double)q.v[b] + (double)m.u[1 + b] * (double)q.dv[b];
    dme += (double)m.u[5 + b] * (double)du[5 + b] + 0.5 * (double)du[5 + b] * (double)du[5 + b];
  }
  const double dp = (gamma - 1.0) * ((double)du[4] - 0.5 * dke - dme);
  q.dpt = (float)(dp + dme);
  q.dEpt = du[4] + q.dpt;
  q.dvB = q.dv[0] * m.u[5] + q.dv[1] * m.u[6] + q.dv[2] * m.u[7] + q.v[0] * du[5] + q.v[1] * du[6] + q.v[2] * du[7];
}

template <int NV, int A>
__device__ __forceinline__ void mhd_dflux(const MeanRef& m, const float* du, const DevPoint& q, float ch2, float* f) {
  const float va = q.v[A], dva = q.dv[A], Ba = q.B[A], dBa = du[5 + A];
  f[0] = du[1 + A];
#pragma unroll
  for (int b = 0; b < 3; ++b) f[1 + b] = (m.u[1 + b] * dva + du[1 + b] * va) - (du[5 + b] * Ba + m.u[5 + b] * dBa);
  f[1 + A] += q.dpt;
  f[4] = (q.dEpt * va + m.ept * dva) - (q.dvB * Ba + m.vb * dBa);
#pragma unroll
  for (int b = 0; b < 3; ++b)
    f[5 + b] = b == A ? 0.0f : (du[5 + b] * va + m.u[5 + b] * dva) - (q.dv[b] * Ba + m.v[b] * dBa);
  if (NV == 9) {
    f[5 + A] = du[8];
    f[8] = ch2 * dBa;
  }
}

// sum_a (|v_a| + c), c = sqrt(gamma p / rho + B^2 / rho), over the first D
// axes; max(p, 0) in the sound speed and no contribution where rho <= 0 (a
// state that the positivity limiter has not seen yet).
template <typename T, int D>
__device__ __forceinline__ double signal_sum(const T* u, double gamma) {
  double r = (double)u[0];
  if (!(r > 0.0)) return (r == r) ? 0.0 : r;
  const double ir = recip(r);
  double p = fmax(pressure64_ir(u, gamma, ir), 0.0);
  double b2 = (double)u[5] * (double)u[5] + (double)u[6] * (double)u[6] + (double)u[7] * (double)u[7];
  double c = sqrt((gamma * p + b2) * ir);
  double s = 0.0;
  for (int a = 0; a < D; ++a) s += fabs((double)u[1 + a]) * ir + c;
  return s;
}

// HLLD in the face frame.  wl/wr: (rho, u, v, w, p, By, Bz); bx common normal
// field.  Output flux of (rho, m_n, m_t1, m_t2, E, B_t1, B_t2) (the normal-B
// flux is zero and not returned).  st (may be null): the state of the fan
// region that contains the face, x/t = 0, as (rho, u, v, w, By, Bz).
template <typename T>
__device__ __forceinline__ void hlld_flux(const T* wl, const T* wr, T bx, double gamma, T* out, T* st = nullptr) {
  // divisions are products with reciprocals computed once (1/(gamma-1),
  // 1/rho per side, 1/den, 1/(S - S_M) per side)
  const T g = (T)gamma;
  const T igm1 = recip(g - T(1));
  T UL[7], UR[7], FL[7], FR[7], EL, ER, ptL, ptR, cfL, cfR;
  auto cf = [&](const T* W, T* U, T* F, T& E, T& pt, T& c) {
    const T rho = W[0], u = W[1], v = W[2], w = W[3], p = W[4], by = W[5], bz = W[6];
    const T irho = recip(rho);
    const T bb = bx * bx + by * by + bz * bz;
    E = p * igm1 + T(0.5) * rho * (u * u + v * v + w * w) + T(0.5) * bb;
    pt = p + T(0.5) * bb;
    const T vb = u * bx + v * by + w * bz;
    U[0] = rho; U[1] = rho * u; U[2] = rho * v; U[3] = rho * w; U[4] = E; U[5] = by; U[6] = bz;
    F[0] = rho * u;
    F[1] = rho * u * u + pt - bx * bx;
    F[2] = rho * v * u - bx * by;
    F[3] = rho * w * u - bx * bz;
    F[4] = (E + pt) * u - vb * bx;
    F[5] = by * u - v * bx;
    F[6] = bz * u - w * bx;
    const T gp = g * p;
    const T s = (gp + bb) * irho;
    T disc = s * s - T(4) * gp * bx * bx * (irho * irho);
    disc = disc > T(0) ? disc : T(0);
    c = sqrt_nr(T(0.5) * (s + sqrt_nr(disc)));
  };
  cf(wl, UL, FL, EL, ptL, cfL);
  cf(wr, UR, FR, ER, ptR, cfR);
  const T uL = wl[1], uR = wr[1], rL = wl[0], rR = wr[0];
  const T cmax = cfL > cfR ? cfL : cfR;
  const T SL = (uL < uR ? uL : uR) - cmax;
  const T SR = (uL > uR ? uL : uR) + cmax;
  auto state = [&](T r, T u, T v, T w, T by, T bz) {
    if (st) { st[0] = r; st[1] = u; st[2] = v; st[3] = w; st[4] = by; st[5] = bz; }
  };
  if (SL > T(0)) {
    for (int k = 0; k < 7; ++k) out[k] = FL[k];
    state(wl[0], wl[1], wl[2], wl[3], wl[5], wl[6]);
    return;
  }
  if (SR <= T(0)) {
    for (int k = 0; k < 7; ++k) out[k] = FR[k];
    state(wr[0], wr[1], wr[2], wr[3], wr[5], wr[6]);
    return;
  }
  const T dL = (SL - uL) * rL, dR = (SR - uR) * rR;
  const T iden = recip(dR - dL);
  const T SM = (dR * uR - dL * uL - ptR + ptL) * iden;
  const T ptS = (dR * ptL - dL * ptR + rL * rR * (SR - uR) * (SL - uL) * (uR - uL)) * iden;
  // outer star states
  T Us[2][7], rs[2], vs[2], ws[2], bys[2], bzs[2], Es[2], vbs[2];
  for (int side = 0; side < 2; ++side) {
    const T* W = side ? wr : wl;
    const T* U = side ? UR : UL;
    const T S = side ? SR : SL;
    const T d = side ? dR : dL;
    const T E = side ? ER : EL, pt = side ? ptR : ptL;
    const T rho = W[0], u = W[1], v = W[2], w = W[3], by = W[5], bz = W[6];
    const T isd = recip(S - SM);
    const T r_s = d * isd;
    const T dd = d * (S - SM) - bx * bx;
    const T sc = rho * (S - u) * (S - u);
    const T thr = T(1e-12) * (sc > bx * bx ? sc : bx * bx);
    T v_s, w_s, by_s, bz_s;
    if (fabs(dd) <= thr) {
      v_s = v; w_s = w; by_s = by; bz_s = bz;
    } else {
      const T idd = recip(dd);
      v_s = v - bx * by * (SM - u) * idd;
      w_s = w - bx * bz * (SM - u) * idd;
      const T fac = (d * (S - u) - bx * bx) * idd;
      by_s = by * fac;
      bz_s = bz * fac;
    }
    const T vb = u * bx + v * by + w * bz;
    const T vb_s = SM * bx + v_s * by_s + w_s * bz_s;
    const T E_s = ((S - u) * E - pt * u + ptS * SM + bx * (vb - vb_s)) * isd;
    rs[side] = r_s; vs[side] = v_s; ws[side] = w_s; bys[side] = by_s; bzs[side] = bz_s;
    Es[side] = E_s; vbs[side] = vb_s;
    Us[side][0] = r_s; Us[side][1] = r_s * SM; Us[side][2] = r_s * v_s; Us[side][3] = r_s * w_s;
    Us[side][4] = E_s; Us[side][5] = by_s; Us[side][6] = bz_s;
    (void)U;
  }
  const T iqL = rsqrt_nr(rs[0]), iqR = rsqrt_nr(rs[1]);  // 1/sqrt(rho*) per side
  const T sqL = rs[0] * iqL, sqR = rs[1] * iqR;
  const T SsL = SM - fabs(bx) * iqL, SsR = SM + fabs(bx) * iqR;
  if (SsL > T(0)) {
    for (int k = 0; k < 7; ++k) out[k] = FL[k] + SL * (Us[0][k] - UL[k]);
    state(rs[0], SM, vs[0], ws[0], bys[0], bzs[0]);
    return;
  }
  if (SsR <= T(0)) {
    for (int k = 0; k < 7; ++k) out[k] = FR[k] + SR * (Us[1][k] - UR[k]);
    state(rs[1], SM, vs[1], ws[1], bys[1], bzs[1]);
    return;
  }
  const T s = bx >= T(0) ? T(1) : T(-1);
  const T isum = recip(sqL + sqR);
  const T vss = (sqL * vs[0] + sqR * vs[1] + (bys[1] - bys[0]) * s) * isum;
  const T wss = (sqL * ws[0] + sqR * ws[1] + (bzs[1] - bzs[0]) * s) * isum;
  const T byss = (sqL * bys[1] + sqR * bys[0] + sqL * sqR * (vs[1] - vs[0]) * s) * isum;
  const T bzss = (sqL * bzs[1] + sqR * bzs[0] + sqL * sqR * (ws[1] - ws[0]) * s) * isum;
  const T vbss = SM * bx + vss * byss + wss * bzss;
  if (SM > T(0)) {
    const T Ess = Es[0] - sqL * (vbs[0] - vbss) * s;
    const T Uss[7] = {rs[0], rs[0] * SM, rs[0] * vss, rs[0] * wss, Ess, byss, bzss};
    for (int k = 0; k < 7; ++k) out[k] = FL[k] + SL * (Us[0][k] - UL[k]) + SsL * (Uss[k] - Us[0][k]);
    state(rs[0], SM, vss, wss, byss, bzss);
  } else {
    const T Ess = Es[1] + sqR * (vbs[1] - vbss) * s;
    const T Uss[7] = {rs[1], rs[1] * SM, rs[1] * vss, rs[1] * wss, Ess, byss, bzss};
    for (int k = 0; k < 7; ++k) out[k] = FR[k] + SR * (Us[1][k] - UR[k]) + SsR * (Uss[k] - Us[1][k]);
    state(rs[1], SM, vss, wss, byss, bzss);
  }
}

// Numerical flux through a face with normal +e_a between traces uL and uR
// (global components).  Writes F (NV components) and returns B^n_F.  vf, bf
// (may be null): velocity and magnetic field of the HLLD interface state
// (global components; its normal field is B^n_F).
template <typename T, int NV, int A>
__device__ __forceinline__ T face_flux_a(const T* uL, const T* uR, double gamma, T ch, T* F, T* vf = nullptr,
                                         T* bf = nullptr) {
  constexpr int n = A, t1 = (A + 1) % 3, t2 = (A + 2) % 3;
  T wl[7], wr[7];
  {
    const T ir = recip(uL[0]);
    wl[0] = uL[0]; wl[1] = uL[1 + n] * ir; wl[2] = uL[1 + t1] * ir; wl[3] = uL[1 + t2] * ir;
    wl[4] = (T)pressure_of(uL, gamma, ir); wl[5] = uL[5 + t1]; wl[6] = uL[5 + t2];
  }
  {
    const T ir = recip(uR[0]);
    wr[0] = uR[0]; wr[1] = uR[1 + n] * ir; wr[2] = uR[1 + t1] * ir; wr[3] = uR[1 + t2] * ir;
    wr[4] = (T)pressure_of(uR, gamma, ir); wr[5] = uR[5 + t1]; wr[6] = uR[5 + t2];
  }
  const T bnL = uL[5 + n], bnR = uR[5 + n];
  const T iL = rsqrt_nr(uL[0]), iR = rsqrt_nr(uR[0]);
  const T bnF = (bnL * iL + bnR * iR) * recip(iL + iR);
  T fn[7], st[6];
  hlld_flux<T>(wl, wr, bnF, gamma, fn, vf ? st : nullptr);
  if (vf) {
    vf[n] = st[1]; vf[t1] = st[2]; vf[t2] = st[3];
    bf[n] = bnF; bf[t1] = st[4]; bf[t2] = st[5];
  }
  F[0] = fn[0];
  F[1 + n] = fn[1]; F[1 + t1] = fn[2]; F[1 + t2] = fn[3];
  F[4] = fn[4];
  F[5 + n] = T(0); F[5 + t1] = fn[5]; F[5 + t2] = fn[6];
  if (NV == 9) {
    const T psL = uL[8], psR = uR[8];
    const T bn_s = T(0.5) * (bnL + bnR) - (psR - psL) * recip(T(2) * ch);
    const T ps_s = T(0.5) * (psL + psR) - T(0.5) * ch * (bnR - bnL);
    F[5 + n] = ps_s;
    F[8] = ch * ch * bn_s;
  }
  return bnF;
}

// The same with a run-time axis (one branch per axis, so that every component
// index inside is a compile-time constant).
template <typename T, int NV>
__device__ __forceinline__ T face_flux(const T* uL, const T* uR, int a, double gamma, T ch, T* F, T* vf = nullptr,
                                       T* bf = nullptr) {
  if (a == 0) return face_flux_a<T, NV, 0>(uL, uR, gamma, ch, F, vf, bf);
  if (a == 1) return face_flux_a<T, NV, 1>(uL, uR, gamma, ch, F, vf, bf);
  return face_flux_a<T, NV, 2>(uL, uR, gamma, ch, F, vf, bf);
}

// q-dagger of eq. powellq-interp for the side whose trace is u (conserved):
// q integrated along the straight path in primitive variables from the
// trace (v_s, B_s) to the interface state (v_F, B_F):
// (0, (B_s + B_F)/2, (2 B_s.v_s + B_s.v_F + B_F.v_s + 2 B_F.v_F)/6, (v_s + v_F)/2).
template <typename T>
__device__ __forceinline__ void powell_q_interp(const T* u, const T* vf, const T* bf, T* q) {
  const T ir = recip(u[0]);
  const T vs[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
  const T bs[3] = {u[5], u[6], u[7]};
  q[0] = T(0);
  T ss = 0, sf = 0, fs = 0, ff_ = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    q[1 + c] = T(0.5) * (bs[c] + bf[c]);
    q[5 + c] = T(0.5) * (vs[c] + vf[c]);
    ss += bs[c] * vs[c];
    sf += bs[c] * vf[c];
    fs += bf[c] * vs[c];
    ff_ += bf[c] * vf[c];
  }
  q[4] = (T(2) * ss + sf + fs + T(2) * ff_) * T(1.0 / 6.0);
}

}  // namespace dgmhd
