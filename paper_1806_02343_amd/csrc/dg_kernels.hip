// gfx950 kernels of the DG right-hand side, stage update, time-step
// reductions and initial projection.
//
// State arrays are SoA: w[mode][cell] with cells fastest, so a wavefront of
// consecutive cells reads each mode row with one coalesced access.
//
// Face kernel (one thread per (axis, face point, face); consecutive threads
// take consecutive faces of the same point, so both traces are coalesced
// reads): traces from both cells, face normal field, HLLD, GLM fluxes; the
// face fluxes go to a face buffer ff[axis][var][point][face] and, for Powell,
// the normal-field jumps to jp[axis][side][point][face].
//
// Cell kernel (one block per tile of TC consecutive cells): the tile's modes
// are staged in LDS; quadrature points are processed in chunks of NT/TC
// points: every thread evaluates one (cell, point) state and its D analytic
// fluxes into LDS, then every thread accumulates its (mode, cell) outputs of
// the volume integral.  The surface integral gathers the 2D face fluxes of
// the cell from the face buffer (owner gather, no atomics, deterministic);
// Powell face terms, GLM damping, the inverse mass and the SSP-RK stage
// combination are fused before the single store.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <type_traits>
#include <vector>

#include "dg_kernels.h"
#include "dg_physics.h"

// The file is compiled as four objects in parallel, one per (precision,
// divergence scheme): DG_PART 0 = FP64 GLM, 1 = FP64 Powell, 2 = FP32 GLM,
// 3 = FP32 Powell.  Part 0 also holds the scalar kernels and host helpers
// shared by all parts and the launcher factory.  Without DG_PART everything
// is built into one object.
#ifndef DG_PART
#define DG_PART -1
#endif
#define DG_SHARED (DG_PART <= 0)

namespace dgmhd {

template <int D, int DEG, int DIVB>
struct Cfg {
  static constexpr int P = DEG + 1;
  static constexpr int N = D == 2 ? (DEG + 1) * (DEG + 2) / 2 : (DEG + 1) * (DEG + 2) * (DEG + 3) / 6;
  static constexpr int NM1 = D == 2 ? DEG * (DEG + 1) / 2 : DEG * (DEG + 1) * (DEG + 2) / 6;
  static constexpr int Q = D == 2 ? P * P : P * P * P;
  static constexpr int FP = D == 2 ? P : P * P;
  // face moments: polynomials of degree <= DEG in the face coordinates
  static constexpr int FM = D == 2 ? P : P * (P + 1) / 2;
  static constexpr int NV = DIVB == GLM ? 9 : 8;
  static constexpr int NLEG = DIVB == GLM ? 9 : (D == 3 ? 5 : 6);
  static constexpr int NLDF = DIVB == GLM ? 0 : D * N - NM1;
  static constexpr int NMODES = NLEG * N + NLDF;
  // conserved variable of Legendre block j
  __host__ __device__ static constexpr int legvar(int j) { return (DIVB == POWELL && j == 5) ? 7 : j; }
};

template <typename T, int D, int DEG, int DIVB>
struct Tile {
  using C = Cfg<D, DEG, DIVB>;
  static constexpr int NT = (sizeof(T) == 8 && D == 3) ? 128 : 256;
  static constexpr int SF = D * C::NV * NT * (int)sizeof(T);
  static constexpr int fit(int tc) { return C::NMODES * tc * (int)sizeof(T) + SF <= 60 * 1024; }
  static constexpr int TC = fit(64) ? 64 : fit(32) ? 32 : fit(16) ? 16 : fit(8) ? 8 : fit(4) ? 4 : fit(2) ? 2 : 1;
  static constexpr int QCH = NT / TC;
};

template <typename T>
struct DevTab {
  const T *V, *GW, *TF, *LF, *Minv, *PV, *PGW, *PTF, *PLF, *Pmean, *Plin, *TFS, *LFS;
};

__device__ __forceinline__ double cell_h(const Grid& g, int64_t K) {
  return g.level ? g.hbase / (double)(1 << g.level[K]) : g.h;
}

// Periodic face neighbour of cell K along axis a (s = +1 or -1) on a uniform
// grid; cell indices fit 32 bits (dg_init rejects larger grids), so the index
// arithmetic is unsigned 32-bit.
__device__ __forceinline__ int64_t nbr(int64_t K, int a, int s, const Grid& g) {
  const uint32_t n0 = (uint32_t)g.n0, n1 = (uint32_t)g.n1, n2 = (uint32_t)g.n2;
  const uint32_t k32 = (uint32_t)K;
  uint32_t i = k32 % n0;
  const uint32_t t = k32 / n0;
  uint32_t j = t % n1;
  uint32_t k = t / n1;
  if (a == 0) i = s > 0 ? (i + 1 == n0 ? 0u : i + 1) : (i == 0 ? n0 - 1 : i - 1);
  else if (a == 1) j = s > 0 ? (j + 1 == n1 ? 0u : j + 1) : (j == 0 ? n1 - 1 : j - 1);
  else k = s > 0 ? (k + 1 == n2 ? 0u : k + 1) : (k == 0 ? n2 - 1 : k - 1);
  return (int64_t)i + (int64_t)n0 * ((int64_t)j + (int64_t)n1 * k);
}

// XCD-aware block order.  Workgroups are dealt round-robin to the 8 XCDs
// (each with its own L2); this maps launch block b to a logical tile so that
// every XCD walks one contiguous 1/8 of the tiles in order, and a cell's
// +y neighbour rows (and the fluxes written for them) are read on the XCD
// whose L2 already holds them.  A bijection on [0, nb).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  constexpr uint32_t NX = 8;
  const uint32_t q = nb / NX, r = nb % NX, x = b % NX, i = b / NX;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ void atomic_max_pos(unsigned long long* addr, double v) {
  // non-negative doubles order like their bit patterns; NaN is mapped above +inf
  unsigned long long b = __double_as_longlong(v);
  if (!(v == v)) b = 0x7ff8000000000000ULL;
  atomicMax(addr, b);
}

// ---------------------------------------------------------------------------
// face kernel

template <typename T, int D, int DEG, int DIVB>
__device__ __forceinline__ T safe_mode_value(int m) {
  using C = Cfg<D, DEG, DIVB>;
  return (m == 0 || m == 4 * C::N) ? T(1) : T(0);
}

// Face tile: TF consecutive faces of one axis (left cells f0 .. f0+TF-1) per
// block; the modes of the TF left and TF right cells are staged in LDS with
// coalesced loads, then each thread evaluates one (face, point) pair.
template <typename T, int D, int DEG, int DIVB>
struct FaceTile {
  using C = Cfg<D, DEG, DIVB>;
  static constexpr int R = 256 / C::FP;
  static constexpr int TF = R >= 64 ? 64 : R >= 32 ? 32 : R >= 16 ? 16 : 8;
  static constexpr int NT = TF * C::FP;
};

template <typename T, int D, int DEG, int DIVB>
__global__ void __launch_bounds__((FaceTile<T, D, DEG, DIVB>::NT))
    k_face(const T* __restrict__ w, T* __restrict__ ff, T* __restrict__ jp, DevTab<T> tb, Grid g,
           const Scal* __restrict__ sc, double gamma, int qint) {
  using C = Cfg<D, DEG, DIVB>;
  constexpr int TF = FaceTile<T, D, DEG, DIVB>::TF, NT = FaceTile<T, D, DEG, DIVB>::NT;
  constexpr int NM = C::NMODES, N = C::N;
  __shared__ T sL[NM * TF];
  __shared__ T sR[NM * TF];
  const int a = blockIdx.y;
  const int64_t f0 = (int64_t)blockIdx.x * TF;
  const int tid = threadIdx.x;
  const int64_t ld = g.ld;
  for (int i = tid; i < NM * TF; i += NT) {
    const int m = i / TF, fl = i % TF;
    const int64_t F = f0 + fl;
    if (F < g.C) {
      sL[i] = w[(int64_t)m * ld + F];
      sR[i] = w[(int64_t)m * ld + nbr(F, a, +1, g)];
    } else {
      sL[i] = safe_mode_value<T, D, DEG, DIVB>(m);
      sR[i] = safe_mode_value<T, D, DEG, DIVB>(m);
    }
  }
  __syncthreads();
  const int fl = tid % TF, r = tid / TF;
  const int64_t f = f0 + fl;
  if (f >= g.C) return;
  T uL[9], uR[9];
  const T* tl = tb.TF + ((a * 2 + 1) * C::FP + r) * N;
  const T* tr = tb.TF + ((a * 2 + 0) * C::FP + r) * N;
  T rowL[N], rowR[N];
#pragma unroll
  for (int l = 0; l < N; ++l) { rowL[l] = tl[l]; rowR[l] = tr[l]; }
#pragma unroll
  for (int j = 0; j < C::NLEG; ++j) {
    T sLv = 0, sRv = 0;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      sLv += rowL[l] * sL[(j * N + l) * TF + fl];
      sRv += rowR[l] * sR[(j * N + l) * TF + fl];
    }
    uL[C::legvar(j)] = sLv;
    uR[C::legvar(j)] = sRv;
  }
  if constexpr (C::NLDF > 0) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const T* pl = tb.PTF + (((a * 2 + 1) * D + c) * C::FP + r) * C::NLDF;
      const T* pr = tb.PTF + (((a * 2 + 0) * D + c) * C::FP + r) * C::NLDF;
      T sLv = 0, sRv = 0;
      for (int l = 0; l < C::NLDF; ++l) {
        sLv += pl[l] * sL[(C::NLEG * N + l) * TF + fl];
        sRv += pr[l] * sR[(C::NLEG * N + l) * TF + fl];
      }
      uL[5 + c] = sLv;
      uR[5 + c] = sRv;
    }
  }
  T F[9];
  if constexpr (DIVB == POWELL) {
    if (qint) {
      // interpolated q-dagger (eq. powellq-interp) with the HLLD interface
      // state: the Powell term of each side is added here, the left cell's
      // face values to ff, the right cell's to jp (same layout as ff)
      T vf[3], bf[3], ql[8], qr[8];
      const T bnF = face_flux<T, C::NV>(uL, uR, a, gamma, (T)sc->ch, F, vf, bf);
      powell_q_interp<T>(uL, vf, bf, ql);
      powell_q_interp<T>(uR, vf, bf, qr);
      const T jl = bnF - uL[5 + a], jr = uR[5 + a] - bnF;
#pragma unroll
      for (int v = 0; v < C::NV; ++v) {
        ff[((int64_t)(a * C::NV + v) * C::FP + r) * ld + f] = F[v] + ql[v] * jl;
        jp[((int64_t)(a * C::NV + v) * C::FP + r) * ld + f] = F[v] - qr[v] * jr;
      }
      return;
    }
  }
  const T bnF = face_flux<T, C::NV>(uL, uR, a, gamma, (T)sc->ch, F);
#pragma unroll
  for (int v = 0; v < C::NV; ++v) ff[((int64_t)(a * C::NV + v) * C::FP + r) * ld + f] = F[v];
  if constexpr (DIVB == POWELL) {
    jp[((int64_t)(a * 2 + 0) * C::FP + r) * ld + f] = bnF - uL[5 + a];
    jp[((int64_t)(a * 2 + 1) * C::FP + r) * ld + f] = uR[5 + a] - bnF;
  }
}

// Face kernel on octree meshes: one thread per (face, point) over the face
// list (sorted by axis); a coarse side evaluates its trace at the points of
// its quarter of the face (L2 prolongation of the coarse trace).
template <typename T, int D, int DEG>
__global__ void __launch_bounds__(256) k_face_amr(const T* __restrict__ w, T* __restrict__ ffa, DevTab<T> tb,
                                                  Grid g, const Scal* __restrict__ sc, double gamma) {
  using C = Cfg<D, DEG, GLM>;
  constexpr int N = C::N, NSUB = 1 + (1 << (D - 1));
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)C::FP * g.NF) return;
  const int64_t f = gid % g.NF;
  const int r = (int)(gid / g.NF);
  int a = 0;
  if (D == 3 && f >= g.face0[2]) a = 2;
  else if (f >= g.face0[1]) a = 1;
  const int64_t L = g.faceL[f], R = g.faceR[f];
  const int sl = g.subL[f] + 1, sr = g.subR[f] + 1;
  const int64_t ld = g.ld;
  const T* tl = tb.TFS + (((a * 2 + 1) * NSUB + sl) * C::FP + r) * N;
  const T* tr = tb.TFS + (((a * 2 + 0) * NSUB + sr) * C::FP + r) * N;
  T uL[9], uR[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    T sLv = 0, sRv = 0;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      sLv += tl[l] * w[(int64_t)(j * N + l) * ld + L];
      sRv += tr[l] * w[(int64_t)(j * N + l) * ld + R];
    }
    uL[j] = sLv;
    uR[j] = sRv;
  }
  T F[9];
  (void)face_flux<T, 9>(uL, uR, a, gamma, (T)sc->ch, F);
#pragma unroll
  for (int v = 0; v < 9; ++v) ffa[((int64_t)v * C::FP + r) * g.ldf + f] = F[v];
}

// ---------------------------------------------------------------------------
// cell kernel


// Tile shape of the cell kernel: TC cells per block, NT threads.  The flux
// phase gives every thread one (cell, point) pair of a chunk of QCH = NT/TC
// points; the contraction phases give every thread IPT items, an item being
// one (Legendre variable or LDF chunk, cell) with N register accumulators.
template <typename T, int D, int DEG, int DIVB, int TC, int NT>
struct CellTile {
  using C = Cfg<D, DEG, DIVB>;
  static constexpr int QCH = NT / TC;
  static constexpr int NLC = C::NLDF ? (C::NLDF + C::N - 1) / C::N : 0;  // LDF chunks of N modes
  static constexpr int NBLK = C::NLEG + NLC;
  static constexpr int NITEM = NBLK * TC;
  static constexpr int IPT = (NITEM + NT - 1) / NT;
  static constexpr int LDS = (C::NMODES * TC + D * C::NV * QCH * TC) * (int)sizeof(T);
  static constexpr bool valid = (NT % TC == 0) && (QCH >= 1) && (LDS <= 160 * 1024) && (IPT <= 4);
};

template <typename T, int D, int DEG, int DIVB, int TC, int NT, int AMR>
__global__ void __launch_bounds__(NT)
    k_cell(const T* w, const T* w0, T* out, const T* __restrict__ ff, const T* __restrict__ jp,
           const T* __restrict__ tV, const T* __restrict__ tGW, const T* __restrict__ tLF,
           const T* __restrict__ tMinv, const T* __restrict__ tPV, const T* __restrict__ tPGW,
           const T* __restrict__ tPLF, const T* __restrict__ tPmean, const T* __restrict__ tLFS, Grid g,
           const Scal* __restrict__ sc, double gamma, double a0, double b0, double cdt, int mode) {
  using C = Cfg<D, DEG, DIVB>;
  using CT = CellTile<T, D, DEG, DIVB, TC, NT>;
  // tables as restrict-qualified arguments: wave-uniform reads become scalar loads
  struct {
    const T *V, *GW, *LF, *Minv, *PV, *PGW, *PLF, *Pmean;
  } tb = {tV, tGW, tLF, tMinv, tPV, tPGW, tPLF, tPmean};
  constexpr int N = C::N, QCH = CT::QCH, IPT = CT::IPT, NITEM = CT::NITEM;
  constexpr int NM = C::NMODES;
  __shared__ T sw[NM * TC];
  __shared__ T sf[D * C::NV * QCH * TC];
  const int64_t c0 = (int64_t)blockIdx.x * TC;
  const int tid = threadIdx.x;
  const int64_t ld = g.ld;
  for (int i = tid; i < NM * TC; i += NT) {
    const int m = i / TC, c = i % TC;
    const int64_t K = c0 + c;
    sw[i] = K < g.C ? w[(int64_t)m * ld + K] : safe_mode_value<T, D, DEG, DIVB>(m);
  }
  const T ch = (T)sc->ch;
  const T ch2 = ch * ch;
  T acc[IPT][N];
#pragma unroll
  for (int k = 0; k < IPT; ++k)
#pragma unroll
    for (int l = 0; l < N; ++l) acc[k][l] = 0;

  for (int qb = 0; qb < C::Q; qb += QCH) {
    __syncthreads();
    {
      const int c = tid % TC, qq = tid / TC, q = qb + qq;
      if (q < C::Q) {
        T u[9];
        T vrow[N];
#pragma unroll
        for (int l = 0; l < N; ++l) vrow[l] = tb.V[q * N + l];
#pragma unroll
        for (int j = 0; j < C::NLEG; ++j) {
          T s = 0;
#pragma unroll
          for (int l = 0; l < N; ++l) s += vrow[l] * sw[(j * N + l) * TC + c];
          u[C::legvar(j)] = s;
        }
        if constexpr (C::NLDF > 0) {
#pragma unroll
          for (int cc = 0; cc < D; ++cc) {
            T s = 0;
            for (int l = 0; l < C::NLDF; ++l) s += tb.PV[(cc * C::Q + q) * C::NLDF + l] * sw[(C::NLEG * N + l) * TC + c];
            u[5 + cc] = s;
          }
        }
#pragma unroll
        for (int a = 0; a < D; ++a) {
          T f[9];
          mhd_flux<T, C::NV>(u, a, gamma, ch2, f);
#pragma unroll
          for (int v = 0; v < C::NV; ++v) sf[((a * C::NV + v) * QCH + qq) * TC + c] = f[v];
        }
      }
    }
    __syncthreads();
    const int qmax = (C::Q - qb) < QCH ? (C::Q - qb) : QCH;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const int it = tid + k * NT;
      if (it >= NITEM) continue;
      const int blk = it / TC, c = it % TC;
      if (blk < C::NLEG) {
        const int v = C::legvar(blk);
        for (int a = 0; a < D; ++a)
          for (int qq = 0; qq < qmax; ++qq) {
            const T f = sf[((a * C::NV + v) * QCH + qq) * TC + c];
            const T* gw = tb.GW + (a * C::Q + qb + qq) * N;
#pragma unroll
            for (int l = 0; l < N; ++l) acc[k][l] += gw[l] * f;
          }
      } else if constexpr (C::NLDF > 0) {
        const int h = blk - C::NLEG;
        for (int a = 0; a < D; ++a)
          for (int cc = 0; cc < D; ++cc)
            for (int qq = 0; qq < qmax; ++qq) {
              const T f = sf[((a * C::NV + 5 + cc) * QCH + qq) * TC + c];
              const T* pg = tb.PGW + ((a * D + cc) * C::Q + qb + qq) * C::NLDF + h * N;
#pragma unroll
              for (int i = 0; i < N; ++i)
                if (h * N + i < C::NLDF) acc[k][i] += pg[i] * f;
            }
      }
    }
  }

  const double dt = sc->dt * cdt;  // the stage's multiple of the step
  const T kappa = (T)sc->kappa;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const int it = tid + k * NT;
    if (it >= NITEM) continue;
    const int blk = it / TC, c = it % TC;
    const int64_t K = c0 + c;
    if (K >= g.C) continue;
    const T two_h = T(2.0 / cell_h(g, K));
    if constexpr (AMR) {
      // owner gather over the faces of each side (1 full face or 2^(D-1) quarters)
      constexpr int NSUB = 1 + (1 << (D - 1)), NQ = 1 << (D - 1);
      const int v = C::legvar(blk);
      for (int a = 0; a < D; ++a)
        for (int sd = 0; sd < 2; ++sd) {
          const int32_t* sl = g.slots + (((int64_t)K * D + a) * 2 + sd) * 4;
          for (int q = 0; q < NQ; ++q) {
            const int32_t f = sl[q];
            if (f < 0) break;
            const int sub = 1 + (sd ? g.subL[f] : g.subR[f]);
            const T sign = sd ? T(-1) : T(1);
            for (int r = 0; r < C::FP; ++r) {
              const T fv = sign * ff[((int64_t)v * C::FP + r) * g.ldf + f];
              const T* lf = tLFS + (((a * 2 + sd) * NSUB + sub) * C::FP + r) * N;
#pragma unroll
              for (int l = 0; l < N; ++l) acc[k][l] += lf[l] * fv;
            }
          }
        }
    }
    T qv[8];
    // interpolated q-dagger (mode bit 2): the face kernel added each side's
    // Powell term to that side's face values (left: ff, right: jp)
    const bool qint = DIVB == POWELL && (mode & 2);
    if constexpr (DIVB == POWELL) {
      // q(<u>_K) = (0, B, v.B, v) from the cell means (eq. powellq-average)
      const T rho = sw[0 * TC + c];
      T bm[3];
      for (int cc = 0; cc < D; ++cc) {
        T b = 0;
        for (int l = 0; l < C::NLDF; ++l) b += tb.Pmean[cc * C::NLDF + l] * sw[(C::NLEG * N + l) * TC + c];
        bm[cc] = b;
      }
      if (D == 2) bm[2] = sw[(5 * N) * TC + c];
      const T v0 = sw[(1 * N) * TC + c] / rho, v1 = sw[(2 * N) * TC + c] / rho, v2 = sw[(3 * N) * TC + c] / rho;
      qv[0] = 0; qv[1] = bm[0]; qv[2] = bm[1]; qv[3] = bm[2];
      qv[4] = v0 * bm[0] + v1 * bm[1] + v2 * bm[2];
      qv[5] = v0; qv[6] = v1; qv[7] = v2;
      if (qint)
        for (int v = 0; v < 8; ++v) qv[v] = T(0);
    }
    for (int a = 0; a < (AMR ? 0 : D); ++a) {
      const int64_t Km = nbr(K, a, -1, g);
      const T* jl = jp + (int64_t)(a * 2 + 0) * C::FP * ld;
      const T* jr = jp + (int64_t)(a * 2 + 1) * C::FP * ld;
      if (blk < C::NLEG) {
        const int v = C::legvar(blk);
        const T* fv = ff + (int64_t)(a * C::NV + v) * C::FP * ld;
        const T* fvm = qint ? jp + (int64_t)(a * C::NV + v) * C::FP * ld : fv;  // the -a face's values
        for (int r = 0; r < C::FP; ++r) {
          const T fp = fv[(int64_t)r * ld + K], fm = fvm[(int64_t)r * ld + Km];
          const T* lfp = tb.LF + ((a * 2 + 1) * C::FP + r) * N;
          const T* lfm = tb.LF + ((a * 2 + 0) * C::FP + r) * N;
#pragma unroll
          for (int l = 0; l < N; ++l) acc[k][l] += lfm[l] * fm - lfp[l] * fp;
          if constexpr (DIVB == POWELL) {
            if (!qint) {
              const T ql = qv[v] * jl[(int64_t)r * ld + K], qr = qv[v] * jr[(int64_t)r * ld + Km];
#pragma unroll
              for (int l = 0; l < N; ++l) acc[k][l] -= lfp[l] * ql + lfm[l] * qr;
            }
          }
        }
      } else if constexpr (C::NLDF > 0) {
        const int h = blk - C::NLEG;
        for (int cc = 0; cc < D; ++cc) {
          const T* fv = ff + (int64_t)(a * C::NV + 5 + cc) * C::FP * ld;
          const T* fvm = qint ? jp + (int64_t)(a * C::NV + 5 + cc) * C::FP * ld : fv;
          for (int r = 0; r < C::FP; ++r) {
            const T fp = fv[(int64_t)r * ld + K], fm = fvm[(int64_t)r * ld + Km];
            const T* pp = tb.PLF + (((a * 2 + 1) * D + cc) * C::FP + r) * C::NLDF + h * N;
            const T* pm = tb.PLF + (((a * 2 + 0) * D + cc) * C::FP + r) * C::NLDF + h * N;
            const T ql = qint ? T(0) : qv[5 + cc] * jl[(int64_t)r * ld + K];
            const T qr = qint ? T(0) : qv[5 + cc] * jr[(int64_t)r * ld + Km];
#pragma unroll
            for (int i = 0; i < N; ++i)
              if (h * N + i < C::NLDF) acc[k][i] += pm[i] * fm - pp[i] * fp - (pp[i] * ql + pm[i] * qr);
          }
        }
      }
    }
    // w0 may alias out (the last stage updates in place): load the item's
    // w0 row together before the stores so the loads are in flight at once
    T base[N];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const int m = blk < C::NLEG ? blk * N + l : C::NLEG * N + (blk - C::NLEG) * N + l;
      base[l] = ((mode & 1) && m < NM) ? w0[(int64_t)m * ld + K] : T(0);
    }
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const int m = blk < C::NLEG ? blk * N + l : C::NLEG * N + (blk - C::NLEG) * N + l;
      if (m >= NM) continue;
      T dw = acc[k][l] * two_h * tb.Minv[m];
      const T wm = sw[m * TC + c];
      if constexpr (DIVB == GLM) {
        if (m >= 8 * N) dw -= kappa * wm;
      }
      if (!(mode & 1)) out[(int64_t)m * ld + K] = dw;
      else out[(int64_t)m * ld + K] = (T)a0 * base[l] + (T)b0 * (wm + (T)dt * dw);
    }
  }
}

// ---------------------------------------------------------------------------
// Cell kernel on the matrix cores (GLM, uniform grids).
//
// One wave owns 16 cells; every contraction of the weak form is a chain of
// 16x16x4 matrix products with the 16 cells as the column index:
//   nodal values   U_v[q][c]  = sum_n V[q][n] w_v[n][c]              (K = modes)
//   volume term    R_v[n][c] += sum_{a,q} GW_a[q][n] f_a,v(U(q,c))   (K = points)
//   surface term   R_v[n][c] += sum_k LFs[n][k] Fhat_v[k][c]         (K = face moments)
// The accumulator layout of the nodal product (lane l, element r: point
// 16 rt + row(l/16, r), cell l % 16) is the B-operand layout of the volume
// product once its K index runs over the same points, so fluxes go from the
// nodal accumulators straight into the next product without any exchange;
// the table operands are stored in that lane order ("fragment order").

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator row held by element r of a lane in k-group k = lane / 16
  static constexpr __host__ __device__ int row(int k, int r) { return k + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static constexpr __host__ __device__ int row(int k, int r) { return 4 * k + r; }
};

// Matrix-core GLM kernels in FP32 on uniform grids: two waves per SIMD
// (256 registers per lane)
template <typename T, bool AMR, int DEG = 3>
constexpr int cell_waves_per_eu() { return ((sizeof(T) == 4 && !AMR) || (AMR && DEG <= 2)) ? 2 : 1; }

template <int D, int DEG>
struct MfmaShape {
  using C = Cfg<D, DEG, GLM>;
  static constexpr int NKS = (C::N + 3) / 4;            // k-steps of the nodal product
  static constexpr int QT = (C::Q + 15) / 16;           // 16-point row tiles
  static constexpr int NMT = (C::N + 15) / 16;          // 16-mode row tiles of the result
  static constexpr int KS = (2 * D * C::FP + 3) / 4;    // k-steps of the surface product
  static constexpr int SZ_V = QT * NKS * 64;
  static constexpr int SZ_G = D * NMT * QT * 4 * 64;
  static constexpr int SZ_L = NMT * KS * 64;
  // modes 16..N-1 when there are at most 4 of them (degree 3: modes 16..19)
  // are accumulated on the vector ALU instead of a 16-row tile that would be
  // mostly padding: per lane 4 modes at its own points / face points
  static constexpr bool XR = NMT == 2 && C::N - 16 <= 4;
  static constexpr int SZ_GX = D * QT * 64;   // [a][rt][j][k][e]
  static constexpr int SZ_LX = KS * 16;       // [s][k][e]
  // surface product over face moments (GLM uniform grids): K = 2 D FM
  static constexpr int KSM = (2 * D * C::FM + 3) / 4;
  // rows per (axis, variable) of the moment buffer: the FM moments, and in
  // the FP32 deviation form two more rows (the face's reference flux minus
  // the left and the right cell's mean flux)
  template <typename T>
  static constexpr int fms() { return sizeof(T) == 4 ? C::FM + 2 : C::FM; }
  // index of the mode xi_a^k (Legendre degree k along axis a, 0 along the
  // others) in the graded order of the modes
  static constexpr int power_mode(int a, int k) {
    int idx = 0;
    for (int g = 0; g <= DEG; ++g)
      for (int k1 = g; k1 >= 0; --k1) {
        if (D == 2) {
          const int e[2] = {k1, g - k1};
          if (e[a] == k && g == k) return idx;
          ++idx;
        } else {
          for (int k2 = g - k1; k2 >= 0; --k2) {
            const int e[3] = {k1, k2, g - k1 - k2};
            if (e[a] == k && g == k) return idx;
            ++idx;
          }
        }
      }
    return -1;
  }
  struct PowModes {
    int m[3][4];
  };
  static constexpr PowModes pow_modes() {
    PowModes p{};
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 4; ++k) p.m[a][k] = (a < D && k <= DEG) ? power_mode(a, k) : 0;
    return p;
  }
  static constexpr int SZ_LM = NMT * KSM * 64;
  static constexpr int SZ_LXM = KSM * 16;
};

// Face moments.  A face flux enters the weak form only through its products
// with the lift rows w_r phi_n(x_r) of the two adjacent cells, which span a
// space of dimension FM (the traces of the basis are polynomials of degree
// <= DEG in the face coordinates, and the two sides differ by signs only).
// With an orthonormal basis Q of that space (FP x FM per axis), the FM
// coordinates M = Q^T F of the point fluxes F carry the whole surface term:
// sum_r LF[n][r] F_r = sum_m (LF Q)[n][m] M_m, exactly up to rounding.
// Q by Gram-Schmidt (two passes) on the lift rows; false if the rank is not
// FM or a row is not reproduced.  qb[a][r][m].
template <int D, int DEG>
bool face_moment_basis(const Tables& t, std::vector<double>& qb) {
  using C = Cfg<D, DEG, GLM>;
  constexpr int N = C::N, FP = C::FP, FM = C::FM;
  qb.assign((size_t)D * FP * FM, 0.0);
  for (int a = 0; a < D; ++a) {
    auto row = [&](int side, int n, int r) { return t.LF[((a * 2 + side) * FP + r) * N + n]; };
    double scale = 0.0;
    for (int side = 0; side < 2; ++side)
      for (int n = 0; n < N; ++n)
        for (int r = 0; r < FP; ++r) scale = std::max(scale, std::fabs(row(side, n, r)));
    std::vector<std::vector<double>> bs;
    for (int side = 0; side < 2; ++side)
      for (int n = 0; n < N; ++n) {
        std::vector<double> x(FP);
        for (int r = 0; r < FP; ++r) x[r] = row(side, n, r);
        for (int pass = 0; pass < 2; ++pass)
          for (const auto& b : bs) {
            double d = 0.0;
            for (int r = 0; r < FP; ++r) d += b[r] * x[r];
            for (int r = 0; r < FP; ++r) x[r] -= d * b[r];
          }
        double nx = 0.0;
        for (int r = 0; r < FP; ++r) nx += x[r] * x[r];
        nx = std::sqrt(nx);
        if (nx > 1e-8 * scale) {
          for (int r = 0; r < FP; ++r) x[r] /= nx;
          bs.push_back(x);
        }
      }
    if ((int)bs.size() != FM) return false;
    for (int r = 0; r < FP; ++r)
      for (int m = 0; m < FM; ++m) qb[((size_t)a * FP + r) * FM + m] = bs[m][r];
    for (int side = 0; side < 2; ++side)
      for (int n = 0; n < N; ++n)
        for (int r = 0; r < FP; ++r) {
          double pr = 0.0;
          for (int m = 0; m < FM; ++m) {
            double d = 0.0;
            for (int rr = 0; rr < FP; ++rr) d += bs[m][rr] * row(side, n, rr);
            pr += d * bs[m][r];
          }
          if (std::fabs(pr - row(side, n, r)) > 1e-13 * scale) return false;
        }
  }
  return true;
}

// Fragment-order lift tables of the GLM cell kernel over face moments:
// entries (LF Q)[a][side][n][m] at K index k = (a * 2 + side) * FM + m
// (negated on the -a side, as the point tables).
template <typename T, int D, int DEG>
void mfma_moment_lift(const Tables& t, const std::vector<double>& qb, std::vector<double>& fl,
                      std::vector<double>& lx) {
  using C = Cfg<D, DEG, GLM>;
  using S = MfmaShape<D, DEG>;
  constexpr int N = C::N, FP = C::FP, FM = C::FM;
  auto lift = [&](int k, int n) {
    const int a = k / (2 * FM), side = (k / FM) % 2, m = k % FM;
    double v = 0.0;
    for (int r = 0; r < FP; ++r) v += t.LF[((a * 2 + side) * FP + r) * N + n] * qb[((size_t)a * FP + r) * FM + m];
    return side ? -v : v;
  };
  fl.assign(S::SZ_LM, 0.0);
  lx.assign(S::SZ_LXM, 0.0);
  for (int mt = 0; mt < S::NMT; ++mt)
    for (int s = 0; s < S::KSM; ++s)
      for (int l = 0; l < 64; ++l) {
        const int k = 4 * s + l / 16, n = 16 * mt + l % 16;
        if (k < 2 * D * FM && n < N) fl[(mt * S::KSM + s) * 64 + l] = lift(k, n);
      }
  for (int s = 0; s < S::KSM; ++s)
    for (int k = 0; k < 4; ++k)
      for (int e = 0; e < 4; ++e) {
        const int kk = 4 * s + k, n = 16 + e;
        if (kk < 2 * D * FM && n < N) lx[(s * 4 + k) * 4 + e] = lift(kk, n);
      }
}

// Fragment-order tables from the plain tables V[q][n], GW[a][q][n] and
// LF[a][side][r][n] (row-major, as uploaded for the other kernels).
template <typename T, int D, int DEG>
void mfma_tables(const Tables& t, std::vector<double>& fv, std::vector<double>& fg, std::vector<double>& fl,
                 std::vector<double>& gx, std::vector<double>& lx) {
  using C = Cfg<D, DEG, GLM>;
  using S = MfmaShape<D, DEG>;
  constexpr int N = C::N, Q = C::Q, FP = C::FP;
  fv.assign(S::SZ_V, 0.0);
  fg.assign(S::SZ_G, 0.0);
  fl.assign(S::SZ_L, 0.0);
  gx.assign(S::SZ_GX, 0.0);
  lx.assign(S::SZ_LX, 0.0);
  for (int a = 0; a < D; ++a)
    for (int rt = 0; rt < S::QT; ++rt)
      for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 4; ++k)
          for (int e = 0; e < 4; ++e) {
            const int q = 16 * rt + Mfma<T>::row(k, j), n = 16 + e;
            if (q < Q && n < N) gx[(((a * S::QT + rt) * 4 + j) * 4 + k) * 4 + e] = t.GW[(a * Q + q) * N + n];
          }
  for (int s = 0; s < S::KS; ++s)
    for (int k = 0; k < 4; ++k)
      for (int e = 0; e < 4; ++e) {
        const int kk = 4 * s + k, n = 16 + e;
        if (kk >= 2 * D * FP || n >= N) continue;
        const int a = kk / (2 * FP), side = (kk / FP) % 2, r = kk % FP;
        const double v = t.LF[((a * 2 + side) * FP + r) * N + n];
        lx[(s * 4 + k) * 4 + e] = side ? -v : v;
      }
  for (int rt = 0; rt < S::QT; ++rt)
    for (int s = 0; s < S::NKS; ++s)
      for (int l = 0; l < 64; ++l) {
        const int q = 16 * rt + l % 16, n = 4 * s + l / 16;
        if (q < Q && n < N) fv[(rt * S::NKS + s) * 64 + l] = t.V[q * N + n];
      }
  for (int a = 0; a < D; ++a)
    for (int mt = 0; mt < S::NMT; ++mt)
      for (int rt = 0; rt < S::QT; ++rt)
        for (int j = 0; j < 4; ++j)
          for (int l = 0; l < 64; ++l) {
            const int q = 16 * rt + Mfma<T>::row(l / 16, j), n = 16 * mt + l % 16;
            if (q < Q && n < N) fg[((((a * S::NMT + mt) * S::QT + rt) * 4 + j) * 64) + l] = t.GW[(a * Q + q) * N + n];
          }
  for (int mt = 0; mt < S::NMT; ++mt)
    for (int s = 0; s < S::KS; ++s)
      for (int l = 0; l < 64; ++l) {
        const int k = 4 * s + l / 16, n = 16 * mt + l % 16;
        if (k >= 2 * D * FP || n >= N) continue;
        const int a = k / (2 * FP), side = (k / FP) % 2, r = k % FP;
        const double v = t.LF[((a * 2 + side) * FP + r) * N + n];
        fl[(mt * S::KS + s) * 64 + l] = side ? -v : v;
      }
}

// The work of one wave on the 16 cells starting at c0 (tables FV, FG, FL in
// global memory or LDS).
// AMR: octree grid; the surface term is then an owner gather of the 1 or
// 2^(D-1) (sub-)face point fluxes of each side, multiplied on the matrix
// cores with the signed sub-face lift tables LFS of each class present.
//
// FP32 deviation form (DEV: FP32 state on uniform grids).  A constant flux c
// added to every volume and face flux of a cell changes nothing in exact
// arithmetic (the quadrature integrates d_a phi over the cell and phi over
// its faces exactly, and the two cancel), but in FP32 the products of a
// large constant background flux leave rounding noise of ~1e-7 of it in
// every mode of a quiet region.  So the FP32 products act on deviations
// only: the nodal product omits mode 0 (the deviation du from the cell
// mean), the volume flux is the flux deviation f_a(mean + du) - f_a(mean)
// in the rearranged form of mhd_dflux, and the face moments are those of
// F* - c with c the FP32-rounded flux of the face's left-cell mean.  The
// face kernel also stores, in two extra rows, c - f_a(mean) of the left and
// of the right cell (FP64 differences, small, rounded to FP32); each cell adds
// the lift of its side's constant over the face, which turns every face term
// into F* minus the cell's own mean flux.  The lift of a constant over a
// face only reaches the modes xi_a^k.  A uniform state gives zero up to FP64
// rounding.
template <typename T, int D, int DEG, bool PF, bool AMR>
__device__ __forceinline__ void cell_tile_mfma(int64_t c0, int lane, const T* w, const T* w0, T* out,
                                               const T* __restrict__ ff, const T* FV, const T* FG, const T* FL,
                                               const T* GX, const T* LX, const T* __restrict__ LFS,
                                               const T* __restrict__ L1, const T* __restrict__ Minv, const Grid& g,
                                               const Scal* __restrict__ sc, double gamma, double a0, double b0, double cdt,
                                               int mode) {
  using C = Cfg<D, DEG, GLM>;
  using S = MfmaShape<D, DEG>;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int N = C::N, Q = C::Q, FP = C::FP, NV = 9;
  constexpr bool XR = S::XR && !AMR;        // last modes on the vector ALU
  constexpr int NMU = XR ? 1 : S::NMT;      // mode tiles on the matrix cores
  constexpr bool DEV = sizeof(T) == 4 && !AMR;
  constexpr int FMS = S::template fms<T>();
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t K = c0 + cl;
  const bool live = K < g.C;
  const int64_t Kc = live ? K : c0;  // ragged tail: dead lanes read a live cell, write nothing
  const int64_t ld = g.ld;
  const T ch = (T)sc->ch;
  const T ch2 = ch * ch;
  // DEV: the cell's mean state as the reference of the flux deviations
  MeanRef mref;
  if constexpr (DEV) {
    float ub[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] = (float)w[(int64_t)(v * N) * ld + Kc];
    mref.init(ub, gamma);
  }
  v4 R[NV][S::NMT];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int mt = 0; mt < S::NMT; ++mt) R[v][mt] = v4{0, 0, 0, 0};
  // XR: partial sums of modes 16..19 over the lane's own points (reduced
  // over the cell's four lanes at the end)
  T RX[NV][4];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) RX[v][e] = T(0);
  // face moments of k-step s (k = 4 s + kq: axis, side, moment);
  // la[NMU] matrix-core table fragments, la[NMU..NMU+3] the XR row values
  constexpr int FM = C::FM;
  auto load_face = [&](int s, T* fv, T* la) {
    const int k = 4 * s + kq;
    const bool kv = k < 2 * D * FM;
    const int a = kv ? k / (2 * FM) : 0, side = (k / FM) % 2, r = k % FM;
    const int64_t Kf = side ? Kc : nbr(Kc, a, -1, g);
#pragma unroll
    for (int v = 0; v < NV; ++v) fv[v] = kv ? ff[((int64_t)(a * NV + v) * FMS + r) * ld + Kf] : T(0);
#pragma unroll
    for (int mt = 0; mt < NMU; ++mt) la[mt] = FL[(mt * S::KSM + s) * 64 + lane];
    if (XR) {
#pragma unroll
      for (int e = 0; e < 4; ++e) la[NMU + e] = LX[(s * 4 + kq) * 4 + e];
    }
  };
  auto surface_step = [&](const T* fv, const T* la) {
#pragma unroll
    for (int mt = 0; mt < NMU; ++mt)
#pragma unroll
      for (int v = 0; v < NV; ++v) R[v][mt] = M::mma(la[mt], fv[v], R[v][mt]);
    if (XR) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) RX[v][e] += la[NMU + e] * fv[v];
    }
  };
  constexpr int NLA = NMU + (XR ? 4 : 0);
  if (PF && !AMR) {
    // batched variant: the surface term first, while the nodal registers are
    // free, with the loads of SB k-steps in flight together
    constexpr int SB = 5;
#pragma unroll 1
    for (int s0 = 0; s0 < S::KSM; s0 += SB) {
      T fv[SB][NV], la[SB][NLA];
#pragma unroll
      for (int b = 0; b < SB; ++b) {
        if (s0 + b < S::KSM) {
          load_face(s0 + b, fv[b], la[b]);
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) fv[b][v] = T(0);
#pragma unroll
          for (int mt = 0; mt < NLA; ++mt) la[b][mt] = T(0);
        }
      }
#pragma unroll
      for (int b = 0; b < SB; ++b) surface_step(fv[b], la[b]);
    }
  }
  // the cell's modes as B operands of the nodal product: in the batched
  // variant loaded once for all row tiles
  T bw[PF ? S::NKS : 1][NV];
  if (PF) {
#pragma unroll
    for (int s = 0; s < S::NKS; ++s)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int n = 4 * s + kq;
        bw[PF ? s : 0][v] = (n < N && !(DEV && n == 0)) ? w[(int64_t)(v * N + n) * ld + Kc] : T(0);
      }
  }

  for (int rt = 0; rt < S::QT; ++rt) {
    v4 U[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v] = v4{0, 0, 0, 0};
    if (PF) {
      T av[S::NKS];
#pragma unroll
      for (int s = 0; s < S::NKS; ++s) av[s] = FV[(rt * S::NKS + s) * 64 + lane];
#pragma unroll
      for (int s = 0; s < S::NKS; ++s)
#pragma unroll
        for (int v = 0; v < NV; ++v) U[v] = M::mma(av[s], bw[PF ? s : 0][v], U[v]);
    } else {
#pragma unroll 1
      for (int s = 0; s < S::NKS; ++s) {
        const int n = 4 * s + kq;
        const T ac = FV[(rt * S::NKS + s) * 64 + lane];
        T bc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) bc[v] = (n < N && !(DEV && n == 0)) ? w[(int64_t)(v * N + n) * ld + Kc] : T(0);
#pragma unroll
        for (int v = 0; v < NV; ++v) U[v] = M::mma(ac, bc[v], U[v]);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool qv = 16 * rt + M::row(kq, j) < Q;
      T u[9];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = U[v][j];
      if (!qv) {  // padding point: a harmless state, its flux is zeroed below
        u[0] = T(1);
        u[4] = T(1);
      }
      DevPoint dq;
      if constexpr (DEV) dev_point(mref, (const float*)u, gamma, dq);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        T f[9];
        if constexpr (DEV) {
          if (a == 0) mhd_dflux<NV, 0>(mref, (const float*)u, dq, (float)ch2, (float*)f);
          else if (a == 1) mhd_dflux<NV, 1>(mref, (const float*)u, dq, (float)ch2, (float*)f);
          else mhd_dflux<NV, 2>(mref, (const float*)u, dq, (float)ch2, (float*)f);
        } else {
          mhd_flux<T, NV>(u, a, gamma, ch2, f);
        }
#pragma unroll
        for (int mt = 0; mt < NMU; ++mt) {
          const T ga = FG[((((a * S::NMT + mt) * S::QT + rt) * 4 + j) * 64) + lane];
#pragma unroll
          for (int v = 0; v < NV; ++v) R[v][mt] = M::mma(ga, qv ? f[v] : T(0), R[v][mt]);
        }
        if (XR) {
          T gx[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) gx[e] = GX[(((a * S::QT + rt) * 4 + j) * 4 + kq) * 4 + e];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const T fq = qv ? f[v] : T(0);
#pragma unroll
            for (int e = 0; e < 4; ++e) RX[v][e] += gx[e] * fq;
          }
        }
      }
    }
  }
  if (!PF && !AMR) {
#pragma unroll 1
    for (int s = 0; s < S::KSM; ++s) {
      T fv[NV], la[NLA];
      load_face(s, fv, la);
      surface_step(fv, la);
    }
  }
  if (XR) {  // sum the partials over the cell's four lanes (every lane of the cell holds the total)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        RX[v][e] += __shfl_xor(RX[v][e], 16);
        RX[v][e] += __shfl_xor(RX[v][e], 32);
      }
  }
  if constexpr (DEV) {
    // each face carries F* - c: add the lift of the stored constant
    // c - f_a(cell mean) of the cell's side over the face (L1[side][a][n],
    // signed as the lift tables; nonzero only for the modes xi_a^k)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T dl[NV], dr[NV];
      const int64_t Kb = nbr(Kc, a, -1, g);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        dl[v] = ff[((int64_t)(a * NV + v) * FMS + C::FM) * ld + Kc];       // +a face: this cell is its left cell
        dr[v] = ff[((int64_t)(a * NV + v) * FMS + C::FM + 1) * ld + Kb];   // -a face: this cell is its right cell
      }
      constexpr typename S::PowModes PM = S::pow_modes();
#pragma unroll
      for (int k = 0; k <= DEG; ++k) {
        const int n = PM.m[a][k];
        const T lp = L1[(1 * D + a) * N + n], lm = L1[(0 * D + a) * N + n];
        const int mt = n / 16, kown = (n % 16) / 4, e = n % 4;  // FP32 accumulator layout: row 4 k + e
        if (XR && mt == 1) {
#pragma unroll
          for (int v = 0; v < NV; ++v) RX[v][n - 16] += lp * dl[v] + lm * dr[v];
        } else if (kq == kown) {
#pragma unroll
          for (int v = 0; v < NV; ++v) R[v][mt][e] += lp * dl[v] + lm * dr[v];
        }
      }
    }
  }
  if constexpr (AMR) {
    // Surface term on the matrix cores: for each side of the cell and each
    // sub-face class (0 the full face, 1 + q quarter q of a side with finer
    // neighbours) one 16x16x4 product chain of the signed lift table of that
    // class (LFS, fragment order, over face moments) with the flux moments of
    // the 16 cells' faces of that class (cells without such a face contribute
    // zero).  A class no cell of the tile has is skipped.
    constexpr int NSUB = 1 + (1 << (D - 1)), NQ = 1 << (D - 1), KS1 = (C::FM + 3) / 4, FMA = C::FM;
    const int64_t ldf = g.ldf;
    for (int a = 0; a < D; ++a)
      for (int sd = 0; sd < 2; ++sd) {
        int32_t fs[NQ], sb[NQ];
        const int32_t* sl = g.slots + (((int64_t)Kc * D + a) * 2 + sd) * 4;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int32_t f = live ? sl[q] : -1;
          fs[q] = f;
          sb[q] = f >= 0 ? 1 + (sd ? g.subL[f] : g.subR[f]) : -1;
        }
        for (int sub = 0; sub < NSUB; ++sub) {
          int32_t f = -1;
#pragma unroll
          for (int q = 0; q < NQ; ++q) f = (sb[q] == sub) ? fs[q] : f;
          if (!__any(f >= 0)) continue;
#pragma unroll
          for (int s = 0; s < KS1; ++s) {
            const int m = 4 * s + kq;
            T bv[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) bv[v] = (f >= 0 && m < FMA) ? ff[((int64_t)v * FMA + m) * ldf + f] : T(0);
#pragma unroll
            for (int mt = 0; mt < S::NMT; ++mt) {
              const T la = LFS[(((((a * 2 + sd) * NSUB + sub) * KS1 + s) * S::NMT + mt) * 64) + lane];
#pragma unroll
              for (int v = 0; v < NV; ++v) R[v][mt] = M::mma(la, bv[v], R[v][mt]);
            }
          }
        }
      }
  }
  if (!live) return;
  const double dt = sc->dt * cdt;  // the stage's multiple of the step
  const T kappa = (T)sc->kappa;
  const T two_h = T(2.0 / cell_h(g, K));
  // out may be w or w0 (stages 2 and 3 update in place), so the compiler
  // keeps every load of an element before its store; loading a variable's
  // elements together first keeps those loads in flight at once.  Each
  // (mode, cell) element belongs to exactly one lane.
  // Each (mode, cell) element belongs to exactly one lane and each variable
  // owns its rows, so the operands of variable v+1 (its state, stage base
  // and inverse-mass entries) may be loaded before the stores of v, even
  // when out aliases w or w0: two variables' loads are in flight while one
  // is combined and stored (FP64; FP32 loads each variable's operands just
  // before it, keeping its registers for two waves per SIMD).  The inverse-
  // mass entries are loaded with the other operands: out is not known not
  // to alias Minv, so a load of Minv after a store would wait for that store.
  constexpr bool AHEAD = sizeof(T) == 8;
  // octree, FP64: the epilogue forms its row offsets afresh rather than
  // keeping those of the mode loads live through the volume loop
  int64_t lde = ld;
  int kqe = kq;
  if constexpr (AMR && sizeof(T) == 8) asm volatile("" : "+s"(lde), "+v"(kqe));
  T ew[2][S::NMT][4], eb[2][S::NMT][4], em[2][S::NMT][4];
  auto eload = [&](int v, T (&wm)[S::NMT][4], T (&base)[S::NMT][4], T (&mi)[S::NMT][4]) {
#pragma unroll
    for (int mt = 0; mt < S::NMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = 16 * mt + M::row(kqe, r);
        const int64_t at = (int64_t)(v * N + (n < N ? n : 0)) * lde + K;
        wm[mt][r] = (v == 8 || (mode & 1)) ? w[at] : T(0);
        base[mt][r] = (mode & 1) ? w0[at] : T(0);
        mi[mt][r] = n < N ? Minv[v * N + n] : T(0);
      }
  };
  eload(0, ew[0], eb[0], em[0]);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (AHEAD && v + 1 < NV) eload(v + 1, ew[(v + 1) & 1], eb[(v + 1) & 1], em[(v + 1) & 1]);
    if (!AHEAD && v > 0) eload(v, ew[v & 1], eb[v & 1], em[v & 1]);
    const auto& wm = ew[v & 1];
    const auto& base = eb[v & 1];
    const auto& mi = em[v & 1];
#pragma unroll
    for (int mt = 0; mt < S::NMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = 16 * mt + M::row(kqe, r);
        if (n >= N) continue;
        const int m = v * N + n;
        T racc = R[v][mt][r];
        if (XR && mt == 1) {
          const int e = n - 16;
          racc = e == 0 ? RX[v][0] : e == 1 ? RX[v][1] : e == 2 ? RX[v][2] : RX[v][3];
        }
        T dw = racc * two_h * mi[mt][r];
        if (v == 8) dw -= kappa * wm[mt][r];
        if (!(mode & 1)) out[(int64_t)m * ld + K] = dw;
        else out[(int64_t)m * ld + K] = (T)a0 * base[mt][r] + (T)b0 * (wm[mt][r] + (T)dt * dw);
      }
  }
}

template <typename T, int D, int DEG, int NW, bool PF, bool AMR>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(cell_waves_per_eu<T, AMR, DEG>())))
    k_cell_mfma(const T* w, const T* w0, T* out, const T* __restrict__ ff, const T* __restrict__ FV,
                const T* __restrict__ FG, const T* __restrict__ FL, const T* __restrict__ GX,
                const T* __restrict__ LX, const T* __restrict__ LFS, const T* __restrict__ L1,
                const T* __restrict__ Minv, Grid g, const Scal* __restrict__ sc, double gamma, double a0, double b0, double cdt,
                int mode) {
  const int64_t c0 = ((int64_t)xcd_block(blockIdx.x, gridDim.x) * NW + (threadIdx.x >> 6)) * 16;
  if (c0 >= g.C) return;  // whole wave; the kernel has no barrier
  cell_tile_mfma<T, D, DEG, PF, AMR>(c0, threadIdx.x & 63, w, w0, out, ff, FV, FG, FL, GX, LX, LFS, L1, Minv, g, sc,
                                     gamma, a0, b0, cdt, mode);
}

// Persistent form: one workgroup per resident slot copies the fragment
// tables into LDS once, then its waves walk a contiguous range of 16-cell
// tiles (ranges dealt XCD by XCD, as in xcd_block).  FP64 on octrees at
// degree <= 2: two waves per SIMD, the cell's modes reloaded per row tile
// (PF off) and the lane's row offsets formed afresh for every tile (hoisted
// out of the walk they would be held in spilled registers).
template <typename T, int D, int DEG, int NW, bool AMR>
__global__ void __launch_bounds__(64 * NW)
    __attribute__((amdgpu_waves_per_eu((AMR && DEG <= 2 && sizeof(T) == 8) ? 2 : 1)))
    k_cell_mfma_p(const T* w, const T* w0, T* out, const T* __restrict__ ff, const T* __restrict__ FV,
                  const T* __restrict__ FG, const T* __restrict__ FL, const T* __restrict__ GX,
                  const T* __restrict__ LX, const T* __restrict__ LFS, const T* __restrict__ L1,
                  const T* __restrict__ Minv, Grid g, const Scal* __restrict__ sc, double gamma, double a0,
                  double b0, double cdt, int mode) {
  using S = MfmaShape<D, DEG>;
  __shared__ T sV[S::SZ_V], sG[S::SZ_G], sL[S::SZ_LM], sGX[S::SZ_GX], sLX[S::SZ_LXM];
  for (int i = threadIdx.x; i < S::SZ_V; i += 64 * NW) sV[i] = FV[i];
  for (int i = threadIdx.x; i < S::SZ_G; i += 64 * NW) sG[i] = FG[i];
  for (int i = threadIdx.x; i < S::SZ_LM; i += 64 * NW) sL[i] = FL[i];
  for (int i = threadIdx.x; i < S::SZ_GX; i += 64 * NW) sGX[i] = GX[i];
  for (int i = threadIdx.x; i < S::SZ_LXM; i += 64 * NW) sLX[i] = LX[i];
  __syncthreads();
  const int64_t ntiles = (g.C + 15) / 16;
  const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int64_t t0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * per;
  const int64_t t1 = t0 + per < ntiles ? t0 + per : ntiles;
  constexpr bool LAUNDER = AMR && DEG <= 2 && sizeof(T) == 8;
  for (int64_t t = t0 + (threadIdx.x >> 6); t < t1; t += NW) {
    const T* mi = Minv;
    Grid gt = g;
    int ln = threadIdx.x & 63;
    if constexpr (LAUNDER) asm volatile("" : "+s"(mi), "+s"(gt.ld), "+v"(ln));
    cell_tile_mfma<T, D, DEG, !LAUNDER, AMR>(t * 16, ln, w, w0, out, ff, sV, sG, sL, sGX, sLX, LFS, L1, mi, gt, sc,
                                             gamma, a0, b0, cdt, mode);
  }
}

// ---------------------------------------------------------------------------
// Cell kernel on the matrix cores for the Powell scheme (uniform grids).
//
// The Legendre variables (rho, m, E; B_z in 2-D) follow the GLM kernel.  The
// magnetic field lives in the locally divergence-free basis: its nodal
// values are products of the per-component tables PV_c with the LDF modes,
// its volume term sums the products of PGW_{a,c} with the flux components
// f_a[B_c], and its surface term the products of the signed PLF_c with the
// face values.  The Powell face term of a face point (eq. powell-src-face
// with q of the cell means) is added to the same B operand as the flux, so it
// costs no extra product: side +a carries F + q (B^n_F - B^n_K), side -a
// F - q (B^n_K' - B^n_F) under the signed tables.

template <int D, int DEG>
struct PowellShape {
  using C = Cfg<D, DEG, POWELL>;
  static constexpr int NKL = (C::NLDF + 3) / 4;      // k-steps over the LDF modes
  static constexpr int NMTL = (C::NLDF + 15) / 16;   // 16-row tiles of the LDF result
  static constexpr int QT = (C::Q + 15) / 16;
  static constexpr int KS = (2 * D * C::FP + 3) / 4;
  // 3-D with the cell-mean q-dagger: the faces carry flux and jump moments
  static constexpr int KSM = (2 * D * C::FM + 3) / 4;
  static constexpr int SZ_PV = D * QT * NKL * 64;
  static constexpr int SZ_PG = D * D * NMTL * QT * 4 * 64;
  static constexpr int SZ_PL = D * NMTL * KS * 64;
  static constexpr int SZ_PLM = D * NMTL * KSM * 64;
};

// LDF lift tables over face moments (3-D, cell-mean q-dagger): entries
// sum_r PLF[a][side][c][r][i] Q[a][r][m] at K index (a * 2 + side) * FM + m,
// negated on the -a side as the point tables.  The LDF components restricted
// to a face are polynomials of degree <= DEG in the face coordinates, so the
// lift rows lie in the span of Q (checked; false otherwise).
template <typename T, int D, int DEG>
bool powell_moment_lift(const Tables& t, const std::vector<double>& qb, std::vector<double>& plm) {
  using C = Cfg<D, DEG, POWELL>;
  using S = PowellShape<D, DEG>;
  constexpr int FP = C::FP, FM = C::FM, L = C::NLDF;
  plm.assign(S::SZ_PLM, 0.0);
  for (int a = 0; a < D; ++a)
    for (int side = 0; side < 2; ++side)
      for (int c = 0; c < D; ++c) {
        const double* rows = &t.PLF[(((size_t)a * 2 + side) * D + c) * FP * L];  // [r][i]
        double scale = 0.0;
        for (int i = 0; i < FP * L; ++i) scale = std::max(scale, std::fabs(rows[i]));
        for (int i = 0; i < L; ++i) {
          double lm[16] = {0.0};
          for (int m = 0; m < FM; ++m)
            for (int r = 0; r < FP; ++r) lm[m] += rows[(size_t)r * L + i] * qb[((size_t)a * FP + r) * FM + m];
          for (int r = 0; r < FP; ++r) {
            double pr = 0.0;
            for (int m = 0; m < FM; ++m) pr += lm[m] * qb[((size_t)a * FP + r) * FM + m];
            if (std::fabs(pr - rows[(size_t)r * L + i]) > 1e-13 * scale) return false;
          }
          for (int m = 0; m < FM; ++m) {
            const int k = (a * 2 + side) * FM + m, s = k / 4, lq = k % 4, mt = i / 16;
            plm[((c * S::NMTL + mt) * S::KSM + s) * 64 + lq * 16 + i % 16] = side ? -lm[m] : lm[m];
          }
        }
      }
  return true;
}

template <typename T, int D, int DEG>
void powell_tables(const Tables& t, std::vector<double>& pv, std::vector<double>& pg, std::vector<double>& pl) {
  using C = Cfg<D, DEG, POWELL>;
  using S = PowellShape<D, DEG>;
  constexpr int Q = C::Q, FP = C::FP, L = C::NLDF;
  pv.assign(S::SZ_PV, 0.0);
  pg.assign(S::SZ_PG, 0.0);
  pl.assign(S::SZ_PL, 0.0);
  for (int c = 0; c < D; ++c)
    for (int rt = 0; rt < S::QT; ++rt)
      for (int s = 0; s < S::NKL; ++s)
        for (int l = 0; l < 64; ++l) {
          const int q = 16 * rt + l % 16, i = 4 * s + l / 16;
          if (q < Q && i < L) pv[((c * S::QT + rt) * S::NKL + s) * 64 + l] = t.PV[(c * Q + q) * L + i];
        }
  for (int a = 0; a < D; ++a)
    for (int c = 0; c < D; ++c)
      for (int mt = 0; mt < S::NMTL; ++mt)
        for (int rt = 0; rt < S::QT; ++rt)
          for (int j = 0; j < 4; ++j)
            for (int l = 0; l < 64; ++l) {
              const int q = 16 * rt + Mfma<T>::row(l / 16, j), i = 16 * mt + l % 16;
              if (q < Q && i < L)
                pg[(((((a * D + c) * S::NMTL + mt) * S::QT + rt) * 4 + j) * 64) + l] = t.PGW[((a * D + c) * Q + q) * L + i];
            }
  for (int c = 0; c < D; ++c)
    for (int mt = 0; mt < S::NMTL; ++mt)
      for (int s = 0; s < S::KS; ++s)
        for (int l = 0; l < 64; ++l) {
          const int k = 4 * s + l / 16, i = 16 * mt + l % 16;
          if (k >= 2 * D * FP || i >= L) continue;
          const int a = k / (2 * FP), side = (k / FP) % 2, r = k % FP;
          const double v = t.PLF[(((a * 2 + side) * D + c) * FP + r) * L + i];
          pl[((c * S::NMTL + mt) * S::KS + s) * 64 + l] = side ? -v : v;
        }
}

// PM (3-D, cell-mean q-dagger): the faces carry moments (face kernel
// variant 1): flux moments at rows a NV FP + v FM + m, the two sides' jump
// moments at a NV FP + 8 FM + side FM + m, and FL / PLt are the lift tables
// over moments.
template <typename T, int D, int DEG, bool PM = false>
__device__ __forceinline__ void cell_tile_mfma_powell(int64_t c0, int lane, const T* w, const T* w0, T* out,
                                                      const T* __restrict__ ff, const T* __restrict__ jp,
                                                      const T* FV, const T* FG, const T* FL, const T* PVt,
                                                      const T* PGt, const T* PLt, const T* __restrict__ Pmean,
                                                      const T* __restrict__ Minv, const Grid& g,
                                                      const Scal* __restrict__ sc, double gamma, double a0, double b0, double cdt,
                                                      int mode) {
  using C = Cfg<D, DEG, POWELL>;
  using S = MfmaShape<D, DEG>;
  using P = PowellShape<D, DEG>;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int N = C::N, Q = C::Q, FP = C::FP, NV = 8, NL = C::NLEG, L = C::NLDF;
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t K = c0 + cl;
  const bool live = K < g.C;
  const int64_t Kc = live ? K : c0;
  const int64_t ld = g.ld;
  v4 R[NL][S::NMT], RB[P::NMTL];
#pragma unroll
  for (int j = 0; j < NL; ++j)
#pragma unroll
    for (int mt = 0; mt < S::NMT; ++mt) R[j][mt] = v4{0, 0, 0, 0};
#pragma unroll
  for (int mt = 0; mt < P::NMTL; ++mt) RB[mt] = v4{0, 0, 0, 0};
  // q(<u>_K) of the lane's cell from the cell means (eq. powellq-average)
  T qv[8];
  {
    const T rho = w[Kc];
    T bm[3];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T b = 0;
      for (int l = 0; l < L; ++l) b += Pmean[c * L + l] * w[(int64_t)(NL * N + l) * ld + Kc];
      bm[c] = b;
    }
    if (D == 2) bm[2] = w[(int64_t)(5 * N) * ld + Kc];
    const T v0 = w[(int64_t)(1 * N) * ld + Kc] / rho, v1 = w[(int64_t)(2 * N) * ld + Kc] / rho,
            v2 = w[(int64_t)(3 * N) * ld + Kc] / rho;
    qv[0] = 0; qv[1] = bm[0]; qv[2] = bm[1]; qv[3] = bm[2];
    qv[4] = v0 * bm[0] + v1 * bm[1] + v2 * bm[2];
    qv[5] = v0; qv[6] = v1; qv[7] = v2;
  }
  const bool qint = (mode & 2) != 0;  // interpolated q-dagger: the Powell terms come with the face values
  if (qint)
#pragma unroll
    for (int v = 0; v < 8; ++v) qv[v] = T(0);
  // surface first: flux + Powell term of face point k = 4 s + kq as one B operand per variable.
  // Face values of k-step s, and the normal-field jump that the Powell term
  // multiplies: side +a: B^n_F - B^n_K at face K; side -a: B^n_K - B^n_F at
  // face K-a (interpolated q-dagger: the face kernel added each side's
  // Powell term to its face values, the left side's in ff, the right side's
  // in jp, and the jump is not read).
  constexpr int FK = PM ? C::FM : FP;                  // face values per face and variable
  constexpr int KSX = PM ? P::KSM : S::KS;            // k-steps of the surface product
  auto load_face = [&](int s, T* fv) {
    const int k = 4 * s + kq;
    const bool kv = k < 2 * D * FK;
    const int a = kv ? k / (2 * FK) : 0, side = (k / FK) % 2, r = k % FK;
    const int64_t Kf = side ? Kc : nbr(Kc, a, -1, g);
    if constexpr (PM) {
      const int64_t base = (int64_t)a * NV * FP;
      fv[NV] = kv ? ff[(base + 8 * FK + (side ? 0 : 1) * FK + r) * ld + Kf] : T(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) fv[v] = kv ? ff[(base + v * FK + r) * ld + Kf] : T(0);
    } else {
      fv[NV] = (kv && !qint) ? jp[((int64_t)(a * 2 + (side ? 0 : 1)) * FP + r) * ld + Kf] : T(0);
      const T* src = (qint && !side) ? jp : ff;
#pragma unroll
      for (int v = 0; v < NV; ++v) fv[v] = kv ? src[((int64_t)(a * NV + v) * FP + r) * ld + Kf] : T(0);
    }
  };
  auto surface_step = [&](int s, const T* fv) {
    const int side = ((4 * s + kq) / FK) % 2;
    T bv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) bv[v] = side ? fv[v] + qv[v] * fv[NV] : fv[v] - qv[v] * fv[NV];
#pragma unroll
    for (int mt = 0; mt < S::NMT; ++mt) {
      const T la = FL[(mt * KSX + s) * 64 + lane];
#pragma unroll
      for (int j = 0; j < NL; ++j) R[j][mt] = M::mma(la, bv[C::legvar(j)], R[j][mt]);
    }
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int mt = 0; mt < P::NMTL; ++mt)
        RB[mt] = M::mma(PLt[((c * P::NMTL + mt) * KSX + s) * 64 + lane], bv[5 + c], RB[mt]);
  };
  // 3-D degree 2: the loads of SB k-steps in flight together (the surface
  // phase holds few registers: the accumulators and q); elsewhere batching
  // measured no gain and raised the persistent kernel's spills
  constexpr int SB = (D == 3 && DEG == 2) ? 7 : 1;
#pragma unroll 1
  for (int s0 = 0; s0 < KSX; s0 += SB) {
    T fv[SB][NV + 1];
#pragma unroll
    for (int b = 0; b < SB; ++b)
      if (s0 + b < KSX) load_face(s0 + b, fv[b]);
#pragma unroll
    for (int b = 0; b < SB; ++b)
      if (s0 + b < KSX) surface_step(s0 + b, fv[b]);
  }
  // the cell's modes as B operands, held for all row tiles
  T bw[NL][S::NKS], bl[P::NKL];
#pragma unroll
  for (int j = 0; j < NL; ++j)
#pragma unroll
    for (int s = 0; s < S::NKS; ++s) {
      const int n = 4 * s + kq;
      bw[j][s] = n < N ? w[(int64_t)(j * N + n) * ld + Kc] : T(0);
    }
#pragma unroll
  for (int s = 0; s < P::NKL; ++s) {
    const int i = 4 * s + kq;
    bl[s] = i < L ? w[(int64_t)(NL * N + i) * ld + Kc] : T(0);
  }
  const T ch2 = T(0);
#pragma unroll 1
  for (int rt = 0; rt < S::QT; ++rt) {
    v4 U[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v] = v4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < S::NKS; ++s) {
      const T av = FV[(rt * S::NKS + s) * 64 + lane];
#pragma unroll
      for (int j = 0; j < NL; ++j) U[C::legvar(j)] = M::mma(av, bw[j][s], U[C::legvar(j)]);
    }
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int s = 0; s < P::NKL; ++s)
        U[5 + c] = M::mma(PVt[((c * S::QT + rt) * P::NKL + s) * 64 + lane], bl[s], U[5 + c]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool qok = 16 * rt + M::row(kq, j) < Q;
      T u[9];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = U[v][j];
      u[8] = T(0);
      if (!qok) {
        u[0] = T(1);
        u[4] = T(1);
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        T f[9];
        mhd_flux<T, NV>(u, a, gamma, ch2, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) f[v] = qok ? f[v] : T(0);
#pragma unroll
        for (int mt = 0; mt < S::NMT; ++mt) {
          const T ga = FG[((((a * S::NMT + mt) * S::QT + rt) * 4 + j) * 64) + lane];
#pragma unroll
          for (int jj = 0; jj < NL; ++jj) R[jj][mt] = M::mma(ga, f[C::legvar(jj)], R[jj][mt]);
        }
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
          for (int mt = 0; mt < P::NMTL; ++mt)
            RB[mt] = M::mma(PGt[(((((a * D + c) * P::NMTL + mt) * S::QT + rt) * 4 + j) * 64) + lane], f[5 + c], RB[mt]);
      }
    }
  }
  if (!live) return;
  const double dt = sc->dt * cdt;  // the stage's multiple of the step
  const T two_h = T(2.0 / g.h);
  // FP64: the epilogue forms its row offsets afresh rather than keeping
  // those of the mode loads live through the volume loop
  int64_t lde = ld;
  int kqe = kq;
  if constexpr (sizeof(T) == 8) asm volatile("" : "+s"(lde), "+v"(kqe));
  auto finish = [&](int m, T racc) {
    T dw = racc * two_h * Minv[m];
    if (!(mode & 1)) return dw;
    return (T)a0 * w0[(int64_t)m * lde + K] + (T)b0 * (w[(int64_t)m * lde + K] + (T)dt * dw);
  };
  // out may alias w or w0: every element's loads precede its store, grouped per block
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    T o[S::NMT][4];
#pragma unroll
    for (int mt = 0; mt < S::NMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = 16 * mt + M::row(kqe, r);
        o[mt][r] = n < N ? finish(j * N + n, R[j][mt][r]) : T(0);
      }
#pragma unroll
    for (int mt = 0; mt < S::NMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = 16 * mt + M::row(kqe, r);
        if (n < N) out[(int64_t)(j * N + n) * lde + K] = o[mt][r];
      }
  }
  {
    T o[P::NMTL][4];
#pragma unroll
    for (int mt = 0; mt < P::NMTL; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * mt + M::row(kqe, r);
        o[mt][r] = i < L ? finish(NL * N + i, RB[mt][r]) : T(0);
      }
#pragma unroll
    for (int mt = 0; mt < P::NMTL; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * mt + M::row(kqe, r);
        if (i < L) out[(int64_t)(NL * N + i) * lde + K] = o[mt][r];
      }
  }
}

// two waves per SIMD where the tile fits 256 registers without spilling
template <typename T, int D, int DEG>
constexpr int powell_cell_waves_per_eu() {
  return (D == 3 && DEG >= 3) ? 1 : 2;
}

template <typename T, int D, int DEG, int NW, bool PM>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(powell_cell_waves_per_eu<T, D, DEG>())))
    k_cell_mfma_powell(const T* w, const T* w0, T* out, const T* __restrict__ ff, const T* __restrict__ jp,
                       const T* __restrict__ FV, const T* __restrict__ FG, const T* __restrict__ FL,
                       const T* __restrict__ PVt, const T* __restrict__ PGt, const T* __restrict__ PLt,
                       const T* __restrict__ Pmean, const T* __restrict__ Minv, Grid g, const Scal* __restrict__ sc,
                       double gamma, double a0, double b0, double cdt, int mode) {
  const int64_t c0 = ((int64_t)xcd_block(blockIdx.x, gridDim.x) * NW + (threadIdx.x >> 6)) * 16;
  if (c0 >= g.C) return;  // whole wave; no barrier in this kernel
  cell_tile_mfma_powell<T, D, DEG, PM>(c0, threadIdx.x & 63, w, w0, out, ff, jp, FV, FG, FL, PVt, PGt, PLt, Pmean, Minv, g,
                                   sc, gamma, a0, b0, cdt, mode);
}

// Persistent form: one workgroup per CU stages every fragment table in LDS
// (157 KB at 3-D degree 2 FP64) and its waves walk a contiguous, XCD-dealt
// range of 16-cell tiles.  Built where the tables fit the 160 KB of LDS.
template <typename T, int D, int DEG, bool PM = false>
struct PowellLds {
  using S = MfmaShape<D, DEG>;
  using P = PowellShape<D, DEG>;
  static constexpr int SZ_L = PM ? S::SZ_LM : S::SZ_L;    // surface lift tables: moments or points
  static constexpr int SZ_PL = PM ? P::SZ_PLM : P::SZ_PL;
  static constexpr size_t bytes = (size_t)(S::SZ_V + S::SZ_G + SZ_L + P::SZ_PV + P::SZ_PG + SZ_PL) * sizeof(T);
  static constexpr bool fits = bytes <= 160 * 1024;
};

template <typename T, int D, int DEG, int NW, bool PM>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(powell_cell_waves_per_eu<T, D, DEG>())))
    k_cell_mfma_powell_p(const T* w, const T* w0, T* out, const T* __restrict__ ff, const T* __restrict__ jp,
                         const T* __restrict__ FV, const T* __restrict__ FG, const T* __restrict__ FL,
                         const T* __restrict__ PVt, const T* __restrict__ PGt, const T* __restrict__ PLt,
                         const T* __restrict__ Pmean, const T* __restrict__ Minv, Grid g, const Scal* __restrict__ sc,
                         double gamma, double a0, double b0, double cdt, int mode) {
  using PL = PowellLds<T, D, DEG, PM>;
  if constexpr (PL::fits) {
    using S = MfmaShape<D, DEG>;
    using P = PowellShape<D, DEG>;
    __shared__ T sV[S::SZ_V], sG[S::SZ_G], sL[PL::SZ_L], sPV[P::SZ_PV], sPG[P::SZ_PG], sPL[PL::SZ_PL];
    for (int i = threadIdx.x; i < S::SZ_V; i += 64 * NW) sV[i] = FV[i];
    for (int i = threadIdx.x; i < S::SZ_G; i += 64 * NW) sG[i] = FG[i];
    for (int i = threadIdx.x; i < PL::SZ_L; i += 64 * NW) sL[i] = FL[i];
    for (int i = threadIdx.x; i < P::SZ_PV; i += 64 * NW) sPV[i] = PVt[i];
    for (int i = threadIdx.x; i < P::SZ_PG; i += 64 * NW) sPG[i] = PGt[i];
    for (int i = threadIdx.x; i < PL::SZ_PL; i += 64 * NW) sPL[i] = PLt[i];
    __syncthreads();
    const int64_t ntiles = (g.C + 15) / 16;
    const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * per;
    const int64_t t1 = t0 + per < ntiles ? t0 + per : ntiles;
    for (int64_t t = t0 + (threadIdx.x >> 6); t < t1; t += NW) {
      // FP64: the per-mode constants and the lane's row offsets (mode x
      // leading dimension) are formed again for every tile: hoisted out of
      // the walk they would be held in (spilled) registers across all tiles
      const T* pm = Pmean;
      const T* mi = Minv;
      Grid gt = g;
      int ln = threadIdx.x & 63;
      if constexpr (sizeof(T) == 8) asm volatile("" : "+s"(pm), "+s"(mi), "+s"(gt.ld), "+v"(ln));
      cell_tile_mfma_powell<T, D, DEG, PM>(t * 16, ln, w, w0, out, ff, jp, sV, sG, sL, sPV, sPG, sPL, pm, mi, gt, sc, gamma,
                                       a0, b0, cdt, mode);
    }
  }
}

// Face kernel on octree meshes on the matrix cores: one wave per tile of 16
// faces of one class (axis, left sub-face, right sub-face), so that both
// trace tables (the full face or the quarter of the coarse side, Sec. 4.4
// prolongation) are shared by the tile's 16 faces; the traces are 16x16x4
// products with the two cells' modes gathered by face, then each lane solves
// the Riemann problems of its four face points, and the face's flux moments
// (Q^T F on the fine face, as on uniform grids) are stored for the cell
// kernels' lift over moments.
template <int D, int DEG>
struct AmrFaceShape {
  using C = Cfg<D, DEG, GLM>;
  static constexpr int NSUB = 1 + (1 << (D - 1));
  static constexpr int NQ = 1 << (D - 1);
  static constexpr int NCL = 1 + 2 * NQ;
  static constexpr int NKS = (C::N + 3) / 4;
  static constexpr int SZ = D * 2 * NSUB * NKS * 64;
  static constexpr int SZM = SZ + D * 4 * 64;  // and the moment tables Q^T, one per axis
  static constexpr int KSM = (C::FM + 3) / 4;  // k-steps of the surface product over moments
};

// Signed sub-face lift tables of the octree surface product in fragment
// order over face moments: [a][side][class][k-step][mode tile][lane],
// A[i][k] = -+ sum_r w_r phi_n(x_r) Q[a][r][m] for moment m = 4 s + k and
// mode n = 16 mt + i, with r the points of the class's (fine) face (side +a:
// minus, side -a: plus; the coarse side's rows are those of its quarter,
// quarter weights included).  The traces of a coarse cell's basis on a
// quarter are polynomials of the same degree in the fine face's coordinates,
// so its lift rows lie in the span of Q (checked; false otherwise): the
// moment form is exact up to rounding.
template <typename T, int D, int DEG>
bool amr_lift_tables(const Tables& t, const std::vector<double>& qb, std::vector<double>& lt) {
  using C = Cfg<D, DEG, GLM>;
  using S = MfmaShape<D, DEG>;
  constexpr int NSUB = 1 + (1 << (D - 1)), KSM = AmrFaceShape<D, DEG>::KSM, FP = C::FP, FM = C::FM, N = C::N;
  lt.assign((size_t)D * 2 * NSUB * KSM * S::NMT * 64, 0.0);
  for (int a = 0; a < D; ++a)
    for (int sd = 0; sd < 2; ++sd)
      for (int sub = 0; sub < NSUB; ++sub) {
        const double* rows = &t.LFS[(((size_t)a * 2 + sd) * NSUB + sub) * FP * N];  // [r][n]
        double scale = 0.0;
        for (int i = 0; i < FP * N; ++i) scale = std::max(scale, std::fabs(rows[i]));
        std::vector<double> lm((size_t)N * FM, 0.0);  // [n][m]
        for (int n = 0; n < N; ++n)
          for (int m = 0; m < FM; ++m)
            for (int r = 0; r < FP; ++r) lm[(size_t)n * FM + m] += rows[(size_t)r * N + n] * qb[((size_t)a * FP + r) * FM + m];
        for (int n = 0; n < N; ++n)  // the rows must lie in the span of Q
          for (int r = 0; r < FP; ++r) {
            double pr = 0.0;
            for (int m = 0; m < FM; ++m) pr += lm[(size_t)n * FM + m] * qb[((size_t)a * FP + r) * FM + m];
            if (std::fabs(pr - rows[(size_t)r * N + n]) > 1e-13 * scale) return false;
          }
        for (int s = 0; s < KSM; ++s)
          for (int mt = 0; mt < S::NMT; ++mt)
            for (int l = 0; l < 64; ++l) {
              const int m = 4 * s + l / 16, n = 16 * mt + l % 16;
              if (m >= FM || n >= N) continue;
              const double v = lm[(size_t)n * FM + m];
              lt[(((((size_t)a * 2 + sd) * NSUB + sub) * KSM + s) * S::NMT + mt) * 64 + l] = sd ? -v : v;
            }
      }
  return true;
}

template <typename T, int D, int DEG>
void amr_face_tables(const Tables& t, const std::vector<double>& qb, std::vector<double>& ft) {
  using C = Cfg<D, DEG, GLM>;
  using S = AmrFaceShape<D, DEG>;
  ft.assign(S::SZM, 0.0);
  // moment tables as in the uniform face kernel (the fine face's points)
  for (int a = 0; a < D; ++a)
    for (int s = 0; s < 4; ++s)
      for (int l = 0; l < 64; ++l) {
        const int m = l % 16, r = Mfma<T>::row(l / 16, s);
        if (m < C::FM && r < C::FP) ft[S::SZ + (a * 4 + s) * 64 + l] = qb[((size_t)a * C::FP + r) * C::FM + m];
      }
  for (int as = 0; as < D * 2 * S::NSUB; ++as)
    for (int s = 0; s < S::NKS; ++s)
      for (int l = 0; l < 64; ++l) {
        const int r = l % 16, n = 4 * s + l / 16;
        if (r < C::FP && n < C::N) ft[(as * S::NKS + s) * 64 + l] = t.TFS[(as * C::FP + r) * C::N + n];
      }
}

template <typename T, int D, int DEG, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(DEG <= 2 ? 2 : 1)))
    k_face_amr_mfma(const T* __restrict__ w, T* __restrict__ ffa,
                                                           const T* __restrict__ FT, Grid g,
                                                           const Scal* __restrict__ sc, double gamma) {
  using C = Cfg<D, DEG, GLM>;
  using S = AmrFaceShape<D, DEG>;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int N = C::N, FP = C::FP, NV = 9;
  const int64_t tile = (int64_t)blockIdx.x * NW + (threadIdx.x >> 6);
  if (tile >= g.nftile) return;  // whole wave; no barrier in this kernel
  const int lane = threadIdx.x & 63, kq = lane >> 4, cl = lane & 15;
  const int cls = g.ftile[2 * tile], off = g.ftile[2 * tile + 1];
  const int a = cls / S::NCL, k = cls % S::NCL;
  const int subL = k <= S::NQ ? -1 : k - 1 - S::NQ, subR = (k >= 1 && k <= S::NQ) ? k - 1 : -1;
  const int32_t f = g.fperm[off + cl];
  const bool live = f >= 0;
  const int32_t fc = live ? f : g.fperm[off];  // the first entry of a tile is a face
  const int64_t L = g.faceL[fc], R = g.faceR[fc];
  const int64_t ld = g.ld;
  const T* tl = FT + ((a * 2 + 1) * S::NSUB + subL + 1) * S::NKS * 64;
  const T* tr = FT + ((a * 2 + 0) * S::NSUB + subR + 1) * S::NKS * 64;
  v4 UL[NV], UR[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    UL[v] = v4{0, 0, 0, 0};
    UR[v] = v4{0, 0, 0, 0};
  }
  // one side's operands of every k-step are loaded together
  {
    T bk[S::NKS][NV], tk[S::NKS];
#pragma unroll
    for (int s = 0; s < S::NKS; ++s) {
      const int n = 4 * s + kq;
      tk[s] = tl[s * 64 + lane];
#pragma unroll
      for (int v = 0; v < NV; ++v) bk[s][v] = n < N ? w[(int64_t)(v * N + n) * ld + L] : T(0);
    }
#pragma unroll
    for (int s = 0; s < S::NKS; ++s)
#pragma unroll
      for (int v = 0; v < NV; ++v) UL[v] = M::mma(tk[s], bk[s][v], UL[v]);
#pragma unroll
    for (int s = 0; s < S::NKS; ++s) {
      const int n = 4 * s + kq;
      tk[s] = tr[s * 64 + lane];
#pragma unroll
      for (int v = 0; v < NV; ++v) bk[s][v] = n < N ? w[(int64_t)(v * N + n) * ld + R] : T(0);
    }
#pragma unroll
    for (int s = 0; s < S::NKS; ++s)
#pragma unroll
      for (int v = 0; v < NV; ++v) UR[v] = M::mma(tk[s], bk[s][v], UR[v]);
  }
  // every lane stays for the moment product below (its A operand is
  // loaded by all lanes); a padding lane solves its tile's first face
  const T ch = (T)sc->ch;
  T FX[NV][4];
  auto riemann = [&](auto axis) {
    constexpr int A = decltype(axis)::value;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = M::row(kq, j);
      T uL[9], uR[9], Fx[9];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        uL[v] = UL[v][j];
        uR[v] = UR[v][j];
        Fx[v] = T(0);
      }
      if (r < FP) (void)face_flux_a<T, NV, A>(uL, uR, gamma, ch, Fx);
#pragma unroll
      for (int v = 0; v < NV; ++v) FX[v][j] = Fx[v];
    }
  };
  if (a == 0) riemann(std::integral_constant<int, 0>{});
  else if (a == 1) riemann(std::integral_constant<int, 1>{});
  else if constexpr (D == 3) riemann(std::integral_constant<int, 2>{});
  // face moments M = Q^T F (16x16x4 products, the point fluxes as B operands
  // as they lie), rows m < FM stored: [v][m] rows of ldf faces
  T mq[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) mq[s] = FT[S::SZ + (a * 4 + s) * 64 + lane];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    v4 acc = v4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = M::mma(mq[s], FX[v][s], acc);
    if (live) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = M::row(kq, e);
        if (m < C::FM) ffa[((int64_t)v * C::FM + m) * g.ldf + f] = acc[e];
      }
    }
  }
}

// Face kernel on the matrix cores (GLM, uniform grids): one wave owns 16
// faces of one axis; the traces of both sides at the face points are 16x16x4
// products of the trace tables with the two cells' modes (faces as columns),
// and each lane then solves the Riemann problems of its four face points.
template <int D, int DEG>
struct MfmaFaceShape {
  using C = Cfg<D, DEG, GLM>;
  static constexpr int NKS = (C::N + 3) / 4;
  static constexpr int SZ = D * 2 * NKS * 64;
  static constexpr int SZM = SZ + D * 4 * 64;  // and the moment tables, one per axis
  static_assert(C::FP <= 16, "face points per face fit one 16-row tile");
};

// Trace tables (A operands: face points x modes), then per axis the moment
// table Q^T (A operand: moments x points) with its K index in the order of
// the flux accumulator rows, so the point fluxes are its B operands as they lie.
template <typename T, int D, int DEG>
void mfma_face_tables(const Tables& t, const std::vector<double>& qb, std::vector<double>& ft) {
  using C = Cfg<D, DEG, GLM>;
  using S = MfmaFaceShape<D, DEG>;
  ft.assign(S::SZM, 0.0);
  for (int a = 0; a < D; ++a)
    for (int side = 0; side < 2; ++side)
      for (int s = 0; s < S::NKS; ++s)
        for (int l = 0; l < 64; ++l) {
          const int r = l % 16, n = 4 * s + l / 16;
          if (r < C::FP && n < C::N) ft[((a * 2 + side) * S::NKS + s) * 64 + l] = t.TF[((a * 2 + side) * C::FP + r) * C::N + n];
        }
  for (int a = 0; a < D; ++a)
    for (int s = 0; s < 4; ++s)
      for (int l = 0; l < 64; ++l) {
        const int m = l % 16, r = Mfma<T>::row(l / 16, s);
        if (m < C::FM && r < C::FP) ft[S::SZ + (a * 4 + s) * 64 + l] = qb[((size_t)a * C::FP + r) * C::FM + m];
      }
}

// Face moments of one wave's 16 faces along axis A from the point fluxes FX
// (accumulator layout: element j of lane l is point row(l/16, j) of face
// l % 16): 16x16x4 products with the moment table; rows < FM stored.
// fx(v, j): the flux of variable v at the lane's point j (ROLL: one variable
// at a time, for fluxes held in LDS).
template <typename T, int D, int DEG, int A, bool ROLL = false, typename FX>
__device__ __forceinline__ void store_face_moments(FX&& fx, const T* __restrict__ FT, T* __restrict__ ff,
                                                   int lane, int64_t F, bool live, int64_t ld) {
  using C = Cfg<D, DEG, GLM>;
  using S = MfmaFaceShape<D, DEG>;
  using M = Mfma<T>;
  using V4 = typename M::v4;
  constexpr int NV = 9, FM = C::FM;
  constexpr int FMS = MfmaShape<D, DEG>::template fms<T>();
  T mt[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) mt[s] = FT[S::SZ + (A * 4 + s) * 64 + lane];
  const int kq = lane >> 4;
#pragma unroll(ROLL ? 1 : NV)
  for (int v = 0; v < NV; ++v) {
    V4 acc = V4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = M::mma(mt[s], fx(v, s), acc);
    if (live) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = M::row(kq, e);
        if (m < FM) ff[((int64_t)(A * NV + v) * FMS + m) * ld + F] = acc[e];
      }
    }
  }
}

// FP32 deviation form of the face kernels (see cell_tile_mfma): the traces
// are FP32 products of the modes above the mean, the Riemann problem is
// solved in FP64 on mean + deviation, and the stored point fluxes are
// F* - c with c the FP32 flux of the left cell's mean (written to the extra
// row of the moment buffer for both cells to use).
template <int NV>
struct FaceDev {
  double ubL[NV], ubR[NV], cL[NV];
  template <int A, int NVS, int FMS, int FM>
  __device__ __forceinline__ void init(const float* __restrict__ w, int N, int64_t ld, int64_t FL, int64_t FR,
                                       double gamma, double ch, float* __restrict__ ff, int64_t F, bool store) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ubL[v] = (double)w[(int64_t)(v * N) * ld + FL];
      ubR[v] = (double)w[(int64_t)(v * N) * ld + FR];
    }
    double fl[NV], fr[NV];
    mhd_flux<double, NV>(ubL, A, gamma, ch * ch, fl);
    mhd_flux<double, NV>(ubR, A, gamma, ch * ch, fr);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      cL[v] = (double)(float)fl[v];
      if (store) {
        ff[((int64_t)(A * NVS + v) * FMS + FM) * ld + F] = (float)(cL[v] - fl[v]);
        ff[((int64_t)(A * NVS + v) * FMS + FM + 1) * ld + F] = (float)(cL[v] - fr[v]);
      }
    }
  }
  template <int A>
  __device__ __forceinline__ void flux(const float* dL, const float* dR, double gamma, double ch, float* Fx) const {
    double uL[NV], uR[NV], F[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uL[v] = ubL[v] + (double)dL[v];
      uR[v] = ubR[v] + (double)dR[v];
    }
    (void)face_flux_a<double, NV, A>(uL, uR, gamma, ch, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) Fx[v] = (float)(F[v] - cL[v]);
  }
};

template <typename T, int D, int DEG, int NW>
__global__ void __launch_bounds__(64 * NW) k_face_mfma(const T* __restrict__ w, T* __restrict__ ff,
                                                       const T* __restrict__ FT, Grid g,
                                                       const Scal* __restrict__ sc, double gamma) {
  using C = Cfg<D, DEG, GLM>;
  using S = MfmaFaceShape<D, DEG>;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int N = C::N, FP = C::FP, NV = 9;
  // this wave's (tile, axis) pair: the D axes of a tile are consecutive, so
  // one XCD reads a cell's modes for all its + faces while they are in its L2
  const int64_t pw = (int64_t)xcd_block(blockIdx.x, gridDim.x) * NW + (threadIdx.x >> 6);
  const int a = (int)(pw % D);
  const int lane = threadIdx.x & 63;
  const int64_t f0 = (pw / D) * 16;
  if (f0 >= g.C) return;  // whole wave; no barrier in this kernel
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t F = f0 + cl;
  const bool live = F < g.C;
  const int64_t FL = live ? F : f0;           // face F lies between cells F (left) and its +a neighbour
  const int64_t FR = nbr(FL, a, +1, g);
  const int64_t ld = g.ld;
  v4 UL[NV], UR[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    UL[v] = v4{0, 0, 0, 0};
    UR[v] = v4{0, 0, 0, 0};
  }
  constexpr bool DEV = sizeof(T) == 4;
  constexpr int FMS = MfmaShape<D, DEG>::template fms<T>();
  // the left cell's operands of every k-step are loaded together, then the
  // right cell's are loaded while the left traces are multiplied
  {
    T bk[S::NKS][NV], tk[S::NKS];
#pragma unroll
    for (int s = 0; s < S::NKS; ++s) {
      const int n = 4 * s + kq;
      tk[s] = FT[((a * 2 + 1) * S::NKS + s) * 64 + lane];
#pragma unroll
      for (int v = 0; v < NV; ++v) bk[s][v] = (n < N && !(DEV && n == 0)) ? w[(int64_t)(v * N + n) * ld + FL] : T(0);
    }
#pragma unroll
    for (int s = 0; s < S::NKS; ++s)
#pragma unroll
      for (int v = 0; v < NV; ++v) UL[v] = M::mma(tk[s], bk[s][v], UL[v]);
#pragma unroll
    for (int s = 0; s < S::NKS; ++s) {
      const int n = 4 * s + kq;
      tk[s] = FT[((a * 2 + 0) * S::NKS + s) * 64 + lane];
#pragma unroll
      for (int v = 0; v < NV; ++v) bk[s][v] = (n < N && !(DEV && n == 0)) ? w[(int64_t)(v * N + n) * ld + FR] : T(0);
    }
#pragma unroll
    for (int s = 0; s < S::NKS; ++s)
#pragma unroll
      for (int v = 0; v < NV; ++v) UR[v] = M::mma(tk[s], bk[s][v], UR[v]);
  }
  const T ch = (T)sc->ch;
  // the axis is uniform over the wave: one branch per axis keeps every
  // component index of the Riemann solver a compile-time constant.  Every
  // lane stays for the moment products (dead lanes and padding rows carry
  // zero fluxes).
  auto riemann = [&](auto axis) {
    constexpr int A = decltype(axis)::value;
    FaceDev<NV> dv;
    if constexpr (DEV)
      dv.template init<A, NV, FMS, C::FM>((const float*)w, N, ld, FL, FR, gamma, sc->ch, (float*)ff, F,
                                          live && kq == 0);
    v4 FX[NV];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = M::row(kq, j);
      T Fx[9];
      if (live && r < FP) {
        T uL[9], uR[9];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          uL[v] = UL[v][j];
          uR[v] = UR[v][j];
        }
        if constexpr (DEV) dv.template flux<A>((const float*)uL, (const float*)uR, gamma, sc->ch, (float*)Fx);
        else (void)face_flux_a<T, NV, A>(uL, uR, gamma, ch, Fx);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx[v] = T(0);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) FX[v][j] = Fx[v];
    }
    store_face_moments<T, D, DEG, A>([&](int v, int j) { return FX[v][j]; }, FT, ff, lane, F, live, ld);
  };
  if (a == 0) riemann(std::integral_constant<int, 0>{});
  else if (a == 1) riemann(std::integral_constant<int, 1>{});
  else if constexpr (D == 3) riemann(std::integral_constant<int, 2>{});
}

// Matrix-core face kernel of the Powell scheme (uniform grids): one wave per
// (tile of 16 faces, axis); the Legendre traces are 16x16x4 products of the
// trace tables with the two cells' modes, the LDF field's traces products of
// the per-component LDF trace tables with the LDF weights; each lane then
// solves the Riemann problems of its four face points and writes the point
// fluxes and the normal-field jumps (or, with the interpolated q-dagger, both
// sides' face values) in the layout of k_face.
template <int D, int DEG>
struct PowellFaceShape {
  using C = Cfg<D, DEG, POWELL>;
  static constexpr int NKS = (C::N + 3) / 4;
  static constexpr int NKL = (C::NLDF + 3) / 4;
  static constexpr int SZL = D * 2 * NKS * 64;          // Legendre traces [a][side][s][lane]
  static constexpr int SZ = SZL + D * 2 * D * NKL * 64;  // then the LDF traces [a][side][c][s][lane]
  static constexpr int SZM = SZ + (D == 3 ? D * 4 * 64 : 0);  // then (3-D) the moment tables Q^T per axis
  static_assert(C::FP <= 16, "face points per face fit one 16-row tile");
};

template <typename T, int D, int DEG>
void powell_face_tables(const Tables& t, const std::vector<double>& qb, std::vector<double>& ft) {
  using C = Cfg<D, DEG, POWELL>;
  using S = PowellFaceShape<D, DEG>;
  ft.assign(S::SZM, 0.0);
  if constexpr (D == 3)  // moment tables as in the GLM face kernel
    for (int a = 0; a < D; ++a)
      for (int s = 0; s < 4; ++s)
        for (int l = 0; l < 64; ++l) {
          const int m = l % 16, r = Mfma<T>::row(l / 16, s);
          if (m < C::FM && r < C::FP) ft[S::SZ + (a * 4 + s) * 64 + l] = qb[((size_t)a * C::FP + r) * C::FM + m];
        }
  for (int a = 0; a < D; ++a)
    for (int side = 0; side < 2; ++side) {
      for (int s = 0; s < S::NKS; ++s)
        for (int l = 0; l < 64; ++l) {
          const int r = l % 16, n = 4 * s + l / 16;
          if (r < C::FP && n < C::N) ft[((a * 2 + side) * S::NKS + s) * 64 + l] = t.TF[((a * 2 + side) * C::FP + r) * C::N + n];
        }
      for (int c = 0; c < D; ++c)
        for (int s = 0; s < S::NKL; ++s)
          for (int l = 0; l < 64; ++l) {
            const int r = l % 16, i = 4 * s + l / 16;
            if (r < C::FP && i < C::NLDF)
              ft[S::SZL + (((a * 2 + side) * D + c) * S::NKL + s) * 64 + l] =
                  t.PTF[(((a * 2 + side) * D + c) * C::FP + r) * C::NLDF + i];
          }
    }
}

template <typename T, int D, int DEG, int NW, bool QINT>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(D == 3 && DEG >= 3 ? 1 : 2)))
    k_face_mfma_powell(const T* __restrict__ w, T* __restrict__ ff, T* __restrict__ jp, const T* __restrict__ FT,
                       Grid g, const Scal* __restrict__ sc, double gamma, int cap) {
  using C = Cfg<D, DEG, POWELL>;
  using S = PowellFaceShape<D, DEG>;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int N = C::N, FP = C::FP, NV = 8, NL = C::NLEG, L = C::NLDF;
  const int64_t pw = (int64_t)xcd_block(blockIdx.x, gridDim.x) * NW + (threadIdx.x >> 6);
  const int a = (int)(pw % D);
  const int lane = threadIdx.x & 63;
  const int64_t f0 = (pw / D) * 16;
  if (f0 >= g.C) return;  // whole wave; no barrier in this kernel
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t F = f0 + cl;
  const bool live = F < g.C;
  const int64_t FL = live ? F : f0;  // face F lies between cells F (left) and its +a neighbour
  const int64_t FR = nbr(FL, a, +1, g);
  const int64_t ld = g.ld;
  v4 UL[NV], UR[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    UL[v] = v4{0, 0, 0, 0};
    UR[v] = v4{0, 0, 0, 0};
  }
  auto traces = [&](v4 (&U)[NV], int64_t K, int side) {
#pragma unroll
    for (int s = 0; s < S::NKS; ++s) {
      const int n = 4 * s + kq;
      const T tk = FT[((a * 2 + side) * S::NKS + s) * 64 + lane];
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        const T b = n < N ? w[(int64_t)(j * N + n) * ld + K] : T(0);
        U[C::legvar(j)] = M::mma(tk, b, U[C::legvar(j)]);
      }
    }
#pragma unroll
    for (int s = 0; s < S::NKL; ++s) {
      const int i = 4 * s + kq;
      const T b = i < L ? w[(int64_t)(NL * N + i) * ld + K] : T(0);
#pragma unroll
      for (int c = 0; c < D; ++c)
        U[5 + c] = M::mma(FT[S::SZL + (((a * 2 + side) * D + c) * S::NKL + s) * 64 + lane], b, U[5 + c]);
    }
  };
  traces(UL, FL, 1);
  traces(UR, FR, 0);
  // 3-D with the cell-mean q-dagger: the point fluxes and the two sides'
  // jumps wait in LDS (lane-private slots) for the moment product; every
  // lane stays (the product's A operand is loaded by all lanes)
  constexpr bool MOM = D == 3 && !QINT;
  constexpr int NVM = MOM ? NV + 2 : 1;
  __shared__ T sU[MOM ? NW : 1][NVM * 4 * 64];
  T* const su = sU[MOM ? (threadIdx.x >> 6) : 0];
  if (!MOM && !live) return;
  const T ch = (T)sc->ch;
  auto riemann = [&](auto axis) {
    constexpr int A = decltype(axis)::value;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = M::row(kq, j);
      if constexpr (MOM) {
        if (r >= FP) {
#pragma unroll
          for (int v = 0; v < NV + 2; ++v) su[(v * 4 + j) * 64 + lane] = T(0);
          continue;
        }
      } else {
        if (r >= FP) continue;
      }
      T uL[9], uR[9], Fx[9];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        uL[v] = UL[v][j];
        uR[v] = UR[v][j];
      }
      if constexpr (QINT) {
        // interpolated q-dagger (eq. powellq-interp): each side's Powell term
        // with the HLLD interface state, left values to ff, right to jp
        T vf[3], bf[3], ql[8], qr[8];
        const T bnF = face_flux_a<T, NV, A>(uL, uR, gamma, ch, Fx, vf, bf);
        powell_q_interp<T>(uL, vf, bf, ql);
        powell_q_interp<T>(uR, vf, bf, qr);
        const T jl = bnF - uL[5 + A], jr = uR[5 + A] - bnF;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          ff[((int64_t)(A * NV + v) * FP + r) * ld + F] = Fx[v] + ql[v] * jl;
          jp[((int64_t)(A * NV + v) * FP + r) * ld + F] = Fx[v] - qr[v] * jr;
        }
      } else {
        const T bnF = face_flux_a<T, NV, A>(uL, uR, gamma, ch, Fx);
        const T jl = bnF - uL[5 + A], jr = uR[5 + A] - bnF;
        if (live && (cap || !MOM)) {  // the jump points feed the time step's Powell cap
          jp[((int64_t)(A * 2 + 0) * FP + r) * ld + F] = jl;
          jp[((int64_t)(A * 2 + 1) * FP + r) * ld + F] = jr;
        }
        if constexpr (MOM) {
#pragma unroll
          for (int v = 0; v < NV; ++v) su[(v * 4 + j) * 64 + lane] = Fx[v];
          su[(NV * 4 + j) * 64 + lane] = jl;
          su[((NV + 1) * 4 + j) * 64 + lane] = jr;
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) ff[((int64_t)(A * NV + v) * FP + r) * ld + F] = Fx[v];
        }
      }
    }
  };
  if (a == 0) riemann(std::integral_constant<int, 0>{});
  else if (a == 1) riemann(std::integral_constant<int, 1>{});
  else if constexpr (D == 3) riemann(std::integral_constant<int, 2>{});
  if constexpr (MOM) {
    // moments Q^T of the fluxes (rows a NV FP + v FM + m) and of the jumps
    // (rows a NV FP + 8 FM + side FM + m): 16x16x4 products with the point
    // values as B operands as they lie in the accumulator rows
    constexpr int FM = C::FM;
    T mq[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) mq[s] = FT[S::SZ + (a * 4 + s) * 64 + lane];
    const int64_t base = (int64_t)a * NV * FP;
#pragma unroll 1
    for (int v = 0; v < NV + 2; ++v) {
      v4 acc = v4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = M::mma(mq[s], su[(v * 4 + s) * 64 + lane], acc);
      if (live) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int m = M::row(kq, e);
          if (m < FM) ff[(base + v * FM + m) * ld + F] = acc[e];
        }
      }
    }
  }
}

// Low-register form of the matrix-core face kernel: the operands are loaded
// one k-step at a time, the right traces wait in LDS, and each lane solves its
// four face points one after another, so that two waves fit on a SIMD and one
// wave's loads run under the other's Riemann solves.
template <typename T, int D, int DEG, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_face_mfma_lr(const T* __restrict__ w, T* __restrict__ ff, const T* __restrict__ FT, Grid g,
               const Scal* __restrict__ sc, double gamma) {
  using C = Cfg<D, DEG, GLM>;
  using S = MfmaFaceShape<D, DEG>;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int N = C::N, FP = C::FP, NV = 9;
  // this wave's (tile, axis) pair: the D axes of a tile are consecutive, so
  // one XCD reads a cell's modes for all its + faces while they are in its L2
  const int64_t pw = (int64_t)xcd_block(blockIdx.x, gridDim.x) * NW + (threadIdx.x >> 6);
  const int a = (int)(pw % D);
  const int lane = threadIdx.x & 63;
  const int64_t f0 = (pw / D) * 16;
  if (f0 >= g.C) return;  // whole wave; no barrier in this kernel
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t F = f0 + cl;
  const bool live = F < g.C;
  const int64_t FL = live ? F : f0;
  const int64_t FR = nbr(FL, a, +1, g);
  const int64_t ld = g.ld;
  constexpr bool DEV = sizeof(T) == 4;
  constexpr int FMS = MfmaShape<D, DEG>::template fms<T>();
  __shared__ T sU[NW][NV * 4 * 64];
  T* const su = sU[threadIdx.x >> 6];
  v4 UL[NV], UR[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    UL[v] = v4{0, 0, 0, 0};
    UR[v] = v4{0, 0, 0, 0};
  }
#pragma unroll
  for (int s = 0; s < S::NKS; ++s) {
    const int n = 4 * s + kq;
    const T tl = FT[((a * 2 + 1) * S::NKS + s) * 64 + lane];
    const T tr = FT[((a * 2 + 0) * S::NKS + s) * 64 + lane];
    T bl[NV], br[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      bl[v] = (n < N && !(DEV && n == 0)) ? w[(int64_t)(v * N + n) * ld + FL] : T(0);
      br[v] = (n < N && !(DEV && n == 0)) ? w[(int64_t)(v * N + n) * ld + FR] : T(0);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      UL[v] = M::mma(tl, bl[v], UL[v]);
      UR[v] = M::mma(tr, br[v], UR[v]);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int j = 0; j < 4; ++j) su[(v * 4 + j) * 64 + lane] = UR[v][j];
  // each lane reads and writes only its own LDS slots: no barrier
  const T ch = (T)sc->ch;
  auto riemann = [&](auto axis) __attribute__((always_inline)) {
    constexpr int A = decltype(axis)::value;
    FaceDev<NV> dv;
    if constexpr (DEV)
      dv.template init<A, NV, FMS, C::FM>((const float*)w, N, ld, FL, FR, gamma, sc->ch, (float*)ff, F,
                                          live && kq == 0);
    // the point fluxes replace the right traces in LDS, slot by slot
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
      const int r = M::row(kq, j);
      T Fx[9];
      if (live && r < FP) {
        T uL[9], uR[9];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          uL[v] = j == 0 ? UL[v][0] : j == 1 ? UL[v][1] : j == 2 ? UL[v][2] : UL[v][3];
          uR[v] = su[(v * 4 + j) * 64 + lane];
        }
        if constexpr (DEV) dv.template flux<A>((const float*)uL, (const float*)uR, gamma, sc->ch, (float*)Fx);
        else (void)face_flux_a<T, NV, A>(uL, uR, gamma, ch, Fx);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx[v] = T(0);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) su[(v * 4 + j) * 64 + lane] = Fx[v];
    }
    store_face_moments<T, D, DEG, A, true>([&](int v, int j) { return su[(v * 4 + j) * 64 + lane]; }, FT, ff, lane,
                                           F, live, ld);
  };
  if (a == 0) riemann(std::integral_constant<int, 0>{});
  else if (a == 1) riemann(std::integral_constant<int, 1>{});
  else if constexpr (D == 3) riemann(std::integral_constant<int, 2>{});
}

// Max signal speed on the matrix cores (GLM, uniform and octree grids): one
// wave evaluates 16 cells at every volume point (row tiles of the nodal
// table) and face point (row tiles of the trace tables) with 16x16x4
// products in the state's precision, the modes held in registers; wave and
// block maxima (NaN-propagating) of the speed and of the speed over the
// cell's size feed one atomic each per block.
template <typename T, int D, int DEG, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2, 2))) k_maxsig_mfma(const T* __restrict__ w, const T* __restrict__ FV,
                                                         const T* __restrict__ FT, Grid g, Scal* sc, double gamma) {
  using C = Cfg<D, DEG, GLM>;
  using S = MfmaShape<D, DEG>;
  using SF = MfmaFaceShape<D, DEG>;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int N = C::N;
  static_assert(SF::NKS == S::NKS, "same k-steps for the volume and face evaluation tables");
  // evaluation rows: the volume row tiles, then the trace rows of each face
  __shared__ T sT[(S::QT + 2 * D) * S::NKS * 64];
  __shared__ double red[NW], red2[NW];
  for (int i = threadIdx.x; i < S::SZ_V; i += 64 * NW) sT[i] = FV[i];
  for (int i = threadIdx.x; i < 2 * D * S::NKS * 64; i += 64 * NW) sT[S::SZ_V + i] = FT[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t ntiles = (g.C + 15) / 16;
  const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int64_t t0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * per;
  const int64_t t1 = t0 + per < ntiles ? t0 + per : ntiles;
  double smax = 0.0, rmax = 0.0;
  for (int64_t t = t0 + wid; t < t1; t += NW) {
    const int64_t c0 = t * 16;
    const int64_t K = c0 + cl;
    const bool live = K < g.C;
    const int64_t Kc = live ? K : c0;
    const double ih = 1.0 / cell_h(g, Kc);
    T bw[8][S::NKS];
#pragma unroll
    for (int v = 0; v < 8; ++v)
#pragma unroll
      for (int s = 0; s < S::NKS; ++s) {
        const int n = 4 * s + kq;
        bw[v][s] = n < N ? w[(int64_t)(v * N + n) * g.ld + Kc] : T(0);
      }
#pragma unroll 1
    for (int rt = 0; rt < S::QT + 2 * D; ++rt) {
      v4 U[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) U[v] = v4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < S::NKS; ++s) {
        const T a = sT[(rt * S::NKS + s) * 64 + lane];
#pragma unroll
        for (int v = 0; v < 8; ++v) U[v] = M::mma(a, bw[v][s], U[v]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = M::row(kq, j);
        const bool valid = live && (rt < S::QT ? (16 * rt + i < C::Q) : (i < C::FP));
        if (!valid) continue;
        T u[9];
#pragma unroll
        for (int v = 0; v < 8; ++v) u[v] = U[v][j];
        u[8] = T(0);
        double sp = signal_sum<T, D>(u, gamma);
        if (!(sp == sp)) sp = __longlong_as_double(0x7ff8000000000000ULL);
        smax = (sp > smax || !(sp == sp)) ? sp : smax;
        const double rt = sp * ih;
        rmax = (rt > rmax || !(rt == rt)) ? rt : rmax;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double x = __shfl_xor(smax, o);
    smax = (x > smax || !(x == x)) ? x : smax;
    const double y = __shfl_xor(rmax, o);
    rmax = (y > rmax || !(y == y)) ? y : rmax;
  }
  if (lane == 0) {
    red[wid] = smax;
    red2[wid] = rmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0], r = red2[0];
    for (int i = 1; i < NW; ++i) {
      m = (red[i] > m || !(red[i] == red[i])) ? red[i] : m;
      r = (red2[i] > r || !(red2[i] == red2[i])) ? red2[i] : r;
    }
    atomic_max_pos(&sc->maxsig_bits, m);
    atomic_max_pos(&sc->maxrate_bits, r);
    if (!(m == m)) atomicAdd(&sc->nonfinite, 1ULL);
  }
}

// Max signal speed on the matrix cores, Powell scheme (uniform grids): one
// wave per 16 cells; the Legendre variables at every volume and face point
// are products of the nodal and trace tables with the cell's modes, the
// field's components products of the LDF tables (PV at volume points, the
// LDF trace tables at face points) with its LDF weights; maxima as in
// k_maxsig_mfma.  Persistent: where the tables fit, each workgroup stages
// them in LDS once and its waves walk a contiguous, XCD-dealt range of
// tiles; otherwise they are read through the L1.
template <typename T, int D, int DEG>
struct PowellSigLds {
  static constexpr int SZ_V = MfmaShape<D, DEG>::SZ_V;
  static constexpr int SZ_PV = PowellShape<D, DEG>::SZ_PV;
  static constexpr int SZ_F = PowellFaceShape<D, DEG>::SZ;
  static constexpr bool fits = (size_t)(SZ_V + SZ_PV + SZ_F) * sizeof(T) <= 128 * 1024;
};

template <typename T, int D, int DEG, int NW>
__device__ __forceinline__ void maxsig_powell_walk(const T* __restrict__ w, const T* FV, const T* PVt, const T* PFT,
                                                   const Grid& g, double gamma, double& smax, double& rmax) {
  using C = Cfg<D, DEG, POWELL>;
  using S = MfmaShape<D, DEG>;
  using P = PowellShape<D, DEG>;
  using F = PowellFaceShape<D, DEG>;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int N = C::N, NL = C::NLEG, L = C::NLDF;
  static_assert(S::NKS == F::NKS && P::NKL == F::NKL, "same k-steps for the volume and face tables");
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t ntiles = (g.C + 15) / 16;
  const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int64_t t0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * per;
  const int64_t t1 = t0 + per < ntiles ? t0 + per : ntiles;
  for (int64_t tt = t0 + wid; tt < t1; tt += NW) {
    const int64_t c0 = tt * 16;
    const int64_t K = c0 + cl;
    const bool live = K < g.C;
    const int64_t Kc = live ? K : c0;
    const double ih = 1.0 / cell_h(g, Kc);
    T bw[NL][S::NKS], bl[P::NKL];
#pragma unroll
    for (int j = 0; j < NL; ++j)
#pragma unroll
      for (int s = 0; s < S::NKS; ++s) {
        const int n = 4 * s + kq;
        bw[j][s] = n < N ? w[(int64_t)(j * N + n) * g.ld + Kc] : T(0);
      }
#pragma unroll
    for (int s = 0; s < P::NKL; ++s) {
      const int i = 4 * s + kq;
      bl[s] = i < L ? w[(int64_t)(NL * N + i) * g.ld + Kc] : T(0);
    }
#pragma unroll 1
    for (int rt = 0; rt < S::QT + 2 * D; ++rt) {
      const bool vol = rt < S::QT;
      const int as = rt - S::QT;  // face (a, side) = as
      v4 U[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) U[v] = v4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < S::NKS; ++s) {
        const T a = vol ? FV[(rt * S::NKS + s) * 64 + lane] : PFT[(as * F::NKS + s) * 64 + lane];
#pragma unroll
        for (int j = 0; j < NL; ++j) U[C::legvar(j)] = M::mma(a, bw[j][s], U[C::legvar(j)]);
      }
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int s = 0; s < P::NKL; ++s) {
          const T a = vol ? PVt[((c * S::QT + rt) * P::NKL + s) * 64 + lane]
                          : PFT[F::SZL + ((as * D + c) * F::NKL + s) * 64 + lane];
          U[5 + c] = M::mma(a, bl[s], U[5 + c]);
        }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = M::row(kq, j);
        const bool valid = live && (vol ? (16 * rt + i < C::Q) : (i < C::FP));
        if (!valid) continue;
        T u[9];
#pragma unroll
        for (int v = 0; v < 8; ++v) u[v] = U[v][j];
        u[8] = T(0);
        double sp = signal_sum<T, D>(u, gamma);
        if (!(sp == sp)) sp = __longlong_as_double(0x7ff8000000000000ULL);
        smax = (sp > smax || !(sp == sp)) ? sp : smax;
        const double rr = sp * ih;
        rmax = (rr > rmax || !(rr == rr)) ? rr : rmax;
      }
    }
  }
}

template <typename T, int D, int DEG, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2)))
    k_maxsig_mfma_powell(const T* __restrict__ w, const T* __restrict__ FV, const T* __restrict__ PVt,
                         const T* __restrict__ PFT, Grid g, Scal* sc, double gamma) {
  using SL = PowellSigLds<T, D, DEG>;
  __shared__ double red[NW], red2[NW];
  double smax = 0.0, rmax = 0.0;
  if constexpr (SL::fits) {
    __shared__ T sT[SL::SZ_V + SL::SZ_PV + SL::SZ_F];
    for (int i = threadIdx.x; i < SL::SZ_V; i += 64 * NW) sT[i] = FV[i];
    for (int i = threadIdx.x; i < SL::SZ_PV; i += 64 * NW) sT[SL::SZ_V + i] = PVt[i];
    for (int i = threadIdx.x; i < SL::SZ_F; i += 64 * NW) sT[SL::SZ_V + SL::SZ_PV + i] = PFT[i];
    __syncthreads();
    maxsig_powell_walk<T, D, DEG, NW>(w, sT, sT + SL::SZ_V, sT + SL::SZ_V + SL::SZ_PV, g, gamma, smax, rmax);
  } else {
    maxsig_powell_walk<T, D, DEG, NW>(w, FV, PVt, PFT, g, gamma, smax, rmax);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double x = __shfl_xor(smax, o);
    smax = (x > smax || !(x == x)) ? x : smax;
    const double y = __shfl_xor(rmax, o);
    rmax = (y > rmax || !(y == y)) ? y : rmax;
  }
  if (lane == 0) {
    red[wid] = smax;
    red2[wid] = rmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0], r = red2[0];
    for (int i = 1; i < NW; ++i) {
      m = (red[i] > m || !(red[i] == red[i])) ? red[i] : m;
      r = (red2[i] > r || !(red2[i] == red2[i])) ? red2[i] : r;
    }
    atomic_max_pos(&sc->maxsig_bits, m);
    atomic_max_pos(&sc->maxrate_bits, r);
    if (!(m == m)) atomicAdd(&sc->nonfinite, 1ULL);
  }
}

// tile-shape variants of the cell kernel offered to the autotuner
template <typename T, int D, int DEG, int DIVB>
struct CellVariants {
  static constexpr int count = 4;
  static constexpr int tc(int i) { return i == 0 ? 16 : i == 1 ? 32 : i == 2 ? 32 : 64; }
  static constexpr int nt(int i) { return i == 0 ? 256 : i == 1 ? 256 : i == 2 ? 512 : 512; }
};

// Time step, c_h and kappa from the reductions (eq. cfl, the GLM rules,
// the Powell cap): s = max signal speed, rate = max speed over cell size,
// pr = Powell rate.
static __device__ __forceinline__ void finalize_dt_dev(Scal* sc, const SchemeParams& sp, int D, int d, int divb,
                                                       double hmin, double s, double rate, double pr) {
  double dt = sp.cfl / (2 * d + 1) / rate;
  double ch = 0.0, kappa = 0.0;
  if (!(s == s) || !(rate > 0.0)) sc->nonfinite += 1ULL;
  if (divb == GLM) {
    if (sp.glm_ch_fixed > 0.0) {
      ch = sp.glm_ch_fixed;
      const double cap = sp.cfl_glm * hmin / ((2 * d + 1) * D * ch);
      dt = fmin(dt, cap);
      if (ch < 2.0 * s / D) sc->n_ch_violation += 1ULL;
    } else {
      ch = (sp.cfl_glm / sp.cfl) * s / D;
    }
    kappa = fmin(ch / sp.glm_cr, 1.0 / (3.0 * dt));
  } else {
    if (pr > 0.0) dt = fmin(dt, sp.powell_eta / pr);
  }
  sc->dt = dt;
  sc->ch = ch;
  sc->kappa = kappa;
  sc->t += dt;
  sc->last_maxsig = s / D;
}

// ---------------------------------------------------------------------------
// max signal speed over volume and face points (eq. cfl; reading: max over
// the cell's quadrature points)

template <typename T, int D, int DEG, int DIVB>
__device__ __forceinline__ void eval_point(const T* sw, int TC, int c, const T* vl, const T* pv, int pvs, T* u) {
  using C = Cfg<D, DEG, DIVB>;
#pragma unroll
  for (int j = 0; j < C::NLEG; ++j) {
    T s = 0;
#pragma unroll
    for (int l = 0; l < C::N; ++l) s += vl[l] * sw[(j * C::N + l) * TC + c];
    u[C::legvar(j)] = s;
  }
  if constexpr (C::NLDF > 0) {
    for (int cc = 0; cc < D; ++cc) {
      T s = 0;
      for (int l = 0; l < C::NLDF; ++l) s += pv[cc * pvs + l] * sw[(C::NLEG * C::N + l) * TC + c];
      u[5 + cc] = s;
    }
  }
}

template <typename T, int D, int DEG, int DIVB>
__global__ void __launch_bounds__(256) k_maxsig(const T* __restrict__ w, DevTab<T> tb, Grid g, Scal* sc,
                                                double gamma, SchemeParams sp, DtFinalize fin, int finalize) {
  using C = Cfg<D, DEG, DIVB>;
  constexpr int TC = Tile<T, D, DEG, DIVB>::TC;
  constexpr int NPT = C::Q + 2 * D * C::FP;
  __shared__ T sw[C::NMODES * TC];
  __shared__ double red[256], red2[256];
  const int64_t c0 = (int64_t)blockIdx.x * TC;
  const int tid = threadIdx.x;
  for (int i = tid; i < C::NMODES * TC; i += 256) {
    const int m = i / TC, c = i % TC;
    const int64_t K = c0 + c;
    sw[i] = K < g.C ? w[(int64_t)m * g.ld + K] : safe_mode_value<T, D, DEG, DIVB>(m);
  }
  __syncthreads();
  double smax = 0.0, rmax = 0.0;
  for (int i = tid; i < NPT * TC; i += 256) {
    const int c = i % TC, p = i / TC;
    if (c0 + c >= g.C) continue;
    const double ih = 1.0 / cell_h(g, c0 + c);
    T u[9];
    if (p < C::Q) {
      eval_point<T, D, DEG, DIVB>(sw, TC, c, tb.V + p * C::N, C::NLDF ? tb.PV + p * C::NLDF : nullptr,
                                  C::Q * C::NLDF, u);
    } else {
      const int fpi = p - C::Q;  // (a*2+s)*FP + r
      const int as = fpi / C::FP, r = fpi % C::FP;
      eval_point<T, D, DEG, DIVB>(sw, TC, c, tb.TF + fpi * C::N,
                                  C::NLDF ? tb.PTF + ((as * D) * C::FP + r) * C::NLDF : nullptr, C::FP * C::NLDF, u);
    }
    double s = signal_sum<T, D>(u, gamma);
    if (!(s == s)) s = __longlong_as_double(0x7ff8000000000000ULL);
    smax = (s > smax || !(s == s)) ? s : smax;
    const double rt = s * ih;
    rmax = (rt > rmax || !(rt == rt)) ? rt : rmax;
  }
  red[tid] = smax;
  red2[tid] = rmax;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      double o = red[tid + st];
      if (o > red[tid] || !(o == o)) red[tid] = o;
      o = red2[tid + st];
      if (o > red2[tid] || !(o == o)) red2[tid] = o;
    }
    __syncthreads();
  }
  if (tid == 0) {
    atomic_max_pos(&sc->maxsig_bits, red[0]);
    atomic_max_pos(&sc->maxrate_bits, red2[0]);
    if (!(red[0] == red[0])) atomicAdd(&sc->nonfinite, 1ULL);
    if (finalize) {
      // the last workgroup to finish reads the maxima, finalises the step
      // and clears them for the next reduction (two launches fewer per step
      // where launches dominate: small grids)
      __threadfence();
      if (atomicAdd(&sc->blocks_done, 1u) == gridDim.x - 1) {
        __threadfence();
        const double s = __longlong_as_double((long long)atomicAdd(&sc->maxsig_bits, 0ULL));
        const double rate = __longlong_as_double((long long)atomicAdd(&sc->maxrate_bits, 0ULL));
        finalize_dt_dev(sc, sp, fin.D, fin.d, fin.divb, fin.hmin, s, rate, 0.0);
        atomicExch(&sc->maxsig_bits, 0ULL);
        atomicExch(&sc->maxrate_bits, 0ULL);
        atomicExch(&sc->powell_rate_bits, 0ULL);
        atomicExch(&sc->blocks_done, 0u);
      }
    }
  }
}

// Powell time-step cap (eq. powell_dt with |div B|_K of eq. divb-cell).
template <typename T, int D, int DEG, int DIVB>
__global__ void __launch_bounds__(256) k_face_jump(const T* __restrict__ w, double* __restrict__ js, DevTab<T> tb,
                                                   Grid g, double gamma) {
  using C = Cfg<D, DEG, DIVB>;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)D * g.C) return;
  const int64_t f = gid % g.C;
  const int a = (int)(gid / g.C);
  const int64_t L = f, R = nbr(f, a, +1, g);
  const int64_t ld = g.ld;
  double jl = 0.0, jr = 0.0;
  for (int r = 0; r < C::FP; ++r) {
    T bl = 0, br = 0, rl = 0, rr = 0;
    const T* tl = tb.TF + ((a * 2 + 1) * C::FP + r) * C::N;
    const T* tr = tb.TF + ((a * 2 + 0) * C::FP + r) * C::N;
    for (int l = 0; l < C::N; ++l) {
      rl += tl[l] * w[(int64_t)l * ld + L];
      rr += tr[l] * w[(int64_t)l * ld + R];
    }
    const T* pl = tb.PTF + (((a * 2 + 1) * D + a) * C::FP + r) * C::NLDF;
    const T* pr = tb.PTF + (((a * 2 + 0) * D + a) * C::FP + r) * C::NLDF;
    for (int l = 0; l < C::NLDF; ++l) {
      bl += pl[l] * w[(int64_t)(C::NLEG * C::N + l) * ld + L];
      br += pr[l] * w[(int64_t)(C::NLEG * C::N + l) * ld + R];
    }
    const double iL = 1.0 / sqrt((double)rl), iR = 1.0 / sqrt((double)rr);
    const double bnF = ((double)bl * iL + (double)br * iR) / (iL + iR);
    double wgt = tb.LF[((a * 2 + 1) * C::FP + r) * C::N + 0];  // w_r * P_0
    jl += wgt * fabs(bnF - (double)bl);
    jr += wgt * fabs((double)br - bnF);
  }
  js[(int64_t)(a * 2 + 0) * g.C + f] = jl;
  js[(int64_t)(a * 2 + 1) * g.C + f] = jr;
}

// The same face-jump integrals from the jumps the face kernel wrote at the
// face points (jp[axis][side][point][face]: B^n_F - B^n_L, B^n_R - B^n_F).
template <typename T, int D, int DEG, int DIVB>
__global__ void __launch_bounds__(256) k_face_jump_jp(const T* __restrict__ jp, double* __restrict__ js, DevTab<T> tb,
                                                      Grid g) {
  using C = Cfg<D, DEG, DIVB>;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)D * g.C) return;
  const int64_t f = gid % g.C;
  const int a = (int)(gid / g.C);
  const int64_t ld = g.ld;
  double jl = 0.0, jr = 0.0;
  for (int r = 0; r < C::FP; ++r) {
    const double wgt = tb.LF[((a * 2 + 1) * C::FP + r) * C::N + 0];  // w_r * P_0
    jl += wgt * fabs((double)jp[((int64_t)(a * 2 + 0) * C::FP + r) * ld + f]);
    jr += wgt * fabs((double)jp[((int64_t)(a * 2 + 1) * C::FP + r) * ld + f]);
  }
  js[(int64_t)(a * 2 + 0) * g.C + f] = jl;
  js[(int64_t)(a * 2 + 1) * g.C + f] = jr;
}

template <typename T, int D, int DEG, int DIVB>
__global__ void __launch_bounds__(256) k_powell_rate(const T* __restrict__ w, const double* __restrict__ js,
                                                     DevTab<T> tb, Grid g, Scal* sc) {
  using C = Cfg<D, DEG, DIVB>;
  __shared__ double red[256];
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double rate = 0.0;
  if (K < g.C) {
    double div = 0.0;
    for (int a = 0; a < D; ++a) div += js[(int64_t)(a * 2 + 0) * g.C + K] + js[(int64_t)(a * 2 + 1) * g.C + nbr(K, a, -1, g)];
    // (1/V_K) int dS with dS = (h/2)^(D-1) dS_xi
    div *= pow(0.5 * g.h, D - 1) / pow(g.h, D);
    const int64_t ld = g.ld;
    const double rho = (double)w[K];
    const double m0 = (double)w[(int64_t)(1 * C::N) * ld + K], m1 = (double)w[(int64_t)(2 * C::N) * ld + K],
                 m2 = (double)w[(int64_t)(3 * C::N) * ld + K];
    const double E = (double)w[(int64_t)(4 * C::N) * ld + K];
    double bm[3] = {0, 0, 0};
    for (int cc = 0; cc < D; ++cc)
      for (int l = 0; l < C::NLDF; ++l) bm[cc] += (double)tb.Pmean[cc * C::NLDF + l] * (double)w[(int64_t)(C::NLEG * C::N + l) * ld + K];
    if (D == 2) bm[2] = (double)w[(int64_t)(5 * C::N) * ld + K];
    const double vb = (m0 * bm[0] + m1 * bm[1] + m2 * bm[2]) / rho;
    const double prod = div * fabs(vb);
    if (prod > 0.0) rate = prod / E;
  }
  red[threadIdx.x] = rate;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomic_max_pos(&sc->powell_rate_bits, red[0]);
}

// ---------------------------------------------------------------------------
// projection of pointwise primitive values (d+3 rule)
//
// One workgroup per tile of PTC cells: the tile's primitive values (a
// contiguous slab of each variable's [ncell][npts] block) are read coalesced,
// converted to conserved variables into LDS, and every (mode, cell) output is
// then a dot product over the tile's points.

template <int D, int DEG>
struct ProjTile {
  static constexpr int NP = (D == 2) ? (DEG + 3) * (DEG + 3) : (DEG + 3) * (DEG + 3) * (DEG + 3);
  static constexpr int TC0 = 131072 / (9 * 8 * NP);
  static constexpr int TC = TC0 > 16 ? 16 : (TC0 < 1 ? 1 : TC0);
};

// Dynamic refinement (Sec. 4.4) on the Legendre basis, one thread per leaf
// (or group).  The smoothness indicator of a field and direction is the
// quadratic form w^T SQ_a w of its weights; the largest over the fields of
// the mask and the directions is stored (NaN propagates).
template <int N, int D>
__device__ __forceinline__ double amr_smax(const double (&u)[N], const double* __restrict__ SQ, double smax) {
  for (int a = 0; a < D; ++a) {
    double q = 0.0;
    for (int n = 0; n < N; ++n) {
      double r = 0.0;
      for (int m = 0; m < N; ++m) r += SQ[(a * N + n) * N + m] * u[m];
      q += u[n] * r;
    }
    smax = (q > smax || q != q) ? q : smax;
  }
  return smax;
}

template <typename T, int D, int DEG>
__global__ void __launch_bounds__(256) k_amr_smooth(const T* __restrict__ w, int64_t ld, int64_t C, uint32_t fields,
                                                    const double* __restrict__ SQ, double* __restrict__ S) {
  constexpr int N = Cfg<D, DEG, GLM>::N;
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= C) return;
  double smax = 0.0;
  for (int v = 0; v < 9; ++v) {
    if (!((fields >> v) & 1u)) continue;
    double u[N];
#pragma unroll
    for (int n = 0; n < N; ++n) u[n] = (double)w[(int64_t)(v * N + n) * ld + K];
    smax = amr_smax<N, D>(u, SQ, smax);
  }
  S[K] = smax;
}

template <typename T, int D, int DEG>
__global__ void __launch_bounds__(256) k_amr_parent_smooth(const T* __restrict__ w, int64_t ld, uint32_t fields,
                                                           const int32_t* __restrict__ groups, int64_t ngroups,
                                                           const double* __restrict__ SQ,
                                                           const double* __restrict__ RES, double* __restrict__ Sp) {
  constexpr int N = Cfg<D, DEG, GLM>::N, NO = 1 << D;
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= ngroups) return;
  double smax = 0.0;
  for (int v = 0; v < 9; ++v) {
    if (!((fields >> v) & 1u)) continue;
    double u[N];
#pragma unroll
    for (int m = 0; m < N; ++m) u[m] = 0.0;
    for (int o = 0; o < NO; ++o) {
      const int64_t K = groups[gi * NO + o];
      for (int n = 0; n < N; ++n) {
        const double x = (double)w[(int64_t)(v * N + n) * ld + K];
#pragma unroll
        for (int m = 0; m < N; ++m) u[m] += RES[(o * N + m) * N + n] * x;
      }
    }
    smax = amr_smax<N, D>(u, SQ, smax);
  }
  Sp[gi] = smax;
}

template <typename T, int D, int DEG>
__global__ void __launch_bounds__(256) k_amr_transfer(const T* __restrict__ wo, int64_t ldo, T* __restrict__ wn,
                                                      int64_t ldn, const int32_t* __restrict__ map,
                                                      const int32_t* __restrict__ kids, int64_t nnew,
                                                      const double* __restrict__ PRO,
                                                      const double* __restrict__ RES) {
  constexpr int N = Cfg<D, DEG, GLM>::N, NO = 1 << D;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnew) return;
  const int kind = map[4 * i], depth = map[4 * i + 2];
  const int64_t src = map[4 * i + 1];
  const uint32_t path = (uint32_t)map[4 * i + 3];
  for (int v = 0; v < 9; ++v) {
    double u[N];
    if (kind == 2) {
#pragma unroll
      for (int m = 0; m < N; ++m) u[m] = 0.0;
      for (int o = 0; o < NO; ++o) {
        const int64_t K = kids[src * NO + o];
        for (int n = 0; n < N; ++n) {
          const double x = (double)wo[(int64_t)(v * N + n) * ldo + K];
#pragma unroll
          for (int m = 0; m < N; ++m) u[m] += RES[(o * N + m) * N + n] * x;
        }
      }
    } else {
#pragma unroll
      for (int n = 0; n < N; ++n) u[n] = (double)wo[(int64_t)(v * N + n) * ldo + src];
      for (int l = 0; l < (kind == 1 ? depth : 0); ++l) {
        const int o = (int)((path >> (3 * (depth - 1 - l))) & 7u);
        double t[N];
#pragma unroll
        for (int m = 0; m < N; ++m) {
          double acc = 0.0;
          for (int n = 0; n < N; ++n) acc += PRO[(o * N + m) * N + n] * u[n];
          t[m] = acc;
        }
#pragma unroll
        for (int m = 0; m < N; ++m) u[m] = t[m];
      }
    }
#pragma unroll
    for (int m = 0; m < N; ++m) wn[(int64_t)(v * N + m) * ldn + i] = (T)u[m];
  }
}

// Conserved state at the points of the projection rule, one thread per
// (cell, point); consecutive threads take consecutive cells of one point.
template <typename T, int D, int DEG, int DIVB>
__global__ void __launch_bounds__(256) k_nodal(const T* __restrict__ w, int64_t cell0, int64_t ncell,
                                               double* __restrict__ out, const double* __restrict__ vp,
                                               const double* __restrict__ pvp, int64_t ld) {
  using C = Cfg<D, DEG, DIVB>;
  constexpr int NP = ProjTile<D, DEG>::NP;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncell * NP) return;
  const int p = (int)(i / ncell);
  const int64_t c = i - (int64_t)p * ncell, K = cell0 + c;
  for (int j = 0; j < C::NLEG; ++j) {
    double s = 0.0;
    for (int l = 0; l < C::N; ++l) s += vp[p * C::N + l] * (double)w[(int64_t)(j * C::N + l) * ld + K];
    out[((int64_t)C::legvar(j) * NP + p) * ncell + c] = s;
  }
  if constexpr (C::NLDF > 0) {
    for (int cc = 0; cc < D; ++cc) {
      double s = 0.0;
      for (int l = 0; l < C::NLDF; ++l)
        s += pvp[(cc * NP + p) * C::NLDF + l] * (double)w[(int64_t)(C::NLEG * C::N + l) * ld + K];
      out[((int64_t)(5 + cc) * NP + p) * ncell + c] = s;
    }
  }
}

template <typename T, int D, int DEG, int DIVB>
__global__ void __launch_bounds__(256) k_project(const double* __restrict__ prim, int64_t cell0, int64_t ncell,
                                                 T* __restrict__ w, const double* __restrict__ vpw,
                                                 const double* __restrict__ pvpw, const double* __restrict__ minv,
                                                 int64_t ld, double gamma) {
  using C = Cfg<D, DEG, DIVB>;
  constexpr int NP = ProjTile<D, DEG>::NP, TC = ProjTile<D, DEG>::TC;
  __shared__ double su[9 * TC * NP];
  const int64_t c0 = (int64_t)blockIdx.x * TC;
  const int nc = (int)((ncell - c0) < TC ? (ncell - c0) : TC);
  for (int i = threadIdx.x; i < nc * NP; i += blockDim.x) {
    const int c = i / NP, p = i - c * NP;
    auto P = [&](int v) { return prim[((int64_t)v * ncell + c0) * NP + i]; };
    const double rho = P(0), vx = P(1), vy = P(2), vz = P(3), pr = P(4);
    const double bx = P(5), by = P(6), bz = P(7);
    const double u[9] = {rho, rho * vx, rho * vy, rho * vz,
                         pr / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) +
                             0.5 * (bx * bx + by * by + bz * bz),
                         bx, by, bz, P(8)};
#pragma unroll
    for (int v = 0; v < 9; ++v) su[(v * TC + c) * NP + p] = u[v];
  }
  __syncthreads();
  for (int o = threadIdx.x; o < C::NMODES * nc; o += blockDim.x) {
    const int m = o / nc, c = o - m * nc;
    double s = 0.0;
    if (m < C::NLEG * C::N) {
      const int j = m / C::N, l = m % C::N;
      const double* uu = su + (C::legvar(j) * TC + c) * NP;
      for (int p = 0; p < NP; ++p) s += vpw[p * C::N + l] * uu[p];
    } else {
      const int l = m - C::NLEG * C::N;
      for (int cc = 0; cc < D; ++cc) {
        const double* uu = su + ((5 + cc) * TC + c) * NP;
        for (int p = 0; p < NP; ++p) s += pvpw[(cc * NP + p) * C::NLDF + l] * uu[p];
      }
    }
    w[(int64_t)m * ld + cell0 + c0 + c] = (T)(s * minv[m]);
  }
}

#if DG_SHARED
// ---------------------------------------------------------------------------
// scalar kernels

__global__ void k_reset_next(Scal* sc) {
  sc->next_maxsig_bits = 0ULL;
  sc->next_maxrate_bits = 0ULL;
}

__global__ void k_take_next(Scal* sc) {
  sc->maxsig_bits = sc->next_maxsig_bits;
  sc->maxrate_bits = sc->next_maxrate_bits;
  sc->powell_rate_bits = 0ULL;
}

__global__ void k_reset_step(Scal* sc) {
  sc->maxrate_bits = 0ULL;
  sc->maxsig_bits = 0ULL;
  sc->powell_rate_bits = 0ULL;
}

__global__ void k_finalize_dt(Scal* sc, SchemeParams sp, int D, int d, int divb, double hmin) {
  finalize_dt_dev(sc, sp, D, d, divb, hmin, __longlong_as_double(sc->maxsig_bits),
                  __longlong_as_double(sc->maxrate_bits), __longlong_as_double(sc->powell_rate_bits));
}

__global__ void k_set_scalars(Scal* sc, double ch, double kappa, double dt) {
  sc->ch = ch;
  sc->kappa = kappa;
  sc->dt = dt;
}

__global__ void k_set_time(Scal* sc, double t) { sc->t = t; }

__global__ void k_reset_stats(Scal* sc) {
  sc->n_tvb = sc->n_pos = sc->n_floor = sc->n_mlp = sc->n_fallback = 0ULL;
  sc->inj_mass = sc->inj_energy = 0.0;
  sc->nonfinite = 0ULL;
  sc->n_ch_violation = 0ULL;
}

// Any non-finite weight in the used columns of the state sets the flag.
template <typename T>
__global__ void __launch_bounds__(256) k_scan_nonfinite(const T* __restrict__ w, int64_t nmodes, int64_t ld,
                                                        int64_t C, Scal* sc) {
  const int64_t n = nmodes * C;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t m = i / C, c = i - m * C;
    const T x = w[m * ld + c];
    bad = bad || !(x - x == T(0));  // NaN and +-inf
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicAdd(&sc->nonfinite, 1ULL);
}

void launch_scan_nonfinite(const void* w, size_t elem, int64_t nmodes, int64_t ld, int64_t C, Scal* sc,
                           hipStream_t s) {
  const int64_t n = nmodes * C;
  const int64_t blocks = (n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  if (elem == 8) k_scan_nonfinite<double><<<grid, 256, 0, s>>>((const double*)w, nmodes, ld, C, sc);
  else k_scan_nonfinite<float><<<grid, 256, 0, s>>>((const float*)w, nmodes, ld, C, sc);
}

void launch_reset_stats(Scal* sc, hipStream_t s) { k_reset_stats<<<1, 1, 0, s>>>(sc); }

void launch_set_time(Scal* sc, double t, hipStream_t s) { k_set_time<<<1, 1, 0, s>>>(sc, t); }
void launch_reset_step(Scal* sc, hipStream_t s) { k_reset_step<<<1, 1, 0, s>>>(sc); }
void launch_reset_next(Scal* sc, hipStream_t s) { k_reset_next<<<1, 1, 0, s>>>(sc); }
void launch_take_next(Scal* sc, hipStream_t s) { k_take_next<<<1, 1, 0, s>>>(sc); }
void launch_finalize_dt(Scal* sc, const SchemeParams& sp, int D, int d, int divb, double hmin, hipStream_t s) {
  k_finalize_dt<<<1, 1, 0, s>>>(sc, sp, D, d, divb, hmin);
}
void launch_set_scalars(Scal* sc, double ch, double kappa, double dt, hipStream_t s) {
  k_set_scalars<<<1, 1, 0, s>>>(sc, ch, kappa, dt);
}

template <typename T>
__global__ void __launch_bounds__(256) k_lincomb(T* out, const T* x0, const T* x1, const T* x2, const T* x3,
                                                 double c0, double c1, double c2, double c3, int64_t nmodes,
                                                 int64_t ld, int64_t C) {
  const int64_t n = nmodes * C;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t m = i / C, at = m * ld + (i - m * C);
    double v = 0.0;
    if (x0) v += c0 * (double)x0[at];
    if (x1) v += c1 * (double)x1[at];
    if (x2) v += c2 * (double)x2[at];
    if (x3) v += c3 * (double)x3[at];
    out[at] = (T)v;
  }
}

void launch_lincomb(void* out, const void* const x[4], const double c[4], size_t elem, int64_t nmodes, int64_t ld,
                    int64_t C, hipStream_t s) {
  const int64_t n = nmodes * C;
  const int64_t blocks = (n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192);
  auto X = [&](int k) { return c[k] != 0.0 ? x[k] : nullptr; };
  if (elem == 8)
    k_lincomb<double><<<grid, 256, 0, s>>>((double*)out, (const double*)X(0), (const double*)X(1),
                                           (const double*)X(2), (const double*)X(3), c[0], c[1], c[2], c[3], nmodes,
                                           ld, C);
  else
    k_lincomb<float><<<grid, 256, 0, s>>>((float*)out, (const float*)X(0), (const float*)X(1), (const float*)X(2),
                                          (const float*)X(3), c[0], c[1], c[2], c[3], nmodes, ld, C);
}
#endif  // DG_SHARED

}  // namespace dgmhd

#include "dg_limiters.inc"

namespace dgmhd {

// ---------------------------------------------------------------------------
// launcher

template <typename T, int D, int DEG, int DIVB>
struct LauncherImpl : Launcher {
  using C = Cfg<D, DEG, DIVB>;
  using TL = Tile<T, D, DEG, DIVB>;
  std::vector<void*> bufs;
  DevTab<T> tb{};
  double *vpw = nullptr, *pvpw = nullptr, *minv64 = nullptr, *vp64 = nullptr, *pvp64 = nullptr;
  double *sq64 = nullptr, *pro64 = nullptr, *res64 = nullptr;
  const T *mfv = nullptr, *mfg = nullptr, *mfl = nullptr;  // fragment-order tables of the matrix-core cell kernel
  const T *mgx = nullptr, *mlx = nullptr;                   // and its vector-ALU rows (modes 16..19)
  const T* ml1 = nullptr;                                   // lift of a constant over each -a face
  // (GLM: mfl and mlx lift face moments; Powell: face points)
  const T *mpv = nullptr, *mpg = nullptr, *mpl = nullptr;  // and its LDF (Powell) tables
  const T* mft = nullptr;                                   // and of the matrix-core face kernel
  const T* mfta = nullptr;                                  // and of its octree form (sub-face tables)
  const T* mlfa = nullptr;                                  // octree surface lift of the cell kernels
  const T* mpft = nullptr;
  const T *mflm = nullptr, *mplm = nullptr;  // Powell lift tables over face moments (3-D)                                  // Powell face trace tables (matrix-core face kernel)
  const double* mpos = nullptr;                             // and of the matrix-core positivity limiter
  int pos_variant = 1;                                      // 1: matrix-core positivity limiter where built
  int face_variant = 1;                                     // default: the matrix-core face kernel

  template <typename U>
  hipError_t up(const std::vector<double>& src, const U*& dst) {
    if (src.empty()) { dst = nullptr; return hipSuccess; }
    std::vector<U> tmp(src.begin(), src.end());
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, tmp.size() * sizeof(U));
    if (e != hipSuccess) return e;
    bufs.push_back(p);
    e = hipMemcpy(p, tmp.data(), tmp.size() * sizeof(U), hipMemcpyHostToDevice);
    dst = (const U*)p;
    return e;
  }

  hipError_t upload_tables(const Tables& t) override {
    if (t.N != C::N || t.Q != C::Q || t.FP != C::FP || t.NMODES != C::NMODES) return hipErrorInvalidValue;
    hipError_t e;
#define UP(src, dst) if ((e = up<T>(t.src, tb.dst)) != hipSuccess) return e;
    UP(V, V) UP(GW, GW) UP(TF, TF) UP(LF, LF) UP(Minv, Minv) UP(PV, PV) UP(PGW, PGW) UP(PTF, PTF) UP(PLF, PLF)
    UP(Pmean, Pmean) UP(Plin, Plin) UP(TFS, TFS) UP(LFS, LFS)
#undef UP
    const double* d1 = nullptr;
    if ((e = up<double>(t.VPW, d1)) != hipSuccess) return e;
    vpw = (double*)d1;
    if ((e = up<double>(t.PVPW, d1)) != hipSuccess) return e;
    pvpw = (double*)d1;
    if ((e = up<double>(t.Minv, d1)) != hipSuccess) return e;
    minv64 = (double*)d1;
    if ((e = up<double>(t.VP, d1)) != hipSuccess) return e;
    vp64 = (double*)d1;
    if ((e = up<double>(t.PVP, d1)) != hipSuccess) return e;
    pvp64 = (double*)d1;
    if ((e = up<double>(t.SQ, d1)) != hipSuccess) return e;
    sq64 = (double*)d1;
    if ((e = up<double>(t.PRO, d1)) != hipSuccess) return e;
    pro64 = (double*)d1;
    if ((e = up<double>(t.RES, d1)) != hipSuccess) return e;
    res64 = (double*)d1;
    if constexpr (DIVB == POWELL) {
      std::vector<double> fv, fg, fl, pv, pg, pl, gx, lx, qb;
      mfma_tables<T, D, DEG>(t, fv, fg, fl, gx, lx);
      powell_tables<T, D, DEG>(t, pv, pg, pl);
      if ((e = up<T>(fv, mfv)) != hipSuccess) return e;
      if ((e = up<T>(fg, mfg)) != hipSuccess) return e;
      if ((e = up<T>(fl, mfl)) != hipSuccess) return e;
      if ((e = up<T>(pv, mpv)) != hipSuccess) return e;
      if ((e = up<T>(pg, mpg)) != hipSuccess) return e;
      if ((e = up<T>(pl, mpl)) != hipSuccess) return e;
      if constexpr (D == 3) {
        // the cell-mean q-dagger's face moments (matrix-core face and cell kernels)
        std::vector<double> flm, lxm, plm;
        if (!face_moment_basis<D, DEG>(t, qb)) return hipErrorInvalidValue;
        mfma_moment_lift<T, D, DEG>(t, qb, flm, lxm);
        if (!powell_moment_lift<T, D, DEG>(t, qb, plm)) return hipErrorInvalidValue;
        if ((e = up<T>(flm, mflm)) != hipSuccess) return e;
        if ((e = up<T>(plm, mplm)) != hipSuccess) return e;
      }
      {
        int dev = 0, ncu = 0, bp = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
        if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        if constexpr (PowellLds<T, D, DEG, false>::fits) {
          if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bp, k_cell_mfma_powell_p<T, D, DEG, 8, false>, 512,
                                                                 0)) != hipSuccess)
            return e;
          persist_powell = bp * ncu;
        }
        if constexpr (D == 3 && PowellLds<T, D, DEG, true>::fits) {
          if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bp, k_cell_mfma_powell_p<T, D, DEG, 8, true>, 512,
                                                                 0)) != hipSuccess)
            return e;
          persist_powell_m = bp * ncu;
        }
      }
      std::vector<double> pft;
      powell_face_tables<T, D, DEG>(t, qb, pft);
      if ((e = up<T>(pft, mpft)) != hipSuccess) return e;
      {  // resident workgroups of the persistent max-signal kernel
        int dev = 0, ncu = 0, bm = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
        if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bm, k_maxsig_mfma_powell<T, D, DEG, 8>, 512, 0)) !=
            hipSuccess)
          return e;
        maxsig_blocks = bm * ncu;
      }
    }
    if constexpr (DIVB == GLM) {
      // uniform grids: the matrix-core face kernels store face moments and
      // the matrix-core cell kernel lifts them (tables over moments)
      std::vector<double> qb, fv, fg, fl, gx, lx, flm, lxm;
      if (!face_moment_basis<D, DEG>(t, qb)) return hipErrorInvalidValue;
      mfma_tables<T, D, DEG>(t, fv, fg, fl, gx, lx);
      mfma_moment_lift<T, D, DEG>(t, qb, flm, lxm);
      if ((e = up<T>(fv, mfv)) != hipSuccess) return e;
      if ((e = up<T>(fg, mfg)) != hipSuccess) return e;
      if ((e = up<T>(flm, mfl)) != hipSuccess) return e;
      if ((e = up<T>(gx, mgx)) != hipSuccess) return e;
      if ((e = up<T>(lxm, mlx)) != hipSuccess) return e;
      // lift of a constant over the -a (side 0) and +a (side 1) face, signed
      // as the lift tables: [side][a][n] = -+ sum_r w_r phi_n (deviation form)
      std::vector<double> l1((size_t)2 * D * C::N, 0.0);
      for (int side = 0; side < 2; ++side)
        for (int a = 0; a < D; ++a)
          for (int n = 0; n < C::N; ++n)
            for (int r = 0; r < C::FP; ++r)
              l1[((size_t)side * D + a) * C::N + n] +=
                  (side ? -1.0 : 1.0) * t.LF[((a * 2 + side) * C::FP + r) * C::N + n];
      if ((e = up<T>(l1, ml1)) != hipSuccess) return e;
      for (int a = 0; a < D; ++a)  // the modes the lift of a constant reaches are the powers xi_a^k
        for (int n = 0; n < C::N; ++n) {
          bool pw = false;
          for (int k = 0; k <= DEG; ++k) pw = pw || MfmaShape<D, DEG>::power_mode(a, k) == n;
          for (int b = 0; b < 3; ++b) {
            const int want = b == a ? -1 : 0;
            if (pw && want == 0 && t.expo[3 * n + b] != 0) return hipErrorInvalidValue;
          }
          if (!pw && (std::fabs(l1[(size_t)a * C::N + n]) > 1e-14 || std::fabs(l1[((size_t)D + a) * C::N + n]) > 1e-14))
            return hipErrorInvalidValue;
        }
      std::vector<double> ft, fta;
      mfma_face_tables<T, D, DEG>(t, qb, ft);
      if ((e = up<T>(ft, mft)) != hipSuccess) return e;
      amr_face_tables<T, D, DEG>(t, qb, fta);
      if ((e = up<T>(fta, mfta)) != hipSuccess) return e;
      std::vector<double> lfa;
      if (!amr_lift_tables<T, D, DEG>(t, qb, lfa)) return hipErrorInvalidValue;
      if ((e = up<T>(lfa, mlfa)) != hipSuccess) return e;
      std::vector<double> pt;
      pos_tables<D, DEG>(t, pt);
      if ((e = up<double>(pt, mpos)) != hipSuccess) return e;
      // resident workgroups of the persistent cell kernels on this device
      int dev = 0, ncu = 0, b4 = 0, b2 = 0, ba4 = 0, ba2 = 0;
      if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
      if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b4, k_cell_mfma_p<T, D, DEG, 4, false>, 256, 0)) !=
          hipSuccess)
        return e;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, k_cell_mfma_p<T, D, DEG, 2, false>, 128, 0)) !=
          hipSuccess)
        return e;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&ba4, k_cell_mfma_p<T, D, DEG, 4, true>, 256, 0)) !=
          hipSuccess)
        return e;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&ba2, k_cell_mfma_p<T, D, DEG, 2, true>, 128, 0)) !=
          hipSuccess)
        return e;
      persist_blocks_amr[0] = ba4 * ncu;
      persist_blocks_amr[1] = ba2 * ncu;
      persist_blocks[0] = b4 * ncu;
      persist_blocks[1] = b2 * ncu;
      int bp = 0, bm = 0;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bp, k_pos_mfma<T, D, DEG, 4, true>, 256, 0)) !=
          hipSuccess)
        return e;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bm, k_maxsig_mfma<T, D, DEG, 4>, 256, 0)) != hipSuccess)
        return e;
      pos_blocks = bp * ncu;
      maxsig_blocks = bm * ncu;

    }
    return hipSuccess;
  }
  void free_tables() override {
    for (void* p : bufs) (void)hipFree(p);
    bufs.clear();
  }
  size_t face_buffer_elems(const Grid& g) const override {
    // uniform grids: point fluxes (FP rows per axis and variable) or face
    // moments (FM rows, FM + 1 in the FP32 deviation form)
    constexpr int rows = C::FP > C::FM + 2 ? C::FP : C::FM + 2;
    return g.level ? (size_t)C::NV * C::FP * g.ldf : (size_t)D * C::NV * rows * g.ld;
  }
  size_t jump_buffer_elems(const Grid& g, int powell_q) const override {
    // Powell: the normal-field jumps, or with the interpolated q-dagger the
    // right cells' face values (the layout of the face buffer)
    if (DIVB != POWELL) return 0;
    return powell_q ? (size_t)D * C::NV * C::FP * g.ld : (size_t)D * 2 * C::FP * g.ld;
  }
  int nmodes() const override { return C::NMODES; }

  void face(const void* w, void* ff, void* jp, const Grid& g, const Scal* sc, const SchemeParams& sp,
            hipStream_t s, bool cap) override {
    if (g.level) {
      if constexpr (DIVB == GLM) {
        if (face_variant >= 1 && mfta && g.nftile > 0) {
          constexpr int NW = 4;
          k_face_amr_mfma<T, D, DEG, NW><<<(unsigned)((g.nftile + NW - 1) / NW), 64 * NW, 0, s>>>(
              (const T*)w, (T*)ff, mfta, g, sc, sp.gamma);
        } else {
          const int64_t total = (int64_t)C::FP * g.NF;
          k_face_amr<T, D, DEG><<<(unsigned)((total + 255) / 256), 256, 0, s>>>((const T*)w, (T*)ff, tb, g, sc,
                                                                                sp.gamma);
        }
      }
      return;
    }
    if constexpr (DIVB == GLM) {
      const int64_t tiles = (g.C + 15) / 16;
      // one wave per (tile, axis) pair
      if (face_variant == 1) {
        constexpr int NW = 4;
        const unsigned grid = (unsigned)((tiles * D + NW - 1) / NW);
        k_face_mfma<T, D, DEG, NW><<<grid, 64 * NW, 0, s>>>((const T*)w, (T*)ff, mft, g, sc, sp.gamma);
        return;
      }
      if (face_variant == 2) {
        const unsigned grid = (unsigned)(tiles * D);
        k_face_mfma<T, D, DEG, 1><<<grid, 64, 0, s>>>((const T*)w, (T*)ff, mft, g, sc, sp.gamma);
        return;
      }
      if (face_variant == 3) {
        constexpr int NW = 1;
        const unsigned grid = (unsigned)((tiles * D + NW - 1) / NW);
        k_face_mfma_lr<T, D, DEG, NW><<<grid, 64 * NW, 0, s>>>((const T*)w, (T*)ff, mft, g, sc, sp.gamma);
        return;
      }
    }
    if constexpr (DIVB == POWELL) {
      if (face_variant == 1 && mpft) {  // matrix-core traces, one wave per (tile, axis) pair
        constexpr int NW = 4;
        const int64_t tiles = (g.C + 15) / 16;
        const unsigned grid = (unsigned)((tiles * D + NW - 1) / NW);
        if (sp.powell_q)
          k_face_mfma_powell<T, D, DEG, NW, true><<<grid, 64 * NW, 0, s>>>((const T*)w, (T*)ff, (T*)jp, mpft, g, sc,
                                                                           sp.gamma, 1);
        else
          k_face_mfma_powell<T, D, DEG, NW, false><<<grid, 64 * NW, 0, s>>>((const T*)w, (T*)ff, (T*)jp, mpft, g, sc,
                                                                            sp.gamma, cap ? 1 : 0);
        return;
      }
    }
    using FT = FaceTile<T, D, DEG, DIVB>;
    dim3 grid((unsigned)((g.C + FT::TF - 1) / FT::TF), D);
    k_face<T, D, DEG, DIVB><<<grid, FT::NT, 0, s>>>((const T*)w, (T*)ff, (T*)jp, tb, g, sc, sp.gamma,
                                                     DIVB == POWELL && sp.powell_q ? 1 : 0);
  }
  int cell_variant = -1;  // -1: default

  // variants 4, 5: the matrix-core cell kernel with 4 or 2 waves per
  // workgroup; 6, 7: the same with batched operand loads (more registers);
  // 8, 9: batched and persistent, the tables in LDS
  static constexpr int NVAR = 10;
  int persist_blocks[2] = {0, 0};      // resident workgroups of the persistent kernels (4 and 2 waves)
  int persist_powell = 0;              // resident workgroups of the persistent Powell cell kernel (8 waves)
  int persist_powell_m = 0;            // the same, face-moment form (3-D, cell-mean q-dagger)
  int persist_blocks_amr[2] = {0, 0};  // the same on octree grids
  int pos_blocks = 0, maxsig_blocks = 0;
  template <int NW>
  bool launch_cell_mfma_p(const void* w, const void* w0, void* out, const void* ff, const Grid& g, const Scal* sc,
                          const SchemeParams& sp, double a0, double b0, double cdt, int mode, hipStream_t s) {
    if constexpr (DIVB == GLM) {
      const int nb = g.level ? persist_blocks_amr[NW == 4 ? 0 : 1] : persist_blocks[NW == 4 ? 0 : 1];
      if (nb <= 0) return false;
      const int64_t groups = ((g.C + 15) / 16 + NW - 1) / NW;
      const unsigned grid = (unsigned)(groups < nb ? groups : nb);
      if (g.level)
        k_cell_mfma_p<T, D, DEG, NW, true><<<grid, 64 * NW, 0, s>>>((const T*)w, (const T*)w0, (T*)out,
                                                                    (const T*)ff, mfv, mfg, mfl, mgx, mlx, mlfa, ml1, tb.Minv, g,
                                                                    sc, sp.gamma, a0, b0, cdt, mode);
      else
        k_cell_mfma_p<T, D, DEG, NW, false><<<grid, 64 * NW, 0, s>>>((const T*)w, (const T*)w0, (T*)out,
                                                                     (const T*)ff, mfv, mfg, mfl, mgx, mlx, tb.LFS, ml1, tb.Minv, g,
                                                                     sc, sp.gamma, a0, b0, cdt, mode);
      return true;
    }
    return false;
  }
  template <int NW, bool PF>
  bool launch_cell_mfma(const void* w, const void* w0, void* out, const void* ff, const Grid& g, const Scal* sc,
                        const SchemeParams& sp, double a0, double b0, double cdt, int mode, hipStream_t s) {
    if constexpr (DIVB == GLM) {
      const int64_t tiles = (g.C + 15) / 16;
      const unsigned grid = (unsigned)((tiles + NW - 1) / NW);
      if (g.level)
        k_cell_mfma<T, D, DEG, NW, PF, true><<<grid, 64 * NW, 0, s>>>((const T*)w, (const T*)w0, (T*)out,
                                                                      (const T*)ff, mfv, mfg, mfl, mgx, mlx, mlfa, ml1, tb.Minv, g,
                                                                      sc, sp.gamma, a0, b0, cdt, mode);
      else
        k_cell_mfma<T, D, DEG, NW, PF, false><<<grid, 64 * NW, 0, s>>>((const T*)w, (const T*)w0, (T*)out,
                                                                       (const T*)ff, mfv, mfg, mfl, mgx, mlx, tb.LFS, ml1, tb.Minv, g,
                                                                       sc, sp.gamma, a0, b0, cdt, mode);
      return true;
    }
    return false;
  }
  bool launch_cell_powell(int nw, const void* w, const void* w0, void* out, const void* ff, const void* jp,
                          const Grid& g, const Scal* sc, const SchemeParams& sp, double a0, double b0, double cdt, int mode,
                          hipStream_t s) {
    if constexpr (DIVB == POWELL) {
      if (g.level) return false;
      // 3-D with the cell-mean q-dagger: the matrix-core face kernel stored
      // face moments; the interpolated q-dagger and 2-D keep the face points
      if constexpr (D == 3) {
        if (!sp.powell_q) return launch_cell_powell_t<true>(nw, w, w0, out, ff, jp, g, sc, sp, a0, b0, cdt, mode, s);
      }
      return launch_cell_powell_t<false>(nw, w, w0, out, ff, jp, g, sc, sp, a0, b0, cdt, mode, s);
    }
    return false;
  }
  template <bool PM>
  bool launch_cell_powell_t(int nw, const void* w, const void* w0, void* out, const void* ff, const void* jp,
                            const Grid& g, const Scal* sc, const SchemeParams& sp, double a0, double b0, double cdt,
                            int mode, hipStream_t s) {
    if constexpr (DIVB == POWELL) {
      const T* fl = PM ? mflm : mfl;
      const T* pl = PM ? mplm : mpl;
      const int pb = PM ? persist_powell_m : persist_powell;
      if (nw == 8) {  // persistent, tables in LDS
        if constexpr (PowellLds<T, D, DEG, PM>::fits) {
          if (pb <= 0) return false;
          const int64_t groups = ((g.C + 15) / 16 + 7) / 8;
          const unsigned grid = (unsigned)(groups < pb ? groups : pb);
          k_cell_mfma_powell_p<T, D, DEG, 8, PM><<<grid, 512, 0, s>>>((const T*)w, (const T*)w0, (T*)out,
                                                                      (const T*)ff, (const T*)jp, mfv, mfg, fl, mpv,
                                                                      mpg, pl, tb.Pmean, tb.Minv, g, sc, sp.gamma, a0,
                                                                      b0, cdt, mode);
          return true;
        }
        return false;
      }
      const unsigned grid = (unsigned)(((g.C + 15) / 16 + nw - 1) / nw);
      if (nw == 4)
        k_cell_mfma_powell<T, D, DEG, 4, PM><<<grid, 256, 0, s>>>((const T*)w, (const T*)w0, (T*)out, (const T*)ff,
                                                                  (const T*)jp, mfv, mfg, fl, mpv, mpg, pl, tb.Pmean,
                                                                  tb.Minv, g, sc, sp.gamma, a0, b0, cdt, mode);
      else
        k_cell_mfma_powell<T, D, DEG, 2, PM><<<grid, 128, 0, s>>>((const T*)w, (const T*)w0, (T*)out, (const T*)ff,
                                                                  (const T*)jp, mfv, mfg, fl, mpv, mpg, pl, tb.Pmean,
                                                                  tb.Minv, g, sc, sp.gamma, a0, b0, cdt, mode);
      return true;
    }
    return false;
  }
  template <int V>
  bool launch_cell_v(const void* w, const void* w0, void* out, const void* ff, const void* jp, const Grid& g,
                     const Scal* sc, const SchemeParams& sp, double a0, double b0, double cdt, int mode, hipStream_t s) {
    constexpr int TC = CellVariants<T, D, DEG, DIVB>::tc(V), NT = CellVariants<T, D, DEG, DIVB>::nt(V);
    if constexpr (CellTile<T, D, DEG, DIVB, TC, NT>::valid) {
      const int nb = (int)((g.C + TC - 1) / TC);
      if (g.level) {
        if constexpr (DIVB == GLM)
          k_cell<T, D, DEG, DIVB, TC, NT, 1><<<nb, NT, 0, s>>>(
              (const T*)w, (const T*)w0, (T*)out, (const T*)ff, (const T*)jp, tb.V, tb.GW, tb.LF, tb.Minv, tb.PV,
              tb.PGW, tb.PLF, tb.Pmean, tb.LFS, g, sc, sp.gamma, a0, b0, cdt, mode);
      } else {
        k_cell<T, D, DEG, DIVB, TC, NT, 0><<<nb, NT, 0, s>>>((const T*)w, (const T*)w0, (T*)out, (const T*)ff,
                                                             (const T*)jp, tb.V, tb.GW, tb.LF, tb.Minv, tb.PV, tb.PGW,
                                                             tb.PLF, tb.Pmean, tb.LFS, g, sc, sp.gamma, a0, b0, cdt, mode);
      }
      return true;
    } else {
      return false;
    }
  }
  bool cell_variant_valid(int v) const override {
    switch (v) {
      case 0: return CellTile<T, D, DEG, DIVB, CellVariants<T, D, DEG, DIVB>::tc(0), CellVariants<T, D, DEG, DIVB>::nt(0)>::valid;
      case 1: return CellTile<T, D, DEG, DIVB, CellVariants<T, D, DEG, DIVB>::tc(1), CellVariants<T, D, DEG, DIVB>::nt(1)>::valid;
      case 2: return CellTile<T, D, DEG, DIVB, CellVariants<T, D, DEG, DIVB>::tc(2), CellVariants<T, D, DEG, DIVB>::nt(2)>::valid;
      case 3: return CellTile<T, D, DEG, DIVB, CellVariants<T, D, DEG, DIVB>::tc(3), CellVariants<T, D, DEG, DIVB>::nt(3)>::valid;
      case 4:
      case 5:
      case 7: return DIVB == GLM;  // the Powell scheme's matrix-core cell forms are 6, 8 and 9
      case 6:
      case 8:
      case 9: return true;
      default: return false;
    }
  }
  int cell_variant_count() const override { return NVAR; }
  // face variants: 0 LDS-staged; GLM uniform grids, matrix cores: 1 four
  // waves per block, 2 one wave per block, 3 low-register form at two waves
  // per SIMD (octree grids run the matrix-core sub-face kernel for 1-3)
  int face_variant_count() const override { return DIVB == GLM ? 4 : 2; }
  // GLM (uniform and octree grids) and 3-D Powell: the LDS kernels (cell
  // 0-3, face 0) exchange point fluxes, the matrix-core ones (cell 4-9, face
  // 1-3) face moments (3-D Powell with the interpolated q-dagger: points in
  // both, paired the same way)
  bool layout_compatible(int cv, int fv, const Grid& g) const override {
    (void)g;
    if (DIVB == POWELL && D == 2) return true;  // 2-D Powell: points throughout
    return (fv >= 1) == (cv >= 4);
  }
  void set_face_variant(int v) override { face_variant = v < 0 ? 1 : v; }
  int get_face_variant() const override { return face_variant; }
  void set_cell_variant(int v) override { cell_variant = v; }
  int get_cell_variant() const override { return cell_variant; }
  void cell(const void* w, const void* w0, void* out, const void* ff, const void* jp, const Grid& g, const Scal* sc,
            const SchemeParams& sp, double a0, double b0, double cdt, int mode_in, hipStream_t s) override {
    // mode bit 1: the stage update; bit 2: interpolated Powell q-dagger
    const int mode = mode_in | ((DIVB == POWELL && sp.powell_q) ? 2 : 0);
    int v = cell_variant;
    if (v < 0) v = DIVB == GLM ? 6 : 8;  // default: a matrix-core kernel
    if (!cell_variant_valid(v)) {
      v = 0;
      while (v < 4 && !cell_variant_valid(v)) ++v;
    }
    if (v == 4 && launch_cell_mfma<4, false>(w, w0, out, ff, g, sc, sp, a0, b0, cdt, mode, s)) return;
    if (v == 5 && launch_cell_mfma<2, false>(w, w0, out, ff, g, sc, sp, a0, b0, cdt, mode, s)) return;
    if (v == 6 && launch_cell_mfma<4, true>(w, w0, out, ff, g, sc, sp, a0, b0, cdt, mode, s)) return;
    if (v == 7 && launch_cell_mfma<2, true>(w, w0, out, ff, g, sc, sp, a0, b0, cdt, mode, s)) return;
    if (v == 8 && launch_cell_mfma_p<4>(w, w0, out, ff, g, sc, sp, a0, b0, cdt, mode, s)) return;
    if (v == 9 && launch_cell_mfma_p<2>(w, w0, out, ff, g, sc, sp, a0, b0, cdt, mode, s)) return;
    if ((v == 8 || v == 9) && launch_cell_powell(v == 8 ? 4 : 2, w, w0, out, ff, jp, g, sc, sp, a0, b0, cdt, mode, s)) return;
    if (v == 6 && launch_cell_powell(8, w, w0, out, ff, jp, g, sc, sp, a0, b0, cdt, mode, s)) return;
    // Powell: a persistent form that cannot be resident runs the plain one
    // (same face layout)
    if (v == 6 && launch_cell_powell(4, w, w0, out, ff, jp, g, sc, sp, a0, b0, cdt, mode, s)) return;
    // GLM: a persistent form that cannot be resident runs the batched one
    // (same face-flux layout)
    if (v >= 8 && launch_cell_mfma<4, true>(w, w0, out, ff, g, sc, sp, a0, b0, cdt, mode, s)) return;
    if (v >= 4) {  // not built for this configuration
      v = 0;
      while (v < 4 && !cell_variant_valid(v)) ++v;
    }
    switch (v) {
      case 0: launch_cell_v<0>(w, w0, out, ff, jp, g, sc, sp, a0, b0, cdt, mode, s); break;
      case 1: launch_cell_v<1>(w, w0, out, ff, jp, g, sc, sp, a0, b0, cdt, mode, s); break;
      case 2: launch_cell_v<2>(w, w0, out, ff, jp, g, sc, sp, a0, b0, cdt, mode, s); break;
      default: launch_cell_v<3>(w, w0, out, ff, jp, g, sc, sp, a0, b0, cdt, mode, s); break;
    }
  }
  bool maxsig_finalizes(const Grid& g) const override {
    if constexpr (DIVB == GLM) return !((g.level || face_variant >= 1) && maxsig_blocks > 0);
    return false;
  }
  bool maxsig(const void* w, const Grid& g, Scal* sc, const SchemeParams& sp, hipStream_t s,
              const DtFinalize* fin) override {
    if constexpr (DIVB == POWELL) {
      if (!g.level && face_variant >= 1 && maxsig_blocks > 0) {
        constexpr int NW = 8;
        const int64_t groups = ((g.C + 15) / 16 + NW - 1) / NW;
        const unsigned grid = (unsigned)(groups < maxsig_blocks ? groups : maxsig_blocks);
        k_maxsig_mfma_powell<T, D, DEG, NW><<<grid, 64 * NW, 0, s>>>((const T*)w, mfv, mpv, mpft, g, sc, sp.gamma);
        return false;
      }
    }
    if constexpr (DIVB == GLM) {
      if ((g.level || face_variant >= 1) && maxsig_blocks > 0) {
        constexpr int NW = 4;
        const int64_t groups = ((g.C + 15) / 16 + NW - 1) / NW;
        const unsigned grid = (unsigned)(groups < maxsig_blocks ? groups : maxsig_blocks);
        k_maxsig_mfma<T, D, DEG, NW><<<grid, 64 * NW, 0, s>>>((const T*)w, mfv, mft, g, sc, sp.gamma);
        return false;
      }
    }
    const int nb = (int)((g.C + TL::TC - 1) / TL::TC);
    const bool f = fin != nullptr && DIVB == GLM;
    k_maxsig<T, D, DEG, DIVB><<<nb, 256, 0, s>>>((const T*)w, tb, g, sc, sp.gamma, sp, f ? *fin : DtFinalize{0, 0, 0, 0.0},
                                                 f ? 1 : 0);
    return f;
  }
  void powell_cap_jp(const void* w, const void* jp, void* jsum, const Grid& g, Scal* sc, hipStream_t s) override {
    if constexpr (DIVB == POWELL) {
      const int64_t nf = (int64_t)D * g.C;
      k_face_jump_jp<T, D, DEG, DIVB><<<(int)((nf + 255) / 256), 256, 0, s>>>((const T*)jp, (double*)jsum, tb, g);
      k_powell_rate<T, D, DEG, DIVB><<<(int)((g.C + 255) / 256), 256, 0, s>>>((const T*)w, (const double*)jsum, tb, g, sc);
    }
  }
  void powell_cap(const void* w, void* jsum, const Grid& g, Scal* sc, const SchemeParams& sp,
                  hipStream_t s) override {
    if constexpr (DIVB == POWELL) {
      const int64_t nf = (int64_t)D * g.C;
      k_face_jump<T, D, DEG, DIVB><<<(int)((nf + 255) / 256), 256, 0, s>>>((const T*)w, (double*)jsum, tb, g, sp.gamma);
      k_powell_rate<T, D, DEG, DIVB><<<(int)((g.C + 255) / 256), 256, 0, s>>>((const T*)w, (const double*)jsum, tb, g, sc);
    }
  }
  void amr_smooth(const void* w, const Grid& g, uint32_t fields, double* S, hipStream_t s) override {
    if constexpr (DIVB == GLM) {
      if (g.C > 0)
        k_amr_smooth<T, D, DEG><<<(unsigned)((g.C + 255) / 256), 256, 0, s>>>((const T*)w, g.ld, g.C, fields, sq64, S);
    }
  }
  void amr_parent_smooth(const void* w, const Grid& g, uint32_t fields, const int32_t* groups, int64_t ngroups,
                         double* Sp, hipStream_t s) override {
    if constexpr (DIVB == GLM) {
      if (ngroups > 0)
        k_amr_parent_smooth<T, D, DEG><<<(unsigned)((ngroups + 255) / 256), 256, 0, s>>>(
            (const T*)w, g.ld, fields, groups, ngroups, sq64, res64, Sp);
    }
  }
  void amr_transfer(const void* w_old, int64_t ld_old, void* w_new, int64_t ld_new, const int32_t* map,
                    const int32_t* kids, int64_t nnew, hipStream_t s) override {
    if constexpr (DIVB == GLM) {
      if (nnew > 0)
        k_amr_transfer<T, D, DEG><<<(unsigned)((nnew + 255) / 256), 256, 0, s>>>(
            (const T*)w_old, ld_old, (T*)w_new, ld_new, map, kids, nnew, pro64, res64);
    }
  }
  void nodal(const void* w, int64_t cell0, int64_t ncell, double* out, const Grid& g, hipStream_t s) override {
    constexpr int NP = ProjTile<D, DEG>::NP;
    if (ncell <= 0) return;
    const int64_t n = ncell * NP;
    k_nodal<T, D, DEG, DIVB><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((const T*)w, cell0, ncell, out, vp64, pvp64,
                                                                         g.ld);
  }
  void project(const double* prim, int64_t cell0, int64_t ncell, void* w, const Grid& g, const SchemeParams& sp,
               hipStream_t s) override {
    constexpr int TC = ProjTile<D, DEG>::TC;
    if (ncell <= 0) return;
    k_project<T, D, DEG, DIVB><<<(unsigned)((ncell + TC - 1) / TC), 256, 0, s>>>(prim, cell0, ncell, (T*)w, vpw,
                                                                                pvpw, minv64, g.ld, sp.gamma);
  }
  void limit(void* w, void* scratch, const Grid& g, Scal* sc, const SchemeParams& sp, hipStream_t s,
             bool next_sig) override {
    launch_limit<T, D, DEG, DIVB>(w, scratch, tb, pos_variant == 1 ? mpos : nullptr, pos_blocks, g, sc, sp, s,
                                  next_sig && fused_signal(g, sp));
  }
  bool fused_signal(const Grid& g, const SchemeParams& sp) const override {
    return DIVB == GLM && !g.level && (sp.limiter & 4) && pos_variant == 1 && mpos && pos_blocks > 0;
  }
  size_t limit_scratch_bytes(const Grid& g) const override { return limit_scratch<T, D, DEG, DIVB>(g); }
  bool mlp_features(const void* w, uint16_t* X, const double* sigma, const Grid& g, hipStream_t s) override {
    if constexpr (DIVB == GLM && DEG <= 3) {
      if (g.level) return false;
      k_mlp_features<T, D, DEG><<<(unsigned)((g.C * 256 + 255) / 256), 256, 0, s>>>((const T*)w, X, sigma, g);
      return true;
    }
    return false;
  }
  bool mlp_scale(const void* w, double* part, double* sigma, const Grid& g, hipStream_t s) override {
    if constexpr (DIVB == GLM) {
      const int64_t nblk = (g.C + 255) / 256;
      k_mean_sq<T, C::N><<<(unsigned)nblk, 256, 0, s>>>((const T*)w, part, g);
      k_scale_final<<<1, 1, 0, s>>>(part, nblk, g.C, sigma);
      return true;
    }
    return false;
  }
  bool mlp_labels(const void* w, float* y, const Grid& g, Scal* sc, const SchemeParams& sp, hipStream_t s) override {
    if constexpr (DIVB == GLM) {
      if (g.level) return false;
      k_tvb_labels<T, D, DEG><<<(unsigned)((g.C + 127) / 128), 128, 0, s>>>((const T*)w, y, g, sc, sp.gamma,
                                                                             sp.tvb_Mtilde * g.h, sp.tvb_beta,
                                                                             sp.tvb_eps, (sp.limiter & 2) ? 1 : 0);
      return true;
    }
    return false;
  }
  bool mlp_record(const void* w, uint16_t* X, float* y, unsigned long long* counter, int64_t cap, double qpos,
                  double q, unsigned long long seed, const Grid& g, Scal* sc, const SchemeParams& sp,
                  hipStream_t s) override {
    if constexpr (DIVB == GLM) {
      if (g.level || !sp.mlp_sigma) return false;
      k_record<T, D, DEG><<<(unsigned)((g.C + 127) / 128), 128, 0, s>>>((const T*)w, X, y, counter, cap, qpos, q, seed, g,
                                                                         sc, sp.mlp_sigma, sp.gamma,
                                                                         sp.tvb_Mtilde * g.h, sp.tvb_beta,
                                                                         sp.tvb_eps);
      k_record_stage_bump<<<1, 1, 0, s>>>(sc);
      return true;
    }
    return false;
  }
  ~LauncherImpl() override { free_tables(); }
};

#define CASE(T, DD, DEG, DIV) \
  if (D == DD && d == DEG) return new LauncherImpl<T, DD, DEG, DIV>();
#define PART(NAME, T, DIV)                                                                            \
  Launcher* NAME(int D, int d) {                                                                      \
    CASE(T, 2, 1, DIV) CASE(T, 2, 2, DIV) CASE(T, 2, 3, DIV) CASE(T, 3, 1, DIV) CASE(T, 3, 2, DIV) \
    CASE(T, 3, 3, DIV) return nullptr;                                                                \
  }
#if DG_PART == -1 || DG_PART == 0
PART(make_launcher_f64_glm, double, GLM)
#endif
#if DG_PART == -1 || DG_PART == 1
PART(make_launcher_f64_powell, double, POWELL)
#endif
#if DG_PART == -1 || DG_PART == 2
PART(make_launcher_f32_glm, float, GLM)
#endif
#if DG_PART == -1 || DG_PART == 3
PART(make_launcher_f32_powell, float, POWELL)
#endif
#undef PART
#undef CASE

#if DG_SHARED
Launcher* make_launcher_f64_glm(int D, int d);
Launcher* make_launcher_f64_powell(int D, int d);
Launcher* make_launcher_f32_glm(int D, int d);
Launcher* make_launcher_f32_powell(int D, int d);

Launcher* make_launcher(int precision, int D, int d, int divb) {
  if (precision == 0) return divb == GLM ? make_launcher_f64_glm(D, d) : make_launcher_f64_powell(D, d);
  return divb == GLM ? make_launcher_f32_glm(D, d) : make_launcher_f32_powell(D, d);
}
#endif

}  // namespace dgmhd
