// Learned troubled-cell indicator: BF16 matrix-core training and inference
// kernels for the 256 -> 64 -> 64 -> 64 -> 1 network (GELU hidden layers,
// sigmoid output, binary cross-entropy), FP32 accumulation, FP32 master
// weights with Adam.
//
// Device parameter layout (FP32 masters and BF16 copies share it): for each
// layer W[fin][fout_pad] row-major then b[fout_pad]; fout_pad = 16 for the
// 1-wide output layer (columns 1..15 stay zero).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <random>
#include <vector>

#include "dg_mlp.h"

namespace dgmhd {

typedef short s16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

// C[i][n] = sum_k A(i,k) B(k,n) (+ beta C), A(i,k) = A[i*ari + k*ark],
// B(k,n) = B[k*brk + n*brn] (BF16), C FP32 row-major.  One wavefront per
// 16x16 output tile with gfx950's v_mfma_f32_16x16x32_bf16: lane l supplies
// A[l%16][8(l/16)+e], B[8(l/16)+e][l%16] (e = 0..7; zero past K) and
// receives C[4(l/16)+j][l%16] (j = 0..3).  M, N, K multiples of 16.
__global__ void __launch_bounds__(256) k_gemm_bf16(const uint16_t* __restrict__ A, int64_t ari, int64_t ark,
                                                   const uint16_t* __restrict__ B, int64_t brk, int64_t brn,
                                                   float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                                   float beta) {
  const int wave = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int ntn = N / 16;
  const int tm = wave / ntn, tn = wave % ntn;
  if (tm >= M / 16) return;
  const int i = tm * 16 + lane % 16, n = tn * 16 + lane % 16, kq = 4 * (lane / 16), k8 = 8 * (lane / 16);
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    s16x8_t a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + k8 + e;
      a[e] = k < K ? (short)A[(int64_t)i * ari + (int64_t)k * ark] : (short)0;
      b[e] = k < K ? (short)B[(int64_t)k * brk + (int64_t)n * brn] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                  acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t r = tm * 16 + kq + j;
    float* c = C + r * ldc + n;
    *c = acc[j] + (beta != 0.f ? beta * *c : 0.f);
  }
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_df(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.3989422804014327f;
}

// Z + b -> Zb (kept for the backward pass) and BF16 GELU(Zb).
__global__ void k_bias_gelu(const float* __restrict__ Z, const float* __restrict__ b, float* __restrict__ Zb,
                            uint16_t* __restrict__ Aout, int64_t rows, int N) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * N) return;
  const float z = Z[t] + b[t % N];
  Zb[t] = z;
  Aout[t] = f2bf(gelu_f(z));
}

// Output layer: p = sigmoid(z + b4); training: dz = (p - y)/B (FP32 for the
// bias gradient, BF16 column 0 of a 16-wide matrix for the weight gradient),
// loss accumulated.  Rows >= nvalid are padding.
__global__ void k_head(const float* __restrict__ Z, const float* __restrict__ b4, const float* __restrict__ y,
                       float* __restrict__ p, float* __restrict__ dz, uint16_t* __restrict__ dzb,
                       float* __restrict__ loss, int64_t rows, int64_t nvalid, float invB) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const float z = Z[r * 16] + b4[0];
  const float pr = 1.0f / (1.0f + expf(-z));
  if (p) p[r] = pr;
  if (dz) {
    const bool ok = r < nvalid;
    const float yy = ok ? y[r] : 0.f;
    const float g = ok ? (pr - yy) * invB : 0.f;
    dz[r] = g;
    dzb[r * 16] = f2bf(g);
    for (int c = 1; c < 16; ++c) dzb[r * 16 + c] = 0;
    if (ok) {
      const float e = 1e-12f;
      const float l = -(yy * logf(fmaxf(pr, e)) + (1.f - yy) * logf(fmaxf(1.f - pr, e)));
      atomicAdd(loss, l * invB);
    }
  }
}

// dZ = dA * GELU'(Zb): FP32 (bias gradient) and BF16 (weight gradient, next dA).
__global__ void k_gelu_back(const float* __restrict__ dA, const float* __restrict__ Zb, float* __restrict__ dZ,
                            uint16_t* __restrict__ dZb, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float g = dA[t] * gelu_df(Zb[t]);
  dZ[t] = g;
  dZb[t] = f2bf(g);
}

// Column sums (bias gradients), one thread per column, fixed order.
// out[c] = sum_r X[r][c]: one block of 256 threads per column, strided
// partial sums and a fixed-order tree (deterministic).
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ X, int64_t rows, int N, int64_t ld,
                                                float* __restrict__ out) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int64_t r = threadIdx.x; r < rows; r += 256) s += X[r * ld + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0 && c < N) out[c] = red[0];
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ Pb, int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float mi = 0.9f * m[i] + 0.1f * g;
  const float vi = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mi;
  v[i] = vi;
  const float p = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  P[i] = p;
  Pb[i] = f2bf(p);
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

__global__ void k_gather_rows(const uint16_t* __restrict__ X, const float* __restrict__ y,
                              const int32_t* __restrict__ idx, int64_t r0, int64_t nrows, int64_t rows,
                              uint16_t* __restrict__ Xb, float* __restrict__ yb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * MLP_NF) return;
  const int64_t r = t / MLP_NF, c = t % MLP_NF;
  const int64_t src = r0 + r;
  if (src < nrows) {
    const int64_t s = idx ? idx[src] : src;
    Xb[t] = X[s * MLP_NF + c];
    if (c == 0) yb[r] = y ? y[s] : 0.f;
  } else {
    Xb[t] = 0;
    if (c == 0) yb[r] = 0.f;
  }
}

// ---------------------------------------------------------------------------
// host side

static const int FIN[4] = {256, 64, 64, 64};
static const int FOUT[4] = {64, 64, 64, 16};

size_t mlp_param_offset(int layer, bool bias) {
  size_t o = 0;
  for (int l = 0; l < layer; ++l) o += (size_t)FIN[l] * FOUT[l] + FOUT[l];
  return o + (bias ? (size_t)FIN[layer] * FOUT[layer] : 0);
}

void mlp_pack(const float* pub, std::vector<float>& dev) {
  dev.assign(MLP_NPARAM_DEV, 0.f);
  size_t q = 0;
  for (int l = 0; l < 4; ++l) {
    const int fo = l == 3 ? 1 : FOUT[l];
    float* W = dev.data() + mlp_param_offset(l, false);
    for (int i = 0; i < FIN[l]; ++i)
      for (int o = 0; o < fo; ++o) W[(size_t)i * FOUT[l] + o] = pub[q++];
    float* b = dev.data() + mlp_param_offset(l, true);
    for (int o = 0; o < fo; ++o) b[o] = pub[q++];
  }
}

void mlp_unpack(const std::vector<float>& dev, float* pub) {
  size_t q = 0;
  for (int l = 0; l < 4; ++l) {
    const int fo = l == 3 ? 1 : FOUT[l];
    const float* W = dev.data() + mlp_param_offset(l, false);
    for (int i = 0; i < FIN[l]; ++i)
      for (int o = 0; o < fo; ++o) pub[q++] = W[(size_t)i * FOUT[l] + o];
    const float* b = dev.data() + mlp_param_offset(l, true);
    for (int o = 0; o < fo; ++o) pub[q++] = b[o];
  }
}

static void gemm(const uint16_t* A, int64_t ari, int64_t ark, const uint16_t* B, int64_t brk, int64_t brn, float* C,
                 int64_t ldc, int M, int N, int K, float beta, hipStream_t s) {
  const int tiles = (M / 16) * (N / 16);
  k_gemm_bf16<<<(tiles + 3) / 4, 256, 0, s>>>(A, ari, ark, B, brk, brn, C, ldc, M, N, K, beta);
}

static unsigned nb(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

bool MlpState::alloc_params(std::string& err) {
  if (P) return true;
  auto m = [&](void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) { err = "mlp allocation"; return false; }
    pbufs.push_back(*p);
    return hipMemset(*p, 0, bytes) == hipSuccess;
  };
  const size_t np = MLP_NPARAM_DEV;
  return m((void**)&P, np * 4) && m((void**)&Pb, np * 2) && m((void**)&G, np * 4) && m((void**)&Mo, np * 4) &&
         m((void**)&Vo, np * 4) && m((void**)&sigma, 16 * 8) && m((void**)&loss, 4 * 4096);
}

bool MlpState::alloc(int batch, std::string& err) {
  if (!alloc_params(err)) return false;
  const int want = (batch + 15) / 16 * 16;
  if (want == B && Xb) return true;
  for (void* p : bufs) (void)hipFree(p);
  bufs.clear();
  B = want;
  auto m = [&](void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) { err = "mlp allocation"; return false; }
    bufs.push_back(*p);
    return hipMemset(*p, 0, bytes) == hipSuccess;
  };
  bool ok = m((void**)&Xb, (size_t)B * MLP_NF * 2) && m((void**)&yb, (size_t)B * 4) && m((void**)&dz4, (size_t)B * 4) &&
            m((void**)&dzb16, (size_t)B * 16 * 2) && m((void**)&pout, (size_t)B * 4);
  for (int l = 0; l < 4 && ok; ++l) {
    ok = m((void**)&Z[l], (size_t)B * FOUT[l] * 4) && m((void**)&Zb[l], (size_t)B * FOUT[l] * 4) &&
         m((void**)&Ab[l], (size_t)B * FOUT[l] * 2) && m((void**)&dA[l], (size_t)B * 64 * 4) &&
         m((void**)&dZ[l], (size_t)B * 64 * 4) && m((void**)&dZbf[l], (size_t)B * 64 * 2);
  }
  return ok;
}

void MlpState::release() {
  for (void* p : bufs) (void)hipFree(p);
  for (void* p : pbufs) (void)hipFree(p);
  bufs.clear();
  pbufs.clear();
  P = G = Mo = Vo = nullptr;
  Pb = nullptr;
  Xb = nullptr;
  B = 0;
}

// forward of the batch in Xb (rows B); returns probabilities in pout
void MlpState::forward(hipStream_t s) {
  const uint16_t* a = Xb;
  for (int l = 0; l < 4; ++l) {
    const uint16_t* W = Pb + mlp_param_offset(l, false);
    gemm(a, FIN[l], 1, W, FOUT[l], 1, Z[l], FOUT[l], B, FOUT[l], FIN[l], 0.f, s);
    if (l < 3) {
      k_bias_gelu<<<nb((int64_t)B * FOUT[l]), 256, 0, s>>>(Z[l], P + mlp_param_offset(l, true), Zb[l], Ab[l], B,
                                                            FOUT[l]);
      a = Ab[l];
    }
  }
}

// forward + backward of the batch in Xb/yb (nvalid real rows); gradients in G
void MlpState::backward(int64_t nvalid, hipStream_t s) {
  forward(s);
  const float invB = 1.0f / (float)nvalid;
  k_head<<<nb(B), 256, 0, s>>>(Z[3], P + mlp_param_offset(3, true), yb, pout, dz4, dzb16, loss + loss_slot, B, nvalid,
                               invB);
  // output layer: dW4 = A3^T dz4, db4 = sum dz4, dA3 = dz4 W4^T
  const uint16_t* dzc = dzb16;
  int ldz = 16;
  const float* dzf = dz4;
  for (int l = 3; l >= 0; --l) {
    const uint16_t* Ain = l == 0 ? Xb : Ab[l - 1];
    float* dW = G + mlp_param_offset(l, false);
    float* db = G + mlp_param_offset(l, true);
    // dW[fin][fout] = sum_b Ain[b][fin] dz[b][fout]
    gemm(Ain, 1, FIN[l], dzc, ldz, 1, dW, FOUT[l], FIN[l], FOUT[l], B, 0.f, s);
    k_colsum<<<l == 3 ? 1 : FOUT[l], 256, 0, s>>>(dzf, B, l == 3 ? 1 : FOUT[l], l == 3 ? 1 : FOUT[l], db);
    if (l > 0) {
      // dA[b][fin] = sum_o dz[b][o] W[fin][o]
      const uint16_t* W = Pb + mlp_param_offset(l, false);
      gemm(dzc, ldz, 1, W, 1, FOUT[l], dA[l - 1], FIN[l], B, FIN[l], FOUT[l], 0.f, s);
      k_gelu_back<<<nb((int64_t)B * FIN[l]), 256, 0, s>>>(dA[l - 1], Zb[l - 1], dZ[l - 1], dZbf[l - 1],
                                                          (int64_t)B * FIN[l]);
      dzc = dZbf[l - 1];
      dzf = dZ[l - 1];
      ldz = FIN[l];
    }
  }
}

void MlpState::adam(float lr, int t, hipStream_t s) {
  const float c1 = 1.f - powf(0.9f, (float)t), c2 = 1.f - powf(0.999f, (float)t);
  k_adam<<<nb(MLP_NPARAM_DEV), 256, 0, s>>>(P, G, Mo, Vo, Pb, MLP_NPARAM_DEV, lr, c1, c2);
}

void MlpState::sync_bf16(hipStream_t s) { k_to_bf16<<<nb(MLP_NPARAM_DEV), 256, 0, s>>>(P, Pb, MLP_NPARAM_DEV); }

__global__ void k_zero_f(float* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

void mlp_zero_loss(MlpState& M, int slot, hipStream_t s) { k_zero_f<<<1, 64, 0, s>>>(M.loss + slot, 1); }

void mlp_head_probs(MlpState& M, hipStream_t s) {
  k_head<<<nb(M.B), 256, 0, s>>>(M.Z[3], M.P + mlp_param_offset(3, true), nullptr, M.pout, nullptr, nullptr, nullptr,
                                 M.B, M.B, 1.f);
}

void MlpState::gather(const uint16_t* X, const float* y, const int32_t* idx, int64_t r0, int64_t nrows,
                      hipStream_t s) {
  k_gather_rows<<<nb((int64_t)B * MLP_NF), 256, 0, s>>>(X, y, idx, r0, nrows, B, Xb, yb);
}

}  // namespace dgmhd
