// Learned troubled-cell indicator: device state and host helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace dgmhd {

constexpr int MLP_NF = 256;                 // input features (234 used, zero padded)
constexpr int MLP_NPARAM = 24833;           // public FP32 parameter count
constexpr int MLP_NPARAM_DEV = 25808;       // device layout (output layer padded to 16 columns)

size_t mlp_param_offset(int layer, bool bias);
void mlp_pack(const float* pub, std::vector<float>& dev);
void mlp_unpack(const std::vector<float>& dev, float* pub);

struct MlpState {
  int B = 0;                                  // batch rows (multiple of 16)
  float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;  // FP32 masters, gradients, Adam moments
  uint16_t* Pb = nullptr;                     // BF16 copy used by the matrix products
  uint16_t* Xb = nullptr;                     // batch features
  float* yb = nullptr;                        // batch labels
  float *Z[4] = {}, *Zb[4] = {}, *dA[4] = {}, *dZ[4] = {};
  uint16_t *Ab[4] = {}, *dZbf[4] = {};
  float *dz4 = nullptr, *pout = nullptr, *loss = nullptr;
  uint16_t* dzb16 = nullptr;
  double* sigma = nullptr;                    // feature scales (9 variables)
  int loss_slot = 0;
  bool have_params = false;
  bool have_sigma = false;
  std::vector<void*> bufs, pbufs;
  bool alloc_params(std::string& err);
  bool alloc(int batch, std::string& err);
  void release();
  void forward(hipStream_t s);
  void backward(int64_t nvalid, hipStream_t s);
  void adam(float lr, int t, hipStream_t s);
  void sync_bf16(hipStream_t s);
  void gather(const uint16_t* X, const float* y, const int32_t* idx, int64_t r0, int64_t nrows, hipStream_t s);
  ~MlpState() { release(); }
};

void mlp_zero_loss(MlpState& M, int slot, hipStream_t s);
void mlp_head_probs(MlpState& M, hipStream_t s);

}  // namespace dgmhd
