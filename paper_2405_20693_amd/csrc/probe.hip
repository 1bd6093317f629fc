// Issue-rate probes of the two VALU operations the render kernels are built
// from: FP32 fused multiply-add (v_fmac_f32, not packed) and the base-2
// exponential (v_exp_f32).  Each lane runs independent dependency chains so
// that the rate, not the latency, is measured; the grid fills every SIMD.
#include "../../include/gs_probe.h"
#include "internal.h"

namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 16;

__global__ __launch_bounds__(256) void k_probe_fma(float *out, int iters, float a, float b) {
  float x[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) x[k] = (float)(threadIdx.x + k) * 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int k = 0; k < kChains; ++k) x[k] = fmaf(x[k], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += x[k];
  if (s == 1234.5f) out[blockIdx.x * 256 + threadIdx.x] = s;  // keeps the chains live
}

__global__ __launch_bounds__(256) void k_probe_exp2(float *out, int iters, float a) {
  float x[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) x[k] = a * (float)(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int k = 0; k < kChains; ++k) x[k] = __builtin_amdgcn_exp2f(x[k]);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += x[k];
  if (s == 1234.5f) out[blockIdx.x * 256 + threadIdx.x] = s;
}

gs_status time_kernel(bool exp2, int blocks, int iters, float *out, hipStream_t s, double *ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return GS_EHIP;
  gs_status st = GS_OK;
  float best = 0.f;
  for (int rep = 0; rep < 4 && st == GS_OK; ++rep) {  // the first launch warms up
    (void)hipEventRecord(e0, s);
    if (exp2)
      hipLaunchKernelGGL(k_probe_exp2, dim3(blocks), dim3(256), 0, s, out, iters, -1e-3f);
    else
      hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
    (void)hipEventRecord(e1, s);
    float t = 0.f;
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess)
      st = GS_EHIP;
    if (rep > 0 && (best == 0.f || t < best)) best = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return st;
}

}  // namespace

extern "C" {

gs_status gs_probe_alu(double *fma_per_s, double *exp2_per_s, hipStream_t stream) {
  if (!fma_per_s || !exp2_per_s) {
    gsk::set_last_error("output pointer is NULL");
    return GS_EINVAL;
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return GS_EHIP;
  const int blocks = cus * 8;  // eight 256-thread workgroups per CU: 8 waves per SIMD
  float *out = nullptr;
  if (hipMalloc(&out, sizeof(float) * 256 * (size_t)blocks) != hipSuccess) return GS_ENOMEM;
  const int iters = 256;
  const double lanes = 256.0 * blocks * iters * kUnroll * kChains;
  double ms = 0.0;
  gs_status st = time_kernel(false, blocks, iters, out, stream, &ms);
  if (st == GS_OK) *fma_per_s = lanes / (ms * 1e-3);
  if (st == GS_OK) st = time_kernel(true, blocks, iters / 4, out, stream, &ms);
  if (st == GS_OK) *exp2_per_s = lanes / 4 / (ms * 1e-3);
  (void)hipFree(out);
  return st;
}

}  // extern "C"
