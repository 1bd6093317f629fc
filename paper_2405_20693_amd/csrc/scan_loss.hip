// Device-wide exclusive scans and the training-loss kernels of Eq. 8:
// L1 + lambda D-SSIM on projection stacks and 3D total variation on a block.
#include <utility>
#include "internal.h"

namespace gsk {

// ----------------------------------------------------------------- scans --

constexpr int kScanThreads = 1024;

// Exclusive scan of n u32 values by one 1024-thread workgroup; out has n + 1
// entries (out[n] = total, truncated to 32 bits); the exact total goes to
// *total.  Each thread owns a contiguous segment.
__device__ void wg_scan(const uint32_t *in, uint32_t *out, int64_t n, unsigned long long *total,
                        unsigned long long *sh) {
  const int tid = threadIdx.x;
  const int64_t per = (n + kScanThreads - 1) / kScanThreads;
  const int64_t b = tid * per, e = min(n, b + per);
  unsigned long long local = 0;
  for (int64_t i = b; i < e; ++i) local += in[i];
  sh[tid] = local;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 1024 segment sums
  for (int d = 1; d < kScanThreads; d <<= 1) {
    unsigned long long y = tid >= d ? sh[tid - d] : 0ull;
    __syncthreads();
    sh[tid] += y;
    __syncthreads();
  }
  unsigned long long run = sh[tid] - local;
  for (int64_t i = b; i < e; ++i) {
    uint32_t x = in[i];
    out[i] = (uint32_t)run;
    run += x;
  }
  if (tid == kScanThreads - 1) {
    out[n] = (uint32_t)sh[tid];
    *total = sh[tid];
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan2(const uint32_t *in0, uint32_t *out0,
                                                        int n0, const uint32_t *in1,
                                                        uint32_t *out1, int n1,
                                                        unsigned long long *totals) {
  __shared__ unsigned long long sh[kScanThreads];
  if (blockIdx.x == 0)
    wg_scan(in0, out0, n0, totals, sh);
  else
    wg_scan(in1, out1, n1, totals + 1, sh);
}

void launch_scan2(const uint32_t *in0, uint32_t *out0, int n0, const uint32_t *in1, uint32_t *out1,
                  int n1, unsigned long long *totals, hipStream_t s) {
  hipLaunchKernelGGL(k_scan2, dim3(in1 ? 2 : 1), dim3(kScanThreads), 0, s, in0, out0, n0, in1,
                     out1, n1, totals);
}

constexpr int kBigBlock = 4096;  // elements per block of the three-phase scan

// Block sums are formed in 64 bits and stored saturated at 2^32 - 1, so that
// the total over the blocks reaches 2^32 - 1 whenever the exact total does
// (the callers reject such totals); below that every block sum is exact.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *in, int64_t n,
                                                        uint32_t *block_sums) {
  __shared__ unsigned long long sh[kBlock];
  const int64_t b = (int64_t)blockIdx.x * kBigBlock;
  unsigned long long s = 0;
  for (int i = threadIdx.x; i < kBigBlock; i += kBlock)
    if (b + i < n) s += in[b + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = (uint32_t)min(sh[0], 0xffffffffull);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(const uint32_t *in, uint32_t *out,
                                                           int64_t n, unsigned long long *total) {
  __shared__ unsigned long long sh[kScanThreads];
  wg_scan(in, out, n, total, sh);
}

// Each block rescans its 4096 elements (16 per thread) from its base.
__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t *in, uint32_t *out, int64_t n,
                                                       const uint32_t *block_base, int64_t nb) {
  __shared__ uint32_t sh[kBlock];
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = block_base[nb];
  constexpr int per = kBigBlock / kBlock;
  const int64_t b = (int64_t)blockIdx.x * kBigBlock + (int64_t)threadIdx.x * per;
  uint32_t v[per];
  uint32_t s = 0;
  for (int i = 0; i < per; ++i) {
    v[i] = (b + i < n) ? in[b + i] : 0u;
    s += v[i];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int d = 1; d < kBlock; d <<= 1) {
    uint32_t y = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0u;
    __syncthreads();
    sh[threadIdx.x] += y;
    __syncthreads();
  }
  uint32_t run = block_base[blockIdx.x] + sh[threadIdx.x] - s;
  for (int i = 0; i < per; ++i) {
    if (b + i < n) out[b + i] = run;
    run += v[i];
  }
}

// out[0..n) = exclusive scan of in, out[n] = total (32 bits); *total exact
// below 2^32 - 1 and at least 2^32 - 1 otherwise.
// block_tmp needs 2 * ceil(n / 4096) + 1 entries.
void launch_scan_big(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *block_tmp,
                     unsigned long long *total, hipStream_t s) {
  int64_t nb = (n + kBigBlock - 1) / kBigBlock;
  if (nb < 1) nb = 1;
  uint32_t *sums = block_tmp, *base = block_tmp + nb;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, sums, base, nb, total);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, base, nb);
}

// ------------------------------------------------------------------ SSIM --
// Tiles of 32 x 32 output pixels per 256-thread workgroup with a 5-pixel halo;
// the 11-tap normalised Gaussian window (sigma 1.5) is separable.  Both passes
// are register-blocked: a thread computes 4 horizontally adjacent outputs of
// the row pass from one 14-value window, and 4 vertically adjacent outputs of
// the column pass from one 14-value window.

constexpr int kSW = 32, kSH = 32, kR = 5, kWin = 2 * kR + 1;
constexpr int kIW = kSW + 2 * kR, kIH = kSH + 2 * kR;  // 42 x 42 input region
constexpr int kRB = 4;                                  // outputs per thread per pass
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;

// The 11-tap Gaussian window (sigma 1.5) normalised to unit sum: weights
// exp(-(i-5)^2 / 4.5) / sum, evaluated in double and rounded to float once.
// Held as literals so that no call has to upload them (no per-device set-up,
// nothing for a graph capture to record).
__constant__ float c_win[kWin] = {
    0x1.0d956cp-10f, 0x1.f1fe02p-8f, 0x1.26eb18p-5f, 0x1.bff0fep-4f, 0x1.b43c40p-3f, 0x1.106560p-2f,
    0x1.b43c40p-3f,  0x1.bff0fep-4f, 0x1.26eb18p-5f, 0x1.f1fe02p-8f, 0x1.0d956cp-10f};

int ssim_num_blocks(int n, int h, int w) {
  return n * ((h + kSH - 1) / kSH) * ((w + kSW - 1) / kSW);
}

// Column pass: 4 consecutive output rows of one column per thread (256 tasks).
template <int Q>
__device__ inline void col_pass(const float (*hz)[kIH][kSW], float (*m)[kRB]) {
  const int c = threadIdx.x & (kSW - 1), r0 = (threadIdx.x / kSW) * kRB;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float win[kRB + kWin - 1];
#pragma unroll
    for (int k = 0; k < kRB + kWin - 1; ++k) win[k] = hz[q][r0 + k][c];
#pragma unroll
    for (int o = 0; o < kRB; ++o) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < kWin; ++k) acc = fmaf(c_win[k], win[o + k], acc);
      m[q][o] = acc;
    }
  }
}

// Computes the per-pixel SSIM map and the coefficient maps
//   D1 = dS/dmu_x - 2 mu_x dS/dsxx - mu_y dS/dsxy,  D2 = dS/dsxx,  D3 = dS/dsxy
// so that d mean(S) / d x = (blur(D1) + 2 x blur(D2) + y blur(D3)) / N.
// coef: [3][n][h][w] (may be NULL).  partials[block] = {sum S, sum |x - y|}.
__global__ __launch_bounds__(kBlock) void k_ssim_coeffs(const float *__restrict__ x,
                                                        const float *__restrict__ y, int n, int h,
                                                        int w, float *__restrict__ coef,
                                                        float *__restrict__ partials) {
  __shared__ float sin_[2][kIH][kIW];   // x, y
  __shared__ float hz[5][kIH][kSW];
  __shared__ float red[2][kBlock];
  const int tiles_x = (w + kSW - 1) / kSW, tiles_y = (h + kSH - 1) / kSH;
  const int b = blockIdx.x;
  const int img = b / (tiles_x * tiles_y), tt = b - img * tiles_x * tiles_y;
  const int ty = tt / tiles_x, tx = tt - ty * tiles_x;
  const int X0 = tx * kSW - kR, Y0 = ty * kSH - kR;
  const float *xi = x + (int64_t)img * h * w, *yi = y + (int64_t)img * h * w;
  const int tid = threadIdx.x;
  for (int i = tid; i < kIW * kIH; i += kBlock) {
    const int r = i / kIW, c = i - r * kIW;
    const int gy = Y0 + r, gx = X0 + c;
    const bool in = gx >= 0 && gx < w && gy >= 0 && gy < h;
    const float xv = in ? xi[(int64_t)gy * w + gx] : 0.f;
    const float yv = in ? yi[(int64_t)gy * w + gx] : 0.f;
    sin_[0][r][c] = xv;
    sin_[1][r][c] = yv;
  }
  __syncthreads();
  // row pass of x, y, x^2, y^2, xy from the x and y windows
  for (int task = tid; task < kIH * (kSW / kRB); task += kBlock) {
    const int r = task / (kSW / kRB), c0 = (task - r * (kSW / kRB)) * kRB;
    float wx[kRB + kWin - 1], wy[kRB + kWin - 1];
#pragma unroll
    for (int k = 0; k < kRB + kWin - 1; ++k) {
      wx[k] = sin_[0][r][c0 + k];
      wy[k] = sin_[1][r][c0 + k];
    }
#pragma unroll
    for (int o = 0; o < kRB; ++o) {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
      for (int k = 0; k < kWin; ++k) {
        const float wk = c_win[k], xv = wx[o + k], yv = wy[o + k];
        a0 = fmaf(wk, xv, a0);
        a1 = fmaf(wk, yv, a1);
        a2 = fmaf(wk, xv * xv, a2);
        a3 = fmaf(wk, yv * yv, a3);
        a4 = fmaf(wk, xv * yv, a4);
      }
      hz[0][r][c0 + o] = a0; hz[1][r][c0 + o] = a1; hz[2][r][c0 + o] = a2;
      hz[3][r][c0 + o] = a3; hz[4][r][c0 + o] = a4;
    }
  }
  __syncthreads();
  float m[5][kRB];
  col_pass<5>(hz, m);
  const int c = tid & (kSW - 1), r0 = (tid / kSW) * kRB;
  const int64_t N = (int64_t)n * h * w;
  float ssum = 0.f, lsum = 0.f;
#pragma unroll
  for (int o = 0; o < kRB; ++o) {
    const int gy = ty * kSH + r0 + o, gx = tx * kSW + c;
    if (gx >= w || gy >= h) continue;
    const float mx = m[0][o], my = m[1][o];
    const float sxx = m[2][o] - mx * mx, syy = m[3][o] - my * my, sxy = m[4][o] - mx * my;
    const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
    const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
    // one hardware reciprocal (about 1 ulp) serves the three quotients:
    // 1/B1 = B2/(B1 B2), 1/B2 = B1/(B1 B2)
    const float iB = __builtin_amdgcn_rcpf(B1 * B2);
    const float S = A1 * A2 * iB;
    const float dmx = 2.f * my * A2 * iB - 2.f * mx * S * (B2 * iB);
    const float dsxx = -S * (B1 * iB);
    const float dsxy = 2.f * A1 * iB;
    const int64_t off = (int64_t)img * h * w + (int64_t)gy * w + gx;
    if (coef) {
      coef[off] = dmx - 2.f * mx * dsxx - my * dsxy;
      coef[N + off] = dsxx;
      coef[2 * N + off] = dsxy;
    }
    ssum += S;
    lsum += fabsf(sin_[0][r0 + o + kR][c + kR] - sin_[1][r0 + o + kR][c + kR]);
  }
  red[0][tid] = ssum;
  red[1][tid] = lsum;
  __syncthreads();
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if (tid < d) {
      red[0][tid] += red[0][tid + d];
      red[1][tid] += red[1][tid + d];
    }
    __syncthreads();
  }
  if (tid == 0) {
    partials[2 * b] = red[0][0];
    partials[2 * b + 1] = red[1][0];
  }
}

void launch_ssim_coeffs(const float *x, const float *y, int n, int h, int w, float *coef,
                        float *partials, hipStream_t s) {
  hipLaunchKernelGGL(k_ssim_coeffs, dim3(ssim_num_blocks(n, h, w)), dim3(kBlock), 0, s, x, y, n, h,
                     w, coef, partials);
}

// Loss and gradient in one pass per 32 x 32 output tile (stacks too small to
// fill the chip with the marching kernel below; grad may be NULL).  The gradient at a
// pixel needs the coefficient maps D1..D3 on a 5-pixel halo, and those need
// the inputs on a further 5-pixel halo, so the workgroup stages x and y over
// 52 x 52, computes the five blurred moments and D1..D3 over the 42 x 42
// coefficient region (zero outside the image: the maps are only defined on
// image pixels), then blurs the coefficients for its 32 x 32 outputs.  Each
// plane is blurred separately (row pass to LDS, column pass to registers) to
// keep LDS at about 32 KB; the coefficient maps overwrite the staged inputs.
// grad = (sign(x - y) - lambda (blur(D1) + 2 x blur(D2) + y blur(D3))) / N;
// partials[block] = {sum S, sum |x - y|} over the tile's image pixels.
constexpr int kDW = kSW + 2 * kR;  // 42: coefficient region edge
constexpr int kXW = kDW + 2 * kR;  // 52: input region edge
constexpr int kF1 = 7;             // stage 1: outputs per row task and per column task
constexpr int kF2 = 8;             // stage 2: outputs per row task
constexpr int kR1 = 11, kRSeg = 4;  // stage 1 row pass: outputs per task, tasks per row
static_assert(kR1 * kRSeg >= kDW && kR1 * (kRSeg - 1) < kDW, "row segments cover the row");

__global__ __launch_bounds__(kBlock) void k_ssim_fused(const float *__restrict__ x,
                                                       const float *__restrict__ y, int n, int h,
                                                       int w, float lambda,
                                                       float *__restrict__ grad,
                                                       float *__restrict__ partials) {
  __shared__ float s_in[2 * kXW * kXW];  // x, y over 52 x 52; later D1..D3 over 42 x 42
  __shared__ float s_h[kXW * kDW];       // row-pass output of one plane
  __shared__ float red[2][kBlock];
  static_assert(3 * kDW * kDW <= 2 * kXW * kXW, "the coefficient maps fit the input buffer");
  float *sx = s_in, *sy = s_in + kXW * kXW;
  const int tiles_x = (w + kSW - 1) / kSW, tiles_y = (h + kSH - 1) / kSH;
  const int b = blockIdx.x;
  const int img = b / (tiles_x * tiles_y), tt = b - img * tiles_x * tiles_y;
  const int ty = tt / tiles_x, tx = tt - ty * tiles_x;
  const int X0 = tx * kSW, Y0 = ty * kSH;  // first output pixel
  const int64_t ib = (int64_t)img * h * w;
  const int tid = threadIdx.x;
  for (int i = tid; i < kXW * kXW; i += kBlock) {
    const int r = i / kXW, c = i - r * kXW;
    const int gy = Y0 - 2 * kR + r, gx = X0 - 2 * kR + c;
    const bool in = gx >= 0 && gx < w && gy >= 0 && gy < h;
    sx[i] = in ? x[ib + (int64_t)gy * w + gx] : 0.f;
    sy[i] = in ? y[ib + (int64_t)gy * w + gx] : 0.f;
  }
  __syncthreads();
  // stage 1: blurred x, y, x^2, y^2, xy at the thread's 7 coefficient positions
  // (column dc, rows dr0 .. dr0 + 6 of the 42 x 42 region; 252 threads)
  const bool t1 = tid < (kDW / kF1) * kDW;
  const int dc = tid % kDW, dr0 = (tid / kDW) * kF1;
  float m[5][kF1];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    // row pass: 52 rows x 4 segments of kR1 outputs (the last one 9), one
    // task per thread
    if (tid < kXW * kRSeg) {
      const int r = tid / kRSeg, c0 = (tid - r * kRSeg) * kR1;
      float win[kR1 + kWin - 1];
#pragma unroll
      for (int k = 0; k < kR1 + kWin - 1; ++k) {
        const bool in = c0 + k < kXW;  // the last segment's window ends at the row
        const float xv = in ? sx[r * kXW + c0 + k] : 0.f, yv = in ? sy[r * kXW + c0 + k] : 0.f;
        win[k] = q == 0 ? xv : q == 1 ? yv : q == 2 ? xv * xv : q == 3 ? yv * yv : xv * yv;
      }
#pragma unroll
      for (int o = 0; o < kR1; ++o) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kWin; ++k) acc = fmaf(c_win[k], win[o + k], acc);
        if (c0 + o < kDW) s_h[r * kDW + c0 + o] = acc;
      }
    }
    __syncthreads();
    if (t1) {
      float win[kF1 + kWin - 1];
#pragma unroll
      for (int k = 0; k < kF1 + kWin - 1; ++k) win[k] = s_h[(dr0 + k) * kDW + dc];
#pragma unroll
      for (int o = 0; o < kF1; ++o) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kWin; ++k) acc = fmaf(c_win[k], win[o + k], acc);
        m[q][o] = acc;
      }
    }
    __syncthreads();
  }
  // SSIM, its derivative maps, and the tile's sums (interior positions only)
  float ssum = 0.f, lsum = 0.f;
  float dv[3][kF1];
#pragma unroll
  for (int o = 0; o < kF1; ++o) {
    dv[0][o] = dv[1][o] = dv[2][o] = 0.f;
    const int dr = dr0 + o;
    const int gy = Y0 - kR + dr, gx = X0 - kR + dc;
    if (!t1 || gx < 0 || gx >= w || gy < 0 || gy >= h) continue;
    const float mx = m[0][o], my = m[1][o];
    const float sxx = m[2][o] - mx * mx, syy = m[3][o] - my * my, sxy = m[4][o] - mx * my;
    const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
    const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
    // one hardware reciprocal (about 1 ulp) serves the three quotients:
    // 1/B1 = B2/(B1 B2), 1/B2 = B1/(B1 B2)
    const float iB = __builtin_amdgcn_rcpf(B1 * B2);
    const float S = A1 * A2 * iB;
    const float dmx = 2.f * my * A2 * iB - 2.f * mx * S * (B2 * iB);
    const float dsxx = -S * (B1 * iB);
    const float dsxy = 2.f * A1 * iB;
    dv[0][o] = dmx - 2.f * mx * dsxx - my * dsxy;
    dv[1][o] = dsxx;
    dv[2][o] = dsxy;
    if (dr >= kR && dr < kR + kSH && dc >= kR && dc < kR + kSW) {
      ssum += S;
      const int i = (dr + kR) * kXW + dc + kR;
      lsum += fabsf(sx[i] - sy[i]);
    }
  }
  red[0][tid] = ssum;
  red[1][tid] = lsum;
  __syncthreads();  // the staged inputs are no longer read
  if (grad) {
    if (t1) {
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int o = 0; o < kF1; ++o) s_in[(q * kDW + dr0 + o) * kDW + dc] = dv[q][o];
    }
    __syncthreads();
    // stage 2: blurred D1..D3 at 4 outputs per thread (column c, rows r0 .. r0 + 3)
    const int c = tid & (kSW - 1), r0 = (tid / kSW) * kRB;
    float bd[3][kRB];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float *D = s_in + q * kDW * kDW;
      for (int task = tid; task < kDW * (kSW / kF2); task += kBlock) {
        const int r = task / (kSW / kF2), c0 = (task - r * (kSW / kF2)) * kF2;
        float win[kF2 + kWin - 1];
#pragma unroll
        for (int k = 0; k < kF2 + kWin - 1; ++k) win[k] = D[r * kDW + c0 + k];
#pragma unroll
        for (int o = 0; o < kF2; ++o) {
          float acc = 0.f;
#pragma unroll
          for (int k = 0; k < kWin; ++k) acc = fmaf(c_win[k], win[o + k], acc);
          s_h[r * kSW + c0 + o] = acc;
        }
      }
      __syncthreads();
      float win[kRB + kWin - 1];
#pragma unroll
      for (int k = 0; k < kRB + kWin - 1; ++k) win[k] = s_h[(r0 + k) * kSW + c];
#pragma unroll
      for (int o = 0; o < kRB; ++o) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < kWin; ++k) acc = fmaf(c_win[k], win[o + k], acc);
        bd[q][o] = acc;
      }
      __syncthreads();
    }
    const float invN = 1.f / (float)((int64_t)n * h * w);
#pragma unroll
    for (int o = 0; o < kRB; ++o) {
      const int gy = Y0 + r0 + o, gx = X0 + c;
      if (gx >= w || gy >= h) continue;
      const int64_t off = ib + (int64_t)gy * w + gx;
      const float xv = x[off], yv = y[off];
      const float dssim = bd[0][o] + 2.f * xv * bd[1][o] + yv * bd[2][o];
      const float d = xv - yv;
      const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
      grad[off] = (sg - lambda * dssim) * invN;
    }
  }
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if (tid < d) {
      red[0][tid] += red[0][tid + d];
      red[1][tid] += red[1][tid + d];
    }
    __syncthreads();
  }
  if (tid == 0) {
    partials[2 * b] = red[0][0];
    partials[2 * b + 1] = red[1][0];
  }
}

void launch_ssim_fused(const float *x, const float *y, int n, int h, int w, float lambda_ssim,
                       float *grad, float *partials, hipStream_t s) {
  hipLaunchKernelGGL(k_ssim_fused, dim3(ssim_num_blocks(n, h, w)), dim3(kBlock), 0, s, x, y, n, h,
                     w, lambda_ssim, grad, partials);
}

// Loss and gradient of L1 + lambda D-SSIM (Eq. 8) in one pass that marches
// down the image.  One wavefront owns a strip of 64 coefficient columns (one
// per lane: the strip's 54 output columns and a 5-column halo on each side)
// and a segment of output rows, and walks the input rows top to bottom:
//   row r of x, y, x^2 + y^2 and x y  -> LDS, blurred along the row (11 taps)
//   the last 11 such rows, held in registers -> blurred moments at row r - 5
//   the SSIM map S and the maps D1..D3 at row r - 5 -> LDS, blurred along the row
//   the last 11 of those rows -> blur(D1..D3) at row r - 10 -> the gradient
// with D2 = dS/dsxx, D3 = dS/dsxy, D1 = dS/dmx - 2 mx D2 - my D3, so that
//   d mean(S) / d x = (blur(D1) + 2 x blur(D2) + y blur(D3)) / N.
// The coefficient maps are zero outside the image (they are only defined on
// image pixels) and the inputs are zero-padded, as in the window sums of the
// definition.  SSIM needs sxx and syy only as their sum, so x^2 and y^2 are
// blurred as one plane.  A strip recomputes 10 halo columns of the first
// stage; a segment recomputes 20 halo rows; nothing else is evaluated twice.
// grad = (sign(x - y) - lambda (blur(D1) + 2 x blur(D2) + y blur(D3))) / N
// (only when kGrad); partials[wave] = {sum S, sum |x - y|} over its output
// pixels, added by the finish kernel in wave order.
constexpr int kMLanes = 64;               // coefficient columns per strip, one per lane
constexpr int kMOut = kMLanes - 2 * kR;   // 54 output columns per strip
constexpr int kMIn = kMLanes + 2 * kR;    // 74 input columns per strip

// The march serves stacks that give it at least 2048 wavefronts with
// segments of 64 rows (two per SIMD); its sequential walk down a segment
// leaves a small stack latency-bound, and those take the tile kernel.
bool loss_use_march(int n, int h, int w) {
  return (int64_t)n * ((w + kMOut - 1) / kMOut) * ((h + 63) / 64) >= 2048;
}

// Output rows per segment: the longest of 256, 128, 64 that still gives the
// launch at least 4096 wavefronts (four per SIMD), or 64.
int loss_march_rows(int n, int h, int w) {
  const int64_t strips = (w + kMOut - 1) / kMOut;
  int rows = 256;
  while (rows > 64 && (int64_t)n * strips * ((h + rows - 1) / rows) < 4096) rows /= 2;
  return rows;
}

// Partial-sum pairs of the loss kernel a stack takes (at most one per 32 x 32
// tile either way).
int loss_image_blocks(int n, int h, int w) {
  if (!loss_use_march(n, h, w)) return ssim_num_blocks(n, h, w);
  const int rows = loss_march_rows(n, h, w);
  return n * ((h + rows - 1) / rows) * ((w + kMOut - 1) / kMOut);
}

// Image access through raw buffer descriptors, one per image and array,
// bounded by the image's bytes: an offset at or beyond the bound reads zero
// and drops a store.  Rows and columns outside the image get such an offset,
// so the zero padding of the window sums needs no branch, and no load or
// store sits under a branch (the compiler can then wait for each load alone
// instead of for every memory operation in flight).
constexpr uint32_t kOutside = 0x80000000u;  // beyond any image of < 2^29 pixels
constexpr int kRsrcWord3 = 0x00020000;      // raw 32-bit access on gfx9-family chips

__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const float *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0, bytes, kRsrcWord3);
}
__device__ __forceinline__ float rsrc_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

// The workgroup is one wavefront, whose LDS operations execute in program
// order (wave_lds_order keeps the compiler from reordering them).

// One wavefront's state; the functions below are inlined into the kernel,
// so it lives in registers (the rings are indexed by compile-time slots).
struct MarchState {
  __amdgpu_buffer_rsrc_t rx, ry, rg;
  int h, w, Y0, rows_here, T, ca, cb, cc, lane;
  bool a_col, b_col, out_col;
  float lambda, invN;
  float r1[4][kWin], r2[3][kWin];  // the last 11 rows of each stage's row blur
  float ssum, lsum;
  float xa, ya, xb, yb;  // the current input row's values
};

// Byte offset of (row r, column c) in an image, or kOutside.
__device__ __forceinline__ uint32_t pix_off(const MarchState &m, int r, int c, bool ok) {
  return ok && r >= 0 && r < m.h ? (uint32_t)(r * m.w + c) * 4u : kOutside;
}

__device__ __forceinline__ void march_load(MarchState &m, int r) {
  const uint32_t oa = pix_off(m, r, m.ca, m.a_col), ob = pix_off(m, r, m.cb, m.b_col);
  m.xa = rsrc_load(m.rx, oa);
  m.ya = rsrc_load(m.ry, oa);
  m.xb = rsrc_load(m.rx, ob);
  m.yb = rsrc_load(m.ry, ob);
}

// Step t of the march (input row Y0 - 10 + t); U = t mod 11 is the ring slot.
template <bool kGrad, int U>
__device__ __forceinline__ void march_step(MarchState &m, int t, float (*s_in)[kMIn],
                                           float (*s_d)[kMLanes]) {
  if (t >= m.T) return;
  const int lane = m.lane;
  const int r = m.Y0 - 2 * kR + t;
  // the inputs at the output pixel whose gradient this step completes (row
  // r - 10), loaded before the next row's prefetch so that waiting for them
  // leaves the prefetch in flight (vector memory counts complete in order)
  const bool gstep = kGrad && t >= 4 * kR && m.out_col;
  const uint32_t goff = pix_off(m, r - 2 * kR, m.cc, gstep);
  float gx = 0.f, gy = 0.f;
  if (kGrad) {
    gx = rsrc_load(m.rx, goff);
    gy = rsrc_load(m.ry, goff);
  }
  // the L1 term at the strip's output pixels of this row (lanes 10..63)
  const bool l1 = r >= m.Y0 && r < m.Y0 + m.rows_here && lane >= 2 * kR && m.a_col;
  m.lsum += l1 ? fabsf(m.xa - m.ya) : 0.f;
  s_in[0][lane] = m.xa;
  s_in[1][lane] = m.ya;
  s_in[2][lane] = fmaf(m.xa, m.xa, m.ya * m.ya);
  s_in[3][lane] = m.xa * m.ya;
  if (lane < 2 * kR) {
    s_in[0][kMLanes + lane] = m.xb;
    s_in[1][kMLanes + lane] = m.yb;
    s_in[2][kMLanes + lane] = fmaf(m.xb, m.xb, m.yb * m.yb);
    s_in[3][kMLanes + lane] = m.xb * m.yb;
  }
  march_load(m, r + 1);  // in flight while this row is blurred
  wave_lds_order();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kWin; ++k) acc = fmaf(c_win[k], s_in[q][lane + k], acc);
    m.r1[q][U] = acc;
  }
  float d1 = 0.f, d2 = 0.f, d3 = 0.f;
  const int rc = r - kR;  // the coefficient row completed by this input row
  if (t >= 2 * kR) {
    // blurred moments at row rc, oldest row first
    float mo[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < kWin; ++k) acc = fmaf(c_win[k], m.r1[q][(U + 1 + k) % kWin], acc);
      mo[q] = acc;
    }
    if (rc >= 0 && rc < m.h && m.cc >= 0 && m.cc < m.w) {
      const float mx = mo[0], my = mo[1];
      const float mm = mx * mx + my * my;
      const float A1 = 2.f * mx * my + kC1, A2 = 2.f * (mo[3] - mx * my) + kC2;
      const float B1 = mm + kC1, B2 = (mo[2] - mm) + kC2;
      // one hardware reciprocal (about 1 ulp) serves the three quotients:
      // 1/B1 = B2/(B1 B2), 1/B2 = B1/(B1 B2)
      const float iB = __builtin_amdgcn_rcpf(B1 * B2);
      const float S = A1 * A2 * iB;
      if (m.out_col && rc >= m.Y0 && rc < m.Y0 + m.rows_here) m.ssum += S;
      if (kGrad) {
        const float dmx = 2.f * my * A2 * iB - 2.f * mx * S * (B2 * iB);
        const float dsxx = -S * (B1 * iB);
        const float dsxy = 2.f * A1 * iB;
        d1 = dmx - 2.f * mx * dsxx - my * dsxy;
        d2 = dsxx;
        d3 = dsxy;
      }
    }
  }
  if (kGrad) {
    s_d[0][lane] = d1;
    s_d[1][lane] = d2;
    s_d[2][lane] = d3;
  }
  wave_lds_order();  // s_d written; every lane has read s_in
  if (!kGrad || t < 2 * kR) return;
  const bool mid = lane >= kR && lane < kR + kMOut;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    float acc = 0.f;
    if (mid) {
#pragma unroll
      for (int k = 0; k < kWin; ++k) acc = fmaf(c_win[k], s_d[q][lane - kR + k], acc);
    }
    m.r2[q][U] = acc;
  }
  if (t >= 4 * kR) {
    // blur(D1..D3) and the gradient at output row rc - 5 (stored by the
    // lanes that own an output pixel; the others' offset is outside)
    float bd[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < kWin; ++k) acc = fmaf(c_win[k], m.r2[q][(U + 1 + k) % kWin], acc);
      bd[q] = acc;
    }
    const float dssim = bd[0] + 2.f * gx * bd[1] + gy * bd[2];
    const float d = gx - gy;
    const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
    const float g = (sg - m.lambda * dssim) * m.invN;
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(g), m.rg, (int)goff, 0, 0);
  }
}

template <bool kGrad, int... U>
__device__ __forceinline__ void march_round(MarchState &m, int t0, float (*s_in)[kMIn],
                                            float (*s_d)[kMLanes],
                                            std::integer_sequence<int, U...>) {
  (march_step<kGrad, U>(m, t0 + U, s_in, s_d), ...);
}

template <bool kGrad>
__global__ __launch_bounds__(kMLanes) void k_ssim_march(const float *__restrict__ x,
                                                        const float *__restrict__ y, int n, int h,
                                                        int w, int rows, float lambda,
                                                        float *__restrict__ grad,
                                                        float *__restrict__ partials) {
  __shared__ float s_in[4][kMIn];    // x, y, x^2 + y^2, x y of the current input row
  __shared__ float s_d[3][kMLanes];  // D1, D2, D3 of the current coefficient row
  const int strips = (w + kMOut - 1) / kMOut, segs = (h + rows - 1) / rows;
  const int b = blockIdx.x;
  const int strip = b % strips, rest = b / strips;
  const int seg = rest % segs, img = rest / segs;
  MarchState m;
  m.lane = threadIdx.x;
  m.h = h;
  m.w = w;
  m.Y0 = seg * rows;  // first output row
  const int X0 = strip * kMOut;  // first output column
  const int64_t ib = (int64_t)img * h * w;
  const int bytes = h * w * 4;  // below 2^31: checked on the host
  m.rx = image_rsrc(x + ib, bytes);
  m.ry = image_rsrc(y + ib, bytes);
  m.rg = image_rsrc(kGrad ? grad + ib : x + ib, kGrad ? bytes : 0);
  m.cc = X0 - kR + m.lane;  // the lane's coefficient column
  m.out_col = m.lane >= kR && m.lane < kR + kMOut && m.cc < w;
  m.rows_here = min(rows, h - m.Y0);
  m.T = m.rows_here + 4 * kR;  // input rows Y0 - 10 .. Y0 + rows_here + 9
  // the lane's input columns: X0 - 10 + lane, and X0 + 54 + lane for lane < 10
  m.ca = X0 - 2 * kR + m.lane;
  m.cb = X0 + kMOut + m.lane;
  m.a_col = m.ca >= 0 && m.ca < w;
  m.b_col = m.lane < 2 * kR && m.cb < w;
  m.lambda = lambda;
  m.invN = 1.f / (float)((int64_t)n * h * w);
  m.ssum = m.lsum = 0.f;
#pragma unroll
  for (int k = 0; k < kWin; ++k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) m.r1[q][k] = 0.f;
#pragma unroll
    for (int q = 0; q < 3; ++q) m.r2[q][k] = 0.f;
  }
  march_load(m, m.Y0 - 2 * kR);
  for (int t0 = 0; t0 < m.T; t0 += kWin)
    march_round<kGrad>(m, t0, s_in, s_d, std::make_integer_sequence<int, kWin>{});
  // the wave's sums, in a fixed order
  float ssum = m.ssum, lsum = m.lsum;
#pragma unroll
  for (int d = kMLanes / 2; d > 0; d >>= 1) {
    ssum += __shfl_down(ssum, d, kMLanes);
    lsum += __shfl_down(lsum, d, kMLanes);
  }
  if (m.lane == 0) {
    partials[2 * b] = ssum;
    partials[2 * b + 1] = lsum;
  }
}

void launch_ssim_march(const float *x, const float *y, int n, int h, int w, float lambda_ssim,
                       float *grad, float *partials, hipStream_t s) {
  if (!loss_use_march(n, h, w)) {
    launch_ssim_fused(x, y, n, h, w, lambda_ssim, grad, partials, s);
    return;
  }
  const int rows = loss_march_rows(n, h, w), nb = loss_image_blocks(n, h, w);
  if (grad)
    hipLaunchKernelGGL(k_ssim_march<true>, dim3(nb), dim3(kMLanes), 0, s, x, y, n, h, w, rows,
                       lambda_ssim, grad, partials);
  else
    hipLaunchKernelGGL(k_ssim_march<false>, dim3(nb), dim3(kMLanes), 0, s, x, y, n, h, w, rows,
                       lambda_ssim, grad, partials);
}

// Sums the per-block partials in double, in a fixed order.
__global__ __launch_bounds__(1024) void k_loss_finish(const float *__restrict__ partials, int n_part,
                                                      double N, float lambda,
                                                      float *__restrict__ out) {
  __shared__ double r0[1024], r1[1024];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n_part; i += 1024) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int d = 512; d > 0; d >>= 1) {
    if (threadIdx.x < d) {
      r0[threadIdx.x] += r0[threadIdx.x + d];
      r1[threadIdx.x] += r1[threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ssim = r0[0] / N, l1 = r1[0] / N;
    out[0] = (float)(l1 + lambda * (1.0 - ssim));
    out[1] = (float)l1;
    out[2] = (float)ssim;
  }
}

void launch_loss_finish(const float *partials, int n_part, int n, int h, int w, float lambda_ssim,
                        float *loss_out, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(1024), 0, s, partials, n_part,
                     (double)n * h * w, lambda_ssim, loss_out);
}

// -------------------------------------------------------------------- TV --

int tv_num_blocks(int nx, int ny, int nz) {
  int64_t n = (int64_t)nx * ny * nz;
  return (int)((n + kBlock - 1) / kBlock);
}

__device__ inline float sgnf(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

// One thread per voxel: its forward differences' share of the TV sum and the
// gradient weight * dTV/dv (each difference pulls its two endpoints).
__global__ __launch_bounds__(kBlock) void k_tv(const float *__restrict__ v, int nx, int ny, int nz,
                                               float weight, float *__restrict__ grad,
                                               int accumulate, float *__restrict__ partials) {
  __shared__ float red[kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t n = (int64_t)nx * ny * nz;
  float s = 0.f;
  if (i < n) {
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / ((int64_t)nx * ny));
    const float c = v[i];
    const float ix = nx > 1 ? 1.f / (float)((int64_t)nz * ny * (nx - 1)) : 0.f;
    const float iy = ny > 1 ? 1.f / (float)((int64_t)nz * (ny - 1) * nx) : 0.f;
    const float iz = nz > 1 ? 1.f / (float)((int64_t)(nz - 1) * ny * nx) : 0.f;
    float g = 0.f;
    if (x + 1 < nx) { float d = v[i + 1] - c; s += fabsf(d) * ix; g -= sgnf(d) * ix; }
    if (x > 0) g += sgnf(c - v[i - 1]) * ix;
    if (y + 1 < ny) { float d = v[i + nx] - c; s += fabsf(d) * iy; g -= sgnf(d) * iy; }
    if (y > 0) g += sgnf(c - v[i - nx]) * iy;
    const int64_t pl = (int64_t)nx * ny;
    if (z + 1 < nz) { float d = v[i + pl] - c; s += fabsf(d) * iz; g -= sgnf(d) * iz; }
    if (z > 0) g += sgnf(c - v[i - pl]) * iz;
    if (grad) grad[i] = accumulate ? grad[i] + weight * g : weight * g;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

void launch_tv(const float *vol, int nx, int ny, int nz, float weight, float *grad, int accumulate,
               float *partials, int *n_part, hipStream_t s) {
  int nb = tv_num_blocks(nx, ny, nz);
  *n_part = nb;
  hipLaunchKernelGGL(k_tv, dim3(nb), dim3(kBlock), 0, s, vol, nx, ny, nz, weight, grad, accumulate,
                     partials);
}

__global__ __launch_bounds__(1024) void k_tv_finish(const float *__restrict__ partials, int n_part,
                                                    float *__restrict__ out) {
  __shared__ double r[1024];
  double a = 0.0;
  for (int i = threadIdx.x; i < n_part; i += 1024) a += partials[i];
  r[threadIdx.x] = a;
  __syncthreads();
  for (int d = 512; d > 0; d >>= 1) {
    if (threadIdx.x < d) r[threadIdx.x] += r[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)r[0];
}

void launch_tv_finish(const float *partials, int n_part, float *loss_out, hipStream_t s) {
  hipLaunchKernelGGL(k_tv_finish, dim3(1), dim3(1024), 0, s, partials, n_part, loss_out);
}

}  // namespace gsk
