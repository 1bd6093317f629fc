// Device-wide exclusive scans and the training-loss kernels of Eq. 8:
// L1 + lambda D-SSIM on projection stacks and 3D total variation on a block.
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

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *in, int64_t n,
                                                        uint32_t *block_sums) {
  __shared__ uint32_t sh[kBlock];
  const int64_t b = (int64_t)blockIdx.x * kBigBlock;
  uint32_t s = 0;
  for (int i = threadIdx.x; i < kBigBlock; i += kBlock)
    if (b + i < n) s += in[b + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = sh[0];
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

// out[0..n) = exclusive scan of in, out[n] = total (32 bits), *total exact.
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

// Loss and gradient in one pass per 32 x 32 output tile.  The gradient at a
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
