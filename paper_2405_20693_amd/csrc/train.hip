// Kernels of the optimisation loop (Sec. 3.3, Sec. 4.1): fused activation +
// Adam update, activation conversions, adaptive density control (count, scan,
// scatter) and the reductions and slice stacks of the 3D metrics.  All are
// HBM-bound elementwise or gather passes; each thread owns whole output
// elements, so there are no atomics and results are deterministic.
#include "internal.h"

namespace gsk {

namespace {

__device__ inline float softplus_f(float x) { return x > 20.f ? x : log1pf(expf(x)); }
__device__ inline float softplus_inv_f(float y) { return y > 20.f ? y : logf(expm1f(y)); }

// One element of the flat parameter vector [mean 3n | log_scale 3n | quat 4n |
// density_raw n]: segment and index inside it.
__device__ inline void segment_of(int64_t e, int64_t n, int &seg, int64_t &i) {
  if (e < 3 * n) {
    seg = 0;
    i = e;
  } else if (e < 6 * n) {
    seg = 1;
    i = e - 3 * n;
  } else if (e < 10 * n) {
    seg = 2;
    i = e - 6 * n;
  } else {
    seg = 3;
    i = e - 10 * n;
  }
}

__global__ __launch_bounds__(kBlock) void k_adam(AdamArgs a) {
  // a guarded step is skipped when a guarding plan recorded a call that
  // overflowed its reservation (its gradients are incomplete)
  for (int k = 0; k < 2; ++k)
    if (a.guard[k] && (a.guard[k][6] | a.guard[k][7])) return;
  const int64_t total = 11 * a.n;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kBlock) {
    int seg;
    int64_t i;
    segment_of(e, a.n, seg, i);
    float *raw = a.raw[seg];
    float x = raw[i];
    float g = a.grad[seg][i];
    if (seg == 1) g *= expf(x);                        // d exp(x) / dx
    else if (seg == 3) g *= 1.f / (1.f + expf(-x));    // d softplus(x) / dx
    float m = a.m[seg][i], v = a.v[seg][i];
    m = a.beta1 * m + a.omb1 * g;
    v = a.beta2 * v + a.omb2 * g * g;
    const float mhat = m * a.bc1_inv, vhat = v * a.bc2_inv;
    x -= a.lr[seg] * mhat / (sqrtf(vhat) + a.eps);
    a.m[seg][i] = m;
    a.v[seg][i] = v;
    raw[i] = x;
    if (seg == 1) a.scale[i] = expf(x);
    else if (seg == 3) a.density[i] = softplus_f(x);
  }
}

__global__ __launch_bounds__(kBlock) void k_activate(float *log_scale, float *density_raw,
                                                     float *scale, float *density, int64_t n,
                                                     int inverse) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < 4 * n;
       e += (int64_t)gridDim.x * kBlock) {
    if (e < 3 * n) {
      if (inverse) log_scale[e] = logf(scale[e]);
      else scale[e] = expf(log_scale[e]);
    } else {
      const int64_t i = e - 3 * n;
      if (inverse) density_raw[i] = softplus_inv_f(density[i]);
      else density[i] = softplus_f(density_raw[i]);
    }
  }
}

unsigned grid_for(int64_t work) {
  int64_t b = (work + kBlock - 1) / kBlock;
  return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

// Action of source Gaussian i (0 removed, 1 kept, 2 cloned, 3 split) and the
// number of Gaussians it emits.
__global__ __launch_bounds__(kBlock) void k_densify_count(DensifyArgs a, int32_t *action,
                                                          uint32_t *count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const float rd = a.src.density_raw[i];
  const int32_t vis = a.visible[i];
  const float avg = vis > 0 ? a.grad_sum[i] / (float)vis : 0.f;
  const bool grow = a.densify && vis > 0 && avg >= a.grad_threshold;
  int act;
  if (!grow) {
    act = rd < a.t_keep ? 0 : 1;
  } else if (rd < a.t_half) {
    act = 0;
  } else {
    const float *ls = a.src.log_scale + 3 * i;
    const float mx = fmaxf(ls[0], fmaxf(ls[1], ls[2]));
    act = mx <= a.t_scale ? 2 : 3;
  }
  action[i] = act;
  count[i] = act == 0 ? 0u : (act == 1 ? 1u : 2u);
}

__device__ inline void copy_n(float *d, const float *s, int k) {
  for (int j = 0; j < k; ++j) d[j] = s[j];
}
__device__ inline void zero_n(float *d, int k) {
  for (int j = 0; j < k; ++j) d[j] = 0.f;
}

// Writes one destination Gaussian o from source i: parameters (raw and
// activated) and moments (copied or zero).
__device__ inline void write_params(const DensifyArgs &a, int64_t i, int64_t o, const float *mean,
                                    const float *log_scale, float dens_raw, bool keep_moments) {
  const ParamPtrs &s = a.src, &d = a.dst;
  copy_n(d.mean + 3 * o, mean, 3);
  copy_n(d.log_scale + 3 * o, log_scale, 3);
  copy_n(d.quat + 4 * o, s.quat + 4 * i, 4);
  d.density_raw[o] = dens_raw;
  for (int j = 0; j < 3; ++j) d.scale[3 * o + j] = expf(log_scale[j]);
  d.density[o] = softplus_f(dens_raw);
  if (keep_moments) {
    copy_n(d.m_mean + 3 * o, s.m_mean + 3 * i, 3);
    copy_n(d.m_scale + 3 * o, s.m_scale + 3 * i, 3);
    copy_n(d.m_quat + 4 * o, s.m_quat + 4 * i, 4);
    d.m_density[o] = s.m_density[i];
    copy_n(d.v_mean + 3 * o, s.v_mean + 3 * i, 3);
    copy_n(d.v_scale + 3 * o, s.v_scale + 3 * i, 3);
    copy_n(d.v_quat + 4 * o, s.v_quat + 4 * i, 4);
    d.v_density[o] = s.v_density[i];
  } else {
    zero_n(d.m_mean + 3 * o, 3);
    zero_n(d.m_scale + 3 * o, 3);
    zero_n(d.m_quat + 4 * o, 4);
    d.m_density[o] = 0.f;
    zero_n(d.v_mean + 3 * o, 3);
    zero_n(d.v_scale + 3 * o, 3);
    zero_n(d.v_quat + 4 * o, 4);
    d.v_density[o] = 0.f;
  }
}

__global__ __launch_bounds__(kBlock) void k_densify_write(DensifyArgs a, const int32_t *action,
                                                          const uint32_t *offset) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int act = action[i];
  if (act == 0) return;
  const int64_t o = offset[i];
  const ParamPtrs &s = a.src;
  const float *p = s.mean + 3 * i, *ls = s.log_scale + 3 * i;
  const float rd = s.density_raw[i];
  if (act == 1) {
    write_params(a, i, o, p, ls, rd, true);
    return;
  }
  const float half = softplus_inv_f(0.5f * softplus_f(rd));
  if (act == 2) {
    write_params(a, i, o, p, ls, half, true);
    write_params(a, i, o + 1, p, ls, half, false);
    return;
  }
  // split: children at p + R (s * z), scales s / 1.6
  const float *q = s.quat + 4 * i;
  const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
  const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                      2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                      2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
  const float sc[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
  const float cls[3] = {ls[0] - a.log_split, ls[1] - a.log_split, ls[2] - a.log_split};
  for (int c = 0; c < 2; ++c) {
    const float *zz = a.normals + 6 * i + 3 * c;
    const float l0 = sc[0] * zz[0], l1 = sc[1] * zz[1], l2 = sc[2] * zz[2];
    float cp[3];
    for (int r = 0; r < 3; ++r) cp[r] = p[r] + (R[3 * r] * l0 + R[3 * r + 1] * l1 + R[3 * r + 2] * l2);
    write_params(a, i, o + c, cp, cls, half, false);
  }
}

// Metrics: per-block partial sums of squared differences (double) and the
// maximum of gt, then one block finishes both.
__global__ __launch_bounds__(kBlock) void k_metric_partials(const float *vol, const float *gt,
                                                            int64_t n, double *part_sse,
                                                            float *part_max) {
  __shared__ double ss[kBlock];
  __shared__ float sm[kBlock];
  double acc = 0.0;
  float mx = -INFINITY;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * kBlock) {
    const double d = (double)vol[e] - (double)gt[e];
    acc += d * d;
    mx = fmaxf(mx, gt[e]);
  }
  ss[threadIdx.x] = acc;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      ss[threadIdx.x] += ss[threadIdx.x + k];
      sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_sse[blockIdx.x] = ss[0];
    part_max[blockIdx.x] = sm[0];
  }
}

__global__ __launch_bounds__(kBlock) void k_metric_finish(const double *part_sse,
                                                          const float *part_max, int nb,
                                                          double *out) {
  __shared__ double ss[kBlock];
  __shared__ float sm[kBlock];
  double acc = 0.0;
  float mx = -INFINITY;
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    acc += part_sse[k];
    mx = fmaxf(mx, part_max[k]);
  }
  ss[threadIdx.x] = acc;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      ss[threadIdx.x] += ss[threadIdx.x + k];
      sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ss[0];
    out[1] = (double)sm[0];
  }
}

// Stack of the slices normal to `axis` (0: x, 1: y, 2: z) of a [nz][ny][nx]
// volume, scaled by 1 / range (range read from device memory): slice s of
// the stack has the two remaining axes in their original order, the slower
// one as rows.  Reads are coalesced along x for axes 1 and 2; for axis 0 the
// gather walks x through consecutive slices.
__global__ __launch_bounds__(kBlock) void k_slices(const float *vol, int nx, int ny, int nz,
                                                   int axis, const double *range, float *out) {
  const int64_t n = (int64_t)nx * ny * nz;
  const float inv = (float)(1.0 / range[1]);
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * kBlock) {
    int64_t src;
    if (axis == 2) {
      src = e;  // slice k = z, rows y, columns x
    } else if (axis == 1) {
      // out [ny][nz][nx]
      const int64_t j = e / ((int64_t)nz * nx), r = e - j * nz * nx;
      const int64_t k = r / nx, i = r - k * nx;
      src = (k * ny + j) * nx + i;
    } else {
      // out [nx][nz][ny]
      const int64_t i = e / ((int64_t)nz * ny), r = e - i * nz * ny;
      const int64_t k = r / ny, j = r - k * ny;
      src = (k * ny + j) * nx + i;
    }
    out[e] = vol[src] * inv;
  }
}

// Philox4x32-10 (Salmon et al., SC 2011) on counter (b, counter_lo,
// counter_hi, 0) and key (seed_lo, seed_hi), then Box-Muller on the four
// words as two pairs; thread b writes normals 4b .. 4b + 3 (in double, then
// rounded: the draws are few and feed positions).
__global__ __launch_bounds__(kBlock) void k_random_normals(uint32_t s0, uint32_t s1, uint32_t c1,
                                                           uint32_t c2, int64_t n,
                                                           float *__restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (4 * b >= n) return;
  uint32_t x0 = (uint32_t)b, x1 = c1, x2 = c2, x3 = 0u, k0 = s0, k1 = s1;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
    const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
    const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  const uint32_t w[4] = {x0, x1, x2, x3};
  double z[4];
  for (int j = 0; j < 4; j += 2) {
    const double u = ((double)w[j] + 0.5) * 0x1p-32, v = ((double)w[j + 1] + 0.5) * 0x1p-32;
    const double r = sqrt(-2.0 * log(u));
    double sn, cs;
    sincospi(2.0 * v, &sn, &cs);
    z[j] = r * cs;
    z[j + 1] = r * sn;
  }
  for (int k = 0; k < 4; ++k)
    if (4 * b + k < n) out[4 * b + k] = (float)z[k];
}

}  // namespace

void launch_random_normals(uint64_t seed, uint64_t counter, int64_t n, float *out, hipStream_t s) {
  const int64_t blocks = (n + 4 * kBlock - 1) / (4 * kBlock);
  hipLaunchKernelGGL(k_random_normals, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                     (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)counter,
                     (uint32_t)(counter >> 32), n, out);
}

void launch_adam(const AdamArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(11 * a.n)), dim3(kBlock), 0, s, a);
}

void launch_activate(float *log_scale, float *density_raw, float *scale, float *density, int64_t n,
                     int inverse, hipStream_t s) {
  hipLaunchKernelGGL(k_activate, dim3(grid_for(4 * n)), dim3(kBlock), 0, s, log_scale, density_raw,
                     scale, density, n, inverse);
}

void launch_densify_count(const DensifyArgs &a, int32_t *action, uint32_t *count, hipStream_t s) {
  const unsigned nb = (unsigned)((a.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_densify_count, dim3(nb), dim3(kBlock), 0, s, a, action, count);
}

void launch_densify_write(const DensifyArgs &a, const int32_t *action, const uint32_t *offset,
                          hipStream_t s) {
  const unsigned nb = (unsigned)((a.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_densify_write, dim3(nb), dim3(kBlock), 0, s, a, action, offset);
}

int metric_num_blocks(int64_t n) {
  int64_t b = (n + kBlock * 16 - 1) / (kBlock * 16);
  return (int)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

void launch_metric_sums(const float *vol, const float *gt, int64_t n, double *part_sse,
                        float *part_max, double *out, hipStream_t s) {
  const int nb = metric_num_blocks(n);
  hipLaunchKernelGGL(k_metric_partials, dim3(nb), dim3(kBlock), 0, s, vol, gt, n, part_sse,
                     part_max);
  hipLaunchKernelGGL(k_metric_finish, dim3(1), dim3(kBlock), 0, s, part_sse, part_max, nb, out);
}

void launch_slices(const float *vol, int nx, int ny, int nz, int axis, const double *range,
                   float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_slices, dim3(grid_for((int64_t)nx * ny * nz)), dim3(kBlock), 0, s, vol, nx,
                     ny, nz, axis, range, out);
}

}  // namespace gsk
