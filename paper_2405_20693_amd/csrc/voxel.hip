// Voxelizer kernels (paper Sec. 3.2.2, Eq. 3-4): per-Gaussian records with 3D
// tile boxes, per-group LDS tile histograms, tile-list scatter, 8^3-tile
// forward and backward, and the per-Gaussian chain rule.
#include "internal.h"

namespace gsk {

__device__ inline uint32_t pack16(int lo, int hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// One thread per Gaussian: precision matrix P = R S^-2 R^T, centre and conic
// in voxel-index units, cutoff bounding box and its 8^3-tile box.
__global__ __launch_bounds__(kBlock) void k_vox_records(VoxArgs a, Rec3 *__restrict__ rec,
                                                        uint32_t *__restrict__ count,
                                                        unsigned long long *skipped) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= a.M) return;
  Gauss G;
  load_gauss(a.mean, a.scale, a.quat, a.dens, g, G);
  Rec3 r;
  r.t0 = pack16(1, 0);  // empty box: tx0 = 1 > tx1 = 0
  r.t1 = pack16(0, 0);
  r.t2 = pack16(0, 0);
  float P[9], Sd[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) {
      float acc = 0.f;
      for (int k = 0; k < 3; ++k) acc += G.R[3 * i + k] * G.R[3 * j + k] / (G.s[k] * G.s[k]);
      P[3 * i + j] = acc;
    }
    float sd = 0.f;
    for (int k = 0; k < 3; ++k) sd += G.R[3 * i + k] * G.R[3 * i + k] * G.s[k] * G.s[k];
    Sd[i] = sd;
  }
  const float *h = a.spacing;
  const int n[3] = {a.nx, a.ny, a.nz};
  bool ok = G.ok;
  for (int i = 0; i < 9; ++i) ok = ok && finitef(P[i]);
  int lo[3], hi[3];
  for (int i = 0; i < 3; ++i) {
    r.c[i] = (G.p[i] - a.origin[i]) / h[i] - 0.5f;
    float rad = a.kappa * sqrtf(Sd[i]) / h[i];
    (&r.rx)[i] = rad;
    float l = fmaxf(ceilf(r.c[i] - rad - 1e-3f), 0.f);
    float u = fminf(floorf(r.c[i] + rad + 1e-3f), (float)(n[i] - 1));
    if (!(l <= u)) ok = false;
    lo[i] = ok ? (int)l : 0;
    hi[i] = ok ? (int)u : 0;
  }
  const float s = -0.5f * kLog2e;
  r.c00 = s * P[0] * h[0] * h[0];
  r.c01 = 2.f * s * P[1] * h[0] * h[1];
  r.c02 = 2.f * s * P[2] * h[0] * h[2];
  r.c11 = s * P[4] * h[1] * h[1];
  r.c12 = 2.f * s * P[5] * h[1] * h[2];
  r.c22 = s * P[8] * h[2] * h[2];
  r.rho = G.rho;
  uint32_t cnt = 0;
  if (ok) {
    int tx0 = lo[0] / kVTile, ty0 = lo[1] / kVTile, tz0 = lo[2] / kVTile;
    int tx1 = hi[0] / kVTile, ty1 = hi[1] / kVTile, tz1 = hi[2] / kVTile;
    r.t0 = pack16(tx0, ty0);
    r.t1 = pack16(tz0, tx1);
    r.t2 = pack16(ty1, tz1);
    cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1) * (tz1 - tz0 + 1));
  } else {
    r.rho = 0.f;
  }
  rec[g] = r;
  count[g] = cnt;
  if (!G.ok) atomicAdd(skipped, 1ull);
}

void launch_vox_records(const VoxArgs &a, Rec3 *rec, uint32_t *count, unsigned long long *skipped,
                        hipStream_t s) {
  unsigned nb = (unsigned)((a.M + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_vox_records, dim3(nb), dim3(kBlock), 0, s, a, rec, count, skipped);
}

// Tile index of (tx, ty, tz) within its group, the group owning z tile layers
// [grp * layers, (grp + 1) * layers).
__device__ inline int group_tile(const VoxArgs &a, int grp, int tx, int ty, int tz) {
  return ((tz - grp * a.layers) * a.TY + ty) * a.TX + tx;
}

// Grid (C, G): LDS histogram of the chunk's tile entries within one group.
__global__ __launch_bounds__(kBlock) void k_vox_hist(VoxArgs a, const Rec3 *__restrict__ rec,
                                                     uint32_t *__restrict__ hist) {
  extern __shared__ uint32_t sh[];
  const int c = blockIdx.x, grp = blockIdx.y, tid = threadIdx.x;
  for (int t = tid; t < a.Tg; t += kBlock) sh[t] = 0;
  __syncthreads();
  const int zl = grp * a.layers, zh = min(zl + a.layers, a.TZ) - 1;
  const int64_t g0 = (int64_t)c * kBlock * a.cpt;
  for (int k = 0; k < a.cpt; ++k) {
    int64_t g = g0 + (int64_t)k * kBlock + tid;
    if (g >= a.M) break;
    Box3 b = unpack_box(rec[g]);
    if (!box_count(b)) continue;
    int z0 = max(b.z0, zl), z1 = min(b.z1, zh);
    for (int tz = z0; tz <= z1; ++tz)
      for (int ty = b.y0; ty <= b.y1; ++ty)
        for (int tx = b.x0; tx <= b.x1; ++tx) atomicAdd(&sh[group_tile(a, grp, tx, ty, tz)], 1u);
  }
  __syncthreads();
  uint32_t *hp = hist + ((int64_t)grp * a.C + c) * a.Tg;
  for (int t = tid; t < a.Tg; t += kBlock) hp[t] = sh[t];
}

void launch_vox_hist(const VoxArgs &a, const Rec3 *rec, uint32_t *hist, hipStream_t s) {
  hipLaunchKernelGGL(k_vox_hist, dim3(a.C, a.G), dim3(kBlock), a.Tg * sizeof(uint32_t), s, a, rec,
                     hist);
}

// Grid (C, G).  Writes the chunk's entries of the group's tiles as a stable
// counting sort, like the projection scatter: a chunk's entries of one tile
// sit in Gaussian order at the tile's cursor, so tile lists are sorted by
// Gaussian index and the same in every run.  Per batch of 256 Gaussians the
// entry counts (boxes clipped to the group's tile layers) are scanned, and
// lanes take entries in rounds of at most 256 entries from at most 64
// consecutive Gaussians, ranked by 64-bit LDS masks per tile (the bit of the
// Gaussian within the round; position = cursor + lower bits set).  Tiles are
// handled in windows of kVoxScatterWindow so that masks and cursors fit LDS.
constexpr int kVoxScatterWindow = 4096;

int vox_scatter_lds(int Tg) { return min(Tg, kVoxScatterWindow) * 12; }

__global__ __launch_bounds__(kBlock) void k_vox_scatter(VoxArgs a, const Rec3 *__restrict__ rec,
                                                        const uint32_t *__restrict__ hist,
                                                        const uint32_t *__restrict__ tile_start,
                                                        uint32_t *__restrict__ list,
                                                        unsigned long long *ctl,
                                                        const unsigned long long *totals) {
  extern __shared__ unsigned long long s_dyn[];  // window masks, then cursors
  __shared__ uint32_t sh4[4];
  __shared__ uint32_t s_off[kBlock + 1];
  __shared__ uint32_t s_org[kBlock];  // box origin in tiles: x0 | y0 << 16
  __shared__ uint32_t s_z0[kBlock];   // first tile layer of the box within the group
  __shared__ uint32_t s_dim[kBlock];  // box extent in tiles: bx | by << 16
  const int c = blockIdx.x, grp = blockIdx.y, tid = threadIdx.x;
  const int Tw = min(a.Tg, kVoxScatterWindow);
  unsigned long long *s_mask = s_dyn;
  uint32_t *cur = reinterpret_cast<uint32_t *>(s_dyn + Tw);
  if (c == 0 && grp == 0 && tid == 0) {  // the binning kernels of this call have finished
    ctl[3] = ctl[1];
    ctl[1] = 0ull;
    const unsigned long long e = totals[0];
    atomicMax(&ctl[5], e);
    if (e > a.cap) {
      atomicAdd(&ctl[7], 1ull);
      if (a.ovf_host) *(volatile unsigned int *)a.ovf_host = 1u;
    }
  }
  const uint32_t *hp = hist + ((int64_t)grp * a.C + c) * a.Tg;
  const uint32_t *ts = tile_start + (int64_t)grp * a.Tg;
  const int zl = grp * a.layers, zh = min(zl + a.layers, a.TZ) - 1;
  const int64_t g0 = (int64_t)c * kBlock * a.cpt;
  for (int w0 = 0; w0 < a.Tg; w0 += Tw) {
    const int wn = min(Tw, a.Tg - w0);
    for (int t = tid; t < wn; t += kBlock) {
      cur[t] = ts[w0 + t] + hp[w0 + t];
      s_mask[t] = 0ull;
    }
    for (int k = 0; k < a.cpt; ++k) {
      const int64_t gk = g0 + (int64_t)k * kBlock;
      if (gk >= a.M) break;
      const int64_t g = gk + tid;
      int n = 0, bx = 0, by = 0, x0 = 0, y0 = 0, z0 = 0;
      if (g < a.M) {
        const Box3 b = unpack_box(rec[g]);
        if (box_count(b)) {
          z0 = max(b.z0, zl);
          const int z1 = min(b.z1, zh);
          bx = b.x1 - b.x0 + 1;
          by = b.y1 - b.y0 + 1;
          x0 = b.x0;
          y0 = b.y0;
          n = z1 >= z0 ? bx * by * (z1 - z0 + 1) : 0;
        }
      }
      uint32_t total;
      const uint32_t ex = block_excl_scan((uint32_t)n, sh4, total);  // synchronizes the workgroup
      s_off[tid] = ex;
      if (tid == 0) s_off[kBlock] = total;
      s_org[tid] = (uint32_t)x0 | ((uint32_t)y0 << 16);
      s_z0[tid] = (uint32_t)z0;
      s_dim[tid] = (uint32_t)bx | ((uint32_t)by << 16);
      __syncthreads();
      for (uint32_t r0 = 0; r0 < total;) {
        const int jA = entry_owner(s_off, r0);  // first Gaussian of the round (uniform)
        const uint32_t r1 = min(r0 + (uint32_t)kBlock, s_off[min(jA + 64, kBlock)]);
        const uint32_t e = r0 + (uint32_t)tid;
        int t = 0, bit = 0;
        bool act = false;
        uint32_t gid = 0;
        if (e < r1) {
          const int j = entry_owner(s_off, e);
          const uint32_t kin = e - s_off[j];
          const uint32_t dim = s_dim[j], org = s_org[j];
          const uint32_t ex_ = dim & 0xffffu, ey_ = dim >> 16, plane = ex_ * ey_;
          const uint32_t lz = kin / plane, rem = kin - lz * plane;
          const uint32_t ly = rem / ex_, lx = rem - ly * ex_;
          const int tx = (int)(org & 0xffffu) + (int)lx, ty = (int)(org >> 16) + (int)ly,
                    tz = (int)s_z0[j] + (int)lz;
          t = group_tile(a, grp, tx, ty, tz) - w0;
          act = t >= 0 && t < wn;
          if (act) {
            gid = (uint32_t)(gk + j);
            bit = j - jA;
            atomicOr(&s_mask[t], 1ull << bit);
          }
        }
        __syncthreads();
        unsigned long long mk = 0ull;
        if (act) {
          mk = s_mask[t];
          const uint32_t pos = cur[t] + (uint32_t)__popcll(mk & ((1ull << bit) - 1ull));
          if (pos < a.cap) list[pos] = gid;
        }
        __syncthreads();
        if (act && (mk >> bit) == 1ull) {  // the round's last entry of this tile
          cur[t] += (uint32_t)__popcll(mk);
          s_mask[t] = 0ull;
        }
        __syncthreads();
        r0 = r1;
      }
      __syncthreads();  // the next batch restages
    }
  }
}

void launch_vox_scatter(const VoxArgs &a, const Rec3 *rec, const uint32_t *hist,
                        const uint32_t *tile_start, uint32_t *list, unsigned long long *ctl,
                        const unsigned long long *totals, hipStream_t s) {
  hipLaunchKernelGGL(k_vox_scatter, dim3(a.C, a.G), dim3(kBlock), vox_scatter_lds(a.Tg), s, a,
                     rec, hist, tile_start, list, ctl, totals);
}

// --------------------------------------------------------------- forward --

struct VoxTile {
  int tx, ty, tz;
  bool valid;
};

__device__ inline VoxTile decode_item(const VoxArgs &a, int item) {
  VoxTile r;
  int grp = item / a.Tg, within = item - grp * a.Tg;
  int plane = a.TX * a.TY;
  int lz = within / plane, rem = within - lz * plane;
  r.ty = rem / a.TX;
  r.tx = rem - r.ty * a.TX;
  r.tz = grp * a.layers + lz;
  r.valid = r.tz < a.TZ;
  return r;
}

// Stage one batch of records in LDS (13 floats each, structure of arrays).
__device__ inline void stage_rec3(const Rec3 &r, float (*s)[kBlock], int tid) {
  s[0][tid] = r.c[0]; s[1][tid] = r.c[1]; s[2][tid] = r.c[2];
  s[3][tid] = r.c00; s[4][tid] = r.c01; s[5][tid] = r.c02;
  s[6][tid] = r.c11; s[7][tid] = r.c12; s[8][tid] = r.c22;
  s[9][tid] = r.rho;
  s[10][tid] = r.rx; s[11][tid] = r.ry; s[12][tid] = r.rz;
}

__device__ inline bool box_hits(const float (*s)[kBlock], int i, float x0, float y0, float z0) {
  const float e = (float)(kVSub - 1);
  const float cx = s[0][i], cy = s[1][i], cz = s[2][i];
  const float rx = s[10][i], ry = s[11][i], rz = s[12][i];
  return (cx + rx >= x0) && (cx - rx <= x0 + e) && (cy + ry >= y0) && (cy - ry <= y0 + e) &&
         (cz + rz >= z0) && (cz - rz <= z0 + e);
}

// Upper bound of the exponent q' (concave: the conic is negative definite)
// over the voxel-centre box [x0, x0 + 3] x [y0, y0 + 3] x [z0, z0 + 3] of a
// 4^3 sub-cube: two sweeps of coordinate ascent give a point y of the box,
// and by concavity q'(x) <= q'(y) + grad q'(y) . (x - y), whose maximum over
// the box is the bound.  It never falls below the true maximum, so culling a
// record whose bound is under the cutoff threshold drops no term; for
// elongated Gaussians it is far tighter than the axis-aligned box.
__device__ inline bool box_may_reach(const float (*s)[kBlock], int i, float x0, float y0, float z0,
                                     float thr) {
  const float e = (float)(kVSub - 1);
  const float c00 = s[3][i], c01 = s[4][i], c02 = s[5][i], c11 = s[6][i], c12 = s[7][i],
              c22 = s[8][i];
  const float lx = x0 - s[0][i], ly = y0 - s[1][i], lz = z0 - s[2][i];
  const float hx = lx + e, hy = ly + e, hz = lz + e;
  const float ix = -0.5f / c00, iy = -0.5f / c11, iz = -0.5f / c22;
  float dx = fminf(fmaxf(0.f, lx), hx), dy = fminf(fmaxf(0.f, ly), hy), dz = fminf(fmaxf(0.f, lz), hz);
  for (int sweep = 0; sweep < 2; ++sweep) {
    dx = fminf(fmaxf((c01 * dy + c02 * dz) * ix, lx), hx);
    dy = fminf(fmaxf((c01 * dx + c12 * dz) * iy, ly), hy);
    dz = fminf(fmaxf((c02 * dx + c12 * dy) * iz, lz), hz);
  }
  const float qy = dx * (c00 * dx + c01 * dy + c02 * dz) + dy * (c11 * dy + c12 * dz) + c22 * dz * dz;
  const float gx = 2.f * c00 * dx + c01 * dy + c02 * dz;
  const float gy = c01 * dx + 2.f * c11 * dy + c12 * dz;
  const float gz = c02 * dx + c12 * dy + 2.f * c22 * dz;
  const float tx = gx > 0.f ? gx * (hx - dx) : gx * (lx - dx);
  const float ty = gy > 0.f ? gy * (hy - dy) : gy * (ly - dy);
  const float tz = gz > 0.f ? gz * (hz - dz) : gz * (lz - dz);
  const float ub = qy + tx + ty + tz;
  // FP32 rounding margin of the bound and of the kernels' own q'
  const float margin = 1e-5f * (fabsf(qy) + fabsf(tx) + fabsf(ty) + fabsf(tz)) + 1e-5f;
  return ub + margin >= thr;
}

__device__ inline float vox_q(const float (*s)[kBlock], int e, float dx, float dy, float dz) {
  return dx * (s[3][e] * dx + s[4][e] * dy + s[5][e] * dz) + dy * (s[6][e] * dy + s[7][e] * dz) +
         s[8][e] * dz * dz;
}

// One workgroup per 8^3 tile; wave w owns the 4^3 sub-cubes w and w + 4.
// For each chunk of 64 staged records, lane i tests record i against the
// sub-cube (box overlap and the concave-bound cull) and, if it may reach it,
// rewrites it relative to the sub-cube centre: with l the voxel offset from
// the centre,
//   q'(l) = K0 + K1 lx + K2 ly + c00 lx^2 + c01 lx ly + c11 ly^2   (lz = -3/2)
// and down z by the differences D0 + c02 lx + c12 ly, stepping by 2 c22.  The
// kept records are compacted and dealt to the wave's four 16-lane quarters;
// a lane evaluates a column of four voxels along z, so one coefficient load
// from LDS serves four voxels.  The quarters' partial sums are added in a
// fixed order at the end.
__global__ __launch_bounds__(kBlock) void k_vox_fwd(VoxArgs a, const Rec3 *__restrict__ rec,
                                                    const uint32_t *__restrict__ list,
                                                    const uint32_t *__restrict__ tile_start,
                                                    float *__restrict__ vol,
                                                    float *__restrict__ partial) {
  __shared__ float s[13][kBlock];
  __shared__ float4 s_k[4][64][3];  // per wave: compacted coefficients of the kept records
  const int wi = xcd_remap(blockIdx.x, gridDim.x);
  const int item = wi / a.parts, part = wi - item * a.parts;
  const VoxTile T = decode_item(a, item);
  if (!T.valid) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the lane's column of four voxels in its quarter's copy of a sub-cube
  const int qd = lane >> 4, j = lane & 15;
  const float hs = 0.5f * (kVSub - 1);
  const float lx = (float)(j & 3) - hs, ly = (float)(j >> 2) - hs;
  const float lxx = lx * lx, lxy = lx * ly, lyy = ly * ly;
  float acc[2][kVSub];
  float ox[2], oy[2], oz[2];
  for (int k = 0; k < 2; ++k) {
    const int sc = w + 4 * k;
    ox[k] = (float)(T.tx * kVTile + (sc & 1) * kVSub);
    oy[k] = (float)(T.ty * kVTile + ((sc >> 1) & 1) * kVSub);
    oz[k] = (float)(T.tz * kVTile + (sc >> 2) * kVSub);
#pragma unroll
    for (int z = 0; z < kVSub; ++z) acc[k][z] = 0.f;
  }
  const float thr = a.thr;
  uint32_t beg, end;
  list_part(min(tile_start[item], a.cap), min(tile_start[item + 1], a.cap), part, a.parts, beg,
            end);
  for (uint32_t base = beg; base < end; base += kBlock) {
    const int n = (int)min((uint32_t)kBlock, end - base);
    __syncthreads();
    if (tid < n) stage_rec3(rec[list[base + tid]], s, tid);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      for (int c0 = 0; c0 < n; c0 += 64) {
        const int i = c0 + lane;
        const bool hit = (i < n) && box_hits(s, i, ox[k], oy[k], oz[k]) &&
                         box_may_reach(s, i, ox[k], oy[k], oz[k], thr);
        float4 k0, k1, k2;
        if (hit) {
          const float c00 = s[3][i], c01 = s[4][i], c02 = s[5][i], c11 = s[6][i], c12 = s[7][i],
                      c22 = s[8][i];
          // record centre relative to the sub-cube centre
          const float u = s[0][i] - (ox[k] + hs), v = s[1][i] - (oy[k] + hs),
                      ww = s[2][i] - (oz[k] + hs);
          const float K0 = u * (c00 * u + c01 * v + c02 * ww) + v * (c11 * v + c12 * ww) + c22 * ww * ww;
          const float K1 = -(2.f * c00 * u + c01 * v + c02 * ww);
          const float K2 = -(c01 * u + 2.f * c11 * v + c12 * ww);
          const float K3 = -(c02 * u + c12 * v + 2.f * c22 * ww);
          // fold lz = -hs into the x-y form, and the first z difference
          k0 = make_float4(K0 - hs * K3 + hs * hs * c22, K1 - hs * c02, K2 - hs * c12, c00);
          k1 = make_float4(c01, c11, K3 + c22 * (1.f - 2.f * hs), c02);
          k2 = make_float4(c12, 2.f * c22, s[9][i], 0.f);
        }
        const uint64_t mask = __ballot(hit);
        const int nk = __popcll(mask);
        if (hit) {
          const int pos = lanes_below(mask);
          s_k[w][pos][0] = k0;
          s_k[w][pos][1] = k1;
          s_k[w][pos][2] = k2;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int r = qd; r < nk; r += 4) {
          const float4 a0 = s_k[w][r][0], a1 = s_k[w][r][1], a2 = s_k[w][r][2];
          float q = fmaf(a0.y, lx, a0.x);
          q = fmaf(a0.z, ly, q);
          q = fmaf(a0.w, lxx, q);
          q = fmaf(a1.x, lxy, q);
          q = fmaf(a1.y, lyy, q);
          float d = fmaf(a1.w, lx, a1.z);  // q'(z + 1) - q'(z) at the first voxel
          d = fmaf(a2.x, ly, d);
#pragma unroll
          for (int z = 0; z < kVSub; ++z) {
            const float e = (q >= thr) ? __builtin_amdgcn_exp2f(q) : 0.f;
            acc[k][z] = fmaf(a2.z, e, acc[k][z]);
            q += d;
            d += a2.y;
          }
        }
        __builtin_amdgcn_wave_barrier();  // the next chunk overwrites this wave's coefficients
      }
    }
  }
  // the four quarters' sums of each voxel (lane x + 4 y + 16 z), in quarter order
  float total[2];
  float *red = reinterpret_cast<float *>(&s_k[w][0][0]);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int z = 0; z < kVSub; ++z) red[qd * 64 + z * 16 + j] = acc[k][z];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    total[k] = ((red[lane] + red[64 + lane]) + red[128 + lane]) + red[192 + lane];
    __builtin_amdgcn_wave_barrier();
  }
  if (a.parts > 1) {
    float *pp = partial + ((int64_t)part * a.G * a.Tg + item) * (2 * kBlock);
    pp[tid] = total[0];
    pp[kBlock + tid] = total[1];
    return;
  }
  for (int k = 0; k < 2; ++k) {
    const int vx = (int)ox[k] + (lane & 3), vy = (int)oy[k] + ((lane >> 2) & 3),
              vz = (int)oz[k] + (lane >> 4);
    if (vx < a.nx && vy < a.ny && vz < a.nz)
      vol[((int64_t)vz * a.ny + vy) * a.nx + vx] = total[k];
  }
}

// Sum of the parts of each tile's voxels, in part order (same voxel mapping
// as the forward: sub-cube w + 4k, lane).
__global__ __launch_bounds__(kBlock) void k_vox_parts(VoxArgs a, const float *__restrict__ partial,
                                                      float *__restrict__ vol) {
  const int item = blockIdx.x;
  const VoxTile T = decode_item(a, item);
  if (!T.valid) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t stride = (int64_t)a.G * a.Tg * (2 * kBlock);
  for (int k = 0; k < 2; ++k) {
    const int sc = w + 4 * k;
    const int vx = T.tx * kVTile + (sc & 1) * kVSub + (lane & 3);
    const int vy = T.ty * kVTile + ((sc >> 1) & 1) * kVSub + ((lane >> 2) & 3);
    const int vz = T.tz * kVTile + (sc >> 2) * kVSub + (lane >> 4);
    const float *p = partial + (int64_t)item * (2 * kBlock) + k * kBlock + tid;
    const float acc = strided_sum(p, stride, a.parts);
    if (vx < a.nx && vy < a.ny && vz < a.nz) vol[((int64_t)vz * a.ny + vy) * a.nx + vx] = acc;
  }
}

void launch_vox_fwd(const VoxArgs &a, const Rec3 *rec, const uint32_t *list,
                    const uint32_t *tile_start, float *volume, float *partial, hipStream_t s) {
  const int n = a.G * a.Tg * a.parts;
  hipLaunchKernelGGL(k_vox_fwd, dim3(n), dim3(kBlock), 0, s, a, rec, list, tile_start, volume,
                     partial);
  if (a.parts > 1)
    hipLaunchKernelGGL(k_vox_parts, dim3(a.G * a.Tg), dim3(kBlock), 0, s, a, partial, volume);
}

// -------------------------------------------------------------- backward --

// Lanes are (record, sub-cube) pairs; each walks the sub-cube's 64 voxels and
// accumulates 10 moments of H e (e = exp2(q')): 1, d_i, d_i d_j (index units,
// d = voxel - centre).  Per-wave LDS accumulators, summed in fixed order.
// Pairs whose form stays below kVChainRange over the sub-cube (its maximum is
// at a corner) step e by multiplication: along x by r = exp2(q(x+1) - q(x)),
// r by exp2(2 c00), and likewise down y and z, so ten exp2 per walk replace
// 64 and every chained value stays a normal FP32 number; the others evaluate
// exp2(q') per voxel.  The two kinds are queued apart (each pair's path is
// its own).  Moments are summed per x column first (dx is constant down a
// column) with cascaded sums over the rows and a fold over the planes, and
// combined once per walk.
constexpr float kVChainRange = 120.f;

__device__ inline float vox_form_max(const float (*s)[kBlock], int i, float x0, float y0,
                                     float z0) {
  // maximum over the 8 corners of the positive form -q' (convex)
  const float e = (float)(kVSub - 1);
  const float c00 = -s[3][i], c01 = -s[4][i], c02 = -s[5][i], c11 = -s[6][i], c12 = -s[7][i],
              c22 = -s[8][i];
  const float xs[2] = {x0 - s[0][i], x0 + e - s[0][i]};
  const float ys[2] = {y0 - s[1][i], y0 + e - s[1][i]};
  const float zs[2] = {z0 - s[2][i], z0 + e - s[2][i]};
  float m = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float dx = xs[a], dy = ys[b], dz = zs[c];
        m = fmaxf(m, dx * (c00 * dx + c01 * dy + c02 * dz) + dy * (c11 * dy + c12 * dz) +
                         c22 * dz * dz);
      }
  return m;
}
__global__ __launch_bounds__(kBlock) void k_vox_bwd(VoxArgs a, const Rec3 *__restrict__ rec,
                                                    const uint32_t *__restrict__ list,
                                                    const uint32_t *__restrict__ tile_start,
                                                    const uint32_t *__restrict__ offsets,
                                                    const float *__restrict__ grad_vol,
                                                    float *__restrict__ slots) {
  __shared__ float s[13][kBlock];
  __shared__ __align__(16) float s_H[kVTile * kVTile * kVTile];
  __shared__ float s_acc[4][10][kBlock];
  __shared__ uint16_t s_q[4][kBlock];
  const int wi = xcd_remap(blockIdx.x, gridDim.x);
  const int item = wi / a.bparts, part = wi - item * a.bparts;
  const VoxTile T = decode_item(a, item);
  if (!T.valid) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < kVTile * kVTile * kVTile; i += kBlock) {
    const int lx = i & 7, ly = (i >> 3) & 7, lz = i >> 6;
    const int x = T.tx * kVTile + lx, y = T.ty * kVTile + ly, z = T.tz * kVTile + lz;
    s_H[i] = (x < a.nx && y < a.ny && z < a.nz) ? grad_vol[((int64_t)z * a.ny + y) * a.nx + x] : 0.f;
  }
  uint32_t beg, end;
  list_part(min(tile_start[item], a.cap), min(tile_start[item + 1], a.cap), part, a.bparts, beg,
            end);
  const float ethr = __builtin_amdgcn_exp2f(a.thr);  // the cutoff on e = exp2(q')
  for (uint32_t base = beg; base < end; base += kBlock) {
    const int n = (int)min((uint32_t)kBlock, end - base);
    __syncthreads();
    uint32_t my_slot = 0;
    if (tid < n) {
      const uint32_t g = list[base + tid];
      const Rec3 r = rec[g];
      stage_rec3(r, s, tid);
      const Box3 b = unpack_box(r);
      const int bx = b.x1 - b.x0 + 1, by = b.y1 - b.y0 + 1;
      my_slot = offsets[g] + (uint32_t)(((T.tz - b.z0) * by + (T.ty - b.y0)) * bx + (T.tx - b.x0));
    }
    for (int k = 0; k < 10; ++k)
      for (int ww = 0; ww < 4; ++ww) s_acc[ww][k][tid] = 0.f;
    __syncthreads();
    for (int kk = 0; kk < 2; ++kk) {
      const int sc = w + 4 * kk;
      const int lx0 = (sc & 1) * kVSub, ly0 = ((sc >> 1) & 1) * kVSub, lz0 = (sc >> 2) * kVSub;
      const float ox = (float)(T.tx * kVTile + lx0), oy = (float)(T.ty * kVTile + ly0),
                  oz = (float)(T.tz * kVTile + lz0);
      int qn = 0, qs = 0;
      for (int c0 = 0; c0 < n; c0 += 64) {
        const int i = c0 + lane;
        const bool hit = (i < n) && box_hits(s, i, ox, oy, oz) && box_may_reach(s, i, ox, oy, oz, a.thr);
        const bool steep = hit && !(vox_form_max(s, i, ox, oy, oz) <= kVChainRange);
        const uint64_t mc = __ballot(hit && !steep), ms = __ballot(steep);
        if (hit && !steep) s_q[w][qn + lanes_below(mc)] = (uint16_t)i;
        if (steep) s_q[w][kBlock - 1 - (qs + lanes_below(ms))] = (uint16_t)i;
        qn += __popcll(mc);
        qs += __popcll(ms);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int pass = 0; pass < 2; ++pass) {
        const bool chain = pass == 0;
        const int cnt = chain ? qn : qs;
        for (int qb = 0; qb < cnt; qb += 64) {
          const int j = qb + lane;
          const bool active = j < cnt;
          const int e = active ? (int)s_q[w][chain ? j : kBlock - 1 - j] : 0;
          const float cx = s[0][e], cy = s[1][e], cz = s[2][e];
          const float c00 = s[3][e], c01 = s[4][e], c02 = s[5][e], c11 = s[6][e], c12 = s[7][e],
                      c22 = s[8][e];
          const float dx0 = ox - cx, dy0 = oy - cy, dz0 = oz - cz;
          // Per x column, a cascade over each z plane's four rows of s = e H:
          // A += s, B += A, C += B (after the rows: row y weighted by 1, 4 - y
          // and (4 - y)(5 - y)/2), folded over the planes into the sums of A,
          // Z A, Z^2 A, B, Z B and C (Z = z - 1.5); the first row and plane
          // start the sums.
          float A[kVSub], B[kVSub], C[kVSub];
          float M0[kVSub], MZ[kVSub], MZZ[kVSub], SB[kVSub], SZB[kVSub], SC[kVSub];
          auto acc_row = [&](int y, const float (&se)[kVSub], const float (&h)[kVSub]) {
#pragma unroll
            for (int x = 0; x < kVSub; ++x) {
              if (y == 0) {
                A[x] = se[x] * h[x];
              } else if (y == 1) {
                const float a1 = fmaf(se[x], h[x], A[x]);
                B[x] = A[x] + a1;
                C[x] = A[x] + B[x];
                A[x] = a1;
              } else {
                A[x] = fmaf(se[x], h[x], A[x]);
                B[x] += A[x];
                C[x] += B[x];
              }
            }
          };
          auto fold_plane = [&](int z) {
            const float Z = (float)z - 0.5f * (kVSub - 1);
#pragma unroll
            for (int x = 0; x < kVSub; ++x) {
              if (z == 0) {
                M0[x] = A[x]; MZ[x] = Z * A[x]; MZZ[x] = (Z * Z) * A[x];
                SB[x] = B[x]; SZB[x] = Z * B[x]; SC[x] = C[x];
              } else {
                M0[x] += A[x]; MZ[x] = fmaf(Z, A[x], MZ[x]); MZZ[x] = fmaf(Z * Z, A[x], MZZ[x]);
                SB[x] += B[x]; SZB[x] = fmaf(Z, B[x], SZB[x]); SC[x] += C[x];
              }
            }
          };
          if (chain) {
            float e_z = __builtin_amdgcn_exp2f(dx0 * (c00 * dx0 + c01 * dy0 + c02 * dz0) +
                                               dy0 * (c11 * dy0 + c12 * dz0) + c22 * dz0 * dz0);
            float rx_z = __builtin_amdgcn_exp2f(c00 * (2.f * dx0 + 1.f) + c01 * dy0 + c02 * dz0);
            float hy_z = __builtin_amdgcn_exp2f(c11 * (2.f * dy0 + 1.f) + c01 * dx0 + c12 * dz0);
            float hz = __builtin_amdgcn_exp2f(c22 * (2.f * dz0 + 1.f) + c02 * dx0 + c12 * dy0);
            const float rxx = __builtin_amdgcn_exp2f(2.f * c00), ryy = __builtin_amdgcn_exp2f(2.f * c11),
                        rzz = __builtin_amdgcn_exp2f(2.f * c22), rxy = __builtin_amdgcn_exp2f(c01),
                        rxz = __builtin_amdgcn_exp2f(c02), ryz = __builtin_amdgcn_exp2f(c12);
#pragma unroll
            for (int z = 0; z < kVSub; ++z) {
              float e_y = e_z, rx_y = rx_z, hy = hy_z;
#pragma unroll
              for (int y = 0; y < kVSub; ++y) {
                const float4 Hr = *reinterpret_cast<const float4 *>(
                    s_H + ((lz0 + z) * kVTile + (ly0 + y)) * kVTile + lx0);
                const float Hx[kVSub] = {Hr.x, Hr.y, Hr.z, Hr.w};
                float se[kVSub];
                float ev = e_y, rx = rx_y;
#pragma unroll
                for (int x = 0; x < kVSub; ++x) {
                  se[x] = (ev >= ethr) ? ev : 0.f;
                  ev *= rx;
                  rx *= rxx;
                }
                acc_row(y, se, Hx);
                e_y *= hy;
                hy *= ryy;
                rx_y *= rxy;
              }
              fold_plane(z);
              e_z *= hz;
              hz *= rzz;
              hy_z *= ryz;
              rx_z *= rxz;
            }
          } else {
#pragma unroll
            for (int z = 0; z < kVSub; ++z) {
              const float dz = oz + (float)z - cz;
#pragma unroll
              for (int y = 0; y < kVSub; ++y) {
                const float dy = oy + (float)y - cy;
                const float *Hrow = s_H + ((lz0 + z) * kVTile + (ly0 + y)) * kVTile + lx0;
                float se[kVSub], Hx[kVSub];
#pragma unroll
                for (int x = 0; x < kVSub; ++x) {
                  const float dx = ox + (float)x - cx;
                  const float q = dx * (c00 * dx + c01 * dy + c02 * dz) + dy * (c11 * dy + c12 * dz) +
                                  c22 * dz * dz;
                  se[x] = (q >= a.thr) ? __builtin_amdgcn_exp2f(q) : 0.f;
                  Hx[x] = Hrow[x];
                }
                acc_row(y, se, Hx);
              }
              fold_plane(z);
            }
          }
          // Sums over the columns (X = x - 1.5), the moments about the
          // sub-cube centre (L_ijk: weight X^i Y^j Z^k; with u = 4 - y =
          // 2.5 - Y, B sums s u and 2 C - B sums s u^2), then shifted to the
          // pair's centre: d = centre offset + (X, Y, Z).
          float sM0 = 0.f, sXM0 = 0.f, sXXM0 = 0.f, sMZ = 0.f, sXMZ = 0.f, sMZZ = 0.f;
          float sSB = 0.f, sXSB = 0.f, sSZB = 0.f, sSC = 0.f;
#pragma unroll
          for (int x = 0; x < kVSub; ++x) {
            const float X = (float)x - 0.5f * (kVSub - 1);
            sM0 += M0[x];
            sXM0 = fmaf(X, M0[x], sXM0);
            sXXM0 = fmaf(X * X, M0[x], sXXM0);
            sMZ += MZ[x];
            sXMZ = fmaf(X, MZ[x], sXMZ);
            sMZZ += MZZ[x];
            sSB += SB[x];
            sXSB = fmaf(X, SB[x], sXSB);
            sSZB += SZB[x];
            sSC += SC[x];
          }
          const float L010 = fmaf(2.5f, sM0, -sSB), L110 = fmaf(2.5f, sXM0, -sXSB);
          const float L011 = fmaf(2.5f, sMZ, -sSZB);
          const float L020 = fmaf(6.25f, sM0, fmaf(-6.f, sSB, 2.f * sSC));
          const float xc = dx0 + 0.5f * (kVSub - 1), yc = dy0 + 0.5f * (kVSub - 1),
                      zc = dz0 + 0.5f * (kVSub - 1);
          float m[10];
          m[0] = sM0;
          m[1] = fmaf(xc, sM0, sXM0);
          m[2] = fmaf(yc, sM0, L010);
          m[3] = fmaf(zc, sM0, sMZ);
          m[4] = fmaf(xc, sXM0 + m[1], sXXM0);
          m[5] = fmaf(yc, m[1], fmaf(xc, L010, L110));
          m[6] = fmaf(zc, m[1], fmaf(xc, sMZ, sXMZ));
          m[7] = fmaf(yc, L010 + m[2], L020);
          m[8] = fmaf(zc, m[2], fmaf(yc, sMZ, L011));
          m[9] = fmaf(zc, sMZ + m[3], sMZZ);
          if (active)
            for (int k = 0; k < 10; ++k) s_acc[w][k][e] += m[k];
        }
      }
    }
    __syncthreads();
    if (tid < n && my_slot < a.cap) {
      float *o = slots + (int64_t)my_slot * 10;
      for (int k = 0; k < 10; ++k)
        o[k] = ((s_acc[0][k][tid] + s_acc[1][k][tid]) + s_acc[2][k][tid]) + s_acc[3][k][tid];
    }
  }
}

void launch_vox_bwd(const VoxArgs &a, const Rec3 *rec, const uint32_t *list,
                    const uint32_t *tile_start, const uint32_t *offsets, const float *grad_volume,
                    float *slots, hipStream_t s) {
  const int n = a.G * a.Tg * a.bparts;
  hipLaunchKernelGGL(k_vox_bwd, dim3(n), dim3(kBlock), 0, s, a, rec, list, tile_start, offsets,
                     grad_volume, slots);
}

// One thread per Gaussian: sum the tile slots' moments and apply the chain
// rule through the index-unit conic, P = R S^-2 R^T and the quaternion.
// Slots are numbered in Gaussian order and the offsets array ends with the
// total, so a Gaussian's slot count is the difference of its offsets; the
// many Gaussians with none (outside the block) read neither their record nor
// their parameters.
__global__ __launch_bounds__(kBlock) void k_vox_chain(VoxArgs a,
                                                      const uint32_t *__restrict__ offsets,
                                                      const float *__restrict__ slots,
                                                      float *g_mean, float *g_scale, float *g_quat,
                                                      float *g_dens, int accumulate) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= a.M || *a.totals > a.cap) return;  // overflow: the slots are incomplete
  float gp[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
  float grho = 0.f;
  const uint32_t off = offsets[g];
  const int cnt = (int)(offsets[g + 1] - off);
  Gauss G;
  G.ok = false;
  if (cnt && (uint64_t)off + (uint64_t)cnt <= a.cap)  // (beyond capacity: dropped)
    load_gauss(a.mean, a.scale, a.quat, a.dens, g, G);
  if (!G.ok && accumulate) return;  // adds nothing
  if (G.ok) {
    float S[10];
    for (int k = 0; k < 10; ++k) S[k] = 0.f;
    const float *sl = slots + (int64_t)off * 10;
    // four slots' loads in flight at a time, added in slot order
    int i = 0;
    for (; i + 4 <= cnt; i += 4) {
      float t[4][10];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 10; ++k) t[u][k] = sl[10 * (i + u) + k];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 10; ++k) S[k] += t[u][k];
    }
    for (; i < cnt; ++i)
      for (int k = 0; k < 10; ++k) S[k] += sl[10 * i + k];
    const float *h = a.spacing;
    // world-unit moments
    const float T[3] = {S[1] * h[0], S[2] * h[1], S[3] * h[2]};
    float Tm[9];
    Tm[0] = S[4] * h[0] * h[0]; Tm[1] = S[5] * h[0] * h[1]; Tm[2] = S[6] * h[0] * h[2];
    Tm[4] = S[7] * h[1] * h[1]; Tm[5] = S[8] * h[1] * h[2]; Tm[8] = S[9] * h[2] * h[2];
    Tm[3] = Tm[1]; Tm[6] = Tm[2]; Tm[7] = Tm[5];
    float P[9], is2[3];
    for (int k = 0; k < 3; ++k) is2[k] = 1.f / (G.s[k] * G.s[k]);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        float acc = 0.f;
        for (int k = 0; k < 3; ++k) acc += G.R[3 * i + k] * G.R[3 * j + k] * is2[k];
        P[3 * i + j] = acc;
      }
    grho = S[0];
    for (int i = 0; i < 3; ++i) gp[i] = G.rho * (P[3 * i] * T[0] + P[3 * i + 1] * T[1] + P[3 * i + 2] * T[2]);
    // dL/dP (each entry) = -rho/2 Tm;  P = R D R^T, D = diag(s^-2)
    float GP[9];
    for (int i = 0; i < 9; ++i) GP[i] = -0.5f * G.rho * Tm[i];
    // dL/dR = 2 dL/dP R D.  The part of D common to the three axes leaves P
    // unchanged under rotation, so it adds exactly zero to dL/dq (R^T dR/dq is
    // antisymmetric, dL/dP symmetric): it is left out, so that a nearly
    // isotropic Gaussian's small rotation gradient is not the FP32
    // remainder of a large cancelling sum
    const float ib2 = (is2[0] + is2[1] + is2[2]) * (1.f / 3.f);
    float gR[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        float acc = 0.f;
        for (int k = 0; k < 3; ++k) acc += GP[3 * i + k] * G.R[3 * k + j];
        gR[3 * i + j] = 2.f * acc * (is2[j] - ib2);
      }
    for (int j = 0; j < 3; ++j) {
      float acc = 0.f;
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) acc += G.R[3 * i + j] * GP[3 * i + k] * G.R[3 * k + j];
      gs[j] = -2.f * acc * is2[j] / G.s[j];
    }
    quat_backward(G, gR, gq);
  }
  if (g_mean)
    for (int i = 0; i < 3; ++i) g_mean[3 * g + i] = accumulate ? g_mean[3 * g + i] + gp[i] : gp[i];
  if (g_scale)
    for (int i = 0; i < 3; ++i)
      g_scale[3 * g + i] = accumulate ? g_scale[3 * g + i] + gs[i] : gs[i];
  if (g_quat)
    for (int i = 0; i < 4; ++i) g_quat[4 * g + i] = accumulate ? g_quat[4 * g + i] + gq[i] : gq[i];
  if (g_dens) g_dens[g] = accumulate ? g_dens[g] + grho : grho;
}

void launch_vox_chain(const VoxArgs &a, const uint32_t *offsets, const float *slots,
                      float *g_mean, float *g_scale, float *g_quat, float *g_dens, int accumulate,
                      hipStream_t s) {
  unsigned nb = (unsigned)((a.M + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_vox_chain, dim3(nb), dim3(kBlock), 0, s, a, offsets, slots, g_mean,
                     g_scale, g_quat, g_dens, accumulate);
}

}  // namespace gsk
