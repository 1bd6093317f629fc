// Internal declarations of the HIP path: device records, per-Gaussian
// projection math and the host launchers of each kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs_train.h"

namespace gsk {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.69314718055994531f;
constexpr float kTwoPi = 6.2831853071795865f;

// Orders one wavefront's LDS accesses across its lanes: a wave's LDS
// operations execute in program order, so no wait is needed, only that the
// compiler keep that order.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reciprocal by the hardware instruction (about 1 ulp; an IEEE division takes
// ten instructions).  The projection chain evaluates a dozen per (view,
// Gaussian), far inside the FP32 tolerances of every result.
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

constexpr int kTile = 16;      // 2D binning tile edge (pixels)
constexpr int kSub = 8;        // 2D per-wave sub-tile edge
constexpr int kVTile = 8;      // 3D binning tile edge (voxels)
constexpr int kVSub = 4;       // 3D per-wave sub-cube edge
constexpr int kBlock = 256;    // threads per workgroup of the binning/render kernels
constexpr int kChunkPerThread = 16;
constexpr int kChunk = kBlock * kChunkPerThread;  // Gaussians per binning chunk
constexpr int kMaxTilesPerGroup = 16384;          // LDS histogram limit (64 KB)

// Per-view constants, precomputed on the host in double precision.
struct DevView {
  float W[9];          // world -> scanner rotation, rows u, v, ray
  float L_SO, L_SD;
  float hu, hv;        // pixel pitch
  float inv_hu, inv_hv;
  float cu, cv;        // pixel coordinate of detector coordinate 0: n/2 - 1/2 - off/h
  int32_t beam;        // 0 parallel, 1 cone
  int32_t pad[3];
};

// Projected Gaussian, one per (view, Gaussian); 32 bytes.
// The centre is in pixel coordinates (pixel a's centre at a).  The conic is
// pre-scaled by -log2(e)/2 so that a term is rho * exp2(q'), with
// q' = c00 dx^2 + c01 dx dy + c11 dy^2 <= 0.
struct Rec2 {
  float pu, pv;
  float c00, c01, c11;
  float rho;           // rectified density rho_hat
  uint32_t r0, r1;     // tile rectangle: tx0 | ty0 << 16, tx1 | ty1 << 16
};

// Voxelization record, one per Gaussian; 64 bytes.  Centre and conic in
// voxel-index coordinates (voxel i's centre at i), conic pre-scaled as above
// with cross terms doubled: q' = sum_i c_ii d_i^2 + c01 d0 d1 + c02 d0 d2 + c12 d1 d2.
struct Rec3 {
  float c[3];
  float c00, c01, c02, c11, c12, c22;
  float rho;
  float rx, ry, rz;    // cutoff bounding-box half extents (voxels)
  uint32_t t0, t1;     // tile box: tx0 | ty0 << 16, tz0 | tx1 << 16
  uint32_t t2;         // ty1 | tz1 << 16
};

__host__ __device__ inline int rect_tx0(uint32_t r0) { return (int)(r0 & 0xffffu); }
__host__ __device__ inline int rect_ty0(uint32_t r0) { return (int)(r0 >> 16); }

struct Rect2 { int x0, y0, x1, y1; };
__device__ inline Rect2 unpack_rect(uint32_t r0, uint32_t r1) {
  return Rect2{(int)(r0 & 0xffffu), (int)(r0 >> 16), (int)(r1 & 0xffffu), (int)(r1 >> 16)};
}
__device__ inline int rect_count(const Rect2 &r) {
  return (r.x1 < r.x0 || r.y1 < r.y0) ? 0 : (r.x1 - r.x0 + 1) * (r.y1 - r.y0 + 1);
}

struct Box3 { int x0, y0, z0, x1, y1, z1; };
__device__ inline Box3 unpack_box(const Rec3 &r) {
  return Box3{(int)(r.t0 & 0xffffu), (int)(r.t0 >> 16), (int)(r.t1 & 0xffffu),
              (int)(r.t1 >> 16),     (int)(r.t2 & 0xffffu), (int)(r.t2 >> 16)};
}
__device__ inline int box_count(const Box3 &b) {
  return (b.x1 < b.x0 || b.y1 < b.y0 || b.z1 < b.z0)
             ? 0
             : (b.x1 - b.x0 + 1) * (b.y1 - b.y0 + 1) * (b.z1 - b.z0 + 1);
}

// ---------------------------------------------------------------- Gaussian --

struct Gauss {
  float p[3], s[3];
  float qn[4];      // normalised quaternion (w, x, y, z)
  float qnorm;
  float rho;
  float R[9];       // rotation, row-major
  bool ok;
};

__device__ inline bool finitef(float x) { return __builtin_isfinite(x); }

// Loads Gaussian i and builds its rotation (Hamilton convention, normalised).
__device__ inline void load_gauss(const float *mean, const float *scale, const float *quat,
                                  const float *dens, int64_t i, Gauss &G) {
  float q[4];
  bool ok = true;
  for (int k = 0; k < 3; ++k) {
    G.p[k] = mean[3 * i + k];
    G.s[k] = scale[3 * i + k];
    ok = ok && finitef(G.p[k]) && finitef(G.s[k]) && G.s[k] > 0.f;
  }
  for (int k = 0; k < 4; ++k) {
    q[k] = quat[4 * i + k];
    ok = ok && finitef(q[k]);
  }
  G.rho = dens[i];
  ok = ok && finitef(G.rho);
  float n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  ok = ok && n2 > 0.f && finitef(n2);
  float n = sqrtf(n2);
  float in = ok ? frcp(n) : 0.f;
  G.qnorm = n;
  float w = q[0] * in, x = q[1] * in, y = q[2] * in, z = q[3] * in;
  G.qn[0] = w; G.qn[1] = x; G.qn[2] = y; G.qn[3] = z;
  G.R[0] = 1.f - 2.f * (y * y + z * z); G.R[1] = 2.f * (x * y - w * z); G.R[2] = 2.f * (x * z + w * y);
  G.R[3] = 2.f * (x * y + w * z); G.R[4] = 1.f - 2.f * (x * x + z * z); G.R[5] = 2.f * (y * z - w * x);
  G.R[6] = 2.f * (x * z - w * y); G.R[7] = 2.f * (y * z + w * x); G.R[8] = 1.f - 2.f * (x * x + y * y);
  G.ok = ok;
}

// Chain rule from dL/dR (row-major 3x3) to dL/dq for the unnormalised input q.
__device__ inline void quat_backward(const Gauss &G, const float *gR, float *gq) {
  float w = G.qn[0], x = G.qn[1], y = G.qn[2], z = G.qn[3];
  float gw = 2.f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
  float gx = 2.f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.f * x * gR[4] - w * gR[5] + z * gR[6] +
                    w * gR[7] - 2.f * x * gR[8]);
  float gy = 2.f * (-2.f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                    z * gR[7] - 2.f * y * gR[8]);
  float gz = 2.f * (-2.f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.f * z * gR[4] +
                    y * gR[5] + x * gR[6] + y * gR[7]);
  float dot = w * gw + x * gx + y * gy + z * gz;
  float in = frcp(G.qnorm);
  gq[0] = (gw - w * dot) * in;
  gq[1] = (gx - x * dot) * in;
  gq[2] = (gy - y * dot) * in;
  gq[3] = (gz - z * dot) * in;
}

// --------------------------------------------------------- 2D projection --

struct Proj2 {
  bool ok;
  float t[3];
  float l;          // |t| (cone)
  float u[3];       // t / |t| (cone)
  float JW[6];      // first two rows of J W (2x3)
  float M[9];       // R S
  float B[6];       // JW M
  float S00, S01, S11, det;
  float A00, A01, A11;
  float ph0, ph1;   // projected centre, detector units
  float d[3];       // unit direction of the ray through the centre (world)
  float r[3];       // R^T d
  float m;          // d^T Sigma^{-1} d
  float mu;         // rectification factor sqrt(2 pi / m)
};

// Transformation + projection + rectification of one Gaussian for one view.
// Cone beam (App. A): t = W p + (0,0,L_SO); p_hat = L_SD (t0, t1) / t2; the
// first two rows of the local affine Jacobian are those of the perspective
// map.  Sigma_hat = B B^T with B = J W R S, so det Sigma_hat is a sum of
// squared 2x2 minors of B (no cancellation).  The rectification factor
// sqrt(2 pi |Sigma_tilde| / |Sigma_hat|) equals sqrt(2 pi / (d^T Sigma^{-1} d))
// with d the world direction of the ray through the centre, because the third
// row of J is t/|t|; the direction form needs no 3x3 determinant.
__device__ inline void project_one(const Gauss &G, const DevView &V, Proj2 &P) {
  const float *W = V.W;
  P.ok = G.ok;
  for (int a = 0; a < 3; ++a)
    P.t[a] = W[3 * a] * G.p[0] + W[3 * a + 1] * G.p[1] + W[3 * a + 2] * G.p[2];
  if (V.beam == 1) {
    P.t[2] += V.L_SO;
    if (!(P.t[2] > 1e-3f * V.L_SO)) P.ok = false;
    float t2 = P.ok ? P.t[2] : 1.f;
    float inv = frcp(t2);
    float L = V.L_SD;
    P.ph0 = L * P.t[0] * inv;
    P.ph1 = L * P.t[1] * inv;
    float a0 = P.t[0] * inv, a1 = P.t[1] * inv, Li = L * inv;
    for (int i = 0; i < 3; ++i) {
      P.JW[i] = Li * (W[i] - a0 * W[6 + i]);
      P.JW[3 + i] = Li * (W[3 + i] - a1 * W[6 + i]);
    }
    P.l = sqrtf(P.t[0] * P.t[0] + P.t[1] * P.t[1] + t2 * t2);
    float il = frcp(P.l);
    P.u[0] = P.t[0] * il; P.u[1] = P.t[1] * il; P.u[2] = t2 * il;
    for (int i = 0; i < 3; ++i) P.d[i] = P.u[0] * W[i] + P.u[1] * W[3 + i] + P.u[2] * W[6 + i];
  } else {
    P.ph0 = P.t[0];
    P.ph1 = P.t[1];
    for (int i = 0; i < 6; ++i) P.JW[i] = W[i];
    P.l = 1.f;
    P.u[0] = P.u[1] = 0.f; P.u[2] = 1.f;
    for (int i = 0; i < 3; ++i) P.d[i] = W[6 + i];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P.M[3 * i + j] = G.R[3 * i + j] * G.s[j];
  for (int a = 0; a < 2; ++a)
    for (int j = 0; j < 3; ++j)
      P.B[3 * a + j] = P.JW[3 * a] * P.M[j] + P.JW[3 * a + 1] * P.M[3 + j] + P.JW[3 * a + 2] * P.M[6 + j];
  const float *b0 = P.B, *b1 = P.B + 3;
  P.S00 = b0[0] * b0[0] + b0[1] * b0[1] + b0[2] * b0[2];
  P.S01 = b0[0] * b1[0] + b0[1] * b1[1] + b0[2] * b1[2];
  P.S11 = b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2];
  float m0 = b0[1] * b1[2] - b0[2] * b1[1];
  float m1 = b0[2] * b1[0] - b0[0] * b1[2];
  float m2 = b0[0] * b1[1] - b0[1] * b1[0];
  P.det = m0 * m0 + m1 * m1 + m2 * m2;
  float idet = frcp(P.det);
  P.A00 = P.S11 * idet;
  P.A01 = -P.S01 * idet;
  P.A11 = P.S00 * idet;
  float m = 0.f;
  for (int j = 0; j < 3; ++j) {
    P.r[j] = G.R[j] * P.d[0] + G.R[3 + j] * P.d[1] + G.R[6 + j] * P.d[2];
    float z = P.r[j] * frcp(G.s[j]);
    m += z * z;
  }
  P.m = m;
  P.mu = sqrtf(kTwoPi * frcp(m));
  P.ok = P.ok && P.det > 0.f && finitef(P.A00) && finitef(P.A11) && finitef(P.A01) && m > 0.f &&
         finitef(P.mu) && finitef(P.ph0) && finitef(P.ph1) && finitef(P.mu * G.rho);
}

// Minimum over a rectangle [x0,x1] x [y0,y1] (offsets from the centre) of the
// positive-definite form a dx^2 + b dx dy + c dy^2; ia = 1/(2a), ic = 1/(2c).
// With the centre outside the rectangle the minimum lies on an edge whose
// half-plane excludes the centre (at a minimum with only the constraints of
// one axis active, the gradient condition puts the centre beyond that edge;
// a corner minimum with neither edge facing the centre would force the corner
// to be the centre).  So only the facing x edge and the facing y edge are
// searched; where no x (y) edge faces the centre, the other axis' edge holds
// the minimum and the extra candidate is just some point of the rectangle.
// Number of set bits of `mask` below the calling lane.
__device__ inline int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Sum of n strided values p[0], p[stride], ... added in index order, with
// four loads in flight (a run-time trip count otherwise issues one at a time).
__device__ inline float strided_sum(const float *__restrict__ p, int64_t stride, int n) {
  float acc = 0.f;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    const float x0 = p[k * stride], x1 = p[(k + 1) * stride], x2 = p[(k + 2) * stride],
                x3 = p[(k + 3) * stride];
    acc += x0;
    acc += x1;
    acc += x2;
    acc += x3;
  }
  for (; k < n; ++k) acc += p[k * stride];
  return acc;
}

// Tile-list entry (Gaussian index | sub-tile mask << kEntryMaskShift, backward
// slot): bit w of the mask is set when the cutoff ellipse meets 8x8 sub-tile w
// of the 16x16 tile (w = (x half) + 2 (y half)).
constexpr int kEntryMaskShift = 28;
constexpr uint32_t kEntryIndexMask = (1u << kEntryMaskShift) - 1u;

__device__ inline float rect_min_form(float a, float b, float c, float ia, float ic, float x0,
                                      float x1, float y0, float y1) {
  if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return 0.f;
  const float xe = x0 > 0.f ? x0 : x1;
  const float ye = y0 > 0.f ? y0 : y1;
  const float dy = fminf(fmaxf(-b * xe * ic, y0), y1);
  const float dx = fminf(fmaxf(-b * ye * ia, x0), x1);
  return fminf(a * xe * xe + b * xe * dy + c * dy * dy, a * dx * dx + b * dx * ye + c * ye * ye);
}

// Workgroup index remapped so that each XCD (workgroups are dealt round-robin
// to the 8 XCDs) receives a contiguous range of items, keeping one view's
// records in one XCD's L2.
__device__ inline int xcd_remap(int b, int n) {
  int xcd = b & 7, r = b >> 3;
  int q = n >> 3, rem = n & 7;
  int start = xcd * q + (xcd < rem ? xcd : rem);
  return start + r;
}

// Part `part` of `parts` of the tile-list range [b, e), split on multiples of
// 64 entries (one wave's batch) so that the parts of a long list get equal work.
__device__ inline void list_part(uint32_t b, uint32_t e, int part, int parts, uint32_t &pb,
                                 uint32_t &pe) {
  if (parts == 1) {
    pb = b;
    pe = e;
    return;
  }
  const uint32_t nb = (e - b + 63) / 64;
  const uint32_t b0 = (uint32_t)(((uint64_t)nb * part) / parts);
  const uint32_t b1 = (uint32_t)(((uint64_t)nb * (part + 1)) / parts);
  pb = min(e, b + 64 * b0);
  pe = min(e, b + 64 * b1);
}

// ---------------------------------------------------- scan primitives --

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan over a 256-thread workgroup; all threads must call it.
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t *sh4, uint32_t &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(x);
  if (lane == 63) sh4[w] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (int i = 0; i < w; ++i) pre += sh4[i];
  total = sh4[0] + sh4[1] + sh4[2] + sh4[3];
  __syncthreads();
  return pre + inc - x;
}

__device__ inline uint32_t block_sum(uint32_t x, uint32_t *sh4) {
  uint32_t t;
  block_excl_scan(x, sh4, t);
  return t;
}

// The last j in [0, 256) with off[j] <= e, off non-decreasing (for e < off[256],
// Gaussian j is the one whose entries hold entry e).
__device__ inline int entry_owner(const uint32_t *off, uint32_t e) {
  int j = 0;
#pragma unroll
  for (int step = kBlock / 2; step > 0; step >>= 1)
    if (off[j + step] <= e) j += step;
  return j;
}

// The same search, for an entry known to belong to one of lo .. hi
// (hi - lo < 64): off[lo] <= e < off[hi + 1].
__device__ inline int entry_owner_in(const uint32_t *off, uint32_t e, int lo, int hi) {
  int j = lo;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1)
    if (j + step <= hi && off[j + step] <= e) j += step;
  return j;
}

// ------------------------------------------------------------ launchers --

// Gaussian set of one view of a multi-model projection call (views of one
// call may render different resident models).
struct ViewSet {
  const float *mean, *scale, *quat, *dens;
  int64_t M;      // Gaussians of the set
  int64_t rbase;  // the view's first record (and slot offset) index
};

struct ProjArgs {
  const float *mean, *scale, *quat, *dens;
  int64_t M;                      // Gaussians (multi-model calls: the largest set)
  int V;
  const DevView *views;
  int width, height, TX, TY, T;   // tiles per view T = TX * TY
  int C;                          // chunks per view
  float kappa, thr, qmax;         // cutoff, exp2-threshold (-qmax), positive-form limit
  int rectify;                    // 1: rho_hat = mu rho (Eq. 7); 0: rho_hat = rho (unrectified)
  int cpt;                        // Gaussians per thread per binning chunk (chunk = kBlock * cpt)
  int parts;                      // workgroups per tile list in the render kernels (>= 1)
  uint32_t cap;                   // tile-list entries the list and slot buffers hold
  const unsigned long long *totals;  // totals[0]: entries this call needs (> cap: overflow)
  unsigned int *ovf_host;         // host-visible overflow flag of the plan (reserved plans), or null
  const ViewSet *sets;            // per-view Gaussian sets (multi-model forward), or null
  int64_t R;                      // records of the call: V M, or the sum of the views' sets
};

// The Gaussian set and record base of view v (the call's one set unless the
// call renders several models).
__device__ inline ViewSet view_set(const ProjArgs &a, int v) {
  if (a.sets) return a.sets[v];
  return ViewSet{a.mean, a.scale, a.quat, a.dens, a.M, (int64_t)v * a.M};
}

void launch_mean_mu(const ProjArgs &a, float *mu_out, float *density_out, hipStream_t s);
void launch_proj_hist(const ProjArgs &a, Rec2 *rec, uint32_t *hist, uint32_t *chunk_cnt,
                      unsigned long long *skipped, hipStream_t s);
void launch_hist_colscan(int groups, int C, int T, uint32_t *hist, uint32_t *tile_total,
                         hipStream_t s);
void launch_scan2(const uint32_t *in0, uint32_t *out0, int n0, const uint32_t *in1, uint32_t *out1,
                  int n1, unsigned long long *totals, hipStream_t s);
// Tile-list entries are (Gaussian index, backward slot) pairs.
// Control words of a plan (unsigned long long [8]): 0, 1 running skipped
// counts of the projection and voxelization binning; 2, 3 the last call's;
// 4, 5 the largest entry count since the last check; 6, 7 the number of calls
// whose entries exceeded the capacity since then.  The projection scatter
// moves 0 to 2, clears 0 and records 4 and 6 from totals[0]; entries at
// positions >= a.cap are dropped, the host-visible flag a.ovf_host is set,
// and the chain kernels of that call write nothing (their slots would be
// incomplete).
void launch_proj_scatter(const ProjArgs &a, const Rec2 *rec, const uint32_t *hist,
                         const uint32_t *tile_start, const uint32_t *chunk_start, uint2 *list,
                         uint32_t *offsets, unsigned long long *ctl,
                         const unsigned long long *totals, hipStream_t s);
// With a.parts > 1, each part of a tile list writes its pixel sums to
// partial [parts][V * T][256] and a second kernel adds the parts in order.
void launch_render_fwd(const ProjArgs &a, const Rec2 *rec, const uint2 *list,
                       const uint32_t *tile_start, float *image, float *partial, hipStream_t s);
void launch_render_bwd(const ProjArgs &a, const Rec2 *rec, const uint2 *list,
                       const uint32_t *tile_start, const float *grad_image, float *slots,
                       hipStream_t s);
int proj_chain_chunks(int n_views);  // partial-gradient chunks (16 or 18 floats per Gaussian each)
// Optional densification statistics of the projection backward: per Gaussian,
// ndc_sum += scale * sum over visible views of |dL/dp_hat| in normalised
// device coordinates, visible += number of those views (no statistics when
// ndc_sum is null).
struct ChainStats {
  float *ndc_sum;
  int32_t *visible;
  float scale;
};
void launch_proj_chain(const ProjArgs &a, const uint32_t *offsets,
                       const float *slots, float *part, float *g_mean, float *g_scale,
                       float *g_quat, float *g_dens, int accumulate, const ChainStats &st,
                       hipStream_t s);

struct VoxArgs {
  const float *mean, *scale, *quat, *dens;
  int64_t M;
  int nx, ny, nz;
  float origin[3], spacing[3];
  int TX, TY, TZ;          // tiles per axis
  int layers;              // z tile layers per group
  int G;                   // groups
  int Tg;                  // tiles per group = TX * TY * layers
  int C;                   // chunks
  float kappa, thr, qmax;
  int cpt;                 // Gaussians per thread per binning chunk (chunk = kBlock * cpt)
  int parts;               // workgroups per tile list in the forward (>= 1)
  int bparts;              // and in the backward (its per-batch setup favours fewer parts)
  uint32_t cap;            // tile-list entries the list and slot buffers hold
  const unsigned long long *totals;  // totals[0]: entries this call needs (> cap: overflow)
  unsigned int *ovf_host;  // host-visible overflow flag of the plan (reserved plans), or null
};

void launch_vox_records(const VoxArgs &a, Rec3 *rec, uint32_t *count,
                        unsigned long long *skipped, hipStream_t s);
void launch_scan_big(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *block_tmp,
                     unsigned long long *total, hipStream_t s);
void launch_vox_hist(const VoxArgs &a, const Rec3 *rec, uint32_t *hist, hipStream_t s);
// Control words as for the projection: moves 1 to 3, clears 1, records 5
// and 7 from totals[0]; entries at positions >= a.cap are dropped.
void launch_vox_scatter(const VoxArgs &a, const Rec3 *rec, const uint32_t *hist,
                        const uint32_t *tile_start, uint32_t *list, unsigned long long *ctl,
                        const unsigned long long *totals, hipStream_t s);
// With a.parts > 1, partial [parts][G * Tg][512] holds each part's voxel sums,
// added in part order by a second kernel.
void launch_vox_fwd(const VoxArgs &a, const Rec3 *rec, const uint32_t *list,
                    const uint32_t *tile_start, float *volume, float *partial, hipStream_t s);
void launch_vox_bwd(const VoxArgs &a, const Rec3 *rec, const uint32_t *list,
                    const uint32_t *tile_start, const uint32_t *offsets, const float *grad_volume,
                    float *slots, hipStream_t s);
void launch_vox_chain(const VoxArgs &a, const uint32_t *offsets, const float *slots,
                      float *g_mean, float *g_scale, float *g_quat, float *g_dens, int accumulate,
                      hipStream_t s);

void launch_ssim_coeffs(const float *x, const float *y, int n, int h, int w, float *coef,
                        float *partials, hipStream_t s);
void launch_loss_finish(const float *partials, int n_part, int n, int h, int w, float lambda_ssim,
                        float *loss_out, hipStream_t s);
void launch_ssim_march(const float *x, const float *y, int n, int h, int w, float lambda_ssim,
                       float *grad, float *partials, hipStream_t s);
int loss_image_blocks(int n, int h, int w);
int ssim_num_blocks(int n, int h, int w);
void launch_tv(const float *vol, int nx, int ny, int nz, float weight, float *grad, int accumulate,
               float *partials, int *n_part, hipStream_t s);
void launch_tv_finish(const float *partials, int n_part, float *loss_out, hipStream_t s);
int tv_num_blocks(int nx, int ny, int nz);

// ------------------------------------------------------ training loop --

// Sets the message gs_last_error returns (for errors found outside api.hip).
void set_last_error(const char *msg);
// A plan's device control words (layout above), or null before its first call.
const unsigned long long *plan_control_words(const gs_plan *p);
// Device word holding the tile-list entries the plan's last projection
// (voxel = 0) or voxelization (voxel = 1) binning needed, or null; and the
// entries a reserved plan holds for that operator (0 if not reserved).
const unsigned long long *plan_entries_needed(const gs_plan *p, int voxel);
int64_t plan_entry_capacity(const gs_plan *p, int voxel);
// The device form of a view.
DevView dev_view(const gs_view &v);
// Forward projection of several models' views on a reserved plan, issuing
// kernel launches only (no copy, memset, event or host synchronization), so
// that a graph captured from it can be replayed for other batches of the same
// shape: the views (DevView[nv]) and per-view Gaussian sets (ViewSet[nv],
// records of view v from sets[v].rbase) are read from device memory, and the
// launch is sized for at most M_bound Gaussians per view and R_bound records,
// so its arguments depend on (nv, detector, bounds, cutoff, image) alone.
// Views beyond a batch's own may carry empty sets (n = 0).  Stage timing must
// be off on the plan.
gs_status project_fwd_device(gs_plan *pl, const DevView *views, const ViewSet *sets, int32_t nv,
                             int32_t width, int32_t height, int64_t M_bound, int64_t R_bound,
                             float cutoff, float *image, hipStream_t s);
// gs_adam_step that does nothing on the device when plan g0 or g1 (either may
// be null) records a call that overflowed its reservation since its last check.
gs_status adam_step_guarded(const gs_params *p, int64_t n, const gs_grads *grads,
                            const gs_adam_config *cfg, const gs_plan *g0, const gs_plan *g1,
                            hipStream_t stream);

struct AdamArgs {
  float *raw[4];         // mean, log_scale, quat, density_raw
  float *m[4], *v[4];
  const float *grad[4];  // with respect to the activated parameters
  float *scale, *density;
  int64_t n;
  float lr[4];
  float beta1, beta2, omb1, omb2;  // beta and 1 - beta, each rounded once from double
  float eps, bc1_inv, bc2_inv;
  // control words of up to two plans (or null): the step does nothing if
  // either records an overflowing call since its last gs_plan_check
  const unsigned long long *guard[2];
};
void launch_adam(const AdamArgs &a, hipStream_t s);
void launch_random_normals(uint64_t seed, uint64_t counter, int64_t n, float *out, hipStream_t s);
void launch_activate(float *log_scale, float *density_raw, float *scale, float *density, int64_t n,
                     int inverse, hipStream_t s);

struct ParamPtrs {
  float *mean, *log_scale, *quat, *density_raw, *scale, *density;
  float *m_mean, *m_scale, *m_quat, *m_density, *v_mean, *v_scale, *v_quat, *v_density;
};
struct DensifyArgs {
  ParamPtrs src, dst;
  int64_t n;
  const float *grad_sum;
  const int32_t *visible;
  const float *normals;
  float grad_threshold;
  float t_keep, t_half, t_scale;  // raw-space thresholds
  float log_split;                // log(1.6)
  int densify;
};
void launch_densify_count(const DensifyArgs &a, int32_t *action, uint32_t *count, hipStream_t s);
void launch_densify_write(const DensifyArgs &a, const int32_t *action, const uint32_t *offset,
                          hipStream_t s);

int metric_num_blocks(int64_t n);
// out[0] = sum of squared differences, out[1] = max(gt)
void launch_metric_sums(const float *vol, const float *gt, int64_t n, double *part_sse,
                        float *part_max, double *out, hipStream_t s);
void launch_slices(const float *vol, int nx, int ny, int nz, int axis, const double *range,
                   float *out, hipStream_t s);

}  // namespace gsk
