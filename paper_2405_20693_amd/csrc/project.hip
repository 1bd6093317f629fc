// X-ray rasterizer kernels: per-(view, Gaussian) projection with tile
// histograms, tile-list scatter, tile render forward/backward and the
// per-Gaussian chain rule (paper Sec. 3.2.1, Eq. 5-7, App. A).
#include <utility>

#include "internal.h"

namespace gsk {

// --------------------------------------------------------- projection ----

// Record (pixel units) and tile rectangle of one projected Gaussian.
__device__ inline Rec2 make_rec2(const Gauss &G, const Proj2 &P, const DevView &V,
                                 const ProjArgs &a) {
  Rec2 r;
  r.r0 = 1u;  // empty rectangle: tx0 = 1 > tx1 = 0
  r.r1 = 0u;
  if (!P.ok) {
    r.pu = r.pv = r.c00 = r.c01 = r.c11 = r.rho = 0.f;
    return r;
  }
  r.pu = P.ph0 * V.inv_hu + V.cu;
  r.pv = P.ph1 * V.inv_hv + V.cv;
  r.c00 = -0.5f * kLog2e * P.A00 * V.hu * V.hu;
  r.c01 = -kLog2e * P.A01 * V.hu * V.hv;
  r.c11 = -0.5f * kLog2e * P.A11 * V.hv * V.hv;
  r.rho = (a.rectify ? P.mu : 1.f) * G.rho;
  float ru = a.kappa * sqrtf(P.S00) * V.inv_hu;
  float rv = a.kappa * sqrtf(P.S11) * V.inv_hv;
  const float eps = 1e-3f;
  float x0 = fmaxf(ceilf(r.pu - ru - eps), 0.f);
  float x1 = fminf(floorf(r.pu + ru + eps), (float)(a.width - 1));
  float y0 = fmaxf(ceilf(r.pv - rv - eps), 0.f);
  float y1 = fminf(floorf(r.pv + rv + eps), (float)(a.height - 1));
  if (x0 <= x1 && y0 <= y1) {
    int tx0 = (int)x0 / kTile, tx1 = (int)x1 / kTile;
    int ty0 = (int)y0 / kTile, ty1 = (int)y1 / kTile;
    r.r0 = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
    r.r1 = (uint32_t)tx1 | ((uint32_t)ty1 << 16);
  }
  return r;
}

// Grid (C chunks, V views).  Projects the chunk's Gaussians for one view,
// writes their records and counts tile entries in an LDS histogram.
__global__ __launch_bounds__(kBlock) void k_proj_hist(ProjArgs a, Rec2 *__restrict__ rec,
                                                      uint32_t *__restrict__ hist,
                                                      uint32_t *__restrict__ chunk_cnt,
                                                      unsigned long long *skipped) {
  extern __shared__ uint32_t sh[];
  __shared__ uint32_t sh4[4];
  const int c = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
  for (int t = tid; t < a.T; t += kBlock) sh[t] = 0;
  __syncthreads();
  const DevView V = a.views[v];
  const ViewSet S = view_set(a, v);
  uint32_t cnt = 0, skip = 0;
  const int64_t g0 = (int64_t)c * kBlock * a.cpt;
  for (int k = 0; k < a.cpt; ++k) {
    int64_t g = g0 + (int64_t)k * kBlock + tid;
    if (g >= S.M) break;
    Gauss G;
    load_gauss(S.mean, S.scale, S.quat, S.dens, g, G);
    Proj2 P;
    project_one(G, V, P);
    Rec2 r = make_rec2(G, P, V, a);
    skip += P.ok ? 0u : 1u;
    rec[S.rbase + g] = r;
    Rect2 rc = unpack_rect(r.r0, r.r1);
    int n = rect_count(rc);
    cnt += (uint32_t)n;
    for (int ty = rc.y0; ty <= rc.y1 && n; ++ty)
      for (int tx = rc.x0; tx <= rc.x1; ++tx) atomicAdd(&sh[ty * a.TX + tx], 1u);
  }
  uint32_t tot = block_sum(cnt, sh4);
  uint32_t sk = block_sum(skip, sh4);
  __syncthreads();
  uint32_t *h = hist + ((int64_t)v * a.C + c) * a.T;
  for (int t = tid; t < a.T; t += kBlock) h[t] = sh[t];
  if (tid == 0) {
    chunk_cnt[v * a.C + c] = tot;
    if (sk) atomicAdd(skipped, (unsigned long long)sk);
  }
}

// Mean over the views of each Gaussian's rectification factor mu (views where
// the Gaussian is culled are left out; 0 if culled in every view), and
// optionally rho / mean(mu).
__global__ __launch_bounds__(kBlock) void k_mean_mu(ProjArgs a, float *__restrict__ mu_out,
                                                    float *__restrict__ density_out) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= a.M) return;
  Gauss G;
  load_gauss(a.mean, a.scale, a.quat, a.dens, g, G);
  float sum = 0.f;
  int n = 0;
  for (int v = 0; v < a.V; ++v) {
    Proj2 P;
    project_one(G, a.views[v], P);
    if (P.ok) {
      sum += P.mu;
      ++n;
    }
  }
  const float m = n ? sum / (float)n : 0.f;
  if (mu_out) mu_out[g] = m;
  if (density_out) density_out[g] = m > 0.f ? G.rho / m : 0.f;
}

void launch_mean_mu(const ProjArgs &a, float *mu_out, float *density_out, hipStream_t s) {
  unsigned nb = (unsigned)((a.M + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_mean_mu, dim3(nb), dim3(kBlock), 0, s, a, mu_out, density_out);
}

void launch_proj_hist(const ProjArgs &a, Rec2 *rec, uint32_t *hist, uint32_t *chunk_cnt,
                      unsigned long long *skipped, hipStream_t s) {
  dim3 grid(a.C, a.V);
  hipLaunchKernelGGL(k_proj_hist, grid, dim3(kBlock), a.T * sizeof(uint32_t), s, a, rec, hist,
                     chunk_cnt, skipped);
}

// Per (group, tile) column: exclusive prefix over the chunks, in place, and
// the tile totals.  A workgroup takes 64 consecutive columns (lane = column,
// so each load instruction reads 256 contiguous bytes) and splits every column
// into kColSeg segments, one per wave: each wave sums its segment, the
// segment sums are scanned through LDS, and each wave rescans its segment
// from its base.  Few-view calls bin in hundreds of small chunks, where one
// thread per column would walk the whole column serially.
constexpr int kColSeg = 16;

__global__ __launch_bounds__(64 * kColSeg) void k_hist_colscan(int groups, int C, int T,
                                                               uint32_t *__restrict__ hist,
                                                               uint32_t *__restrict__ tile_total) {
  __shared__ uint32_t s_sum[kColSeg][64];
  const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = col < (int64_t)groups * T;
  const int grp = ok ? (int)(col / T) : 0, t = ok ? (int)(col - (int64_t)grp * T) : 0;
  uint32_t *h = hist + (int64_t)grp * C * T + t;
  const int L = (C + kColSeg - 1) / kColSeg;
  const int c0 = min(C, seg * L), c1 = min(C, c0 + L);
  uint32_t sum = 0;
  if (ok) {
    int c = c0;
    for (; c + 8 <= c1; c += 8) {  // batches of 8 independent loads
      uint32_t x[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = h[(int64_t)(c + k) * T];
#pragma unroll
      for (int k = 0; k < 8; ++k) sum += x[k];
    }
    for (; c < c1; ++c) sum += h[(int64_t)c * T];
  }
  s_sum[seg][lane] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (int k = 0; k < seg; ++k) run += s_sum[k][lane];
  if (!ok) return;
  if (seg == kColSeg - 1) tile_total[col] = run + sum;
  int c = c0;
  for (; c + 8 <= c1; c += 8) {
    uint32_t x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = h[(int64_t)(c + k) * T];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      h[(int64_t)(c + k) * T] = run;
      run += x[k];
    }
  }
  for (; c < c1; ++c) {
    const uint32_t x = h[(int64_t)c * T];
    h[(int64_t)c * T] = run;
    run += x;
  }
}

void launch_hist_colscan(int groups, int C, int T, uint32_t *hist, uint32_t *tile_total,
                         hipStream_t s) {
  const int64_t n = (int64_t)groups * T;
  hipLaunchKernelGGL(k_hist_colscan, dim3((unsigned)((n + 63) / 64)), dim3(64 * kColSeg), 0, s,
                     groups, C, T, hist, tile_total);
}

// Grid (C, V).  Writes each Gaussian's tile entries and the base index of
// its backward slots (Gaussian order within the chunk).  The placement is a
// stable counting sort: a chunk's entries of one tile sit in Gaussian order at
// the tile's cursor, so every tile list is sorted by Gaussian index and any
// two runs of the binning give the same lists (the forward's sums then run in
// a fixed order).  Lanes take entries, not Gaussians: after the scan of the
// 256 Gaussians' entry counts, an entry finds its Gaussian by binary search of
// the staged offsets, so Gaussians covering many tiles do not idle the rest
// of their wave.  Entries are placed in rounds of at most 256 entries from at
// most 64 consecutive Gaussians: each entry sets its Gaussian's bit (index
// within the round) in its tile's 64-bit LDS mask; after a barrier its
// position is the tile's cursor plus the number of lower bits set, and the
// entry holding the highest bit then advances the cursor and clears the mask.
// Tiles are handled in windows of kScatterWindow so that masks and cursors
// fit LDS.  Detectors of more than 2048 tiles use 32-bit masks (rounds of at
// most 32 Gaussians) so that three workgroups fit a CU; the lists are the
// same with either width, only the rounds differ.  Each entry carries the mask of the tile's 8x8 sub-tiles that the
// cutoff ellipse meets (exact minimum of the quadratic form over each
// sub-tile's pixel-centre rectangle).
constexpr int kScatterWindow = 4096;

constexpr int kScatterWideTiles = 2048;  // above this, 32-bit masks

template <typename MaskT>
int proj_scatter_lds(int T) { return min(T, kScatterWindow) * (int)(sizeof(MaskT) + 4); }

__device__ inline int mask_popc(uint32_t m) { return __popc(m); }
__device__ inline int mask_popc(unsigned long long m) { return __popcll(m); }

template <typename MaskT>
__global__ __launch_bounds__(kBlock) void k_proj_scatter(ProjArgs a, const Rec2 *__restrict__ rec,
                                                         const uint32_t *__restrict__ hist,
                                                         const uint32_t *__restrict__ tile_start,
                                                         const uint32_t *__restrict__ chunk_start,
                                                         uint2 *__restrict__ list,
                                                         uint32_t *__restrict__ offsets,
                                                         unsigned long long *ctl,
                                                         const unsigned long long *totals) {
  constexpr int kRoundG = 8 * (int)sizeof(MaskT);  // Gaussians per placement round
  extern __shared__ unsigned long long s_dyn[];     // window masks, then cursors
  __shared__ uint32_t sh4[4];
  __shared__ uint32_t s_off[kBlock + 1];  // exclusive entry offsets of the 256 Gaussians
  __shared__ uint32_t s_org[kBlock];      // rectangle origin tx0 | ty0 << 16
  __shared__ float s_w[kBlock];           // rectangle width in tiles
  __shared__ float s_pu[kBlock], s_pv[kBlock], s_fa[kBlock], s_fb[kBlock], s_fc[kBlock];
  __shared__ float s_ia[kBlock], s_ic[kBlock];
  __shared__ int s_jnext;                 // owner of the round's last entry
  const int c = blockIdx.x, v = blockIdx.y, tid = threadIdx.x;
  const int Tw = min(a.T, kScatterWindow);
  MaskT *s_mask = reinterpret_cast<MaskT *>(s_dyn);
  uint32_t *cur = reinterpret_cast<uint32_t *>(s_mask + Tw);
  if (c == 0 && v == 0 && tid == 0) {  // the binning kernels of this call have finished
    ctl[2] = ctl[0];
    ctl[0] = 0ull;
    const unsigned long long e = totals[0];
    atomicMax(&ctl[4], e);
    if (e > a.cap) {
      atomicAdd(&ctl[6], 1ull);
      if (a.ovf_host) *(volatile unsigned int *)a.ovf_host = 1u;
    }
  }
  const uint32_t *h = hist + ((int64_t)v * a.C + c) * a.T;
  const uint32_t *ts = tile_start + (int64_t)v * a.T;
  const int64_t g0 = (int64_t)c * kBlock * a.cpt;
  const ViewSet S = view_set(a, v);
  uint32_t base = 0;
  for (int w0 = 0; w0 < a.T; w0 += Tw) {
    const int wn = min(Tw, a.T - w0);
    for (int t = tid; t < wn; t += kBlock) {
      cur[t] = ts[w0 + t] + h[w0 + t];
      s_mask[t] = 0;
    }
    base = chunk_start[v * a.C + c];
    // each batch's records are loaded one batch ahead (zero past the set)
    Rec2 r_next{};
    if (g0 + tid < S.M) r_next = rec[S.rbase + g0 + tid];
    for (int k = 0; k < a.cpt; ++k) {
      const int64_t gk = g0 + (int64_t)k * kBlock;
      if (gk >= S.M) break;
      const int64_t g = gk + tid;
      const bool valid = g < S.M;
      const Rec2 r = r_next;
      if (k + 1 < a.cpt) {
        Rec2 rn{};
        if (g + kBlock < S.M) rn = rec[S.rbase + g + kBlock];
        r_next = rn;
      }
      Rect2 rc{1, 0, 0, 0};
      if (valid) rc = unpack_rect(r.r0, r.r1);
      const int n = valid ? rect_count(rc) : 0;
      uint32_t total;
      const uint32_t ex = block_excl_scan((uint32_t)n, sh4, total);  // synchronizes the workgroup
      if (valid && w0 == 0) offsets[S.rbase + g] = base + ex;
      s_off[tid] = ex;
      if (tid == 0) s_off[kBlock] = total;
      s_org[tid] = (uint32_t)rc.x0 | ((uint32_t)rc.y0 << 16);
      s_w[tid] = (float)(rc.x1 - rc.x0 + 1);
      s_pu[tid] = r.pu;
      s_pv[tid] = r.pv;
      s_fa[tid] = -r.c00;
      s_fb[tid] = -r.c01;
      s_fc[tid] = -r.c11;
      s_ia[tid] = -0.5f * frcp(r.c00);
      s_ic[tid] = -0.5f * frcp(r.c11);
      __syncthreads();
      // jA: a Gaussian at or below the owner of the round's first entry
      // (uniform).  The round ends at r1 <= s_off[jA + kRoundG], so its
      // entries belong to jA .. jA + kRoundG - 1 and the bit j - jA fits the
      // mask; the next round starts at jA + kRoundG if that bound ended this
      // one, else at the owner of this round's last entry.
      int jA = 0;
      for (uint32_t r0 = 0; r0 < total;) {
        const int jE = min(jA + kRoundG, kBlock);
        const uint32_t rG = s_off[jE];
        const uint32_t r1 = min(r0 + (uint32_t)kBlock, rG);
        const uint32_t e = r0 + (uint32_t)tid;
        int t = 0, bit = 0;
        bool act = false;
        uint2 ent;
        if (e < r1) {
          const int j = entry_owner_in(s_off, e, jA, jE - 1);
          if (e + 1 == r1) s_jnext = j;
          const uint32_t kin = e - s_off[j];
          const float wf = s_w[j];
          int ry = (int)((float)kin * frcp(wf));  // row within the rectangle, corrected below
          const int wi = (int)wf;
          if ((uint32_t)((ry + 1) * wi) <= kin) ++ry;
          if ((uint32_t)(ry * wi) > kin) --ry;
          const int rx = (int)kin - ry * wi;
          const uint32_t org = s_org[j];
          const int tx = (int)(org & 0xffffu) + rx, ty = (int)(org >> 16) + ry;
          t = ty * a.TX + tx - w0;
          act = t >= 0 && t < wn;
          if (act) {
            const float pu = s_pu[j], pv = s_pv[j], fa = s_fa[j], fb = s_fb[j], fc = s_fc[j];
            const float ia = s_ia[j], ic = s_ic[j];
            // the minimum of the form over each sub-tile's pixel-centre
            // rectangle (rect_min_form), with the terms of its column and of
            // its row formed once for the two sub-tiles that share them
            float x0[2], x1[2], xe[2], ys[2], y0[2], y1[2], ye[2], xs[2];
            bool xin[2], yin[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              const int sx = tx * kTile + k * kSub, sy = ty * kTile + k * kSub;
              x0[k] = (float)sx - pu;
              x1[k] = (float)(sx + kSub - 1) - pu;
              y0[k] = (float)sy - pv;
              y1[k] = (float)(sy + kSub - 1) - pv;
              xin[k] = x0[k] <= 0.f && x1[k] >= 0.f;
              yin[k] = y0[k] <= 0.f && y1[k] >= 0.f;
              xe[k] = x0[k] > 0.f ? x0[k] : x1[k];
              ye[k] = y0[k] > 0.f ? y0[k] : y1[k];
              ys[k] = -fb * xe[k] * ic;  // the minimising y on the facing x edge
              xs[k] = -fb * ye[k] * ia;  // the minimising x on the facing y edge
            }
            uint32_t m = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
              const int c = w & 1, r = w >> 1;
              float f = 0.f;
              if (!(xin[c] && yin[r])) {
                // clamps to the edges (y0 < y1, x0 < x1), one med3 each
                const float dy = __builtin_amdgcn_fmed3f(ys[c], y0[r], y1[r]);
                const float dx = __builtin_amdgcn_fmed3f(xs[r], x0[c], x1[c]);
                f = fminf(fa * xe[c] * xe[c] + fb * xe[c] * dy + fc * dy * dy,
                          fa * dx * dx + fb * dx * ye[r] + fc * ye[r] * ye[r]);
              }
              m |= (f <= a.qmax ? 1u : 0u) << w;
            }
            ent = make_uint2((uint32_t)(gk + j) | (m << kEntryMaskShift), base + e);
            bit = j - jA;
            atomicOr(&s_mask[t], (MaskT)1 << bit);
          }
        }
        __syncthreads();
        // read between the round's first and last barriers: the next round
        // writes s_jnext only after the last one
        const int jn = s_jnext;
        MaskT mk = 0;
        if (act) {
          mk = s_mask[t];
          const uint32_t pos = cur[t] + (uint32_t)mask_popc((MaskT)(mk & (((MaskT)1 << bit) - 1)));
          if (pos < a.cap) list[pos] = ent;
        }
        __syncthreads();
        if (act && (mk >> bit) == 1) {  // the round's last entry of this tile
          cur[t] += (uint32_t)mask_popc(mk);
          s_mask[t] = 0;
        }
        __syncthreads();
        jA = r1 == rG ? jE : jn;
        r0 = r1;
      }
      base += total;
      __syncthreads();  // the next batch restages
    }
  }
  // the slot total closes the offsets array (offsets[R]); the last chunk of
  // the last view ends there
  if (v == a.V - 1 && c == a.C - 1 && tid == 0) offsets[a.R] = base;
}

void launch_proj_scatter(const ProjArgs &a, const Rec2 *rec, const uint32_t *hist,
                         const uint32_t *tile_start, const uint32_t *chunk_start, uint2 *list,
                         uint32_t *offsets, unsigned long long *ctl,
                         const unsigned long long *totals, hipStream_t s) {
  dim3 grid(a.C, a.V);
  if (a.T > kScatterWideTiles)
    hipLaunchKernelGGL(k_proj_scatter<uint32_t>, grid, dim3(kBlock), proj_scatter_lds<uint32_t>(a.T),
                       s, a, rec, hist, tile_start, chunk_start, list, offsets, ctl, totals);
  else
    hipLaunchKernelGGL(k_proj_scatter<unsigned long long>, grid, dim3(kBlock),
                       proj_scatter_lds<unsigned long long>(a.T), s, a, rec, hist, tile_start,
                       chunk_start, list, offsets, ctl, totals);
}

// ------------------------------------------------------- render forward --

// One workgroup per (view, 16x16 tile); wave w owns the 8x8 sub-tile
// (w & 1, w >> 1).  The tile's records are staged in LDS in batches of 256,
// each expanded once about the tile centre.  For each chunk of 64 records,
// lane i takes record i if its entry's mask marks the wave's sub-tile (set by
// the scatter) and shifts the expansion to the sub-tile centre: with x, y the
// pixel offsets from that centre,
//   q' + log2|rho_hat| = A0 + A1 x + c00 x^2          on the first row,
// stepping down a column by D(y) = B0 + c01 x, D itself by 2 c11.  The kept
// records are compacted and dealt to the wave's eight 8-lane groups in turn;
// each lane evaluates one column of eight pixels.  Where every value of
// e = exp2(q') over the sub-tile is a normal FP32 number (form at most
// kFwdChainRange there, its maximum being at a corner, where the exponent is
// least, and |rho_hat| not tiny), e is stepped down the column by multiplication, e *= exp2(D),
// exp2(D) *= exp2(2 c11): two exp2 per column instead of eight; the sign of
// rho_hat rides on e and the cutoff becomes |e| >= exp2(threshold).  Other
// records keep exp2 per pixel with q' forward-differenced; the two kinds are
// queued apart, so a record's path is its own, and each queue runs in whole
// passes of the eight groups, its remainder carried to the next chunk.  The
// pixel sums
// sign(rho_hat) exp2(...) over the kept records (a plain sum: Eq. 7 composes
// 2D Gaussians additively, so the order is free); the groups' partial sums
// are added in a fixed order at the end.
constexpr float kFwdChainRange = 100.f;

__global__ __launch_bounds__(kBlock) void k_render_fwd(ProjArgs a, const Rec2 *__restrict__ rec,
                                                       const uint2 *__restrict__ list,
                                                       const uint32_t *__restrict__ tile_start,
                                                       float *__restrict__ image,
                                                       float *__restrict__ partial) {
  // staged records, relative to the tile centre, for the exponent
  // q' + log2|rho_hat| = K0 + K1 x + K2 y + c00 x^2 + c01 x y + c11 y^2:
  // (Pt = K0 + (kShift^2 + hs^2)(c00 + c11), K1, K2, c00), (c01, c11,
  // sign(rho_hat) S, -et' S) of the cutoff factor for the threshold
  // et = exp2(threshold + log2|rho_hat|), (threshold + log2|rho_hat|, the
  // least exponent the multiplicative walk accepts, or +inf when et is too
  // small for the factor), and the entry's sub-tile mask (empty for a zero
  // density)
  __shared__ float4 s_r0[kBlock], s_r1[kBlock];
  __shared__ float2 s_r2[kBlock];
  __shared__ uint8_t s_m[kBlock];
  __shared__ uint8_t s_h[4][kBlock];  // per wave: the batch's records that mark its sub-tile
  // per wave: the kept records' coefficients, compacted, two float4 each in
  // two arrays, so that the eight groups read eight consecutive float4:
  // multiplicative records queue from the front, per-pixel exp2 records from
  // the back.  Each queue is evaluated in whole passes of eight records; up
  // to seven left over wait at its head for the next chunk, so that only the
  // last pass of the tile list runs part-filled (64 new records and two
  // remainders of seven fit the 78 places; 20 KB in all keeps eight
  // workgroups per CU)
  constexpr int kQ = 78;
  __shared__ float4 s_k[4][2][kQ];
  const int wi = xcd_remap(blockIdx.x, gridDim.x);
  const int item = wi / a.parts, part = wi - item * a.parts;
  const int v = item / a.T, t = item - v * a.T;
  const int ty = t / a.TX, tx = t - ty * a.TX;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int sx0 = tx * kTile + (w & 1) * kSub, sy0 = ty * kTile + (w >> 1) * kSub;
  const int px = sx0 + (lane & 7), py = sy0 + (lane >> 3);
  const float hs = 0.5f * (kSub - 1);
  constexpr float kShift = 0.5f * (kTile - kSub);  // sub-tile centre from the tile centre
  // the tile centre, and the sub-tile centre relative to it
  const float cxt = (float)(tx * kTile) + 0.5f * (kTile - 1), cyt = (float)(ty * kTile) + 0.5f * (kTile - 1);
  const float du = (float)((w & 1) * kSub) + hs - 0.5f * (kTile - 1);
  const float dv = (float)((w >> 1) * kSub) + hs - 0.5f * (kTile - 1);
  // the lane's column: x = lane & 7 of its group's copy of the sub-tile
  const int grp = lane >> 3;
  const float lx = (float)(lane & 7) - hs, lxx = lx * lx;
  uint32_t beg, end;
  list_part(min(tile_start[item], a.cap), min(tile_start[item + 1], a.cap), part, a.parts, beg,
            end);
  const Rec2 *rv = rec + (a.sets ? a.sets[v].rbase : (int64_t)v * a.M);
  const float thr = a.thr;
  float acc[kSub];
#pragma unroll
  for (int y = 0; y < kSub; ++y) acc[y] = 0.f;
  // the next batch's entries are loaded while this batch renders
  // the queues' first n records, dealt to the eight groups in turn
  // The cutoff |e| >= et as a 0/1 factor in one clamped FMA:
  // m = clamp(|e| S - et' S, 0, 1), et' the float below et and S = 2^(24 - E)
  // for et in [2^E, 2^(E+1)).  S is a power of two, so |e| S and et' S are
  // exact, and et - et' >= 2^(E - 24) puts every |e| >= et at or above 1 and
  // every |e| <= et' at or below 0: m is exactly 1 or 0, and acc + m e is the
  // same sum as with the comparison.
  auto chain_pass = [&](int n) {
    for (int r = grp; r < n; r += 8) {
      const float4 a0 = s_k[w][0][r], a1 = s_k[w][1][r];
      const float q0 = fmaf(a0.z, lxx, fmaf(a0.y, lx, a0.x));
      const float d0 = fmaf(a1.x, lx, a0.w);
      float e = copysignf(__builtin_amdgcn_exp2f(q0), a1.z);
      float rr = __builtin_amdgcn_exp2f(d0);
      const float S = fabsf(a1.z), cS = a1.w, R = a1.y;
#pragma unroll
      for (int y = 0; y < kSub; ++y) {
        const float m = __builtin_amdgcn_fmed3f(fmaf(fabsf(e), S, cS), 0.f, 1.f);
        acc[y] = fmaf(m, e, acc[y]);
        e *= rr;
        rr *= R;
      }
    }
  };
  auto pixel_pass = [&](int n) {
    for (int r = grp; r < n; r += 8) {
      const float4 a0 = s_k[w][0][kQ - 1 - r], a1 = s_k[w][1][kQ - 1 - r];
      float q = fmaf(a0.z, lxx, fmaf(a0.y, lx, a0.x));
      float d = fmaf(a1.x, lx, a0.w);
#pragma unroll
      for (int y = 0; y < kSub; ++y) {
        const float ev = (q >= a1.z) ? __builtin_amdgcn_exp2f(q) : 0.f;
        acc[y] = fmaf(a1.w, ev, acc[y]);
        q += d;
        d += a1.y;
      }
    }
  };
  int qc = 0, qe = 0;  // records waiting in the two queues (wave-uniform)
  uint32_t ex_next = beg + tid < end ? list[beg + tid].x : 0u;
  for (uint32_t base = beg; base < end; base += kBlock) {
    const int n = (int)min((uint32_t)kBlock, end - base);
    __syncthreads();
    if (tid < n) {
      // once per record: its exponent relative to the tile centre
      const uint32_t ex = ex_next;
      const float4 *p = reinterpret_cast<const float4 *>(rv + (ex & kEntryIndexMask));
      const float4 r0 = p[0], r1 = p[1];
      const float c00 = r0.z, c01 = r0.w, c11 = r1.x, rho = r1.y;
      const float lr = __log2f(fabsf(rho));
      const float U = r0.x - cxt, V = r0.y - cyt;
      const float K0 = U * (c00 * U + c01 * V) + c11 * V * V + lr;
      const float K1 = -(2.f * c00 * U + c01 * V), K2 = -(c01 * U + 2.f * c11 * V);
      // the sub-tile centres lie at (+-kShift, +-kShift) from the tile
      // centre: Pt + du K1 + dv K2 + du dv c01 is the exponent at a sub-tile
      // centre plus hs^2 (c00 + c11)
      const float Pt = fmaf(kShift * kShift + hs * hs, c00 + c11, K0);
      // the cutoff factor's scale S and offset -et' S (et = 0: no cutoff,
      // m = 1); thresholds under 2^-100 keep the per-pixel path
      const float et = __builtin_amdgcn_exp2f(thr + lr);
      const uint32_t etb = __float_as_uint(et) >> 23;  // biased exponent
      const float S = et > 0.f ? __uint_as_float((278u - etb) << 23) : 0.f;
      const float cS = et > 0.f ? -__uint_as_float(__float_as_uint(et) - 1u) * S : 1.f;
      const bool chain_ok = et == 0.f || etb >= 27u;
      s_r0[tid] = make_float4(Pt, K1, K2, c00);
      s_r1[tid] = make_float4(c01, c11, copysignf(S, rho), cS);
      s_r2[tid] = make_float2(thr + lr, chain_ok ? fmaxf(lr, 0.f) - kFwdChainRange : INFINITY);
      s_m[tid] = rho != 0.f ? (uint8_t)(ex >> kEntryMaskShift) : (uint8_t)0;
    }
    ex_next = base + kBlock + tid < end ? list[base + kBlock + tid].x : 0u;
    __syncthreads();
    // the indices of the batch's records that mark this wave's sub-tile, in
    // entry order, so that the chunks below are whole chunks of them
    int nh = 0;
    for (int c0 = 0; c0 < n; c0 += 64) {
      const int i = c0 + lane;
      const bool h = i < n && ((s_m[i] >> w) & 1u);
      const uint64_t mh = __ballot(h);
      if (h) s_h[w][nh + lanes_below(mh)] = (uint8_t)i;
      nh += __popcll(mh);
    }
    wave_lds_order();
    for (int c0 = 0; c0 < nh; c0 += 64) {
      const bool hit = c0 + lane < nh;
      const int i = hit ? (int)s_h[w][c0 + lane] : 0;
      bool chain = false;
      float4 k0, k1;
      if (hit) {
        // the exponent relative to the sub-tile centre (the tile's
        // expansion shifted by (du, dv)): on the first row
        //   A0 + A1 x + c00 x^2, stepping down a column by B0 + c01 x
        const float4 r0 = s_r0[i], r1 = s_r1[i];
        const float2 r2 = s_r2[i];
        const float c00 = r0.w, c01 = r1.x, c11 = r1.y;
        const float K1 = fmaf(2.f * c00, du, fmaf(c01, dv, r0.y));
        const float K2 = fmaf(c01, du, fmaf(2.f * c11, dv, r0.z));
        // P: the exponent at the sub-tile centre plus hs^2 (c00 + c11)
        const float P = fmaf(du, r0.y, fmaf(dv, r0.z, fmaf(du * dv, c01, r0.x)));
        const float A0 = fmaf(-hs, K2, fmaf(-hs * hs, c00, P)), A1 = fmaf(-hs, c01, K1);
        const float B0 = fmaf(c11, 1.f - 2.f * hs, K2);
        // the least exponent over the sub-tile is at a corner (+-hs, +-hs):
        // P + c +- a on one diagonal, P - c +- b on the other
        const float ea = hs * (K1 + K2), eb = hs * (K1 - K2), ec = hs * hs * c01;
        const float qmin = P + fminf(ec - fabsf(ea), -ec - fabsf(eb));
        chain = qmin >= r2.y;
        k0 = make_float4(A0, A1, c00, B0);
        k1 = chain ? make_float4(c01, __builtin_amdgcn_exp2f(2.f * c11), r1.z, r1.w)
                   : make_float4(c01, 2.f * c11, r2.x, copysignf(1.f, r1.z));
      }
      // compact: multiplicative records from the front, the others from the back
      const uint64_t mc = __ballot(hit && chain), me = __ballot(hit && !chain);
      if (hit) {
        const int pos = chain ? qc + lanes_below(mc) : kQ - 1 - (qe + lanes_below(me));
        s_k[w][0][pos] = k0;
        s_k[w][1][pos] = k1;
      }
      qc += __popcll(mc);
      qe += __popcll(me);
      wave_lds_order();
      const int fc = qc & ~7, fe = qe & ~7;  // whole passes
      chain_pass(fc);
      pixel_pass(fe);
      wave_lds_order();
      // the remainders move to the queue heads (disjoint from their sources:
      // fewer than eight records, moved only past a whole pass)
      if (fc > 0 && lane < qc - fc) {
        s_k[w][0][lane] = s_k[w][0][fc + lane];
        s_k[w][1][lane] = s_k[w][1][fc + lane];
      }
      if (fe > 0 && lane < qe - fe) {
        s_k[w][0][kQ - 1 - lane] = s_k[w][0][kQ - 1 - fe - lane];
        s_k[w][1][kQ - 1 - lane] = s_k[w][1][kQ - 1 - fe - lane];
      }
      qc -= fc;
      qe -= fe;
      wave_lds_order();
    }
  }
  // the last, part-filled passes
  chain_pass(qc);
  pixel_pass(qe);
  wave_lds_order();
  // the eight groups' sums of each pixel (lane x + 8 y), added in group order
  float *red = reinterpret_cast<float *>(&s_k[w][0][0]);  // 512 floats per wave
#pragma unroll
  for (int y = 0; y < kSub; ++y) red[grp * 64 + y * kSub + (lane & 7)] = acc[y];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  float total = 0.f;
#pragma unroll
  for (int g = 0; g < 8; ++g) total += red[g * 64 + lane];
  if (a.parts > 1)
    partial[((int64_t)part * a.V * a.T + item) * kBlock + tid] = total;
  else if (px < a.width && py < a.height)
    image[((int64_t)v * a.height + py) * a.width + px] = total;
}

// Sum of the parts of each tile's pixels, in part order.
__global__ __launch_bounds__(kBlock) void k_render_parts(ProjArgs a, const float *__restrict__ partial,
                                                         float *__restrict__ image) {
  const int item = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int v = item / a.T, t = item - v * a.T;
  const int ty = t / a.TX, tx = t - ty * a.TX;
  const int px = tx * kTile + (w & 1) * kSub + (lane & 7);
  const int py = ty * kTile + (w >> 1) * kSub + (lane >> 3);
  const int64_t stride = (int64_t)a.V * a.T * kBlock;
  const float *p = partial + (int64_t)item * kBlock + tid;
  const float acc = strided_sum(p, stride, a.parts);
  if (px < a.width && py < a.height) image[((int64_t)v * a.height + py) * a.width + px] = acc;
}

void launch_render_fwd(const ProjArgs &a, const Rec2 *rec, const uint2 *list,
                       const uint32_t *tile_start, float *image, float *partial, hipStream_t s) {
  const int n = a.V * a.T * a.parts;
  hipLaunchKernelGGL(k_render_fwd, dim3(n), dim3(kBlock), 0, s, a, rec, list, tile_start, image,
                     partial);
  if (a.parts > 1)
    hipLaunchKernelGGL(k_render_parts, dim3(a.V * a.T), dim3(kBlock), 0, s, a, partial, image);
}

// ------------------------------------------------------ render backward --

constexpr float kChainRange = 120.f;  // exp2 range of the multiplicative walk

// Eight consecutive floats of a 16-B aligned LDS row.
__device__ inline void load_row8(const float *p, float (&g)[kSub]) {
  const float4 a = reinterpret_cast<const float4 *>(p)[0], b = reinterpret_cast<const float4 *>(p)[1];
  g[0] = a.x; g[1] = a.y; g[2] = a.z; g[3] = a.w;
  g[4] = b.x; g[5] = b.y; g[6] = b.z; g[7] = b.w;
}

// Same tiling as the forward.  For the upstream gradient G of one tile and
// each (record, sub-tile) pair that the cutoff keeps, one lane walks the
// sub-tile's 64 pixels and accumulates the moments
//   S0 = sum G e, S1 = sum G e dx, S2 = sum G e dy,
//   S3 = sum G e dx^2, S4 = sum G e dx dy, S5 = sum G e dy^2
// (pixel units, e = exp2(q'), d = pixel - centre), which determine the
// gradients with respect to rho_hat, the centre and the conic.  Down each
// column the walk keeps three cascaded sums, A += e G, B += A, C += B, one
// row at a time: after the eight rows A, B and C weight row r by 1, 8 - r and
// (8 - r)(9 - r)/2, which span 1, Y and Y^2 (Y the row relative to the
// sub-tile centre), so a pixel costs one FMA and two adds.  The x moments and
// the shift to the pair's centre follow once per walk.  Wave w culls
// the batch's records against sub-tile w; the workgroup then walks the kept
// pairs of all four sub-tiles as one queue in chunks of 64, dealt to the
// waves in turn, so that lanes stay busy and load is balanced.  Lanes are
// pairs, so no cross-lane reduction is needed; each pair's moments depend on
// that pair alone, and the four sub-tiles' moments are summed in a fixed
// order and written to the entry's slot (deterministic).
__global__ __launch_bounds__(kBlock) void k_render_bwd(ProjArgs a, const Rec2 *__restrict__ rec,
                                                       const uint2 *__restrict__ list,
                                                       const uint32_t *__restrict__ tile_start,
                                                       const float *__restrict__ grad_image,
                                                       float *__restrict__ slots) {
  __shared__ float s_pu[kBlock], s_pv[kBlock], s_c00[kBlock], s_c01[kBlock], s_c11[kBlock];
  __shared__ uint8_t s_m[kBlock];
  __shared__ __align__(16) float s_G[kTile * kTile];
  __shared__ float s_acc[4][6][kBlock];
  __shared__ uint16_t s_q[4][kBlock];
  __shared__ int s_cnt[2][4];  // per sub-tile: chained pairs, per-pixel exp2 pairs
  const int wi = xcd_remap(blockIdx.x, gridDim.x);
  const int item = wi / a.parts, part = wi - item * a.parts;
  const int v = item / a.T, t = item - v * a.T;
  const int ty = t / a.TX, tx = t - ty * a.TX;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int sxl = (w & 1) * kSub, syl = (w >> 1) * kSub;  // sub-tile origin within the tile
  const int sx0 = tx * kTile + sxl, sy0 = ty * kTile + syl;
  const float rx0 = (float)sx0, rx1 = (float)(sx0 + kSub - 1);
  const float ry0 = (float)sy0, ry1 = (float)(sy0 + kSub - 1);
  {
    const int lx = tid & (kTile - 1), ly = tid / kTile;
    const int gx = tx * kTile + lx, gy = ty * kTile + ly;
    s_G[tid] = (gx < a.width && gy < a.height)
                   ? grad_image[((int64_t)v * a.height + gy) * a.width + gx]
                   : 0.f;
  }
  uint32_t beg, end;
  list_part(min(tile_start[item], a.cap), min(tile_start[item + 1], a.cap), part, a.parts, beg,
            end);
  const Rec2 *rv = rec + (int64_t)v * a.M;
  const float ethr = __builtin_amdgcn_exp2f(a.thr);  // the cutoff on e = exp2(q)
  // Software pipeline over the batches: entries are loaded two batches
  // ahead and records one batch ahead, so staging does not wait on memory.
  uint2 ent_cur = make_uint2(0u, 0u), ent_next = ent_cur;
  float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0;
  if (beg + tid < end) {
    ent_cur = list[beg + tid];
    const float4 *p = reinterpret_cast<const float4 *>(rv + (ent_cur.x & kEntryIndexMask));
    q0 = p[0];
    q1 = p[1];
  }
  if (beg + kBlock + tid < end) ent_next = list[beg + kBlock + tid];
  for (uint32_t base = beg; base < end; base += kBlock) {
    const int n = (int)min((uint32_t)kBlock, end - base);
    __syncthreads();
    uint32_t my_slot = 0;
    if (tid < n) {
      my_slot = ent_cur.y;
      s_pu[tid] = q0.x; s_pv[tid] = q0.y; s_c00[tid] = q0.z; s_c01[tid] = q0.w;
      s_c11[tid] = q1.x;
      s_m[tid] = (uint8_t)(ent_cur.x >> kEntryMaskShift);
    }
    if (base + kBlock + tid < end) {
      const float4 *p = reinterpret_cast<const float4 *>(rv + (ent_next.x & kEntryIndexMask));
      q0 = p[0];
      q1 = p[1];
    }
    ent_cur = ent_next;
    ent_next = (base + 2 * kBlock + tid < end) ? list[base + 2 * kBlock + tid] : make_uint2(0u, 0u);
    __syncthreads();
    // Compact the records whose entry mask marks this wave's sub-tile (the
    // cutoff ellipse meets it; set by the scatter) into two queues.
    // Entries whose form stays below kChainRange over the whole sub-tile
    // (its maximum is at a corner) go to the front: their walk steps
    // e = exp2(q) by multiplication, along a row by r = exp2(q(x+1) - q(x)),
    // r itself by exp2(2 c00), and down the first column likewise, so every
    // chained value and factor is a normal FP32 number and six exp2 per walk
    // replace 64.  The others go to the back and evaluate exp2(q) per pixel
    // with q forward-differenced.  Each entry's path is its own, so its
    // moments do not depend on which entries share its wave.
    int qn = 0, qs = 0;
    for (int c0 = 0; c0 < n; c0 += 64) {
      const int i = c0 + lane;
      bool hit = false, steep = false;
      if (i < n && ((s_m[i] >> w) & 1u)) {
        const float pu = s_pu[i], pv = s_pv[i];
        const float fa = -s_c00[i], fb = -s_c01[i], fc = -s_c11[i];
        const float x0 = rx0 - pu, x1 = rx1 - pu, y0 = ry0 - pv, y1 = ry1 - pv;
        hit = true;
        const float ax0 = fa * x0 * x0, ax1 = fa * x1 * x1, cy0 = fc * y0 * y0, cy1 = fc * y1 * y1;
        const float fmax = fmaxf(fmaxf(fmaf(fb * x0, y0, ax0 + cy0), fmaf(fb * x1, y0, ax1 + cy0)),
                                 fmaxf(fmaf(fb * x0, y1, ax0 + cy1), fmaf(fb * x1, y1, ax1 + cy1)));
        steep = !(fmax <= kChainRange);
      }
      const uint64_t mc = __ballot(hit && !steep), ms = __ballot(hit && steep);
      if (hit && !steep) s_q[w][qn + lanes_below(mc)] = (uint16_t)i;
      if (hit && steep) s_q[w][kBlock - 1 - (qs + lanes_below(ms))] = (uint16_t)i;
      qn += __popcll(mc);
      qs += __popcll(ms);
    }
    if (lane == 0) {
      s_cnt[0][w] = qn;
      s_cnt[1][w] = qs;
    }
    __syncthreads();
    // The workgroup's queue: the chained pairs of sub-tiles 0..3, then their
    // per-pixel pairs, in chunks of 64 (a chunk holds pairs of one kind).
    const int kc = (s_cnt[0][0] + s_cnt[0][1] + s_cnt[0][2] + s_cnt[0][3] + 63) >> 6;
    const int kall = kc + ((s_cnt[1][0] + s_cnt[1][1] + s_cnt[1][2] + s_cnt[1][3] + 63) >> 6);
    for (int k = w; k < kall; k += 4) {
      {
        const bool chain = k < kc;
        const int kind = chain ? 0 : 1;
        const int b1 = s_cnt[kind][0], b2 = b1 + s_cnt[kind][1], b3 = b2 + s_cnt[kind][2];
        const int btot = b3 + s_cnt[kind][3];
        int pidx = (chain ? k : k - kc) * 64 + lane;
        const bool active = pidx < btot;
        const int sw = (pidx >= b1) + (pidx >= b2) + (pidx >= b3);
        pidx -= sw == 0 ? 0 : sw == 1 ? b1 : sw == 2 ? b2 : b3;
        const int e = active ? (int)s_q[sw][chain ? pidx : kBlock - 1 - pidx] : 0;
        const int pxl = (sw & 1) * kSub, pyl = (sw >> 1) * kSub;  // the pair's sub-tile
        const float ox = (float)(tx * kTile + pxl), oy = (float)(ty * kTile + pyl);
        const int goff = pyl * kTile + pxl;
        const float pu = s_pu[e], pv = s_pv[e];
        const float c00 = s_c00[e], c01 = s_c01[e], c11 = s_c11[e];
        const float dx0 = ox - pu, dy0 = oy - pv;
        // per column, the cascaded sums over the rows of e G
        float A[kSub], B[kSub], C[kSub];
        if (chain) {
          float e_row = __builtin_amdgcn_exp2f(dx0 * (c00 * dx0 + c01 * dy0) + c11 * dy0 * dy0);
          float rx_row = __builtin_amdgcn_exp2f(c00 * (2.f * dx0 + 1.f) + c01 * dy0);
          float hr = __builtin_amdgcn_exp2f(c01 * dx0 + c11 * (2.f * dy0 + 1.f));
          const float rxx = __builtin_amdgcn_exp2f(2.f * c00);
          const float rxy = __builtin_amdgcn_exp2f(c01);
          const float ryy = __builtin_amdgcn_exp2f(2.f * c11);
          // rows 0 and 1 start the cascade without zeroed sums: after row 0,
          // A = B = C = e G; row 1 forms B and C from that
          {
            float g[kSub];
            load_row8(s_G + goff, g);
            float ev = e_row, rx = rx_row;
#pragma unroll
            for (int col = 0; col < kSub; ++col) {
              A[col] = ((ev >= ethr) ? ev : 0.f) * g[col];
              ev *= rx;
              rx *= rxx;
            }
            e_row *= hr;
            hr *= ryy;
            rx_row *= rxy;
          }
          {
            float g[kSub];
            load_row8(s_G + goff + kTile, g);
            float ev = e_row, rx = rx_row;
#pragma unroll
            for (int col = 0; col < kSub; ++col) {
              const float a = fmaf((ev >= ethr) ? ev : 0.f, g[col], A[col]);
              B[col] = A[col] + a;
              C[col] = A[col] + B[col];
              A[col] = a;
              ev *= rx;
              rx *= rxx;
            }
            e_row *= hr;
            hr *= ryy;
            rx_row *= rxy;
          }
#pragma unroll 2
          for (int r = 2; r < kSub; ++r) {
            float g[kSub];
            load_row8(s_G + goff + r * kTile, g);
            float ev = e_row, rx = rx_row;
#pragma unroll
            for (int col = 0; col < kSub; ++col) {
              const float se = (ev >= ethr) ? ev : 0.f;
              A[col] = fmaf(se, g[col], A[col]);
              B[col] += A[col];
              C[col] += B[col];
              ev *= rx;
              rx *= rxx;
            }
            e_row *= hr;
            hr *= ryy;
            rx_row *= rxy;
          }
        } else {
#pragma unroll
          for (int col = 0; col < kSub; ++col) A[col] = B[col] = C[col] = 0.f;
          const float dd = 2.f * c00;
          const float thr = a.thr;
#pragma unroll 2
          for (int r = 0; r < kSub; ++r) {
            const float dy = oy + (float)r - pv;
            float q = dx0 * (c00 * dx0 + c01 * dy) + c11 * dy * dy;
            float d = c00 * (2.f * dx0 + 1.f) + c01 * dy;
            float g[kSub];
            load_row8(s_G + goff + r * kTile, g);
#pragma unroll
            for (int col = 0; col < kSub; ++col) {
              const float se = (q >= thr) ? __builtin_amdgcn_exp2f(q) : 0.f;
              A[col] = fmaf(se, g[col], A[col]);
              B[col] += A[col];
              C[col] += B[col];
              q += d;
              d += dd;
            }
          }
        }
        // Sums over the columns with weights 1, X, X^2 (X = column - 3.5):
        // with u = 8 - r = 4.5 - Y, B sums e G u and 2 C - B sums e G u^2, so
        // sum e G Y = 4.5 A - B and sum e G Y^2 = 20.25 A - 10 B + 2 C.
        float sA = 0.f, sXA = 0.f, sXXA = 0.f, sB = 0.f, sXB = 0.f, sC = 0.f;
#pragma unroll
        for (int col = 0; col < kSub; ++col) {
          const float X = (float)col - 0.5f * (kSub - 1);
          sA += A[col];
          sXA = fmaf(X, A[col], sXA);
          sXXA = fmaf(X * X, A[col], sXXA);
          sB += B[col];
          sXB = fmaf(X, B[col], sXB);
          sC += C[col];
        }
        // moments about the sub-tile centre (L_ij: weight X^i Y^j) ...
        const float L00 = sA, L10 = sXA, L20 = sXXA;
        const float L01 = fmaf(4.5f, sA, -sB);
        const float L11 = fmaf(4.5f, sXA, -sXB);
        const float L02 = fmaf(20.25f, sA, fmaf(-10.f, sB, 2.f * sC));
        // ... shifted to the pair's centre: dx = xc + X, dy = yc + Y
        const float xc = dx0 + 0.5f * (kSub - 1), yc = dy0 + 0.5f * (kSub - 1);
        const float S0 = L00;
        const float S1 = fmaf(xc, L00, L10);
        const float S2 = fmaf(yc, L00, L01);
        const float S3 = fmaf(xc, L10 + S1, L20);
        const float S4 = fmaf(yc, S1, fmaf(xc, L01, L11));
        const float S5 = fmaf(yc, L01 + S2, L02);
        if (active) {
          s_acc[sw][0][e] = S0; s_acc[sw][1][e] = S1; s_acc[sw][2][e] = S2;
          s_acc[sw][3][e] = S3; s_acc[sw][4][e] = S4; s_acc[sw][5][e] = S5;
        }
      }
    }
    __syncthreads();
    if (tid < n && my_slot < a.cap) {
      // every sub-tile the entry's mask marks was walked and wrote its
      // moments; the others count as zero (their accumulators hold older
      // batches' values, cleared here bit by bit, without a branch)
      const uint32_t mk = s_m[tid];
      const int z0 = -(int)(mk & 1u), z1 = -(int)((mk >> 1) & 1u), z2 = -(int)((mk >> 2) & 1u),
                z3 = -(int)((mk >> 3) & 1u);
      float *o = slots + (int64_t)my_slot * 6;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const float a0 = __int_as_float(__float_as_int(s_acc[0][k][tid]) & z0);
        const float a1 = __int_as_float(__float_as_int(s_acc[1][k][tid]) & z1);
        const float a2 = __int_as_float(__float_as_int(s_acc[2][k][tid]) & z2);
        const float a3 = __int_as_float(__float_as_int(s_acc[3][k][tid]) & z3);
        o[k] = ((a0 + a1) + a2) + a3;
      }
    }
  }
}

void launch_render_bwd(const ProjArgs &a, const Rec2 *rec, const uint2 *list,
                       const uint32_t *tile_start, const float *grad_image, float *slots,
                       hipStream_t s) {
  const int n = a.V * a.T * a.parts;
  hipLaunchKernelGGL(k_render_bwd, dim3(n), dim3(kBlock), 0, s, a, rec, list, tile_start,
                     grad_image, slots);
}

// ------------------------------------------------- per-Gaussian chain rule --

// Per (Gaussian, chunk of views), views in order (deterministic): sums the
// moments of its tile slots, converts them to the gradients of rho_hat, the
// projected centre and the conic, and applies the chain rule through the
// inverse, Sigma_hat = B B^T with B = J W R S, the rectification factor
// mu = sqrt(2 pi / (d^T Sigma^{-1} d)), the perspective Jacobian J(t), the
// perspective division and t = W p + t0.  Writes the chunk's partial
// gradients with respect to p, s, R and rho (16 values, component-major);
// k_proj_chain_reduce sums the chunks in order and finishes the quaternion.
constexpr int kChainViews = 16;
constexpr int kChainParts = 16;  // gradient parts; +2 with statistics (NDC norm sum, views)

// A wave's 64 consecutive Gaussians own one contiguous run of slots per view
// (offsets follow Gaussian order), so the wave stages that run in LDS with
// 16-byte loads, in rounds of up to 8 KB, and each lane sums its own slots
// from LDS.  The slot buffer carries 16 bytes of padding for the rounded-up
// last load.
constexpr int kChainStage = 512;         // float4 per wave (8 KB)
constexpr uint32_t kChainRound = 340u;   // slots per staging round
constexpr int kChainLoads = kChainStage / 64;  // 16-byte loads per lane and round
typedef float f32x4 __attribute__((ext_vector_type(4)));

// A round's float4 i = I * 64 + lane into register I (indices fixed at
// compile time, so the array stays in registers).  Lanes past the round
// reload its last float4: with a branch around each load the compiler waits
// for every load before issuing the next, and the round then costs up to
// eight memory latencies instead of one.
template <int... I>
__device__ __forceinline__ void chain_round_load(f32x4 (&r)[kChainLoads], const float4 *src,
                                                 int lane, int n4, std::integer_sequence<int, I...>) {
  const f32x4 *s = reinterpret_cast<const f32x4 *>(src);
  ((r[I] = s[min(I * 64 + lane, n4 - 1)]), ...);
}
// ... and all of them to the wave's staging buffer of kChainStage float4
// (the copies past the round land where the round's sums never read).
template <int... I>
__device__ __forceinline__ void chain_round_stage(const f32x4 (&r)[kChainLoads], float4 *dst,
                                                  int lane, std::integer_sequence<int, I...>) {
  f32x4 *d = reinterpret_cast<f32x4 *>(dst);
  ((d[I * 64 + lane] = r[I]), ...);
}

__global__ __launch_bounds__(kBlock) void k_proj_chain(ProjArgs a,
                                                       const uint32_t *__restrict__ offsets,
                                                       const float *__restrict__ slots,
                                                       float *__restrict__ part, int stats) {
  __shared__ float4 s_st[4][kChainStage];
  if (*a.totals > a.cap) return;  // the call overflowed its reservation: slots are incomplete
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = g < a.M;
  const int vc = blockIdx.y;
  const int n_parts = kChainParts + (stats ? 2 : 0);
  float ndc_sum = 0.f, n_vis = 0.f;
  Gauss G;
  G.ok = false;
  if (active) load_gauss(a.mean, a.scale, a.quat, a.dens, g, G);
  float gp[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, gR[9] = {0.f};
  float grho = 0.f;
  const int v0 = vc * kChainViews, v1 = min(v0 + kChainViews, a.V);
  const float4 *slots4 = reinterpret_cast<const float4 *>(slots);
  {
    // The slots of (view, Gaussian) vg are [offsets[vg], offsets[vg + 1]):
    // slots are numbered in (view, Gaussian) order and the array ends with the
    // total.  The next view's pair of offsets is loaded one view ahead.
    uint2 off_next = make_uint2(0u, 0u);
    if (G.ok && v0 < v1) {
      const int64_t vg = (int64_t)v0 * a.M + g;
      off_next = make_uint2(offsets[vg], offsets[vg + 1]);
    }
    for (int v = v0; v < v1; ++v) {
      int cnt = 0;
      uint32_t off = 0;
      if (G.ok) {
        off = off_next.x;
        cnt = (int)(off_next.y - off_next.x);
        if ((uint64_t)off + (uint64_t)cnt > a.cap) cnt = 0;  // (beyond capacity: dropped)
        if (v + 1 < v1) {
          const int64_t vg = (int64_t)(v + 1) * a.M + g;
          off_next = make_uint2(offsets[vg], offsets[vg + 1]);
        }
      }
      const uint64_t have = __ballot(cnt > 0);
      if (!have) continue;
      const int fl = __builtin_ctzll(have), ll = 63 - __builtin_clzll(have);
      const uint32_t lo = (uint32_t)__shfl((int)off, fl);
      const uint32_t hi = (uint32_t)__shfl((int)(off + (uint32_t)cnt), ll);
      // the run in rounds of kChainRound slots (at most 511 float4 with the
      // alignment slack); each lane sums, in slot order, its slots in the round
      float S[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      for (uint64_t clo = lo; clo < hi; clo += kChainRound) {  // 64-bit: no wrap near 2^32
        const uint64_t chi = min((uint64_t)hi, clo + kChainRound);
        const uint64_t b4 = (clo * 6u) >> 2, e4 = (chi * 6u + 3u) >> 2;
        const int n4 = (int)(e4 - b4);
        {
          f32x4 r[kChainLoads];
          chain_round_load(r, slots4 + b4, lane, n4, std::make_integer_sequence<int, kChainLoads>{});
          chain_round_stage(r, s_st[w], lane, std::make_integer_sequence<int, kChainLoads>{});
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint64_t k0 = max((uint64_t)off, clo), k1 = min((uint64_t)off + (uint64_t)cnt, chi);
        if (cnt && k0 < k1) {
          const float *sl = reinterpret_cast<const float *>(s_st[w]) + (k0 * 6u - b4 * 4u);
          for (int k = 0; k < (int)(k1 - k0); ++k)
#pragma unroll
            for (int j = 0; j < 6; ++j) S[j] += sl[6 * k + j];
        }
        __builtin_amdgcn_wave_barrier();  // the next round restages
      }
      if (!cnt) continue;
      const DevView V = a.views[v];
      Proj2 P;
      project_one(G, V, P);
      const float mu = a.rectify ? P.mu : 1.f;
      const float rh = mu * G.rho;
      // world-unit moments
      const float T1 = S[1] * V.hu, T2 = S[2] * V.hv;
      const float T3 = S[3] * V.hu * V.hu, T4 = S[4] * V.hu * V.hv, T5 = S[5] * V.hv * V.hv;
      const float g_rh = S[0];
      const float gph0 = rh * (P.A00 * T1 + P.A01 * T2);
      const float gph1 = rh * (P.A01 * T1 + P.A11 * T2);
      if (stats) {  // |dL/dp_hat| in normalised device coordinates (half-width = 1)
        const float nu = gph0 * V.hu * (0.5f * a.width), nv = gph1 * V.hv * (0.5f * a.height);
        ndc_sum += sqrtf(nu * nu + nv * nv);
        n_vis += 1.f;
      }
      // dL/dA as a symmetric matrix (each entry), then dL/dSigma_hat = -A Gb A
      const float Gb00 = -0.5f * rh * T3, Gb01 = -0.5f * rh * T4, Gb11 = -0.5f * rh * T5;
      const float X00 = P.A00 * Gb00 + P.A01 * Gb01, X01 = P.A00 * Gb01 + P.A01 * Gb11;
      const float X10 = P.A01 * Gb00 + P.A11 * Gb01, X11 = P.A01 * Gb01 + P.A11 * Gb11;
      const float gS00 = -(X00 * P.A00 + X01 * P.A01);
      const float gS01 = -0.5f * ((X00 * P.A01 + X01 * P.A11) + (X10 * P.A00 + X11 * P.A01));
      const float gS11 = -(X10 * P.A01 + X11 * P.A11);
      // Sigma_hat = B B^T
      float gB[6];
      for (int j = 0; j < 3; ++j) {
        gB[j] = 2.f * (gS00 * P.B[j] + gS01 * P.B[3 + j]);
        gB[3 + j] = 2.f * (gS01 * P.B[j] + gS11 * P.B[3 + j]);
      }
      // B = JW M
      float gJW[6];
      for (int aa = 0; aa < 2; ++aa)
        for (int i = 0; i < 3; ++i)
          gJW[3 * aa + i] = gB[3 * aa] * P.M[3 * i] + gB[3 * aa + 1] * P.M[3 * i + 1] +
                            gB[3 * aa + 2] * P.M[3 * i + 2];
      // dL/dR = dL/dM S.  The part of S^2 common to the three axes leaves
      // Sigma = R S^2 R^T unchanged under rotation, so it adds exactly zero
      // to dL/dq (R^T dR/dq is antisymmetric, dL/dSigma symmetric): it is
      // left out here, so that a nearly isotropic Gaussian's small rotation
      // gradient is not the FP32 remainder of a large cancelling sum.  With
      // dL/dM_ij = 2 (Y R S)_ij, dL/dM_ij (s_j - sbar^2 / s_j) = 2 (Y R (S^2 - sbar^2))_ij.
      const float sb2 = (G.s[0] * G.s[0] + G.s[1] * G.s[1] + G.s[2] * G.s[2]) * (1.f / 3.f);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const float gM = P.JW[i] * gB[j] + P.JW[3 + i] * gB[3 + j];
          gR[3 * i + j] += gM * (G.s[j] - sb2 * frcp(G.s[j]));
          gs[j] += gM * G.R[3 * i + j];
        }
      // rho_hat = mu rho,  mu = sqrt(2 pi / m),  m = sum_j (r_j / s_j)^2,  r = R^T d
      grho += mu * g_rh;
      // the rectification factor's own dependence on p, s, q (none when unrectified)
      const float gmu = a.rectify ? G.rho * g_rh : 0.f;
      const float gm = gmu * (-0.5f * P.mu / P.m);
      // m = d^T R S^-2 R^T d: as above, the part of S^-2 common to the
      // three axes adds nothing to dL/dq and is left out of dL/dR
      float gd[3] = {0.f, 0.f, 0.f};
      float is1[3], is2[3];
      for (int j = 0; j < 3; ++j) {
        is1[j] = frcp(G.s[j]);
        is2[j] = is1[j] * is1[j];
      }
      const float ib2 = (is2[0] + is2[1] + is2[2]) * (1.f / 3.f);
      for (int j = 0; j < 3; ++j) {
        const float gr = gm * 2.f * P.r[j] * is2[j];
        const float grR = gm * 2.f * P.r[j] * (is2[j] - ib2);
        gs[j] += gm * (-2.f * P.r[j] * P.r[j] * is2[j] * is1[j]);
        for (int i = 0; i < 3; ++i) {
          gR[3 * i + j] += P.d[i] * grR;
          gd[i] += G.R[3 * i + j] * gr;
        }
      }
      float gt[3] = {0.f, 0.f, 0.f};
      const float *W = V.W;
      if (V.beam == 1) {
        // d = W^T u, u = t / |t|
        float gu[3];
        for (int aa = 0; aa < 3; ++aa)
          gu[aa] = W[3 * aa] * gd[0] + W[3 * aa + 1] * gd[1] + W[3 * aa + 2] * gd[2];
        const float ug = P.u[0] * gu[0] + P.u[1] * gu[1] + P.u[2] * gu[2];
        const float il = frcp(P.l);
        for (int aa = 0; aa < 3; ++aa) gt[aa] += (gu[aa] - P.u[aa] * ug) * il;
        // JW = J2 W
        float gJ[6];
        for (int aa = 0; aa < 2; ++aa)
          for (int k = 0; k < 3; ++k)
            gJ[3 * aa + k] = gJW[3 * aa] * W[3 * k] + gJW[3 * aa + 1] * W[3 * k + 1] +
                             gJW[3 * aa + 2] * W[3 * k + 2];
        const float L = V.L_SD, t0 = P.t[0], t1 = P.t[1], inv = frcp(P.t[2]);
        const float Li2 = L * inv * inv;
        gt[0] += -gJ[2] * Li2;
        gt[1] += -gJ[5] * Li2;
        gt[2] += -(gJ[0] + gJ[4]) * Li2 + (gJ[2] * t0 + gJ[5] * t1) * 2.f * Li2 * inv;
        // p_hat = L (t0, t1) / t2
        gt[0] += L * inv * gph0;
        gt[1] += L * inv * gph1;
        gt[2] += -Li2 * (t0 * gph0 + t1 * gph1);
      } else {
        gt[0] += gph0;
        gt[1] += gph1;
      }
      for (int i = 0; i < 3; ++i) gp[i] += W[i] * gt[0] + W[3 + i] * gt[1] + W[6 + i] * gt[2];
    }
  }
  if (!active) return;
  float *o = part + (int64_t)vc * n_parts * a.M + g;
  for (int i = 0; i < 3; ++i) o[(int64_t)i * a.M] = gp[i];
  for (int i = 0; i < 3; ++i) o[(int64_t)(3 + i) * a.M] = gs[i];
  for (int i = 0; i < 9; ++i) o[(int64_t)(6 + i) * a.M] = gR[i];
  o[(int64_t)15 * a.M] = grho;
  if (stats) {
    o[(int64_t)16 * a.M] = ndc_sum;
    o[(int64_t)17 * a.M] = n_vis;
  }
}

__global__ __launch_bounds__(kBlock) void k_proj_chain_reduce(ProjArgs a, int n_chunks,
                                                              const float *__restrict__ part,
                                                              float *g_mean, float *g_scale,
                                                              float *g_quat, float *g_dens,
                                                              int accumulate, ChainStats st) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= a.M || *a.totals > a.cap) return;
  const int stats = st.ndc_sum != nullptr;
  const int n_parts = kChainParts + (stats ? 2 : 0);
  float sum[kChainParts + 2];
  for (int k = 0; k < kChainParts + 2; ++k) sum[k] = 0.f;
  for (int c = 0; c < n_chunks; ++c) {
    const float *o = part + (int64_t)c * n_parts * a.M + g;
    for (int k = 0; k < kChainParts; ++k) sum[k] += o[(int64_t)k * a.M];
    if (stats) {
      sum[16] += o[(int64_t)16 * a.M];
      sum[17] += o[(int64_t)17 * a.M];
    }
  }
  if (stats) {
    st.ndc_sum[g] += st.scale * sum[16];
    st.visible[g] += (int)sum[17];
  }
  Gauss G;
  load_gauss(a.mean, a.scale, a.quat, a.dens, g, G);
  float gq[4] = {0.f, 0.f, 0.f, 0.f};
  if (G.ok) quat_backward(G, sum + 6, gq);
  if (g_mean)
    for (int i = 0; i < 3; ++i) g_mean[3 * g + i] = accumulate ? g_mean[3 * g + i] + sum[i] : sum[i];
  if (g_scale)
    for (int i = 0; i < 3; ++i)
      g_scale[3 * g + i] = accumulate ? g_scale[3 * g + i] + sum[3 + i] : sum[3 + i];
  if (g_quat)
    for (int i = 0; i < 4; ++i) g_quat[4 * g + i] = accumulate ? g_quat[4 * g + i] + gq[i] : gq[i];
  if (g_dens) g_dens[g] = accumulate ? g_dens[g] + sum[15] : sum[15];
}

int proj_chain_chunks(int n_views) { return (n_views + kChainViews - 1) / kChainViews; }

void launch_proj_chain(const ProjArgs &a, const uint32_t *offsets,
                       const float *slots, float *part, float *g_mean, float *g_scale,
                       float *g_quat, float *g_dens, int accumulate, const ChainStats &st,
                       hipStream_t s) {
  unsigned nb = (unsigned)((a.M + kBlock - 1) / kBlock);
  const int nc = proj_chain_chunks(a.V);
  const int stats = st.ndc_sum != nullptr;
  hipLaunchKernelGGL(k_proj_chain, dim3(nb, nc), dim3(kBlock), 0, s, a, offsets, slots, part, stats);
  hipLaunchKernelGGL(k_proj_chain_reduce, dim3(nb), dim3(kBlock), 0, s, a, nc, part, g_mean,
                     g_scale, g_quat, g_dens, accumulate, st);
}

}  // namespace gsk
