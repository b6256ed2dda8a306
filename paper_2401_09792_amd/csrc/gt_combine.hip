// Channel matrices at general coefficient vectors: mode 3 of the channel tensor holds P path /
// delay submatrices, and the channel at time or frequency point t is their combination by the
// row u_t = c*(t) (Section 2.2, equation "channel submatrices, tensor"):
//   full        H(t)  = X x3 u_t = sum_s u_t[s] H_s                         [nr x nt]
//   compressed  Ht(t) = G x3 (u_t C) = sum_g sum_q w_g,q(t) G_g[q],
//               w_g,q(t) = sum_{s in g} u_t[s] C[s,q]                       [m x n]
// (Section 3.3, equation "compressed matrix SINR reduction"; with the groupwise model every
// group contributes its own core combined by its own rows of C).  The selector u_t = e_s gives
// the slice H_s and the per-subcarrier Ht_s of gt_tucker_reconstruct.
//
// Layouts per channel c (complex, row-major): U [n_pts][nsc] at n_pts * offsets.sc; H
// [n_pts][nr][nt] at n_pts * (sum of nr nt over the channels before c); Ht [n_pts][m][n] at
// n_pts * (sum of m n over the channels before c).
#include <hip/hip_runtime.h>

#include "gt_device.h"
#include "gt_internal.h"

namespace gt {

__device__ __forceinline__ void cfma2(float2& acc, float2 a, float2 b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
}

// Compressed combination, a product per channel Ht (n_pts x m n) = W (n_pts x groups p) times
// the stacked cores (groups p x m n), with W's columns of group g, w_g(t) = u_t,g C_g, formed
// per group in LDS: block tile 32 points x 64 entries; per group the block stages its 32 rows
// of U on the group (up to 32 submatrices) and C_g, forms the 32 x p_g weights (a dot product
// over the group per weight), stages G_g's p_g x 64 tile and accumulates.  Thread (ty, tx)
// owns points ty, ty + 16 and entries tx + 16 j.
__global__ void __launch_bounds__(256) k_combine_core(const DevChan* __restrict__ chans, int n_pts,
                                                      const float2* __restrict__ C,
                                                      const float2* __restrict__ G,
                                                      const float2* __restrict__ U,
                                                      float2* __restrict__ Ht) {
  const DevChan& ch = chans[blockIdx.z];
  const int mn = ch.m * ch.n, p = ch.p, nsc = ch.nsc;
  const int e0 = blockIdx.x * 64, t0 = blockIdx.y * 32;
  if (e0 >= mn || t0 >= n_pts) return;
  __shared__ float2 us[32][kMaxGroup + 1];
  __shared__ float2 cs[kMaxGroup][kMaxGroup + 1];
  __shared__ float2 ws[32][kMaxGroup + 1];
  __shared__ float2 gs_[kMaxGroup][64];
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  const float2* Uc = U + (int64_t)ch.sc * n_pts;
  float2 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_float2(0.f, 0.f);
  for (int g = 0; g < ch.ngroups; ++g) {
    const int s0 = g * ch.gs, sz = min(ch.gs, nsc - s0), pg = min(p, sz);
    for (int idx = tid; idx < 32 * sz; idx += 256) {
      const int r = idx / sz, k = idx - r * sz;
      us[r][k] = t0 + r < n_pts ? Uc[(int64_t)(t0 + r) * nsc + s0 + k] : make_float2(0.f, 0.f);
    }
    for (int idx = tid; idx < sz * pg; idx += 256) {
      const int k = idx / pg, q = idx - k * pg;
      cs[k][q] = C[ch.c + (int64_t)(s0 + k) * p + q];
    }
    const float2* Gg = G + ch.g + (int64_t)g * p * mn;
    for (int idx = tid; idx < pg * 64; idx += 256) {
      const int q = idx / 64, c = idx % 64;
      gs_[q][c] = e0 + c < mn ? Gg[(int64_t)q * mn + e0 + c] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int idx = tid; idx < 32 * pg; idx += 256) {
      const int r = idx / pg, q = idx - r * pg;
      float2 v = make_float2(0.f, 0.f);
      for (int k = 0; k < sz; ++k) cfma2(v, us[r][k], cs[k][q]);
      ws[r][q] = v;
    }
    __syncthreads();
    for (int q = 0; q < pg; ++q) {
      const float2 w0 = ws[ty][q], w1 = ws[ty + 16][q];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float2 gv = gs_[q][tx + 16 * j];
        cfma2(acc[0][j], w0, gv);
        cfma2(acc[1][j], w1, gv);
      }
    }
    __syncthreads();
  }
  float2* out = Ht + ch.mn_off * n_pts;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int t = t0 + ty + 16 * i;
    if (t < n_pts)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int e = e0 + tx + 16 * j;
        if (e < mn) out[(int64_t)t * mn + e] = acc[i][j];
      }
  }
}

// Full combination, a complex product per channel: H (n_pts x nr nt) = U (n_pts x nsc) times
// X (nsc x nr nt).  Block tile 32 points x 64 entries, K chunks of 16 slices staged in LDS;
// thread (ty, tx) owns points ty, ty + 16 and entries tx + 16 j.
__global__ void __launch_bounds__(256) k_combine_full(const DevChan* __restrict__ chans, int n_pts,
                                                      const float2* __restrict__ X,
                                                      const float2* __restrict__ U,
                                                      float2* __restrict__ H) {
  const DevChan& ch = chans[blockIdx.z];
  const int ne = ch.nr * ch.nt, nsc = ch.nsc;
  const int e0 = blockIdx.x * 64, t0 = blockIdx.y * 32;
  if (e0 >= ne || t0 >= n_pts) return;
  __shared__ float2 us[32][17];
  __shared__ float2 xs[16][64];
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  const float2* Uc = U + (int64_t)ch.sc * n_pts;
  const float2* Xc = X + ch.x;
  float2 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_float2(0.f, 0.f);
  for (int k0 = 0; k0 < nsc; k0 += 16) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int idx = tid + 256 * j, r = idx / 16, k = idx % 16;
      us[r][k] = (t0 + r < n_pts && k0 + k < nsc) ? Uc[(int64_t)(t0 + r) * nsc + k0 + k]
                                                   : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int idx = tid + 256 * j, k = idx / 64, c = idx % 64;
      xs[k][c] = (k0 + k < nsc && e0 + c < ne) ? Xc[(int64_t)(k0 + k) * ne + e0 + c]
                                                : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const float2 u0 = us[ty][k], u1 = us[ty + 16][k];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float2 xv = xs[k][tx + 16 * j];
        cfma2(acc[0][j], u0, xv);
        cfma2(acc[1][j], u1, xv);
      }
    }
    __syncthreads();
  }
  float2* out = H + ch.rt_off * n_pts;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int t = t0 + ty + 16 * i;
    if (t < n_pts)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int e = e0 + tx + 16 * j;
        if (e < ne) out[(int64_t)t * ne + e] = acc[i][j];
      }
  }
}

#define GT_LAUNCH(name, grid, block, ...)                            \
  do {                                                               \
    prof_begin(#name, L.stream);                                     \
    hipLaunchKernelGGL(name, grid, block, 0, L.stream, __VA_ARGS__); \
    prof_end(L.stream);                                              \
    hipError_t e_ = hipGetLastError();                               \
    if (e_ != hipSuccess) {                                          \
      set_error_detail(#name, e_);                                   \
      return GT_ERR_HIP;                                             \
    }                                                                \
  } while (0)

gt_status launch_combine_core(const LaunchCtx& L, int n_pts, const float2* C, const float2* G,
                              const float2* U, float2* Ht) {
  const unsigned ex = (unsigned)((L.max_m * L.max_n + 63) / 64), ty = (unsigned)((n_pts + 31) / 32);
  GT_LAUNCH(k_combine_core, dim3(ex, ty, L.n_channels), dim3(256), L.d_chans, n_pts, C, G, U, Ht);
  return GT_OK;
}

gt_status launch_combine_full(const LaunchCtx& L, int n_pts, const float2* X, const float2* U,
                              float2* H) {
  const unsigned ex = (unsigned)((L.max_nr * L.max_nt + 63) / 64), ty = (unsigned)((n_pts + 31) / 32);
  GT_LAUNCH(k_combine_full, dim3(ex, ty, L.n_channels), dim3(256), L.d_chans, n_pts, X, U, H);
  return GT_OK;
}

}  // namespace gt
