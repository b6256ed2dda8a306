// Reconstruction from the compressed form and its adjoint.
//   Ht_s   = sum_q C[s,q] G_g[q]            (equation "compressed matrix SINR reduction")
//   Xhat_s = A Ht_s B^H                     (equation "three matrix factorization")
// Adjoint for upstream gradients dHt_s, dXhat_s (dl/dRe + i dl/dIm):
//   dHt_s(total) = dHt_s + A^H dXhat_s B
//   dA = sum_s dXhat_s B Ht_s^H,  dB = sum_s dXhat_s^H A Ht_s
//   dG_g[q] = sum_{s in g} conj(C[s,q]) dHt_s(total),  dC[s,q] = <dHt_s(total), G_g[q]>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gt_device.h"
#include "gt_internal.h"

namespace gt {

constexpr int kRecMaxNt = 256;
constexpr int kRecMaxMN = kMaxNr * 64;  // m * n staged per subcarrier

__device__ __forceinline__ void find_sub(const DevChan* chans, int n_channels, int64_t gsc,
                                         int& c) {
  int lo = 0, hi = n_channels - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (chans[mid].sc <= gsc)
      lo = mid;
    else
      hi = mid - 1;
  }
  c = lo;
}

// Ht_s into LDS (m x n), from C and G.
__device__ void stage_ht(const DevChan& ch, int64_t s, const float2* __restrict__ C,
                         const float2* __restrict__ G, float2* sh) {
  const int g = (int)(s / ch.gs);
  const int pg = min(ch.p, min(ch.gs, ch.nsc - g * ch.gs));
  const int mn = ch.m * ch.n;
  const float2* Cs = C + ch.c + s * ch.p;
  const float2* Gg = G + ch.g + (int64_t)g * ch.p * mn;
  for (int e = threadIdx.x; e < mn; e += blockDim.x) {
    Cx<float> acc{0.f, 0.f};
    for (int q = 0; q < pg; ++q) cfma(acc, ld(Cs + q), ld(Gg + (int64_t)q * mn + e));
    sh[e] = make_float2(acc.re, acc.im);
  }
}

// one block per subcarrier
__global__ void __launch_bounds__(256) k_reconstruct(const DevChan* __restrict__ chans, int n_channels,
                                                     const float2* __restrict__ A,
                                                     const float2* __restrict__ B,
                                                     const float2* __restrict__ C,
                                                     const float2* __restrict__ G, float2* Ht,
                                                     float2* Xhat) {
  __shared__ float2 sh[kRecMaxMN];
  __shared__ float2 ah[kMaxNr * 64];
  const int64_t gsc = blockIdx.x;
  int c;
  find_sub(chans, n_channels, gsc, c);
  const DevChan& ch = chans[c];
  const int64_t s = gsc - ch.sc;
  const int m = ch.m, n = ch.n, nr = ch.nr, nt = ch.nt;
  stage_ht(ch, s, C, G, sh);
  __syncthreads();
  if (Ht)
    for (int e = threadIdx.x; e < m * n; e += blockDim.x) Ht[ch.ht + s * m * n + e] = sh[e];
  if (!Xhat) return;
  // A Ht  (nr x n)
  for (int e = threadIdx.x; e < nr * n; e += blockDim.x) {
    const int i = e / n, b = e % n;
    Cx<float> acc{0.f, 0.f};
    for (int a = 0; a < m; ++a) cfma(acc, ld(A + ch.a + i * m + a), Cx<float>{sh[a * n + b].x, sh[a * n + b].y});
    ah[e] = make_float2(acc.re, acc.im);
  }
  __syncthreads();
  float2* X = Xhat + ch.x + s * nr * nt;
  for (int e = threadIdx.x; e < nr * nt; e += blockDim.x) {
    const int i = e / nt, j = e % nt;
    Cx<float> acc{0.f, 0.f};
    const float2* Bj = B + ch.b + (int64_t)j * n;
    for (int b = 0; b < n; ++b) cfmac(acc, ld(Bj + b), Cx<float>{ah[i * n + b].x, ah[i * n + b].y});
    X[e] = make_float2(acc.re, acc.im);
  }
}

// Ht only (no Xhat): one block per group; a thread owns entry e of Ht_s for SC consecutive
// subcarriers, so each entry of G_g is read once per chunk of subcarriers rather than once per
// subcarrier.  The group's C rows are staged in LDS (every thread of a chunk reads the same
// entry), and the cores are read four q at a time with their loads issued before the products.
// The sum over q runs in the same order as in stage_ht.
__global__ void __launch_bounds__(256) k_reconstruct_ht(const DevChan* __restrict__ chans,
                                                        const GroupItem* __restrict__ items,
                                                        const float2* __restrict__ C,
                                                        const float2* __restrict__ G, float2* Ht) {
  __shared__ float2 cs[kMaxGroup * kMaxGroup];
  const GroupItem it = items[blockIdx.x];
  const DevChan& ch = chans[it.ch];
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  const int p = ch.p, pg = min(p, sz);
  const int mn = ch.m * ch.n;
  const float2* Gg = G + ch.g + (int64_t)it.g * p * mn;
  for (int e = threadIdx.x; e < sz * p; e += blockDim.x) cs[e] = C[ch.c + (int64_t)s0 * p + e];
  __syncthreads();
  constexpr int SC = 6, QU = 4;
  const int nch = (sz + SC - 1) / SC;
  for (int o = threadIdx.x; o < nch * mn; o += blockDim.x) {
    const int sc = o / mn, e = o - sc * mn;
    const float2* cr = cs + sc * SC * p;  // C row of this chunk's first subcarrier
    Cx<float> acc[SC];
#pragma unroll
    for (int j = 0; j < SC; ++j) acc[j] = Cx<float>{0.f, 0.f};
    int q = 0;
    for (; q + QU <= pg; q += QU) {
      Cx<float> gv[QU];
#pragma unroll
      for (int u = 0; u < QU; ++u) gv[u] = ld(Gg + (int64_t)(q + u) * mn + e);
#pragma unroll
      for (int u = 0; u < QU; ++u)
#pragma unroll
        for (int j = 0; j < SC; ++j)
          if (sc * SC + j < sz) {
            const float2 cv = cr[j * p + q + u];
            cfma(acc[j], Cx<float>{cv.x, cv.y}, gv[u]);
          }
    }
    for (; q < pg; ++q) {
      const Cx<float> gv = ld(Gg + (int64_t)q * mn + e);
#pragma unroll
      for (int j = 0; j < SC; ++j)
        if (sc * SC + j < sz) {
          const float2 cv = cr[j * p + q];
          cfma(acc[j], Cx<float>{cv.x, cv.y}, gv);
        }
    }
#pragma unroll
    for (int j = 0; j < SC; ++j)
      if (sc * SC + j < sz)
        Ht[ch.ht + (int64_t)(s0 + sc * SC + j) * mn + e] = make_float2(acc[j].re, acc[j].im);
  }
}

// Adjoint, one block per subcarrier: dHt(total) into the workspace, and the per-subcarrier
// contributions to dA and dB accumulated per group by k_rec_bwd_group.
__global__ void __launch_bounds__(256) k_rec_bwd_sub(const DevChan* __restrict__ chans, int n_channels,
                                                     const float2* __restrict__ A,
                                                     const float2* __restrict__ B,
                                                     const float2* __restrict__ gHt,
                                                     const float2* __restrict__ gX, char* ws) {
  __shared__ float2 agx[kMaxNr * kRecMaxNt];  // A^H dXhat_s  (m x nt)
  const int64_t gsc = blockIdx.x;
  int c;
  find_sub(chans, n_channels, gsc, c);
  const DevChan& ch = chans[c];
  const int64_t s = gsc - ch.sc;
  const int m = ch.m, n = ch.n, nr = ch.nr, nt = ch.nt;
  float2* out = reinterpret_cast<float2*>(ws + ch.w_gH) + s * m * n;
  if (gX) {
    const float2* gXs = gX + ch.x + s * nr * nt;
    for (int e = threadIdx.x; e < m * nt; e += blockDim.x) {
      const int a = e / nt, j = e % nt;
      Cx<float> acc{0.f, 0.f};
      for (int i = 0; i < nr; ++i) cfmac(acc, ld(A + ch.a + i * m + a), ld(gXs + (int64_t)i * nt + j));
      agx[e] = make_float2(acc.re, acc.im);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int a = e / n, b = e % n;
    Cx<float> acc{0.f, 0.f};
    if (gHt) acc = ld(gHt + ch.ht + s * m * n + e);
    if (gX)
      for (int j = 0; j < nt; ++j)
        cfma(acc, Cx<float>{agx[a * nt + j].x, agx[a * nt + j].y}, ld(B + ch.b + (int64_t)j * n + b));
    out[e] = make_float2(acc.re, acc.im);
  }
}

// Per group: partial dA (nr x m) and dB (nt x n) from the group's subcarriers.
__global__ void __launch_bounds__(256) k_rec_bwd_group(const DevChan* __restrict__ chans,
                                                       const GroupItem* __restrict__ items,
                                                       const float2* __restrict__ A,
                                                       const float2* __restrict__ B,
                                                       const float2* __restrict__ C,
                                                       const float2* __restrict__ G,
                                                       const float2* __restrict__ gX, char* ws) {
  __shared__ float2 sh[kRecMaxMN];
  __shared__ float2 ah[kMaxNr * 64];            // A Ht_s (nr x n)
  __shared__ float2 bh[kRecMaxNt * kMaxNr];     // B Ht_s^H (nt x m)
  const GroupItem it = items[blockIdx.x];
  const DevChan& ch = chans[it.ch];
  const int m = ch.m, n = ch.n, nr = ch.nr, nt = ch.nt;
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  float2* pA = reinterpret_cast<float2*>(ws + ch.w_gAp) + (int64_t)it.g * nr * m;
  float2* pB = reinterpret_cast<float2*>(ws + ch.w_gBp) + (int64_t)it.g * nt * n;
  // each output element is owned by one thread, which accumulates it in place
  for (int e = threadIdx.x; e < nr * m; e += blockDim.x) pA[e] = make_float2(0.f, 0.f);
  for (int e = threadIdx.x; e < nt * n; e += blockDim.x) pB[e] = make_float2(0.f, 0.f);
  for (int i0 = 0; i0 < sz; ++i0) {
    const int64_t s = s0 + i0;
    __syncthreads();
    stage_ht(ch, s, C, G, sh);
    __syncthreads();
    for (int e = threadIdx.x; e < nr * n; e += blockDim.x) {
      const int i = e / n, b = e % n;
      Cx<float> acc{0.f, 0.f};
      for (int a = 0; a < m; ++a) cfma(acc, ld(A + ch.a + i * m + a), Cx<float>{sh[a * n + b].x, sh[a * n + b].y});
      ah[e] = make_float2(acc.re, acc.im);
    }
    for (int e = threadIdx.x; e < nt * m; e += blockDim.x) {
      const int j = e / m, a = e % m;
      Cx<float> acc{0.f, 0.f};
      for (int b = 0; b < n; ++b)  // B[j][b] conj(Ht[a][b])
        cfmac(acc, Cx<float>{sh[a * n + b].x, sh[a * n + b].y}, ld(B + ch.b + (int64_t)j * n + b));
      bh[e] = make_float2(acc.re, acc.im);
    }
    __syncthreads();
    const float2* gXs = gX + ch.x + s * nr * nt;
    for (int e = threadIdx.x; e < nr * m; e += blockDim.x) {  // dA[i][a]
      const int i = e / m, a = e % m;
      Cx<float> acc = ld(pA + e);
      for (int j = 0; j < nt; ++j)
        cfma(acc, ld(gXs + (int64_t)i * nt + j), Cx<float>{bh[j * m + a].x, bh[j * m + a].y});
      st(pA + e, acc);
    }
    for (int e = threadIdx.x; e < nt * n; e += blockDim.x) {  // dB[j][b]
      const int j = e / n, b = e % n;
      Cx<float> acc = ld(pB + e);
      for (int i = 0; i < nr; ++i)
        cfmac(acc, ld(gXs + (int64_t)i * nt + j), Cx<float>{ah[i * n + b].x, ah[i * n + b].y});
      st(pB + e, acc);
    }
  }
}

// dA, dB = sums of the group partials (fixed order)
__global__ void __launch_bounds__(256) k_rec_bwd_ab(const DevChan* __restrict__ chans, char* ws,
                                                    float2* gA, float2* gB, int have_gx) {
  const DevChan& ch = chans[blockIdx.y];
  const int na = ch.nr * ch.m, nb = ch.nt * ch.n;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < na) {
    Cx<float> acc{0.f, 0.f};
    if (have_gx) {
      const float2* P = reinterpret_cast<const float2*>(ws + ch.w_gAp);
      for (int g = 0; g < ch.ngroups; ++g) {
        float2 v = P[(int64_t)g * na + e];
        acc.re += v.x;
        acc.im += v.y;
      }
    }
    st(gA + ch.a + e, acc);
  }
  if (e < nb) {
    Cx<float> acc{0.f, 0.f};
    if (have_gx) {
      const float2* P = reinterpret_cast<const float2*>(ws + ch.w_gBp);
      for (int g = 0; g < ch.ngroups; ++g) {
        float2 v = P[(int64_t)g * nb + e];
        acc.re += v.x;
        acc.im += v.y;
      }
    }
    st(gB + ch.b + e, acc);
  }
}

gt_status launch_grad_cg(const LaunchCtx& L, const float2* C, const float2* G, float2* gC, float2* gG);

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

gt_status launch_reconstruct(const LaunchCtx& L, int64_t total_sc, const float2* A, const float2* B,
                             const float2* C, const float2* G, float2* Ht, float2* Xhat) {
  if (!Xhat) {
    if (Ht) GT_LAUNCH(k_reconstruct_ht, dim3(L.total_groups), dim3(256), L.d_chans, L.d_groups, C, G, Ht);
    return GT_OK;
  }
  GT_LAUNCH(k_reconstruct, dim3((unsigned)total_sc), dim3(256), L.d_chans, L.n_channels, A, B, C, G, Ht,
            Xhat);
  return GT_OK;
}

gt_status launch_reconstruct_bwd(const LaunchCtx& L, int64_t total_sc, const float2* A,
                                 const float2* B, const float2* C, const float2* G,
                                 const float2* gHt, const float2* gX, float2* gA, float2* gB,
                                 float2* gC, float2* gG) {
  GT_LAUNCH(k_rec_bwd_sub, dim3((unsigned)total_sc), dim3(256), L.d_chans, L.n_channels, A, B, gHt, gX,
            L.ws);
  if (gX)
    GT_LAUNCH(k_rec_bwd_group, dim3(L.total_groups), dim3(256), L.d_chans, L.d_groups, A, B, C, G, gX,
              L.ws);
  const int maxe = std::max(L.max_nr * L.max_m, L.max_nt * L.max_n);
  GT_LAUNCH(k_rec_bwd_ab, dim3((maxe + 255) / 256, L.n_channels), dim3(256), L.d_chans, L.ws, gA, gB,
            gX ? 1 : 0);
  return launch_grad_cg(L, C, G, gC, gG);
}

}  // namespace gt
