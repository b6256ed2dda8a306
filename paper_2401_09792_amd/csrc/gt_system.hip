// The multi-cell system of the groupwise model (Sections 2.2, 3.2 and 3.3): factor sharing in
// the fit, and the per-subcarrier SINR of every UE with intra- and inter-cell interference from
// the compressed channels.
//
// Sharing (equation "three matrix factorization"): channels with the same a_id share the
// mode-1 factor A (a UE's channels from every BS), channels with the same b_id the mode-2
// factor B (every UE's channel from one BS).  The updates of A and B are eigenvectors of the
// Grams summed over the sharing channels (equations "update A", "update B"); k_share_gram forms
// those sums between each channel's own Gram reduction and the eigensolves, which then run per
// channel on identical inputs and give every member the same factor.
//
// SINR (equations "signal receiving", "covariance matrix", "compressed pre", "Cov", "MMSE
// receive filter", "s_r^ij", "SINR formula"): UE u, served by BS i, sees transmissions t = (BS
// k, UE v served by k) through its compressed channels Ht_{u,k}; with V~_v the precoder of v
// (first ns right singular vectors of v's serving channel Ht_{v,k}),
//   G_t = Ht_{u,k} V~_v  (m x ns),  Q~ = sum_t G_t G_t^H + s2 I_m,
//   W~ = Q~^{-1} G_own,  SINR_r = |w_r^H g_own,r|^2 / (w_r^H Q~ w_r - |w_r^H g_own,r|^2),
// everything in the m-dimensional basis of A_u and the n-dimensional bases of the B_k, which
// cancel (the reduced inversion of the interference matrix).  The denominator is evaluated as
// s2 ||w_r||^2 + sum_{k != r} |w_r^H g_own,k|^2 + w_r^H R w_r with R = sum over the other
// transmissions of G_t G_t^H: the same quantity without subtracting the signal power.
#include <hip/hip_runtime.h>

#include "gt_rows.h"

namespace gt {

// One block per sharing group: every member's Gram (S1 for which = 0, S2 for which = 1) is
// replaced by the sum over the members, added in the group's fixed member order.
__global__ void __launch_bounds__(256) k_share_gram(const DevChan* __restrict__ chans,
                                                    const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ members, int which,
                                                    char* ws) {
  const int b = off[blockIdx.x], e = off[blockIdx.x + 1];
  const DevChan& c0 = chans[members[b]];
  const int d = which == 0 ? c0.nr : c0.nt;
  const int64_t cnt = (int64_t)d * d;
  for (int64_t x = threadIdx.x; x < cnt; x += blockDim.x) {
    float sr = 0.f, si = 0.f;
    for (int k = b; k < e; ++k) {
      const DevChan& ch = chans[members[k]];
      const float2 v = reinterpret_cast<const float2*>(ws + (which == 0 ? ch.w_S1 : ch.w_S2))[x];
      sr += v.x;
      si += v.y;
    }
    for (int k = b; k < e; ++k) {
      const DevChan& ch = chans[members[k]];
      reinterpret_cast<float2*>(ws + (which == 0 ? ch.w_S1 : ch.w_S2))[x] = make_float2(sr, si);
    }
  }
}

// Channel of global subcarrier position pos (channels hold consecutive subcarrier ranges).
__device__ __forceinline__ int sys_locate(const DevChan* chans, int n_channels, int64_t pos) {
  int lo = 0, hi = n_channels - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (chans[mid].sc <= pos)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int MP, int NS>
struct SysLds {
  RowsLds<MP, NS> b;
  float2 g[MP][NS];  // rows of U_ns (precoder pass) or of one transmission's G_t (SINR pass)
};

// Pointers to row r (clamped to the channel's m rows) of subcarrier s of channel ch.
struct SysRow {
  const float2* Cs;
  const float2* Gr;
  int64_t gq;
  int pg;
};

__device__ __forceinline__ SysRow sys_row(const DevChan& ch, int64_t s, int r, const float2* C,
                                          const float2* G) {
  SysRow o;
  const int g = (int)(s / ch.gs);
  o.pg = min(ch.p, min(ch.gs, ch.nsc - g * ch.gs));
  const int rr = min(r, ch.m - 1);
  o.Cs = C + ch.c + s * ch.p;
  o.Gr = G + ch.g + ((int64_t)g * ch.p * ch.m + rr) * ch.n;
  o.gq = (int64_t)ch.m * ch.n;
  return o;
}

// Precoders of the serving links: V~ = Ht^H U_ns Sigma_ns^{-1}, the first ns right singular
// vectors of the serving channel (equation "precoding matrix"), [nsc][n][ns] into the serving
// channel's scratch.  Streams below the zero-stream floor get a zero column.
template <int MP, int NS>
__global__ void __launch_bounds__(256) k_sys_precoder(const DevChan* __restrict__ chans,
                                                      const int32_t* __restrict__ serving,
                                                      int n_channels, int64_t total_sc,
                                                      const float2* __restrict__ C,
                                                      const float2* __restrict__ G, char* ws,
                                                      int32_t* status) {
  constexpr int SPB = 256 / MP;
  __shared__ SysLds<MP, NS> lds[SPB];
  const int sub = threadIdx.x / MP, r = threadIdx.x % MP;
  SysLds<MP, NS>& S = lds[sub];
  const int64_t pos = (int64_t)blockIdx.x * SPB + sub;
  if (pos >= total_sc) return;
  const int c = sys_locate(chans, n_channels, pos);
  if (!serving[c]) return;  // the whole group leaves together
  const DevChan& ch = chans[c];
  const int64_t s = pos - ch.sc;
  const bool row = r < ch.m;
  const int n = ch.n, ns = ch.ns;
  const SysRow h = sys_row(ch, s, r, C, G);
  float kr[MP], ki[MP], vr[MP], vi[MP];
  rows_gram<MP, NS>(S.b, r, row, n, h.pg, h.Cs, h.Gr, h.gq, kr, ki);
  uint32_t bits = rows_eig<MP>(S.b.rot, r, kr, ki, vr, vi) ? 0u : GT_DEV_EIG_SWEEPS;
  float sig[NS], ur[NS], ui[NS], hvr[NS], hvi[NS];
  rows_hv<MP, NS>(S.b, r, row, ns, kr, vr, vi, sig, ur, ui, hvr, hvi, bits);
  float inv[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) {
    const bool live = a < ns && sig[a] > 1.0e-3f * sig[0];
    inv[a] = live ? 1.f / sig[a] : 0.f;
    S.g[r][a] = make_float2(ur[a], ui[a]);
  }
  wave_sync();
  float2* V = reinterpret_cast<float2*>(ws + ch.w_gH) + s * n * ns;
  for (int j0 = 0; j0 < n; j0 += kRowsChunk) {
    float hr[kRowsChunk], hi[kRowsChunk];
    rows_ht_chunk<MP, kRowsChunk>(row, j0, n, h.pg, h.Cs, h.Gr, h.gq, hr, hi);
#pragma unroll
    for (int jj = 0; jj < kRowsChunk; ++jj) S.b.u.ht[r][jj] = make_float2(hr[jj], hi[jj]);
    wave_sync();
    // column jj of the chunk in lane jj mod MP: V~[j][a] = sum_i conj(Ht[i][j]) U[i][a] / sigma_a
    for (int jj = r; jj < kRowsChunk; jj += MP) {
      const int j = j0 + jj;
      float ar[NS], ai[NS];
#pragma unroll
      for (int a = 0; a < NS; ++a) ar[a] = ai[a] = 0.f;
#pragma unroll
      for (int i = 0; i < MP; ++i) {
        const float2 x = S.b.u.ht[i][jj];
#pragma unroll
        for (int a = 0; a < NS; ++a) {
          const float2 u = S.g[i][a];
          ar[a] += x.x * u.x + x.y * u.y;
          ai[a] += x.x * u.y - x.y * u.x;
        }
      }
      if (j < n) {
#pragma unroll
        for (int a = 0; a < NS; ++a)
          if (a < ns) V[(int64_t)j * ns + a] = make_float2(ar[a] * inv[a], ai[a] * inv[a]);
      }
    }
    wave_sync();
  }
  bits = rows_or<MP>(bits);
  if (status && bits && r == 0) atomicOr(reinterpret_cast<unsigned int*>(status + c), bits);
}

// SINR of every UE at its serving channel's subcarriers; terms[2 t] is the channel Ht_{u,k} of
// transmission t and terms[2 t + 1] the serving channel whose precoder BS k uses; the UE's own
// transmission is its first term.  Subcarriers of the other channels are written as zero.
template <int MP, int NS>
__global__ void __launch_bounds__(256) k_sys_sinr(const DevChan* __restrict__ chans,
                                                  const int32_t* __restrict__ term_off,
                                                  const int32_t* __restrict__ terms, int n_channels,
                                                  int64_t total_sc, const float2* __restrict__ C,
                                                  const float2* __restrict__ G, RowsSnr snr,
                                                  float* __restrict__ out, int ns_max,
                                                  const char* __restrict__ ws, int32_t* status) {
  constexpr int SPB = 256 / MP;
  __shared__ SysLds<MP, NS> lds[SPB];
  const int sub = threadIdx.x / MP, r = threadIdx.x % MP;
  SysLds<MP, NS>& S = lds[sub];
  const int64_t pos = (int64_t)blockIdx.x * SPB + sub;
  if (pos >= total_sc) return;
  const int c = sys_locate(chans, n_channels, pos);
  const int t0 = term_off[c], t1 = term_off[c + 1];
  if (t0 == t1) {  // not a serving channel
    for (int k = 0; k < snr.n; ++k)
      for (int q = r; q < ns_max; q += MP) out[((int64_t)k * total_sc + pos) * ns_max + q] = 0.f;
    return;
  }
  const DevChan& ch = chans[c];
  const int64_t s = pos - ch.sc;
  const int m = ch.m, ns = ch.ns;
  const bool row = r < m;
  // rows of P = G_own G_own^H and R = sum of the other G_t G_t^H
  float pr[MP], pi[MP], qr[MP], qi[MP], hvr[NS], hvi[NS];
#pragma unroll
  for (int j = 0; j < MP; ++j) pr[j] = pi[j] = qr[j] = qi[j] = 0.f;
#pragma unroll
  for (int a = 0; a < NS; ++a) hvr[a] = hvi[a] = 0.f;
  for (int t = t0; t < t1; ++t) {
    const DevChan& cu = chans[terms[2 * t]];
    const DevChan& cv = chans[terms[2 * t + 1]];
    const int n = cu.n;
    const SysRow h = sys_row(cu, s, r, C, G);
    const float2* V = reinterpret_cast<const float2*>(ws + cv.w_gH) + s * n * ns;
    float gr[NS], gi[NS];  // row r of G_t = Ht_{u,k} V~_v
#pragma unroll
    for (int a = 0; a < NS; ++a) gr[a] = gi[a] = 0.f;
    for (int j0 = 0; j0 < n; j0 += kRowsChunk) {
      float hr[kRowsChunk], hi[kRowsChunk];
      rows_ht_chunk<MP, kRowsChunk>(row, j0, n, h.pg, h.Cs, h.Gr, h.gq, hr, hi);
#pragma unroll
      for (int jj = 0; jj < kRowsChunk; ++jj) {
        const int j = min(j0 + jj, n - 1);  // columns past n have hr = hi = 0
#pragma unroll
        for (int a = 0; a < NS; ++a) {
          const float2 v = (a < ns) ? V[(int64_t)j * ns + a] : make_float2(0.f, 0.f);
          gr[a] += hr[jj] * v.x - hi[jj] * v.y;
          gi[a] += hr[jj] * v.y + hi[jj] * v.x;
        }
      }
    }
#pragma unroll
    for (int a = 0; a < NS; ++a) S.g[r][a] = make_float2(gr[a], gi[a]);
    wave_sync();
    const bool own = t == t0;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      float ar = 0.f, ai = 0.f;
#pragma unroll
      for (int a = 0; a < NS; ++a) {  // g_r conj(g_j)
        const float2 y = S.g[j][a];
        ar += gr[a] * y.x + gi[a] * y.y;
        ai += gi[a] * y.x - gr[a] * y.y;
      }
      pr[j] += own ? ar : 0.f;
      pi[j] += own ? ai : 0.f;
      qr[j] += own ? 0.f : ar;
      qi[j] += own ? 0.f : ai;
    }
    if (own) {
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        hvr[a] = gr[a];
        hvi[a] = gi[a];
      }
    }
    wave_sync();
  }
  uint32_t bits = 0;
  for (int kk = 0; kk < snr.n; ++kk) {
    const float s2 = snr.s2[kk];
    float lr[MP], li[MP];
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      lr[j] = row ? pr[j] + qr[j] + ((j == r) ? s2 : 0.f) : ((j == r) ? 1.f : 0.f);
      li[j] = row ? pi[j] + qi[j] : 0.f;
    }
    bool ok;
    float rd;
    rows_chol_factor<MP, NS>(S.b, r, lr, li, ok, rd);
    float wr[NS], wi[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      wr[a] = hvr[a];
      wi[a] = hvi[a];
    }
    rows_solve<MP, NS>(S.b, r, lr, li, rd, wr, wi);  // W rows; the y table holds all of them
    // z = R W, row r (W rows from the y table), then w_a^H R w_a summed over the rows
    float zr[NS], zi[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) zr[a] = zi[a] = 0.f;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        const float2 w = S.b.u.m.y[j][a];
        zr[a] += qr[j] * w.x - qi[j] * w.y;
        zi[a] += qr[j] * w.y + qi[j] * w.x;
      }
    }
    float sinr_me = 0.f;
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      const float interf = rows_sum<MP>(wr[a] * zr[a] + wi[a] * zi[a]);
      float sig_p = 0.f, den = s2 * rows_sum<MP>(wr[a] * wr[a] + wi[a] * wi[a]) + interf;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const float cr = rows_sum<MP>(wr[a] * hvr[k] + wi[a] * hvi[k]);
        const float ci = rows_sum<MP>(wr[a] * hvi[k] - wi[a] * hvr[k]);
        const float pw = cr * cr + ci * ci;
        if (k == a)
          sig_p = pw;
        else
          den += pw;
      }
      sinr_me = (a == r) ? sig_p / den : sinr_me;
    }
    const bool any_bad = rows_or<MP>(ok ? 0u : 1u) != 0u;
    if (any_bad) bits |= GT_DEV_CHOLESKY;
    float v = (r < ns && !any_bad) ? sinr_me : 0.f;
    if (!(v == v) || v > 3.0e38f) {
      v = 0.f;
      bits |= GT_DEV_NONFINITE;
    }
    for (int q = r; q < ns_max; q += MP)
      out[((int64_t)kk * total_sc + pos) * ns_max + q] = (q == r) ? v : 0.f;
    wave_sync();
  }
  bits = rows_or<MP>(bits);
  if (status && bits && r == 0) atomicOr(reinterpret_cast<unsigned int*>(status + c), bits);
}

// ---------------------------------------------------------------------------------------

gt_status launch_share_gram(const LaunchCtx& L, int which) {
  const int n = L.n_share[which];
  if (n == 0) return GT_OK;
  prof_begin("k_share_gram", L.stream);
  hipLaunchKernelGGL(k_share_gram, dim3(n), dim3(256), 0, L.stream, L.d_chans, L.d_share_off[which],
                     L.d_share_ch[which], which, L.ws);
  prof_end(L.stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error_detail("k_share_gram", e);
    return GT_ERR_HIP;
  }
  return GT_OK;
}

template <int MP, int NS>
static gt_status sys_launch_t(const LaunchCtx& L, int64_t total_sc, const int32_t* terms_off,
                              const int32_t* terms, const float2* C, const float2* G,
                              const RowsSnr& a, float* out, int ns_max, int32_t* status) {
  constexpr int SPB = 256 / MP;
  const unsigned grid = (unsigned)((total_sc + SPB - 1) / SPB);
  prof_begin("k_sys_precoder", L.stream);
  hipLaunchKernelGGL((k_sys_precoder<MP, NS>), dim3(grid), dim3(256), 0, L.stream, L.d_chans,
                     L.d_sys_serving, L.n_channels, total_sc, C, G, L.ws, status);
  prof_end(L.stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error_detail("k_sys_precoder", e);
    return GT_ERR_HIP;
  }
  prof_begin("k_sys_sinr", L.stream);
  hipLaunchKernelGGL((k_sys_sinr<MP, NS>), dim3(grid), dim3(256), 0, L.stream, L.d_chans, terms_off,
                     terms, L.n_channels, total_sc, C, G, a, out, ns_max, L.ws, status);
  prof_end(L.stream);
  e = hipGetLastError();
  if (e != hipSuccess) {
    set_error_detail("k_sys_sinr", e);
    return GT_ERR_HIP;
  }
  return GT_OK;
}

// Precoders of every serving link, then the SINR of every UE with the transmissions of the
// chosen interference table.
gt_status launch_sinr_system(const LaunchCtx& L, int64_t total_sc, const int32_t* terms_off,
                             const int32_t* terms, const float2* C, const float2* G,
                             const float* s2, int n_snr, float* out, int ns_max, int32_t* status) {
  RowsSnr a{};
  a.n = n_snr;
  for (int k = 0; k < n_snr; ++k) a.s2[k] = s2[k];
  if (L.max_m <= 4) {
    if (L.max_ns <= 2) return sys_launch_t<4, 2>(L, total_sc, terms_off, terms, C, G, a, out, ns_max, status);
    return sys_launch_t<4, 4>(L, total_sc, terms_off, terms, C, G, a, out, ns_max, status);
  }
  return sys_launch_t<8, 4>(L, total_sc, terms_off, terms, C, G, a, out, ns_max, status);
}

}  // namespace gt
