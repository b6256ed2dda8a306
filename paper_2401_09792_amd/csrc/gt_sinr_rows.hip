// Per-subcarrier SINR from the compressed form (Section 3.3), row-parallel form.
//
// MP lanes of one wave (an aligned group, MP = 4, 8 or 16 >= m) handle one subcarrier; lane r
// owns row r of every m x m matrix of the chain and keeps it in registers:
//   Ht_s = sum_q C[s,q] G_g[q]   (equation "compressed matrix SINR reduction"), row r formed
//                                by lane r, kRowsChunk columns at a time;
//   K = Ht Ht^H                  rows from the staged chunk of Ht rows in LDS;
//   K = U diag(sigma^2) U^H      parallel two-sided Jacobi: in step t of a sweep lane r is
//                                paired with lane r xor t (t = 1 .. MP-1, so every pair of
//                                indices meets once per sweep); partner rows are exchanged with
//                                ds_swizzle, and the column rotations of the other pairs read
//                                their (c, s) from LDS;
//   HV = U_ns Sigma_ns           precoder of equation "precoding matrix" (HV = Ht V_ns);
//   M = HV^H HV                  ns x ns, summed over the group by swizzles, held by every lane;
//   W = Q^{-1} HV = HV P^{-1}    the MMSE filter with Q = HV HV^H + s2 I_m (equation "MMSE
//                                receive filter"), through the push-through identity with
//                                P = M + s2 I_ns: the ns x ns system replaces the m x m one, as
//                                the Woodbury step of Section 3.3 replaces M x M by m x m;
//   c_jk = w_j^H hv_k = (P^{-1} M)_jk,   ||w_j||^2 = (P^{-1} M P^{-1})_jj: lane j factors P by
//                                Cholesky, solves P y = e_j and forms z = M y, so c_jk = conj(z_k)
//                                and ||w_j||^2 = y^H z;
//   SINR_j = |c_jj|^2 / (s2 ||w_j||^2 + sum_{k != j} |c_jk|^2)   (equations "s_r^ij" and
//                                "SINR formula"; the denominator equals w_j^H Q w_j - s_j).
// Instantiations with NS = MP, and the adjoint kernel (whose back-propagation runs through it),
// keep the m x m chain: Q = HV HV^H + s2 I = L L^H by a left-looking Cholesky over the rows,
// W = Q^{-1} HV by substitutions, c_jk = w_j^H hv_k summed over the group by swizzles.
// Spreading a subcarrier over MP lanes gives a launch MP times as many waves as one lane per
// subcarrier, so the long serial chain of each small eigenproblem overlaps with others.
#include <hip/hip_runtime.h>

#include "gt_rows.h"

namespace gt {

// M = HV^H HV from the rows of HV held by the MP lanes of a group (ns x ns, zero past ns), the
// same in every lane.
template <int MP, int NS>
__device__ __forceinline__ void pt_gram(const float (&hvr)[NS], const float (&hvi)[NS],
                                        float (&mr)[NS][NS], float (&mi)[NS][NS]) {
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int k = i; k < NS; ++k) {
      const float re = rows_sum<MP>(hvr[i] * hvr[k] + hvi[i] * hvi[k]);
      const float im = (k == i) ? 0.f : rows_sum<MP>(hvr[i] * hvi[k] - hvi[i] * hvr[k]);
      mr[i][k] = re;
      mi[i][k] = im;
      mr[k][i] = re;
      mi[k][i] = -im;
    }
}

// P = M + s2 I = L L^H (Cholesky, lower, in registers); dinv[i] = 1 / L[i][i].  ok turns false
// if a pivot is not positive.
template <int NS>
__device__ __forceinline__ void pt_chol(const float (&mr)[NS][NS], const float (&mi)[NS][NS],
                                        float s2, float (&lr)[NS][NS], float (&li)[NS][NS],
                                        float (&dinv)[NS], bool& ok) {
#pragma unroll
  for (int i = 0; i < NS; ++i) {
#pragma unroll
    for (int k = 0; k <= i; ++k) {
      float sr = mr[i][k] + (i == k ? s2 : 0.f), si = (i == k) ? 0.f : mi[i][k];
#pragma unroll
      for (int l = 0; l < k; ++l) {  // - L[i][l] conj(L[k][l])
        sr -= lr[i][l] * lr[k][l] + li[i][l] * li[k][l];
        si -= li[i][l] * lr[k][l] - lr[i][l] * li[k][l];
      }
      if (i == k) {
        ok = ok && sr > 0.f;
        dinv[i] = __builtin_amdgcn_rsqf(sr > 0.f ? sr : 1.f);
      } else {
        lr[i][k] = sr * dinv[k];
        li[i][k] = si * dinv[k];
      }
    }
  }
}

// y = P^{-1} e_j = L^{-H} L^{-1} e_j; returns P^{-1}_jj = ||L^{-1} e_j||^2 (real by construction).
template <int NS>
__device__ __forceinline__ float pt_solve(const float (&lr)[NS][NS], const float (&li)[NS][NS],
                                          const float (&dinv)[NS], int j, float (&yr)[NS],
                                          float (&yi)[NS]) {
  float ur[NS], ui[NS], xjj = 0.f;
#pragma unroll
  for (int i = 0; i < NS; ++i) {  // L u = e_j
    float sr = (i == j) ? 1.f : 0.f, si = 0.f;
#pragma unroll
    for (int l = 0; l < i; ++l) {
      sr -= lr[i][l] * ur[l] - li[i][l] * ui[l];
      si -= lr[i][l] * ui[l] + li[i][l] * ur[l];
    }
    ur[i] = sr * dinv[i];
    ui[i] = si * dinv[i];
    xjj += ur[i] * ur[i] + ui[i] * ui[i];
  }
#pragma unroll
  for (int i = NS - 1; i >= 0; --i) {  // L^H y = u
    float sr = ur[i], si = ui[i];
#pragma unroll
    for (int l = i + 1; l < NS; ++l) {  // - conj(L[l][i]) y[l]
      sr -= lr[l][i] * yr[l] + li[l][i] * yi[l];
      si -= lr[l][i] * yi[l] - li[l][i] * yr[l];
    }
    yr[i] = sr * dinv[i];
    yi[i] = si * dinv[i];
  }
  return xjj;
}

// SINR of stream j of the MMSE filter from M = HV^H HV (NS x NS Hermitian, zero past ns) and the
// noise level s2: y = P^{-1} e_j, z = M y; c_jk = conj(z_k), ||w_j||^2 = y^H z.  ok turns false
// if a pivot of P is not positive.
template <int NS>
__device__ __forceinline__ float pt_stream_sinr(const float (&mr)[NS][NS], const float (&mi)[NS][NS],
                                                float s2, int j, bool& ok) {
  float lr[NS][NS], li[NS][NS], dinv[NS], yr[NS], yi[NS];
  pt_chol<NS>(mr, mi, s2, lr, li, dinv, ok);
  pt_solve<NS>(lr, li, dinv, j, yr, yi);
  // z = M y; signal |z_j|^2, interference sum_{k != j} |z_k|^2, ||w_j||^2 = Re(y^H z)
  float sig_p = 0.f, den = 0.f, wn = 0.f;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    float zr = 0.f, zi = 0.f;
#pragma unroll
    for (int l = 0; l < NS; ++l) {
      zr += mr[k][l] * yr[l] - mi[k][l] * yi[l];
      zi += mr[k][l] * yi[l] + mi[k][l] * yr[l];
    }
    const float pw = zr * zr + zi * zi;
    if (k == j)
      sig_p = pw;
    else
      den += pw;
    wn += yr[k] * zr + yi[k] * zi;
  }
  return sig_p / (den + s2 * wn);
}

// Compressed-channel SINR for channels with m <= MP and ns <= NS, 256 / MP subcarriers per
// block of 256 lanes.
template <int MP, int NS>
__global__ void __launch_bounds__(256, 4) k_sinr_rows(const DevChan* __restrict__ chans, RowsRange R,
                                                    int64_t total_sc, const float2* __restrict__ C,
                                                    const float2* __restrict__ G, RowsSnr snr,
                                                    float* __restrict__ out, int ns_max,
                                                    int32_t* status) {
  constexpr int SPB = 256 / MP;
  __shared__ RowsLds<MP, NS, 16> lds[SPB];
  const int sub = threadIdx.x / MP, r = threadIdx.x % MP;
  RowsLds<MP, NS, 16>& S = lds[sub];
  const int64_t it = (int64_t)blockIdx.x * SPB + sub;
  const bool valid = it < R.count;
  int64_t gsc = 0;
  const int c = valid ? rows_locate(R, chans, it, gsc) : R.ch[0];
  const DevChan& ch = chans[c];
  const int64_t s = valid ? gsc - ch.sc : 0;
  const int m = valid ? ch.m : 0;
  const int n = valid ? ch.n : 0;
  const int ns = valid ? ch.ns : 0;
  const int g = (int)(s / ch.gs);
  const int pg = min(ch.p, min(ch.gs, ch.nsc - g * ch.gs));
  const bool row = r < m;
  // row r of G_g[q] (padding rows read row m - 1 and are zeroed)
  const int rr = min(r, max(ch.m - 1, 0));
  const float2* Cs = C + ch.c + s * ch.p;
  const float2* Gr = G + ch.g + ((int64_t)g * ch.p * ch.m + rr) * ch.n;
  const int64_t gq = (int64_t)ch.m * ch.n;

  float kr[MP], ki[MP], vr[MP], vi[MP];
  {
    // the cores of the wave's groups staged in the wave's own (not yet used) part of lds
    constexpr int MAXG = kRowsMaxG<MP>;
    const RowsWave<MAXG> W = rows_wave_groups<MP, MAXG>(
        valid, c, g, ch.g + (int64_t)g * ch.p * ch.m * ch.n, m, n, pg);
    float2* stage = reinterpret_cast<float2*>(&lds[(threadIdx.x / 64) * (64 / MP)]);
    rows_gram<MP, NS, 16, MAXG, true>(S, r, row, n, pg, Cs, Gr, gq, kr, ki, &W, stage, G);
  }
  // the forward stops the sweeps at a squared off-diagonal norm of 1e6 eps^2 (3.6e-9) of the
  // diagonal's: relative off-diagonal entries of 6e-5 tilt the precoder by about that over the
  // eigenvalue gap, which moves an SINR by its square (second order, about 1e-4 dB at 20 dB);
  // the adjoint keeps the tight test, since gradients are first order in the eigenvectors
  uint32_t bits = rows_eig_x<MP>(S.rot, r, kr, ki, vr, vi, false, 1.0e6f) ? 0u : GT_DEV_EIG_SWEEPS;
  float sig[NS], ur[NS], ui[NS], hvr[NS], hvi[NS];
  rows_hv<MP, NS, 16, true>(S, r, row, ns, kr, vr, vi, sig, ur, ui, hvr, hvi, bits);

  // with ns < m the ns x ns push-through form of the MMSE filter; with ns = m the m x m chain
  constexpr bool kPT = NS < MP;
  float mr[kPT ? NS : 1][kPT ? NS : 1], mi[kPT ? NS : 1][kPT ? NS : 1];
  bool live = true;
  int js = 0;
  if constexpr (kPT) {
    pt_gram<MP, NS>(hvr, hvi, mr, mi);  // M = HV^H HV
    js = min(r, NS - 1);  // this lane's stream
    float sig_me = sig[0];
#pragma unroll
    for (int k = 1; k < NS; ++k) sig_me = (k == js) ? sig[k] : sig_me;
    live = sig_me > 1.0e-3f * sig[0];  // zero-stream rule
  }
  for (int kk = 0; kk < snr.n; ++kk) {
    const float s2 = snr.s2[kk];
    bool ok = true;
    float sinr_me = 0.f;
    if constexpr (kPT) {
      sinr_me = pt_stream_sinr<NS>(mr, mi, s2, js, ok);
      if (!live) sinr_me = 0.f;
    } else {
      float lr[MP], li[MP];
      float rd;
      rows_chol<MP, NS>(S, r, row, s2, hvr, hvi, lr, li, ok, rd);
      float wr[NS], wi[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        wr[k] = hvr[k];
        wi[k] = hvi[k];
      }
      rows_solve<MP, NS>(S, r, lr, li, rd, wr, wi);
      // c_jk = w_j^H hv_k, ||w_j||^2, SINR_j
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        float sig_p = 0.f, den = 0.f;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const float cr = rows_sum<MP>(wr[j] * hvr[k] + wi[j] * hvi[k]);
          const float ci = rows_sum<MP>(wr[j] * hvi[k] - wi[j] * hvr[k]);
          const float pw = cr * cr + ci * ci;
          if (k == j)
            sig_p = pw;
          else
            den += pw;
        }
        den += s2 * rows_sum<MP>(wr[j] * wr[j] + wi[j] * wi[j]);
        float v = sig_p / den;
        if (!(sig[j] > 1.0e-3f * sig[0])) v = 0.f;
        sinr_me = (j == r) ? v : sinr_me;
      }
    }
    const bool any_bad = rows_or<MP>(ok ? 0u : 1u) != 0u;
    if (any_bad) bits |= GT_DEV_CHOLESKY;
    float v = (r < ns && !any_bad) ? sinr_me : 0.f;
    if (!(v == v) || v > 3.0e38f) {
      v = 0.f;
      bits |= GT_DEV_NONFINITE;
    }
    if (valid) {
      float* o = out + ((int64_t)kk * total_sc + gsc) * ns_max;
      for (int q = r; q < ns_max; q += MP) o[q] = (q == r) ? v : 0.f;
    }
  }
  bits = rows_or<MP>(bits);
  if (valid && status && bits && r == 0) atomicOr(reinterpret_cast<unsigned int*>(status + c), bits);
}

// Adjoint of k_sinr_rows: recomputes Ht, its eigendecomposition and, per noise level, the MMSE
// chain.  With ns < m it runs in the ns x ns push-through form (see the loop); otherwise it
// recomputes L and W and back-propagates dl/dSINR through SINR_j = s_j / d_j, s_j = |c_jj|^2,
// d_j = s2 ||w_j||^2 + sum_{k != j} |c_jk|^2 with c_jk = w_j^H hv_k, W = Q^{-1} HV and
// Q = HV HV^H + s2 I to dl/dHV:
//   C-bar_jk = 2 (k == j ? g_j / d_j : -g_j s_j / d_j^2) c_jk,   N-bar_j = -s2 g_j s_j / d_j^2,
//   W-bar = HV C-bar^H + 2 W diag(N-bar),   Lambda = Q^{-1} W-bar,
//   dl/dHV += W C-bar + Lambda - Lambda (W^H HV) - W (Lambda^H HV);
// then through HV = U_ns Sigma_ns with the kept-block singular-vector adjoint
//   P = U_ns^H dl/dHV,  D_aa = Re P_aa,
//   D_ab = (sigma_b^2 P_ab - sigma_a sigma_b conj(P_ba)) / (sigma_b^2 - sigma_a^2)  (a != b,
//          zero for numerically equal sigma),
//   dl/dHt = U_ns D V_ns^H = E Ht,  E = U_ns D Sigma^{-1} U_ns^H,
// row i of dl/dHt from row i of E and the recomputed rows of Ht.  Streams forced to zero by
// the zero-stream rule carry no gradient.  dl/dHt goes to the workspace; the per-group
// reduction forms dl/dC and dl/dG.
template <int MP, int NS>
__global__ void __launch_bounds__(256, 3) k_sinr_bwd_rows(const DevChan* __restrict__ chans,
                                                        RowsRange R, int64_t total_sc,
                                                        const float2* __restrict__ C,
                                                        const float2* __restrict__ G, RowsSnr snr,
                                                        const float* __restrict__ gsinr,
                                                        int ns_max, char* ws, int32_t* status) {
  constexpr int SPB = 256 / MP;
  __shared__ RowsLds<MP, NS> lds[SPB];
  const int sub = threadIdx.x / MP, r = threadIdx.x % MP;
  RowsLds<MP, NS>& S = lds[sub];
  const int64_t it = (int64_t)blockIdx.x * SPB + sub;
  const bool valid = it < R.count;
  int64_t gsc = 0;
  const int c = valid ? rows_locate(R, chans, it, gsc) : R.ch[0];
  const DevChan& ch = chans[c];
  const int64_t s = valid ? gsc - ch.sc : 0;
  const int m = valid ? ch.m : 0;
  const int n = valid ? ch.n : 0;
  const int ns = valid ? ch.ns : 0;
  const int g = (int)(s / ch.gs);
  const int pg = min(ch.p, min(ch.gs, ch.nsc - g * ch.gs));
  const bool row = r < m;
  const int rr = min(r, max(ch.m - 1, 0));
  const float2* Cs = C + ch.c + s * ch.p;
  const float2* Gr = G + ch.g + ((int64_t)g * ch.p * ch.m + rr) * ch.n;
  const int64_t gq = (int64_t)ch.m * ch.n;

  float kr[MP], ki[MP], vr[MP], vi[MP];
  // the cores of the wave's groups staged in the wave's own part of lds (while it is free)
  constexpr int MAXG = kRowsMaxG<MP>;
  const RowsWave<MAXG> W = rows_wave_groups<MP, MAXG>(
      valid, c, g, ch.g + (int64_t)g * ch.p * ch.m * ch.n, m, n, pg);
  float2* stage = reinterpret_cast<float2*>(&lds[(threadIdx.x / 64) * (64 / MP)]);
  rows_gram<MP, NS, kRowsChunk, MAXG, true>(S, r, row, n, pg, Cs, Gr, gq, kr, ki, &W, stage, G);
  uint32_t bits = rows_eig_x<MP>(S.rot, r, kr, ki, vr, vi) ? 0u : GT_DEV_EIG_SWEEPS;
  float sig[NS], ur[NS], ui[NS], hvr[NS], hvi[NS];
  rows_hv<MP, NS, kRowsChunk, true>(S, r, row, ns, kr, vr, vi, sig, ur, ui, hvr, hvi, bits);
  bool live[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) live[k] = k < ns && sig[k] > 1.0e-3f * sig[0];

  float br[NS], bi[NS];  // row r of dl/dHV
#pragma unroll
  for (int k = 0; k < NS; ++k) br[k] = bi[k] = 0.f;
  if constexpr (NS < MP) {
    // ns < m: with X = P^{-1}, P = HV^H HV + s2 I_ns, the SINR of the MMSE filter is
    // SINR_j = 1 / (s2 X_jj) - 1 (the chain's c and ||w_j||^2 in terms of X), so
    // dl/dM = sum_j g_j / (s2 X_jj^2) x_j x_j^H (x_j = X e_j) and dl/dHV = 2 HV dl/dM
    float mr[NS][NS], mi[NS][NS], gmr[NS][NS], gmi[NS][NS];
    pt_gram<MP, NS>(hvr, hvi, mr, mi);
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int l = 0; l < NS; ++l) gmr[k][l] = gmi[k][l] = 0.f;
    for (int kk = 0; kk < snr.n; ++kk) {
      const float s2 = snr.s2[kk];
      float lr[NS][NS], li[NS][NS], dinv[NS];
      bool ok = true;
      pt_chol<NS>(mr, mi, s2, lr, li, dinv, ok);
      const bool any_bad = rows_or<MP>(ok ? 0u : 1u) != 0u;
      if (any_bad) bits |= GT_DEV_CHOLESKY;
      const float* gk = gsinr + ((int64_t)kk * total_sc + gsc) * ns_max;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        // streams past ns, zero streams and broken-down noise levels carry no gradient
        const bool on = valid && live[j] && !any_bad;
        const float gj = on ? gk[j] : 0.f;
        float yr[NS], yi[NS];
        const float xjj = pt_solve<NS>(lr, li, dinv, j, yr, yi);
        const float aj = on ? gj / (s2 * xjj * xjj) : 0.f;
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
          for (int l = 0; l < NS; ++l) {  // a_j y_k conj(y_l)
            gmr[k][l] += aj * (yr[k] * yr[l] + yi[k] * yi[l]);
            gmi[k][l] += aj * (yi[k] * yr[l] - yr[k] * yi[l]);
          }
      }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {  // row r of 2 HV dl/dM
      float ar = 0.f, ai = 0.f;
#pragma unroll
      for (int l = 0; l < NS; ++l) {
        ar += hvr[l] * gmr[l][k] - hvi[l] * gmi[l][k];
        ai += hvr[l] * gmi[l][k] + hvi[l] * gmr[l][k];
      }
      br[k] = 2.f * ar;
      bi[k] = 2.f * ai;
    }
  } else {
    for (int kk = 0; kk < snr.n; ++kk) {
      const float s2 = snr.s2[kk];
      float lr[MP], li[MP];
      bool ok;
      float rd;
      rows_chol<MP, NS>(S, r, row, s2, hvr, hvi, lr, li, ok, rd);
      const bool any_bad = rows_or<MP>(ok ? 0u : 1u) != 0u;
      if (any_bad) bits |= GT_DEV_CHOLESKY;
      float wr[NS], wi[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        wr[k] = hvr[k];
        wi[k] = hvi[k];
      }
      rows_solve<MP, NS>(S, r, lr, li, rd, wr, wi);
      float cr[NS][NS], ci[NS][NS];  // c_jk = w_j^H hv_k
      rows_inner<MP, NS>(wr, wi, hvr, hvi, cr, ci);
      // C-bar (in place of c) and N-bar
      float nb[NS];
      const float* gk = gsinr + ((int64_t)kk * total_sc + gsc) * ns_max;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const float nw = rows_sum<MP>(wr[j] * wr[j] + wi[j] * wi[j]);
        float sv = 0.f, dv = s2 * nw;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const float pw = cr[j][k] * cr[j][k] + ci[j][k] * ci[j][k];
          if (k == j)
            sv = pw;
          else
            dv += pw;
        }
        // streams past ns (zero columns of W and HV, d_j = 0), zero streams and broken-down
        // noise levels carry no gradient
        const bool on = valid && live[j] && !any_bad;
        const float gj = on ? gk[j] : 0.f;
        const float sbar = on ? gj / dv : 0.f;
        const float dbar = on ? -gj * sv / (dv * dv) : 0.f;
        nb[j] = s2 * dbar;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const float f = (k == j) ? 2.f * sbar : 2.f * dbar;
          cr[j][k] *= f;
          ci[j][k] *= f;
        }
      }
      // c (needed below) is recomputed from W and HV after W-bar: keep C-bar in cr/ci
      // W-bar row r: sum_k hv[r][k] conj(Cbar[j][k]) + 2 nb_j w[r][j]
      float lmr[NS], lmi[NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        float ar = 2.f * nb[j] * wr[j], ai = 2.f * nb[j] * wi[j];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          ar += hvr[k] * cr[j][k] + hvi[k] * ci[j][k];
          ai += hvi[k] * cr[j][k] - hvr[k] * ci[j][k];
        }
        lmr[j] = ar;
        lmi[j] = ai;
      }
      // dl/dHV += W C-bar
#pragma unroll
      for (int k = 0; k < NS; ++k) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          br[k] += wr[j] * cr[j][k] - wi[j] * ci[j][k];
          bi[k] += wr[j] * ci[j][k] + wi[j] * cr[j][k];
        }
      }
      rows_solve<MP, NS>(S, r, lr, li, rd, lmr, lmi);  // Lambda = Q^{-1} W-bar
      // c again (C-bar overwrote it), then X = Lambda^H HV
      rows_inner<MP, NS>(wr, wi, hvr, hvi, cr, ci);
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        float ar = lmr[k], ai = lmi[k];
#pragma unroll
        for (int j = 0; j < NS; ++j) {  // - Lambda[r][j] c_jk
          ar -= lmr[j] * cr[j][k] - lmi[j] * ci[j][k];
          ai -= lmr[j] * ci[j][k] + lmi[j] * cr[j][k];
        }
        br[k] += ar;
        bi[k] += ai;
      }
      rows_inner<MP, NS>(lmr, lmi, hvr, hvi, cr, ci);  // X_jk = lambda_j^H hv_k
#pragma unroll
      for (int k = 0; k < NS; ++k) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {  // - W[r][j] X_jk
          br[k] -= wr[j] * cr[j][k] - wi[j] * ci[j][k];
          bi[k] -= wr[j] * ci[j][k] + wi[j] * cr[j][k];
        }
      }
    }
  }
  // singular-vector stage: P = U_ns^H dl/dHV, D, E row r
  float pr[NS][NS], pi[NS][NS];
  rows_inner<MP, NS>(ur, ui, br, bi, pr, pi);
  const float lam1 = sig[0] * sig[0];
  float dr[NS][NS], di[NS][NS];
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = 0; b < NS; ++b) {
      const float sa = sig[a], sb = sig[b];
      const float gap = sb * sb - sa * sa;
      float xr = 0.f, xi = 0.f;
      if (a == b) {
        xr = pr[a][a];
      } else if (__builtin_fabsf(gap) > 1e-5f * lam1) {
        xr = (sb * sb * pr[a][b] - sa * sb * pr[b][a]) / gap;
        xi = (sb * sb * pi[a][b] + sa * sb * pi[b][a]) / gap;
      }
      const float inv = (live[b] && sb > 0.f) ? 1.f / sb : 0.f;  // D Sigma^{-1}
      dr[a][b] = (a < ns && b < ns) ? xr * inv : 0.f;
      di[a][b] = (a < ns && b < ns) ? xi * inv : 0.f;
    }
  // row r of F = U_ns D Sigma^{-1}; E[r][j] = sum_b F[r][b] conj(U[j][b]) with the U rows in LDS
  float fr[NS], fi[NS];
#pragma unroll
  for (int b = 0; b < NS; ++b) {
    float ar = 0.f, ai = 0.f;
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      ar += ur[a] * dr[a][b] - ui[a] * di[a][b];
      ai += ur[a] * di[a][b] + ui[a] * dr[a][b];
    }
    fr[b] = ar;
    fi[b] = ai;
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) S.u.m.hv[r][k] = make_float2(ur[k], ui[k]);
  wave_sync();
  float er[MP], ei[MP];
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    float ar = 0.f, ai = 0.f;
#pragma unroll
    for (int b = 0; b < NS; ++b) {  // F[r][b] conj(U[j][b])
      const float2 u = S.u.m.hv[j][b];
      ar += fr[b] * u.x + fi[b] * u.y;
      ai += fi[b] * u.x - fr[b] * u.y;
    }
    er[j] = ar;
    ei[j] = ai;
  }
  wave_sync();
  // dl/dHt row r = sum_j E[r][j] Ht[j][:], chunk by chunk of recomputed Ht rows
  float2* gH = reinterpret_cast<float2*>(ws + ch.w_gH) + (s * ch.m + rr) * ch.n;
  const bool staged = W.ngrp <= MAXG;  // the same in every lane of the wave
  int jend = n;
  if (staged) {
    jend = 0;
#pragma unroll
    for (int k = 0; k < MAXG; ++k)
      if (k < W.ngrp) jend = max(jend, W.nk[k]);
  }
  for (int j0 = 0; j0 < jend; j0 += kRowsChunk) {
    float hr[kRowsChunk], hi[kRowsChunk];
    if (staged)
      rows_ht_chunk_staged<MP, kRowsChunk, MAXG>(stage, W, G, r, row, j0, n, pg, Cs, hr, hi);
    else
      rows_ht_chunk<MP, kRowsChunk>(row, j0, n, pg, Cs, Gr, gq, hr, hi);
#pragma unroll
    for (int jj = 0; jj < kRowsChunk; ++jj) S.u.ht[r][jj] = make_float2(hr[jj], hi[jj]);
    wave_sync();
#pragma unroll
    for (int jj = 0; jj < kRowsChunk; ++jj) hr[jj] = hi[jj] = 0.f;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
#pragma unroll
      for (int jj = 0; jj < kRowsChunk; jj += 2) {
        const float4 h = *reinterpret_cast<const float4*>(&S.u.ht[j][jj]);
        hr[jj] += er[j] * h.x - ei[j] * h.y;
        hi[jj] += er[j] * h.y + ei[j] * h.x;
        hr[jj + 1] += er[j] * h.z - ei[j] * h.w;
        hi[jj + 1] += er[j] * h.w + ei[j] * h.z;
      }
    }
    if (valid && row) {
#pragma unroll
      for (int jj = 0; jj < kRowsChunk; ++jj)
        if (j0 + jj < n) gH[j0 + jj] = make_float2(hr[jj], hi[jj]);
    }
    wave_sync();
  }
  bits = rows_or<MP>(bits);
  if (valid && status && bits && r == 0) atomicOr(reinterpret_cast<unsigned int*>(status + c), bits);
}

// ---------------------------------------------------------------------------------------

template <int MP, int NS>
static gt_status rows_launch_t(const LaunchCtx& L, const RowsRange& R, int64_t total_sc,
                               const float2* C, const float2* G, const RowsSnr& a, float* out,
                               int ns_max, int32_t* status) {
  constexpr int SPB = 256 / MP;
  const unsigned grid = (unsigned)((R.count + SPB - 1) / SPB);
  prof_begin("k_sinr_rows", L.stream);
  hipLaunchKernelGGL((k_sinr_rows<MP, NS>), dim3(grid), dim3(256), 0, L.stream, L.d_chans, R,
                     total_sc, C, G, a, out, ns_max, status);
  prof_end(L.stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error_detail("k_sinr_rows", e);
    return GT_ERR_HIP;
  }
  return GT_OK;
}

// The compressed SINR of the classes [k0, k1) on the row-parallel kernel (m <= mp <= 8,
// ns <= nsm).
gt_status launch_sinr_rows(const LaunchCtx& L, int k0, int k1, int mp, int nsm, int64_t total_sc,
                           const float2* C, const float2* G, const float* s2, int n_snr,
                           float* out, int ns_max, int32_t* status) {
  RowsRange R;
  const int j0 = L.sc_j[k0], j1 = L.sc_j[k1];
  R.ch = L.d_sc_ch + j0;
  R.off = L.d_sc_off + j0;
  R.n = j1 - j0;
  R.base = L.sc_base[k0];
  R.count = L.sc_base[k1] - L.sc_base[k0];
  if (R.count == 0) return GT_OK;
  RowsSnr a{};
  a.n = n_snr;
  for (int k = 0; k < n_snr; ++k) a.s2[k] = s2[k];
  if (mp <= 4) {
    if (nsm <= 2) return rows_launch_t<4, 2>(L, R, total_sc, C, G, a, out, ns_max, status);
    return rows_launch_t<4, 4>(L, R, total_sc, C, G, a, out, ns_max, status);
  }
  if (nsm <= 4) return rows_launch_t<8, 4>(L, R, total_sc, C, G, a, out, ns_max, status);
  return rows_launch_t<8, 8>(L, R, total_sc, C, G, a, out, ns_max, status);
}


template <int MP, int NS>
static gt_status rows_bwd_launch_t(const LaunchCtx& L, const RowsRange& R, int64_t total_sc,
                                   const float2* C, const float2* G, const RowsSnr& a,
                                   const float* gs, int ns_max, int32_t* status) {
  constexpr int SPB = 256 / MP;
  const unsigned grid = (unsigned)((R.count + SPB - 1) / SPB);
  prof_begin("k_sinr_bwd_rows", L.stream);
  hipLaunchKernelGGL((k_sinr_bwd_rows<MP, NS>), dim3(grid), dim3(256), 0, L.stream, L.d_chans, R,
                     total_sc, C, G, a, gs, ns_max, L.ws, status);
  prof_end(L.stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error_detail("k_sinr_bwd_rows", e);
    return GT_ERR_HIP;
  }
  return GT_OK;
}

// dl/dHt of the classes [k0, k1) on the row-parallel adjoint (m <= mp, ns <= nsm) into the
// workspace.
gt_status launch_sinr_bwd_rows(const LaunchCtx& L, int k0, int k1, int mp, int nsm,
                               int64_t total_sc, const float2* C, const float2* G, const float* s2,
                               int n_snr, const float* gsinr, int ns_max, int32_t* status) {
  RowsRange R;
  const int j0 = L.sc_j[k0], j1 = L.sc_j[k1];
  R.ch = L.d_sc_ch + j0;
  R.off = L.d_sc_off + j0;
  R.n = j1 - j0;
  R.base = L.sc_base[k0];
  R.count = L.sc_base[k1] - L.sc_base[k0];
  if (R.count == 0) return GT_OK;
  RowsSnr a{};
  a.n = n_snr;
  for (int k = 0; k < n_snr; ++k) a.s2[k] = s2[k];
  if (mp <= 4) {
    if (nsm <= 2) return rows_bwd_launch_t<4, 2>(L, R, total_sc, C, G, a, gsinr, ns_max, status);
    return rows_bwd_launch_t<4, 4>(L, R, total_sc, C, G, a, gsinr, ns_max, status);
  }
  if (nsm <= 4) return rows_bwd_launch_t<8, 4>(L, R, total_sc, C, G, a, gsinr, ns_max, status);
  return rows_bwd_launch_t<8, 8>(L, R, total_sc, C, G, a, gsinr, ns_max, status);
}

}  // namespace gt
