// Fused per-group kernels of the alternating sweep (Section 3.2, equations "update A",
// "update B", "update C" and "kernel"), used when a group's intermediates fit in LDS.
//
// k_fused_t reads a group's slices H_s once: T_s = H_s B and, for a C-step, Yh_s = A^H T_s and
// the group's mode-3 Gram.  After the batched mode-3 eigensolve, k_fused_z forms the A-step
// partial Gram from T and the new C (the C-step of sweep s and the A-step of sweep s+1 use the
// same B, so one pass over X serves both, in the algorithm's Gauss-Seidel order), or the cores.
//
// k_fused_b, one block per chunk of groups, reads the slices once more and accumulates
//   W_q = sum_s conj(C[s,q]) A^H H_s,   S2 partial += sum_{q} W_q^H W_q
// with the Gram tile of each thread in registers.
#include <hip/hip_runtime.h>

#include "gt_device.h"
#include "gt_internal.h"

namespace gt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ void k_reduce_S2(const DevChan* __restrict__ chans, char* ws);

// S3[s][t] = <Yh_s, Yh_t> for one group: 16 lanes per output read consecutive elements
// (conflict-free LDS access) and combine by shuffles.
__device__ __forceinline__ void group_gram_s3(const float2* Yh, float2* S3, int gs, int sz, int mn,
                                              int tid) {
  const int l16 = tid % 16;
  for (int o = tid / 16; o < gs * gs; o += 16) {
    const int s = o / gs, t = o % gs;
    float ar = 0.f, ai = 0.f;
    if (s < sz && t < sz)
      for (int e = l16; e < mn; e += 16) {
        const float2 x = Yh[s * mn + e], y = Yh[t * mn + e];
        ar += x.x * y.x + x.y * y.y;
        ai += x.y * y.x - x.x * y.y;
      }
#pragma unroll
    for (int d = 8; d > 0; d >>= 1) {
      ar += __shfl_xor(ar, d, 64);
      ai += __shfl_xor(ai, d, 64);
    }
    if (l16 == 0) S3[o] = make_float2(ar, ai);
  }
}

__device__ __forceinline__ float2* wsp2(char* ws, int64_t off) {
  return reinterpret_cast<float2*>(ws + off);
}
__device__ __forceinline__ double* wsd2(char* ws, int64_t off) {
  return reinterpret_cast<double*>(ws + off);
}

// k_fused_t, one block per group: T_s = H_s B for the group's subcarriers (to the workspace)
// and, for a C-step, Yh_s = A^H T_s and the group's Gram S3[s,t] = <Yh_s, Yh_t>.
// do_c: 0 = T only; 1 = also Yh (in LDS) and S3; 2 = as 1 and Yh to the workspace (the
// cores of the last sweep read it).
__global__ void __launch_bounds__(256) k_fused_t(const DevChan* __restrict__ chans,
                                                  const GroupItem* __restrict__ items,
                                                  const float2* __restrict__ X,
                                                  const float2* __restrict__ A,
                                                  const float2* __restrict__ B, char* ws,
                                                  int do_c) {
  extern __shared__ float2 smem[];
  const GroupItem it = items[blockIdx.x];
  const DevChan& ch = chans[it.ch];
  const int nr = ch.nr, nt = ch.nt, m = ch.m, n = ch.n;
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  const int tid = threadIdx.x;
  float2* Bs = smem;                    // nt x n
  float2* As = Bs + nt * n;             // nr x m
  float2* Ts = As + nr * m;             // sz x nr x n
  float2* Yh = Ts + ch.gs * nr * n;     // sz x m x n
  for (int e = tid; e < nt * n; e += 256) Bs[e] = B[ch.b + e];
  for (int e = tid; e < nr * m; e += 256) As[e] = A[ch.a + e];
  __syncthreads();
  const float2* Xg = X + ch.x + (int64_t)s0 * nr * nt;
  float2* Tg = wsp2(ws, ch.w_T) + (int64_t)s0 * nr * n;
  float2* Xs = Yh + ch.gs * m * n;  // one slice, nr x nt
  constexpr int XPT = 4;            // nr * nt <= 1024
  float2 xn[XPT];
#pragma unroll
  for (int u = 0; u < XPT; ++u) {
    const int e = tid + 256 * u;
    xn[u] = e < nr * nt ? Xg[e] : make_float2(0.f, 0.f);
  }
  for (int s = 0; s < sz; ++s) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int e = tid + 256 * u;
      if (e < nr * nt) Xs[e] = xn[u];
    }
    __syncthreads();
    if (s + 1 < sz) {
#pragma unroll
      for (int u = 0; u < XPT; ++u) {
        const int e = tid + 256 * u;
        if (e < nr * nt) xn[u] = Xg[(int64_t)(s + 1) * nr * nt + e];
      }
    }
    // T_s[i][b] = sum_j H_s[i][j] B[j][b]
    for (int o = tid; o < nr * n; o += 256) {
      const int b = o % n, i = o / n;
      const float2* row = Xs + i * nt;
      float ar0 = 0.f, ai0 = 0.f, ar1 = 0.f, ai1 = 0.f;
      int j = 0;
      for (; j + 2 <= nt; j += 2) {
        float2 x0 = row[j], x1 = row[j + 1];
        float2 b0 = Bs[j * n + b], b1 = Bs[(j + 1) * n + b];
        ar0 += x0.x * b0.x - x0.y * b0.y;
        ai0 += x0.x * b0.y + x0.y * b0.x;
        ar1 += x1.x * b1.x - x1.y * b1.y;
        ai1 += x1.x * b1.y + x1.y * b1.x;
      }
      for (; j < nt; ++j) {
        float2 x0 = row[j], b0 = Bs[j * n + b];
        ar0 += x0.x * b0.x - x0.y * b0.y;
        ai0 += x0.x * b0.y + x0.y * b0.x;
      }
      const float2 v = make_float2(ar0 + ar1, ai0 + ai1);
      Ts[s * nr * n + o] = v;
      Tg[(int64_t)s * nr * n + o] = v;
    }
  }
  if (!do_c) return;
  __syncthreads();
  float2* Yg = wsp2(ws, ch.w_Yh) + (int64_t)s0 * m * n;
  for (int o = tid; o < sz * m * n; o += 256) {
    const int b = o % n;
    const int a = (o / n) % m;
    const int s = o / (m * n);
    Cx<float> acc{0.f, 0.f};
    for (int i = 0; i < nr; ++i) cfmac(acc, ld(As + i * m + a), ld(Ts + (s * nr + i) * n + b));
    const float2 v = make_float2(acc.re, acc.im);
    Yh[o] = v;
    if (do_c == 2) Yg[o] = v;
  }
  __syncthreads();
  group_gram_s3(Yh, wsp2(ws, ch.w_S3) + (int64_t)it.g * ch.gs * ch.gs, ch.gs, sz, m * n, tid);
}

// The group's mode-3 Gram on matrix cores, for gs <= 16 and m n a multiple of 8, by four waves:
// the real Gram P = R^T R of the mn x 32 matrix R[e][c] = Re Yh_c[e] (c < gs), Im Yh_{c-gs}[e]
// (gs <= c < 2 gs), zero for other c and for subcarriers past the group, with the mn entries
// split over the waves (32 x 32 x 2 products, one operand register for both sides).  The
// waves' partials go through `part` (4 x 1024 floats, which may alias Yh: the waves are past
// their reads of Yh before it is written), then S3[s][t] = sum_e Yh_s[e] conj(Yh_t[e]) =
// (P[s][t] + P[gs+s][gs+t]) + i (P[gs+s][t] - P[s][gs+t]).  Yh rows start ys apart.
__device__ __forceinline__ void group_gram_s3_mfma(const float2* Yh, int ys, float* part, float2* S3,
                                                   int gs, int sz, int mn, int tid) {
  const int wave = tid / 64, lane = tid % 64, c = lane % 32, h = lane / 32;
  const int sl = c < gs ? c : c - gs;
  const bool live = c < 2 * gs && sl < sz;
  const float* yb = reinterpret_cast<const float*>(Yh + (live ? sl : 0) * ys) + (c < gs ? 0 : 1);
  const int kq = mn / 4, e0 = wave * kq;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int k = 0; k < kq; k += 2) {
    const float v0 = yb[2 * (e0 + k + h)];
    const float v = live ? v0 : 0.f;
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(v, v, acc, 0, 0, 0);
  }
  __syncthreads();  // every wave has read its entries of Yh
  // accumulator layout: lane l, register r -> row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
#pragma unroll
  for (int r = 0; r < 16; ++r) part[wave * 1024 + (8 * (r / 4) + 4 * h + (r % 4)) * 32 + c] = acc[r];
  __syncthreads();
  auto P = [&](int i, int j) {
    const int o = i * 32 + j;
    return (part[o] + part[1024 + o]) + (part[2048 + o] + part[3072 + o]);
  };
  for (int o = tid; o < gs * gs; o += 256) {
    const int s = o / gs, t = o - s * gs;
    S3[o] = make_float2(P(s, t) + P(gs + s, gs + t), P(gs + s, t) - P(s, gs + t));
  }
}

// The part of the T pass after the product: T (accumulators of 32 x 32 tiles over rows (s, i)
// and the 2 n real columns) to LDS and the workspace, then for a C-step Yh = A^H T and the
// group's mode-3 Gram.
// yh_cap: complex elements of LDS from Yh on that the caller owns (the matrix-core Gram writes
// its partials there).
template <int TPW>
__device__ __forceinline__ void fused_t_finish(const DevChan& ch, const GroupItem& it, int s0, int sz,
                                               int rows, int ntile, float2* Ts, float2* Yh,
                                               int yh_cap, const float2* As, char* ws, int do_c,
                                               f32x16 (&acc)[TPW], int wave, int half, int col,
                                               int tid) {
  const int nr = ch.nr, m = ch.m, n = ch.n;
  const int mode = do_c & T_MODE;
  // accumulator element (row 8 (r / 4) + 4 half + r % 4, column col) of tile -> T
  float2* Tg = wsp2(ws, ch.w_T) + (int64_t)s0 * nr * n;
  float* Tsf = reinterpret_cast<float*>(Ts);
  float* Tgf = reinterpret_cast<float*>(Tg);
  const bool keep_t = (do_c & T_NO_STORE) == 0;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int tile = wave + 4 * u;
    if (tile < ntile && col < 2 * n) {
      const int c = col < n ? col : col - n;
      const int part = col < n ? 0 : 1;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = tile * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        if (row < rows) {
          Tsf[2 * (row * n + c) + part] = acc[u][r];
          if (keep_t) Tgf[2 * (row * n + c) + part] = acc[u][r];
        }
      }
    }
  }
  if (!mode) return;
  __syncthreads();
  float2* Yg = wsp2(ws, ch.w_Yh) + (int64_t)s0 * m * n;
  const int ys = m * n + 2;  // LDS stride of Yh_s (complex): consecutive subcarriers 4 banks apart
  if ((do_c & T_GRAM_OF_T) && mode == 1 && m == nr) {
    // A square and unitary: <Yh_s, Yh_t> = <T_s, T_t>, so the Gram is taken of T itself
    // (copied to the padded Yh layout) and Yh is not formed
    const int mn = m * n;
    for (int e = tid; e < sz * mn; e += 256) {
      const int s = e / mn;
      Yh[s * ys + (e - s * mn)] = Ts[e];
    }
  } else if (m <= 8 && n <= 16 && nr <= 16) {
    // Yh_s = A^H T_s on 16 x 16 x 4 matrix cores, one subcarrier per wave at a time: rows
    // (a, re/im), columns b, K = (i, re/im) in steps of 4 (lane l: row / column l % 16,
    // k' = 4 t + l / 16); the A operand is the sign-arranged real form of A^H
    const int lane = tid % 64, r16 = lane % 16, k4 = lane / 16;
    const int nst = (nr + 1) / 2;
    const float* Tsf = reinterpret_cast<const float*>(Ts);
    float* Yhf = reinterpret_cast<float*>(Yh);
    float* Ygf = reinterpret_cast<float*>(Yg);
    float aop[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int kk = 4 * t + k4, i = kk >> 1, kp = kk & 1, a = r16 >> 1, pp = r16 & 1;
      const float2 av = As[min(i, nr - 1) * m + min(a, m - 1)];
      const float v = pp == 0 ? (kp == 0 ? av.x : av.y) : (kp == 0 ? -av.y : av.x);
      aop[t] = (t < nst && a < m && i < nr) ? v : 0.f;
    }
    for (int s = wave; s < sz; s += 4) {
      f32x4 acc4;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc4[r] = 0.f;
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (t < nst) {
          const int kk = 4 * t + k4, i = kk >> 1;
          const float y = Tsf[2 * ((s * nr + min(i, nr - 1)) * n + min(r16, n - 1)) + (kk & 1)];
          acc4 = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[t], (i < nr && r16 < n) ? y : 0.f, acc4, 0, 0, 0);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * k4 + r, a = row >> 1;
        if (a < m && r16 < n) {
          const int o = 2 * ((s * m + a) * n + r16) + (row & 1);
          Yhf[2 * s * ys + o - 2 * s * m * n] = acc4[r];
          if (mode == 2) Ygf[o] = acc4[r];
        }
      }
    }
  } else {
    // a thread owns column b of one T_s (in registers) and forms all m rows
    for (int sb = tid; sb < sz * n; sb += 256) {
      const int s = sb / n, b = sb - s * n;
      float2 tc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i)
        tc[i] = i < nr ? Ts[(s * nr + i) * n + b] : make_float2(0.f, 0.f);
      for (int a = 0; a < m; ++a) {
        float yr = 0.f, yi = 0.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          if (i < nr) {
            const float2 av = As[i * m + a];
            yr += av.x * tc[i].x + av.y * tc[i].y;
            yi += av.x * tc[i].y - av.y * tc[i].x;
          }
        }
        const int o = (s * m + a) * n + b;
        Yh[s * ys + a * n + b] = make_float2(yr, yi);
        if (mode == 2) Yg[o] = make_float2(yr, yi);
      }
    }
  }
  __syncthreads();
  // S3[s][t] = <Yh_s, Yh_t>: on matrix cores split over the four waves where the shapes allow
  // (Yh sits in region 0, which also holds the waves' partials), else on the vector ALU on the
  // upper triangle (16 lanes per entry), mirrored below (zero where t is past the group)
  const int gs = ch.gs, mn = m * n;
  float2* S3 = wsp2(ws, ch.w_S3) + (int64_t)it.g * gs * gs;
  if (gs <= 16 && (mn & 7) == 0 && yh_cap >= 2048) {
    group_gram_s3_mfma(Yh, ys, reinterpret_cast<float*>(Yh), S3, gs, sz, mn, tid);
  } else {
    const int l16 = tid % 16;
    for (int k = tid / 16; k < gs * (gs + 1) / 2; k += 16) {
      int s = 0, rem = k;
      while (rem >= gs - s) {
        rem -= gs - s;
        ++s;
      }
      const int t = s + rem;
      float ar = 0.f, ai = 0.f;
      if (t < sz) {
#pragma unroll 8
        for (int e = l16; e < mn; e += 16) {
          const float2 x = Yh[s * ys + e], y = Yh[t * ys + e];
          ar += x.x * y.x + x.y * y.y;
          ai += x.y * y.x - x.x * y.y;
        }
      }
#pragma unroll
      for (int d = 8; d > 0; d >>= 1) {
        ar += __shfl_xor(ar, d, 64);
        ai += __shfl_xor(ai, d, 64);
      }
      if (l16 == 0) {
        S3[s * gs + t] = make_float2(ar, ai);
        if (t != s) S3[t * gs + s] = make_float2(ar, -ai);
      }
    }
  }
}

// Matrix-core variant of k_fused_t.  Stacking the group's rows (s, i) of H gives
// T = H B as one complex (sz nr) x nt by nt x n product.  In real form the K index runs over
// (j, re/im) pairs, k' = 2 j + part, which matches the interleaved storage of H, and
//   A[(s,i)][k'] = (part 0: Re H, part 1: Im H)[s][i][j]
//   Bt[k'][c]    = part 0: (c < n: Re B[j][c], else Im B[j][c - n])
//                  part 1: (c < n: -Im B[j][c], else Re B[j][c - n])
// so that the real product A Bt is [Re T | Im T].  Output tiles are 32 x 32 over rows
// (s, i) and the 2 n real columns (n <= 16: one column tile); tile r goes to wave r % 4.  The
// bounds ask for four resident blocks per CU (at most 128 registers): without them the
// accumulators went to 32 extra AGPRs, three blocks fitted, and the pass took 25 % longer.
template <int TPW>
__global__ void __launch_bounds__(256, 4) k_fused_t_mfma(const DevChan* __restrict__ chans,
                                                      const GroupItem* __restrict__ items,
                                                      const float2* __restrict__ X,
                                                      const float2* __restrict__ A,
                                                      const float2* __restrict__ B, char* ws,
                                                      int do_c) {
  extern __shared__ float2 smem[];
  const GroupItem it = items[blockIdx.x];
  const DevChan& ch = chans[it.ch];
  const int nr = ch.nr, nt = ch.nt, m = ch.m, n = ch.n;
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  // region 0 holds the real-form B ([2 nt][32] floats) for the product and Yh (sz x m x n)
  // afterwards
  const int reg0 = max(nt * 32, ch.gs * (m * n + 2));
  float* Bt = reinterpret_cast<float*>(smem);
  float2* Yh = smem;
  float2* As = smem + reg0;                           // nr x m
  float2* Ts = As + nr * m;                           // sz x nr x n
  const int rows = sz * nr;
  const int ntile = (rows + 31) / 32;
  const float* Xf = reinterpret_cast<const float*>(X + ch.x + (int64_t)s0 * nr * nt);
  const int half = lane / 32, col = lane % 32;
  // K order: with nt % 4 == 0 and 16-byte aligned rows, step 4 u + v takes real index
  // k' = 8 u + 4 half + v in lane half, so each lane reads 16 contiguous bytes per four steps
  // (the same permutation indexes Bt); otherwise k' = 2 j + half.
  const bool vec4 = (nt % 4) == 0 && ((reinterpret_cast<uintptr_t>(Xf) & 15) == 0);
  // nt = 64, one tile per wave: the lane's whole half-row (16 x 16 bytes) is requested first,
  // so that its latency overlaps the staging of B
  const bool whole = TPW == 1 && vec4 && nt == 64;
  float4 a4[16];
  if (whole) {
    const int row = min(wave * 32 + col, rows - 1);
    const float4* xrow4 = reinterpret_cast<const float4*>(Xf + (int64_t)row * 2 * nt);
#pragma unroll
    for (int w = 0; w < 16; ++w) a4[w] = xrow4[2 * w + half];
  }
  {
    // all loads of the real-form B are issued before any is used (clamped indices)
    constexpr int NE = 2 * 64 * 32 / 256;
    float2 bv[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = tid + 256 * k, kk = e / 32, c = e % 32;
      const int j = min(kk / 2, nt - 1), cc = min(c < n ? c : c - n, n - 1);
      bv[k] = B[ch.b + j * n + max(cc, 0)];
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = tid + 256 * k, kk = e / 32, c = e % 32, part = kk % 2;
      float v = (part == 0) ? (c < n ? bv[k].x : bv[k].y) : (c < n ? -bv[k].y : bv[k].x);
      if (c >= 2 * n) v = 0.f;
      if (e < 2 * nt * 32) Bt[e] = v;
    }
  }
  for (int e = tid; e < nr * m; e += 256) As[e] = A[ch.a + e];
  __syncthreads();
  f32x16 acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[u][r] = 0.f;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int tile = wave + 4 * u;
    if (tile < ntile) {
      const int row = tile * 32 + col;
      const bool rv = row < rows;
      if (whole) {
        // products alternate between two accumulators
        const float* bcol = Bt + 4 * half * 32 + col;
        f32x16 acc_b;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc_b[r] = 0.f;
#pragma unroll
        for (int w = 0; w < 16; w += 2) {
          const float* bw = bcol + 8 * w * 32;
          const float4 x0 = rv ? a4[w] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float4 x1 = rv ? a4[w + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, bw[0], acc[u], 0, 0, 0);
          acc_b = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.x, bw[256], acc_b, 0, 0, 0);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.y, bw[32], acc[u], 0, 0, 0);
          acc_b = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.y, bw[288], acc_b, 0, 0, 0);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.z, bw[64], acc[u], 0, 0, 0);
          acc_b = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.z, bw[320], acc_b, 0, 0, 0);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.w, bw[96], acc[u], 0, 0, 0);
          acc_b = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.w, bw[352], acc_b, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[u][r] += acc_b[r];
      } else if (vec4) {
        const float4* xrow4 = reinterpret_cast<const float4*>(Xf + (int64_t)(rv ? row : 0) * 2 * nt);
        const float* bcol = Bt + 4 * half * 32 + col;
#pragma unroll 2
        for (int w = 0; w < nt / 4; ++w) {
          const float4 a4 = rv ? xrow4[2 * w + half] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float* bw = bcol + 8 * w * 32;
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, bw[0], acc[u], 0, 0, 0);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, bw[32], acc[u], 0, 0, 0);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, bw[64], acc[u], 0, 0, 0);
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, bw[96], acc[u], 0, 0, 0);
        }
      } else {
        const float* xrow = Xf + (int64_t)(rv ? row : 0) * 2 * nt + half;
        const float* bcol = Bt + half * 32 + col;
#pragma unroll 8
        for (int j = 0; j < nt; ++j) {
          const float av = rv ? xrow[2 * j] : 0.f;
          const float bv = bcol[j * 64];
          acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[u], 0, 0, 0);
        }
      }
    }
  }
  fused_t_finish<TPW>(ch, it, s0, sz, rows, ntile, Ts, Yh, reg0, As, ws, do_c, acc, wave, half, col,
                      tid);
}

// ---------------------------------------------------------------------------------------
// 16-bit contraction operands (precision form).  PREC 1: BF16, 2: FP16, 3: split BF16
// (x = hi + lo with hi = bf16(x), lo = bf16(x - hi); products hi hi + hi lo + lo hi).  The
// products accumulate in FP32 on 32 x 32 x 8 matrix cores; operand lane layout: lane l holds
// A[l % 32][4 (l / 32) + v] and B[4 (l / 32) + v][l % 32], v = 0..3.
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {  // round to nearest even
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }
__device__ __forceinline__ unsigned short f2h(float x) {
  return __builtin_bit_cast(unsigned short, (_Float16)x);
}
template <int PREC>
__device__ __forceinline__ unsigned short q_hi(float x) { return PREC == 2 ? f2h(x) : f2bf(x); }
template <int PREC>
__device__ __forceinline__ unsigned short q_lo(float x) {
  return PREC == 3 ? f2bf(x - bf2f(f2bf(x))) : (unsigned short)0;
}

template <int PREC>
__device__ __forceinline__ f32x16 mfma16(s16x4 a, s16x4 b, f32x16 c) {
  if constexpr (PREC == 2)
    return __builtin_amdgcn_mfma_f32_32x32x8f16(__builtin_bit_cast(f16x4, a), __builtin_bit_cast(f16x4, b),
                                                 c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ s16x4 pack4(unsigned short a, unsigned short b, unsigned short c,
                                       unsigned short d) {
  s16x4 v;
  v[0] = (short)a;
  v[1] = (short)b;
  v[2] = (short)c;
  v[3] = (short)d;
  return v;
}

// 16-bit copy of each channel's X in the workspace, same element order (hi, then lo for the
// split form).
template <int PREC>
__global__ void __launch_bounds__(256) k_convert_x(const DevChan* __restrict__ chans,
                                                   const float2* __restrict__ X, char* ws) {
  const DevChan& ch = chans[blockIdx.y];
  const int64_t total = (int64_t)ch.nsc * ch.nr * ch.nt;
  unsigned short* hi = reinterpret_cast<unsigned short*>(ws + ch.w_Xq);
  unsigned short* lo = hi + 2 * total;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const float2 v = X[ch.x + e];
    const unsigned short hr = q_hi<PREC>(v.x), hm = q_hi<PREC>(v.y);
    *reinterpret_cast<ushort2*>(hi + 2 * e) = make_ushort2(hr, hm);
    if (PREC == 3) *reinterpret_cast<ushort2*>(lo + 2 * e) = make_ushort2(q_lo<PREC>(v.x), q_lo<PREC>(v.y));
  }
}

// Precision-form T pass: T = H B on 16-bit operands (one 32-row tile per wave, nt % 4 == 0),
// then the same finish as the FP32 pass.  B is staged in LDS in real form as [32 c][2 nt k'].
template <int PREC>
__global__ void __launch_bounds__(256) k_fused_t_lp(const DevChan* __restrict__ chans,
                                                    const GroupItem* __restrict__ items,
                                                    const float2* __restrict__ A,
                                                    const float2* __restrict__ B, char* ws,
                                                    int do_c) {
  extern __shared__ float2 smem[];
  const GroupItem it = items[blockIdx.x];
  const DevChan& ch = chans[it.ch];
  const int nr = ch.nr, nt = ch.nt, m = ch.m, n = ch.n;
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int half = lane / 32, col = lane % 32;
  constexpr int NQ = PREC == 3 ? 2 : 1;
  unsigned short* Bq = reinterpret_cast<unsigned short*>(smem);  // [NQ][32][2 nt]
  float2* As = smem + NQ * 32 * 2 * nt * 2 / 8;                 // nr x m
  float2* Ts = As + nr * m;
  float2* Yh = Ts + ch.gs * nr * n;
  const int rows = sz * nr;
  const int ntile = (rows + 31) / 32;
  const int64_t xtot = (int64_t)ch.nsc * nr * nt;
  const unsigned short* Xh = reinterpret_cast<const unsigned short*>(ws + ch.w_Xq);
  const int K8 = 2 * nt / 8;  // K steps of 8 real indices
  // the lane's half-row: K index k' = 8 t + 4 half + v, 8 contiguous bytes per step
  const int row = min(wave * 32 + col, rows - 1);
  const bool rv = wave * 32 + col < rows;
  const uint2* xr = reinterpret_cast<const uint2*>(Xh + 2 * ((int64_t)s0 * nr * nt + (int64_t)row * nt));
  uint2 ah[16], al[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    ah[t] = t < K8 ? xr[2 * t + half] : make_uint2(0u, 0u);
    if (PREC == 3) al[t] = t < K8 ? xr[2 * t + half + xtot / 2] : make_uint2(0u, 0u);
  }
  for (int e = tid; e < 32 * 2 * nt; e += 256) {
    const int c = e / (2 * nt), kk = e % (2 * nt), j = kk / 2, part = kk % 2;
    float v = 0.f;
    if (c < 2 * n) {
      const float2 b = B[ch.b + j * n + (c < n ? c : c - n)];
      v = (part == 0) ? (c < n ? b.x : b.y) : (c < n ? -b.y : b.x);
    }
    Bq[e] = q_hi<PREC>(v);
    if (PREC == 3) Bq[32 * 2 * nt + e] = q_lo<PREC>(v);
  }
  for (int e = tid; e < nr * m; e += 256) As[e] = A[ch.a + e];
  __syncthreads();
  f32x16 acc[1];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[0][r] = 0.f;
  if (wave < ntile) {
    const uint2* bq = reinterpret_cast<const uint2*>(Bq + col * 2 * nt) + half;
    const uint2* bl = reinterpret_cast<const uint2*>(Bq + 32 * 2 * nt + col * 2 * nt) + half;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      if (t < K8) {
        const uint2 a2 = rv ? ah[t] : make_uint2(0u, 0u);
        const uint2 b2 = bq[2 * t];
        const s16x4 a = __builtin_bit_cast(s16x4, a2), b = __builtin_bit_cast(s16x4, b2);
        acc[0] = mfma16<PREC>(a, b, acc[0]);
        if (PREC == 3) {
          const uint2 a2l = rv ? al[t] : make_uint2(0u, 0u);
          const uint2 b2l = bl[2 * t];
          acc[0] = mfma16<PREC>(a, __builtin_bit_cast(s16x4, b2l), acc[0]);
          acc[0] = mfma16<PREC>(__builtin_bit_cast(s16x4, a2l), b, acc[0]);
        }
      }
    }
  }
  fused_t_finish<1>(ch, it, s0, sz, rows, ntile, Ts, Yh, ch.gs * (m * n + 2), As, ws, do_c, acc, wave,
                    half, col, tid);
}

// k_fused_z, one block per group, after the mode-3 eigensolve: the A-step partial Gram
// S1 = sum_q Z_q Z_q^H with Z_q = sum_s conj(C[s,q]) T_s, and/or the cores
// G_g[q] = sum_s conj(C[s,q]) Yh_s.
__global__ void __launch_bounds__(256) k_fused_z(const DevChan* __restrict__ chans,
                                                  const GroupItem* __restrict__ items,
                                                  const float2* __restrict__ C, float2* G,
                                                  char* ws, int do_a, int do_core) {
  extern __shared__ float2 smem[];
  const GroupItem it = items[blockIdx.x];
  const DevChan& ch = chans[it.ch];
  const int nr = ch.nr, m = ch.m, n = ch.n, p = ch.p;
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  const int pg = min(p, sz);
  const int tid = threadIdx.x;
  float2* Cs = smem;             // sz x p
  float2* Zs = Cs + ch.gs * p;   // p x nr x n
  for (int e = tid; e < sz * p; e += 256) Cs[e] = C[ch.c + (int64_t)s0 * p + e];
  __syncthreads();
  if (do_a) {
    // a thread owns entry e of T_s for QC consecutive q: each T entry is read from memory once
    // per chunk of q, not once per q
    const float2* Tg = wsp2(ws, ch.w_T) + (int64_t)s0 * nr * n;
    constexpr int QC = 6;
    const int nrn = nr * n, nqc = (pg + QC - 1) / QC;
    for (int o = tid; o < nqc * nrn; o += 256) {
      const int qc = o / nrn, e = o - qc * nrn;
      Cx<float> z[QC];
#pragma unroll
      for (int j = 0; j < QC; ++j) z[j] = Cx<float>{0.f, 0.f};
      // the T entries of four subcarriers are loaded before their products
      constexpr int SU = 4;
      int s = 0;
      for (; s + SU <= sz; s += SU) {
        Cx<float> tv[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) tv[u] = ld(Tg + (s + u) * nrn + e);
#pragma unroll
        for (int u = 0; u < SU; ++u)
#pragma unroll
          for (int j = 0; j < QC; ++j)
            if (qc * QC + j < pg) cfmac(z[j], ld(Cs + (s + u) * p + qc * QC + j), tv[u]);
      }
      for (; s < sz; ++s) {
        const Cx<float> tv = ld(Tg + s * nrn + e);
#pragma unroll
        for (int j = 0; j < QC; ++j)
          if (qc * QC + j < pg) cfmac(z[j], ld(Cs + s * p + qc * QC + j), tv);
      }
#pragma unroll
      for (int j = 0; j < QC; ++j)
        if (qc * QC + j < pg) Zs[(qc * QC + j) * nrn + e] = make_float2(z[j].re, z[j].im);
    }
    __syncthreads();
    // S1[i][k] = sum_{q, b} Z_q[i][b] conj(Z_q[k][b]); four threads per output split b, in
    // passes of 64 outputs (nr up to 16: 256 outputs).  The four threads of an output are
    // aligned lanes of one pass, so they stay active together for the shuffles.
    for (int o4 = tid; o4 < 4 * nr * nr; o4 += 256) {
      const int o = o4 / 4, part = o4 % 4;
      const int i = o / nr, k = o % nr;
      float ar = 0.f, ai = 0.f;
      for (int q = 0; q < pg; ++q) {
        const float2* zq = Zs + q * nr * n;
        for (int b = part; b < n; b += 4) {
          float2 zi = zq[i * n + b], zk = zq[k * n + b];
          ar += zi.x * zk.x + zi.y * zk.y;
          ai += zi.y * zk.x - zi.x * zk.y;
        }
      }
      ar += __shfl_xor(ar, 1, 64);
      ai += __shfl_xor(ai, 1, 64);
      ar += __shfl_xor(ar, 2, 64);
      ai += __shfl_xor(ai, 2, 64);
      if (part == 0) wsp2(ws, ch.w_S1p)[(int64_t)it.g * nr * nr + o] = make_float2(ar, ai);
    }
  }
  if (do_core) {
    // a thread owns entry e of G_g[q] for QC consecutive q (each Yh entry is read once per
    // chunk of q) and loads the Yh entries of four subcarriers before their products; rows
    // q >= p_g are written as zero
    const int mn = m * n;
    const float2* Yg = wsp2(ws, ch.w_Yh) + (int64_t)s0 * mn;
    float2* Gg = G + ch.g + (int64_t)it.g * p * mn;
    constexpr int QC = 6, SU = 4;
    const int nqc = (p + QC - 1) / QC;
    for (int o = tid; o < nqc * mn; o += 256) {
      const int qc = o / mn, e = o - qc * mn;
      Cx<float> acc[QC];
#pragma unroll
      for (int j = 0; j < QC; ++j) acc[j] = Cx<float>{0.f, 0.f};
      int s = 0;
      for (; s + SU <= sz; s += SU) {
        Cx<float> yv[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) yv[u] = ld(Yg + (s + u) * mn + e);
#pragma unroll
        for (int u = 0; u < SU; ++u)
#pragma unroll
          for (int j = 0; j < QC; ++j)
            if (qc * QC + j < pg) cfmac(acc[j], ld(Cs + (s + u) * p + qc * QC + j), yv[u]);
      }
      for (; s < sz; ++s) {
        const Cx<float> yv = ld(Yg + s * mn + e);
#pragma unroll
        for (int j = 0; j < QC; ++j)
          if (qc * QC + j < pg) cfmac(acc[j], ld(Cs + s * p + qc * QC + j), yv);
      }
#pragma unroll
      for (int j = 0; j < QC; ++j)
        if (qc * QC + j < p) Gg[(int64_t)(qc * QC + j) * mn + e] = make_float2(acc[j].re, acc[j].im);
    }
  }
}

// ---------------------------------------------------------------------------------------

// one block per (chunk of groups, channel); 4 x 4 tile of the nt x nt Gram per thread
__global__ void __launch_bounds__(256) k_fused_b(const DevChan* __restrict__ chans,
                                                  const float2* __restrict__ X,
                                                  const float2* __restrict__ A,
                                                  const float2* __restrict__ C, char* ws) {
  extern __shared__ float2 Ws[];  // [p*m][nt] of the current group, then A and C rows
  const DevChan& ch = chans[blockIdx.y];
  const int split = blockIdx.x;
  if (split >= ch.nsplit) return;
  const int nr = ch.nr, nt = ch.nt, m = ch.m, p = ch.p;
  float2* As = Ws + p * m * nt;  // nr x m
  float2* Cs = As + nr * m;      // gs x p
  const int g0 = (int)((int64_t)split * ch.ngroups / ch.nsplit);
  const int g1 = (int)((int64_t)(split + 1) * ch.ngroups / ch.nsplit);
  const int tid = threadIdx.x;
  const int bi = (tid / 16) * 4, bj = (tid % 16) * 4;
  float ar[4][4], ai[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) ar[a][b] = ai[a][b] = 0.f;
  for (int e = tid; e < nr * m; e += 256) As[e] = A[ch.a + e];
  const int mnt = m * nt;
  for (int g = g0; g < g1; ++g) {
    const int s0 = g * ch.gs;
    const int sz = min(ch.gs, ch.nsc - s0);
    const int pg = min(p, sz);
    const float2* Xg = X + ch.x + (int64_t)s0 * nr * nt;
    for (int e = tid; e < sz * p; e += 256) Cs[e] = C[ch.c + (int64_t)s0 * p + e];
    __syncthreads();
    // W[q][a][j] for the (a, j) pairs of this thread, accumulated over s in registers
    for (int aj = tid; aj < mnt; aj += 256) {
      const int a = aj / nt, j = aj % nt;
      float wr[kMaxGroup], wi[kMaxGroup];
#pragma unroll
      for (int q = 0; q < kMaxGroup; ++q) wr[q] = wi[q] = 0.f;
      for (int s = 0; s < sz; ++s) {
        float yr = 0.f, yi = 0.f;  // Y_s[a][j] = sum_i conj(A[i][a]) H_s[i][j]
        const float2* xs = Xg + (int64_t)s * nr * nt + j;
        for (int i = 0; i < nr; ++i) {
          const float2 av = As[i * m + a];
          const float2 xv = xs[(int64_t)i * nt];
          yr += av.x * xv.x + av.y * xv.y;
          yi += av.x * xv.y - av.y * xv.x;
        }
        const float2* Cr = Cs + s * p;
#pragma unroll
        for (int q = 0; q < kMaxGroup; ++q) {
          if (q < pg) {  // conj(C[s,q]) y
            const float2 cv = Cr[q];
            wr[q] += cv.x * yr + cv.y * yi;
            wi[q] += cv.x * yi - cv.y * yr;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < kMaxGroup; ++q)
        if (q < p) Ws[(q * m + a) * nt + j] = (q < pg) ? make_float2(wr[q], wi[q]) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    // Gram tile: sum over rows (q, a) of conj(W[row][bi+x]) W[row][bj+y]
    if (bi < nt && bj < nt) {
      const int rows = pg * m;
      for (int row = 0; row < rows; ++row) {
        const float2* w = Ws + row * nt;
        float xr[4], xi[4], yr[4], yi[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          float2 u = (bi + x < nt) ? w[bi + x] : make_float2(0.f, 0.f);
          float2 v = (bj + x < nt) ? w[bj + x] : make_float2(0.f, 0.f);
          xr[x] = u.x;
          xi[x] = u.y;
          yr[x] = v.x;
          yi[x] = v.y;
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) {
            ar[x][y] += xr[x] * yr[y] + xi[x] * yi[y];
            ai[x][y] += xr[x] * yi[y] - xi[x] * yr[y];
          }
      }
    }
    __syncthreads();
  }
  float2* P = wsp2(ws, ch.w_S2p) + (int64_t)split * nt * nt;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
      if (bi + x < nt && bj + y < nt) P[(bi + x) * nt + bj + y] = make_float2(ar[x][y], ai[x][y]);
}

// ---------------------------------------------------------------------------------------
// B-step pass with the mode-2 Gram on FP32 matrix cores.
//
// With R = [Re W | Im W] (rows (q, a), 2 * 64 columns, zero beyond nt), R^T R holds
// Re(W^H W) = R_re^T R_re + R_im^T R_im and Im(W^H W) = R_re^T R_im - R_im^T R_re in its
// blocks.  R^T R is symmetric, so only its 10 upper 32 x 32 tiles are accumulated (with
// v_mfma_f32_32x32x2f32, K = 2 rows per instruction) across the chunk's groups; the
// reduction kernel forms the complex Gram from the blocks.  Wave w owns tiles kTile[w].
__device__ __forceinline__ void tile_of(int w, int k, int& I, int& J) {
  // wave 0: (0,0) (0,1) (0,2); wave 1: (0,3) (1,1) (1,2); wave 2: (1,3) (2,2); wave 3: (2,3) (3,3)
  const int ti[4][3] = {{0, 0, 0}, {0, 1, 1}, {1, 2, -1}, {2, 3, -1}};
  const int tj[4][3] = {{0, 1, 2}, {3, 1, 2}, {3, 2, -1}, {3, 3, -1}};
  I = ti[w][k];
  J = tj[w][k];
}

template <int APER, int PMAX>
__global__ void __launch_bounds__(256) k_fused_b_mfma(const DevChan* __restrict__ chans,
                                                      const float2* __restrict__ X,
                                                      const float2* __restrict__ A,
                                                      const float2* __restrict__ C, char* ws) {
  extern __shared__ float smf[];
  const DevChan& ch = chans[blockIdx.y];
  const int split = blockIdx.x;
  if (split >= ch.nsplit) return;
  const int nr = ch.nr, nt = ch.nt, m = ch.m, p = ch.p;
  const int rowsmax = p * m + 1;
  float* Wre = smf;                          // [p*m + 1][64]
  float* Wim = Wre + rowsmax * 64;           // [p*m + 1][64]
  float2* Xs = reinterpret_cast<float2*>(Wim + rowsmax * 64);  // [nr][nt] of one subcarrier
  float2* As = Xs + nr * nt;                 // [nr][m]
  float2* Cs = As + nr * m;                  // [gs][p]
  const int g0 = (int)((int64_t)split * ch.ngroups / ch.nsplit);
  const int g1 = (int)((int64_t)(split + 1) * ch.ngroups / ch.nsplit);
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  for (int e = tid; e < nr * m; e += 256) As[e] = A[ch.a + e];
  f32x16 acc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;
  const int ntiles = wave < 2 ? 3 : 2;
  const int mnt = m * nt;
  for (int g = g0; g < g1; ++g) {
    const int s0 = g * ch.gs;
    const int sz = min(ch.gs, ch.nsc - s0);
    const int pg = min(p, sz);
    for (int e = tid; e < sz * p; e += 256) Cs[e] = C[ch.c + (int64_t)s0 * p + e];
    // W[q][a][j] = sum_s conj(C[s,q]) sum_i conj(A[i][a]) H_s[i][j], (a, j) pairs in registers
    float wr[APER][PMAX], wi[APER][PMAX];
#pragma unroll
    for (int u = 0; u < APER; ++u)
#pragma unroll
      for (int q = 0; q < PMAX; ++q) wr[u][q] = wi[u][q] = 0.f;
    // the slice of the next subcarrier is loaded into registers while this one is used
    constexpr int XPT = 4;  // nr * nt <= 1024 elements per slice
    float2 xn[XPT];
    {
      const float2* xs = X + ch.x + (int64_t)s0 * nr * nt;
#pragma unroll
      for (int u = 0; u < XPT; ++u) {
        const int e = tid + 256 * u;
        xn[u] = e < nr * nt ? xs[e] : make_float2(0.f, 0.f);
      }
    }
    for (int s = 0; s < sz; ++s) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < XPT; ++u) {
        const int e = tid + 256 * u;
        if (e < nr * nt) Xs[e] = xn[u];
      }
      __syncthreads();
      if (s + 1 < sz) {
        const float2* xs = X + ch.x + (int64_t)(s0 + s + 1) * nr * nt;
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
          const int e = tid + 256 * u;
          if (e < nr * nt) xn[u] = xs[e];
        }
      }
      const float2* Cr = Cs + s * p;
#pragma unroll
      for (int u = 0; u < APER; ++u) {
        const int aj = tid + 256 * u;
        if (aj < mnt) {
          const int a = aj / nt, j = aj % nt;
          float yr = 0.f, yi = 0.f;
          for (int i = 0; i < nr; ++i) {
            const float2 av = As[i * m + a], xv = Xs[i * nt + j];
            yr += av.x * xv.x + av.y * xv.y;
            yi += av.x * xv.y - av.y * xv.x;
          }
#pragma unroll
          for (int q = 0; q < PMAX; ++q) {
            if (q < pg) {
              const float2 cv = Cr[q];
              wr[u][q] += cv.x * yr + cv.y * yi;
              wi[u][q] += cv.x * yi - cv.y * yr;
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < APER; ++u) {
      const int aj = tid + 256 * u;
      if (aj < mnt) {
        const int a = aj / nt, j = aj % nt;
#pragma unroll
        for (int q = 0; q < PMAX; ++q)
          if (q < pg) {
            Wre[(q * m + a) * 64 + j] = wr[u][q];
            Wim[(q * m + a) * 64 + j] = wi[u][q];
          }
      }
    }
    // zero the padding columns j in [nt, 64) of the used rows
    if (nt < 64)
      for (int e = tid; e < pg * m * (64 - nt); e += 256) {
        const int row = e / (64 - nt), j = nt + e % (64 - nt);
        Wre[row * 64 + j] = 0.f;
        Wim[row * 64 + j] = 0.f;
      }
    __syncthreads();
    // R^T R on the matrix cores: rows (q, a) for q < pg, two rows per instruction; an odd
    // row count is padded with a zero row.  Each lane walks fixed column pointers.
    const int rows = pg * m;
    if (rows & 1) {
      for (int j = tid; j < 64; j += 256) {
        Wre[rows * 64 + j] = 0.f;
        Wim[rows * 64 + j] = 0.f;
      }
      __syncthreads();
    }
    const int half = lane / 32, col = lane % 32;
    const float* pa[3];
    const float* pb[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      int I = 0, J = 0;
      if (t < ntiles) tile_of(wave, t, I, J);
      const int ca = 32 * I + col, cb = 32 * J + col;
      pa[t] = (ca < 64 ? Wre + ca : Wim + (ca - 64)) + half * 64;
      pb[t] = (cb < 64 ? Wre + cb : Wim + (cb - 64)) + half * 64;
    }
    if (ntiles == 3) {
      for (int k0 = 0; k0 < rows; k0 += 2) {
        const int o = k0 * 64;
        const float a0 = pa[0][o], b0 = pb[0][o], a1 = pa[1][o], b1 = pb[1][o];
        const float a2 = pa[2][o], b2 = pb[2][o];
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, b2, acc[2], 0, 0, 0);
      }
    } else {
      for (int k0 = 0; k0 < rows; k0 += 2) {
        const int o = k0 * 64;
        const float a0 = pa[0][o], b0 = pb[0][o], a1 = pa[1][o], b1 = pb[1][o];
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // accumulator layout: lane l, register r -> row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
  float* P = reinterpret_cast<float*>(ws + ch.w_S2p) + (int64_t)split * 128 * 128;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (t < ntiles) {
      int I, J;
      tile_of(wave, t, I, J);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * I + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
        const int col = 32 * J + lane % 32;
        P[row * 128 + col] = acc[t][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// B-step pass with all three contractions on FP32 matrix cores, 8 waves per block.  Per
// group, in real form (each complex product split into re/im rows and columns):
//   1. Hc_q = sum_s conj(C[s,q]) H_s for q < p_g: rows (q, re/im), K over (s, re/im), N over
//      the nr nt entries (i, j) of a slice.  Those are contiguous in X, so the B operand is
//      read straight from HBM, coalesced.
//   2. W_q = A^H Hc_q: rows (a, re/im), K over (i, re/im), N over j (two 32-column tiles,
//      zero beyond nt).  Each wave takes whole q's and overwrites Hc_q by W_q (planar).
//   3. The real Gram R^T R of R = [Re W | Im W] on the 10 upper 32 x 32 tiles (two tiles
//      for waves 0 and 1, one for the others), accumulated over the block's groups.
// LDS holds one slot per q of max(2 nr nt, 2 m 64) floats and the step-2 A operand.
__host__ __device__ __forceinline__ int bmm_slot(int nr, int nt, int m) {
  const int a = 2 * nr * nt, b = 2 * m * 64;
  return a > b ? a : b;
}

// upper 32 x 32 tile k of the 128 x 128 real Gram: (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3)
// (2,2) (2,3) (3,3)
__device__ __forceinline__ void gram_tile(int k, int& I, int& J) {
  I = k < 4 ? 0 : (k < 7 ? 1 : (k < 9 ? 2 : 3));
  J = k < 4 ? k : (k < 7 ? k - 3 : (k < 9 ? k - 5 : 3));
}

// Step-1 operands of group g for this lane, loaded one group ahead: the real (h = 0) or
// imaginary (h = 1) part of slice s at column c = 32 (wave + 8 u) + lane % 32, and the
// component of C[s, q] that the A operand of row (q, part) = lane % 32 at K index (s, h)
// needs (its sign is applied at use).  Indices are clamped into the group so that every load
// is unconditional (no wait is forced inside the prefetch); rows q >= p_g, columns beyond
// nr nt and slices s >= size_g only reach outputs that are never stored or MFMAs that are
// skipped.
template <int NT1W, int SMAX>
__device__ __forceinline__ void bmm_prefetch(float (&xp)[SMAX][NT1W], float (&cp)[SMAX],
                                             const float2* __restrict__ X,
                                             const float2* __restrict__ C, const DevChan& ch,
                                             int g, int nrnt, int wave, int col, int h) {
  const int s0 = g * ch.gs, sz = min(ch.gs, ch.nsc - s0);
  const int pg = min(ch.p, sz);
  const float* xg = reinterpret_cast<const float*>(X + ch.x + (int64_t)s0 * nrnt) + h;
  const int q = min(col >> 1, pg - 1), part = col & 1;
  const float* cg = reinterpret_cast<const float*>(C + ch.c + (int64_t)s0 * ch.p + q) + (part ^ h);
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    const int sc = min(s, sz - 1);
#pragma unroll
    for (int u = 0; u < NT1W; ++u) {
      const int c = min(32 * (wave + 8 * u) + col, nrnt - 1);
      xp[s][u] = xg[2 * ((int64_t)sc * nrnt + c)];
    }
    cp[s] = cg[2 * (int64_t)sc * ch.p];
  }
}

// Step-1 operands of group g on 16-bit data: B operand (slices 4 t + 2 h and 4 t + 2 h + 1, re
// and im, column c) from the 16-bit copy of X, A operand from C quantised here; indices
// clamped into the group, A zeroed for slices beyond the group or rows q >= p_g.
template <int NT1W, int SMAX, int PREC>
__device__ __forceinline__ void bmm_prefetch_lp(uint2 (&xq)[PREC == 3 ? 2 : 1][(2 * SMAX + 7) / 8][NT1W],
                                                uint2 (&cq)[PREC == 3 ? 2 : 1][(2 * SMAX + 7) / 8],
                                                const float2* __restrict__ C, const char* ws,
                                                const DevChan& ch, int g, int nrnt, int wave,
                                                int col, int h) {
  constexpr int S8 = (2 * SMAX + 7) / 8;
  const int s0 = g * ch.gs, sz = min(ch.gs, ch.nsc - s0);
  const int pg = min(ch.p, sz);
  const int64_t total = (int64_t)ch.nsc * nrnt;
  const unsigned* xg = reinterpret_cast<const unsigned*>(ws + ch.w_Xq) + (int64_t)s0 * nrnt;
  const int q = col >> 1, po = col & 1;
  const int qc = min(q, pg - 1);
#pragma unroll
  for (int t = 0; t < S8; ++t) {
    const int sa = 4 * t + 2 * h, sb = sa + 1;
    const int sac = min(sa, sz - 1), sbc = min(sb, sz - 1);
#pragma unroll
    for (int u = 0; u < NT1W; ++u) {
      const int c = min(32 * (wave + 8 * u) + col, nrnt - 1);
      xq[0][t][u] = make_uint2(xg[(int64_t)sac * nrnt + c], xg[(int64_t)sbc * nrnt + c]);
      if (PREC == 3)
        xq[PREC == 3 ? 1 : 0][t][u] = make_uint2(xg[total + (int64_t)sac * nrnt + c],
                                                 xg[total + (int64_t)sbc * nrnt + c]);
    }
    const float2 ca = C[ch.c + (int64_t)(s0 + sac) * ch.p + qc];
    const float2 cb = C[ch.c + (int64_t)(s0 + sbc) * ch.p + qc];
    const bool va = sa < sz && q < pg, vb = sb < sz && q < pg;
    // A[(q, po)][(s, pi)]: po 0: (Re C, Im C)[pi]; po 1: (-Im C, Re C)[pi]
    const float a0 = va ? (po == 0 ? ca.x : -ca.y) : 0.f, a1 = va ? (po == 0 ? ca.y : ca.x) : 0.f;
    const float b0 = vb ? (po == 0 ? cb.x : -cb.y) : 0.f, b1 = vb ? (po == 0 ? cb.y : cb.x) : 0.f;
    cq[0][t] = __builtin_bit_cast(uint2, pack4(q_hi<PREC>(a0), q_hi<PREC>(a1), q_hi<PREC>(b0), q_hi<PREC>(b1)));
    if (PREC == 3)
      cq[PREC == 3 ? 1 : 0][t] =
          __builtin_bit_cast(uint2, pack4(q_lo<PREC>(a0), q_lo<PREC>(a1), q_lo<PREC>(b0), q_lo<PREC>(b1)));
  }
}

// Step-1 output (re, im) of Hc_q at column c = i nt + j into the q slot: interleaved for step 2,
// or, when step 2 is skipped (m == nr), in the layout step 2 would write (real parts of the m
// rows of 64 columns, then the imaginary parts).
__device__ __forceinline__ void bmm_store_hc(float* slot, int c, int nt, int m, bool skip2,
                                             float re, float im) {
  if (skip2) {
    const int i = c / nt, j = c - i * nt;
    slot[i * 64 + j] = re;
    slot[m * 64 + i * 64 + j] = im;
  } else {
    *reinterpret_cast<float2*>(slot + 2 * c) = make_float2(re, im);
  }
}

// PF: the next group's step-1 operands are loaded while the current group's steps 2 and 3
// run (more registers, one block per CU); otherwise they are loaded at the start of step 1
// and latency is hidden by a second resident block.  SLC: the per-q LDS slot stride in
// floats when every channel of the launch fits it (a compile-time stride turns the slot
// offsets into instruction immediates instead of per-lane addresses held across the group
// loop), or 0 for the channel's own stride.
// QL (every channel m == nr <= 8, SLC 1024): each q slot holds the 8 x 128 real rows of Hc in
// row quads, element (a, c') at (a / 4) 512 + 4 c' + a % 4, rows m..7 and columns past nt zero.
// A lane then reads the four rows a K quad needs as one 16-byte load: the Gram takes its K
// steps in the order 4 h + v (lane half h, step v) over the rows of each q, so that one q is
// four products per tile fed by two loads, with no per-step address or mask arithmetic.
template <int NT1W, int SMAX, bool PF, int PREC, int SLC, bool QL = false>
__global__ void __launch_bounds__(512, PF ? 2 : 4) k_fused_b_mm(const DevChan* __restrict__ chans,
                                                       const float2* __restrict__ X,
                                                       const float2* __restrict__ A,
                                                       const float2* __restrict__ C, char* ws) {
  extern __shared__ float smf[];
  const DevChan& ch = chans[blockIdx.y];
  const int split = blockIdx.x;
  if (split >= ch.nsplit) return;
  const int nr = ch.nr, nt = ch.nt, m = ch.m, p = ch.p;
  const int nrnt = nr * nt;
  const int SL = SLC ? SLC : bmm_slot(nr, nt, m);
  // with a compile-time stride, all 16 q slots exist and step 1 stores its rows q >= p_g
  // unconditionally (steps 2 and 3 read only q < p_g)
  float* aop = smf + (SLC ? 16 * SLC : max(p * SL, 2048));  // [nr][64] step-2 A operand
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int h = lane / 32, col = lane % 32;
  // step-2 A operand.  m <= 8 (16 real rows) uses 16 x 16 x 4 products: lane l at K step t
  // holds row l % 16 = (a, re/im) and k' = 4 t + l / 16 = (i, re/im).  Otherwise 32 x 32 x 2:
  // lane l at K step i holds row l % 32 = (a, re/im) and k = (i, l / 32).
  const bool w16 = m <= 8;
  // m == nr: A is square and unitary (every B-step follows an eigensolve of the mode-1 Gram),
  // so W_q^H W_q = Hc_q^H A A^H Hc_q = Hc_q^H Hc_q: step 1 writes Hc in the layout step 3
  // reads and step 2 is skipped
  const bool skip2 = QL || m == nr;
  if (QL) {
    // rows m..7 and columns past nt of every slot stay zero (the Gram reads them)
    if (m < 8 || nt < 64)
      for (int e = tid; e < 16 * 1024; e += 512) {
        const int o = e & 1023, a = ((o >> 9) << 2) | (o & 3), cc = (o & 511) >> 2;
        if (a >= m || (cc & 63) >= nt) smf[e] = 0.f;
      }
  } else if (skip2 && nt < 64) {  // the Gram reads 64 columns; those past nt stay zero
    const int per = 2 * m * 64;
    for (int e = tid; e < (SLC ? 16 : p) * per; e += 512) {
      const int q = e / per, o = e - q * per;
      if ((o & 63) >= nt) smf[q * SL + o] = 0.f;
    }
  }
  for (int e = tid; e < (skip2 ? 0 : nr * 64); e += 512) {
    const int st = e / 64, l = e % 64;
    int a, part, i, kp;
    if (w16) {
      a = (l % 16) >> 1;
      part = l & 1;
      const int kk = 4 * st + l / 16;
      i = kk >> 1;
      kp = kk & 1;
    } else {
      a = (l % 32) >> 1;
      part = l & 1;
      i = st;
      kp = l / 32;
    }
    float v = 0.f;
    if (a < m && i < nr) {
      const float2 av = A[ch.a + i * m + a];
      v = part == 0 ? (kp == 0 ? av.x : av.y) : (kp == 0 ? -av.y : av.x);
    }
    aop[e] = v;
  }
  // Gram tiles: wave w owns tile w; tiles 8 and 9 are shared, waves 0 and 1 taking them over
  // even q and waves 2 and 3 over odd q, so that each SIMD carries two and a half tiles
  const int nt2 = wave < 4 ? 2 : 1;
  f32x16 gacc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) gacc[t][r] = 0.f;
  const int g0 = (int)((int64_t)split * ch.ngroups / ch.nsplit);
  const int g1 = (int)((int64_t)(split + 1) * ch.ngroups / ch.nsplit);
  // QL: offset of this lane's step-1 output (q = 2 h, row i, real column j) for each of its
  // column tiles c = 32 (wave + 8 u) + col = i nt + j
  int qo[NT1W];
#pragma unroll
  for (int u = 0; u < NT1W; ++u) {
    const int c = 32 * (wave + 8 * u) + col, i = c / nt, j = c - i * nt;
    qo[u] = QL ? h * 2 * 1024 + (i >> 2) * 512 + 4 * j + (i & 3) : 0;
  }
  float xp[SMAX][NT1W], cp[SMAX];
  if (PF && g0 < g1) bmm_prefetch<NT1W, SMAX>(xp, cp, X, C, ch, g0, nrnt, wave, col, h);
  __syncthreads();
  for (int g = g0; g < g1; ++g) {
    const int s0 = g * ch.gs;
    const int sz = min(ch.gs, ch.nsc - s0);
    const int pg = min(p, sz);
    int ol1 = lane;  // opaque copy: step 1's per-lane addresses are recomputed per group
    asm volatile("" : "+v"(ol1));
    const int h = ol1 / 32, col = ol1 % 32;
    if (PREC != 0) {
      // 1. Hc on 16-bit operands, K steps of 8 = two subcarriers x (re, im) per lane half
      constexpr int S8 = (2 * SMAX + 7) / 8;
      constexpr int NQ = PREC == 3 ? 2 : 1;
      uint2 xq[NQ][S8][NT1W], cq[NQ][S8];
      bmm_prefetch_lp<NT1W, SMAX, PREC>(xq, cq, C, ws, ch, g, nrnt, wave, col, h);
#pragma unroll
      for (int u = 0; u < NT1W; ++u) {
        f32x16 acc1;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc1[r] = 0.f;
#pragma unroll
        for (int t = 0; t < S8; ++t)
          if (8 * t < 2 * sz) {
            const s16x4 a = __builtin_bit_cast(s16x4, cq[0][t]), b = __builtin_bit_cast(s16x4, xq[0][t][u]);
            acc1 = mfma16<PREC>(a, b, acc1);
            if (PREC == 3) {
              acc1 = mfma16<PREC>(a, __builtin_bit_cast(s16x4, xq[NQ - 1][t][u]), acc1);
              acc1 = mfma16<PREC>(__builtin_bit_cast(s16x4, cq[NQ - 1][t]), b, acc1);
            }
          }
        const int c = 32 * (wave + 8 * u) + col;
        if (c < nrnt)
#pragma unroll
          for (int r = 0; r < 16; r += 2) {
            const int q = 4 * (r / 4) + 2 * h + ((r % 4) >> 1);
            if (QL) {
              float* d = smf + qo[u] + (4 * (r / 4) + ((r % 4) >> 1)) * 1024;
              d[0] = acc1[r];
              d[256] = acc1[r + 1];
            } else if (SLC || q < pg) {
              bmm_store_hc(smf + q * SL, c, nt, m, skip2, acc1[r], acc1[r + 1]);
            }
          }
      }
    } else {
    if (!PF) bmm_prefetch<NT1W, SMAX>(xp, cp, X, C, ch, g, nrnt, wave, col, h);
    // 1. Hc: this wave's 32-column tiles c = 32 (wave + 8 u) + col, one tile at a time
    // A[(q, part)][(s, h)] = part 0: (Re C, Im C)[h], part 1: (-Im C, Re C)[h]
    {
      const float csign = ((col & 1) == 1 && h == 0) ? -1.f : 1.f;
#pragma unroll
      for (int u = 0; u < NT1W; ++u) {
        f32x16 acc1;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc1[r] = 0.f;
#pragma unroll
        for (int s = 0; s < SMAX; ++s)
          if (s < sz) acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(csign * cp[s], xp[s][u], acc1, 0, 0, 0);
        // register pair (r, r + 1), r % 4 in {0, 2}, holds (re, im) of q = row / 2
        const int c = 32 * (wave + 8 * u) + col;
        if (c < nrnt)
#pragma unroll
          for (int r = 0; r < 16; r += 2) {
            const int q = 4 * (r / 4) + 2 * h + ((r % 4) >> 1);
            if (QL) {
              float* d = smf + qo[u] + (4 * (r / 4) + ((r % 4) >> 1)) * 1024;
              d[0] = acc1[r];
              d[256] = acc1[r + 1];
            } else if (SLC || q < pg) {
              bmm_store_hc(smf + q * SL, c, nt, m, skip2, acc1[r], acc1[r + 1]);
            }
          }
      }
    }
    if (PF && g + 1 < g1) bmm_prefetch<NT1W, SMAX>(xp, cp, X, C, ch, g + 1, nrnt, wave, col, h);
    }
    __syncthreads();
    // 2. W_q = A^H Hc_q, in place (skipped for m == nr)
    if (!skip2) {
    // both column tiles are read before either is written back; loads are unconditional
    // (clamped) and out-of-range operands are zeroed by selects, four K steps per batch
    if (w16) {
      // rows (a, re/im) < 16, four 16-column tiles of j, K = (i, re/im) in steps of 4; every
      // operand of four K steps is loaded before their products (nr <= 16: at most 8).  Lane
      // (k4, r16) at step t reads Hc[i = 2 t + k4 / 2][j = 16 jt + r16], part k4 % 2: one
      // per-lane base plus a uniform step offset and an immediate tile offset.  Reads past row
      // nr - 1 or column nt - 1 stay inside the block's LDS (the allocation is padded) and are
      // zeroed by selects.
      int ol = lane;  // opaque copy: the per-lane offsets below are recomputed per group
      asm volatile("" : "+v"(ol));
      const int r16 = ol % 16, k4 = ol / 16;
      const int nst = (nr + 1) / 2;
      const int lb = 2 * (k4 >> 1) * nt + 2 * r16 + (k4 & 1);
      bool jv[4];
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) jv[jt] = 16 * jt + r16 < nt;
      for (int q = wave; q < pg; q += 8) {
        float* slot = smf + q * SL;
        const float* src = slot + lb;
        f32x4 acc4[4];
#pragma unroll
        for (int jt = 0; jt < 4; ++jt)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc4[jt][r] = 0.f;
#pragma unroll
        for (int tb = 0; tb < 8; tb += 4)
          if (tb < nst) {  // four K steps: all loads, then the products
            float av[4], bv[4][4];
#pragma unroll
            for (int d = 0; d < 4; ++d)
              if (tb + d < nst) {
                const int t = tb + d;
                const bool iv = 2 * t + (k4 >> 1) < nr;
                av[d] = aop[t * 64 + lane];
#pragma unroll
                for (int jt = 0; jt < 4; ++jt) {
                  const float y = src[t * 4 * nt + 32 * jt];
                  bv[d][jt] = (iv && jv[jt]) ? y : 0.f;
                }
              }
#pragma unroll
            for (int d = 0; d < 4; ++d)
              if (tb + d < nst)
#pragma unroll
                for (int jt = 0; jt < 4; ++jt)
                  acc4[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[d], bv[d][jt], acc4[jt], 0, 0, 0);
          }
        // accumulator (lane l, register r) = row 4 (l / 16) + r, column 16 jt + l % 16
#pragma unroll
        for (int jt = 0; jt < 4; ++jt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 4 * k4 + r, a = row >> 1;
            if (a < m) slot[((row & 1) ? m * 64 : 0) + a * 64 + 16 * jt + r16] = acc4[jt][r];
          }
      }
    } else
    for (int q = wave; q < pg; q += 8) {
      float* slot = smf + q * SL;
      f32x16 acc2[2];
#pragma unroll
      for (int jt = 0; jt < 2; ++jt)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc2[jt][r] = 0.f;
      const int j0 = min(col, nt - 1), j1 = min(32 + col, nt - 1);
      const bool jv0 = col < nt, jv1 = 32 + col < nt;
      for (int i0 = 0; i0 < nr; i0 += 4) {
        float av[4], b0[4], b1[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const int i = min(i0 + d, nr - 1);
          const bool iv = i0 + d < nr;
          const float x = aop[i * 64 + lane];
          const float y0 = slot[2 * (i * nt + j0) + h], y1 = slot[2 * (i * nt + j1) + h];
          av[d] = iv ? x : 0.f;
          b0[d] = jv0 ? y0 : 0.f;
          b1[d] = jv1 ? y1 : 0.f;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          acc2[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[d], b0[d], acc2[0], 0, 0, 0);
          acc2[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[d], b1[d], acc2[1], 0, 0, 0);
        }
      }
#pragma unroll
      for (int jt = 0; jt < 2; ++jt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 8 * (r / 4) + 4 * h + (r % 4);
          const int a = row >> 1;
          if (a < m) slot[((row & 1) ? m * 64 : 0) + a * 64 + 32 * jt + col] = acc2[jt][r];
        }
    }
    __syncthreads();
    }
    // 3. Gram over the rows (q, a) of W, q < p_g
    if constexpr (QL) {
      // row quads: per q, lane half h supplies rows 4 h + v at step v, so each tile takes
      // four products per q from one 16-byte load of each operand; two q per batch (the
      // second clamped, its products skipped past p_g), all branches wave-uniform
      const int wu = __builtin_amdgcn_readfirstlane(wave);
      int ol = lane;
      asm volatile("" : "+v"(ol));
      const int base = (ol >> 5) * 512 + 4 * (ol & 31);
      int I0, J0, I1, J1;
      gram_tile(wu, I0, J0);
      gram_tile(8 + (wu & 1), I1, J1);
      const float* pa0 = smf + base + 128 * I0;
      const float* pb0 = smf + base + 128 * J0;
      const float* pa1 = smf + base + 128 * I1;
      const float* pb1 = smf + base + 128 * J1;
      const bool t2 = wu < 4;
      const int par = (wu >> 1) & 1;
      for (int q = 0; q < pg; q += 2) {
        const bool more = q + 1 < pg;
        const int q1 = more ? q + 1 : q;
        const float4 x0 = *reinterpret_cast<const float4*>(pa0 + q * 1024);
        const float4 y0 = *reinterpret_cast<const float4*>(pb0 + q * 1024);
        const float4 x1 = *reinterpret_cast<const float4*>(pa0 + q1 * 1024);
        const float4 y1 = *reinterpret_cast<const float4*>(pb0 + q1 * 1024);
        // the shared tile on the q of this wave's parity (waves 0, 1 even q, waves 2, 3 odd)
        const int qt = par ? q1 : q;
        float4 u0, w0;  // read and used by waves 0..3 only
        if (t2) {
          u0 = *reinterpret_cast<const float4*>(pa1 + qt * 1024);
          w0 = *reinterpret_cast<const float4*>(pb1 + qt * 1024);
        }
        gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, y0.x, gacc[0], 0, 0, 0);
        gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.y, y0.y, gacc[0], 0, 0, 0);
        gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.z, y0.z, gacc[0], 0, 0, 0);
        gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.w, y0.w, gacc[0], 0, 0, 0);
        if (t2 && (par == 0 || more)) {
          gacc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(u0.x, w0.x, gacc[1], 0, 0, 0);
          gacc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(u0.y, w0.y, gacc[1], 0, 0, 0);
          gacc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(u0.z, w0.z, gacc[1], 0, 0, 0);
          gacc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(u0.w, w0.w, gacc[1], 0, 0, 0);
        }
        if (more) {
          gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.x, y1.x, gacc[0], 0, 0, 0);
          gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.y, y1.y, gacc[0], 0, 0, 0);
          gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.z, y1.z, gacc[0], 0, 0, 0);
          gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.w, y1.w, gacc[0], 0, 0, 0);
        }
      }
    } else {
    // two rows a0 + h of one q per step (an odd m pads each q with a zero row); two steps per
    // batch, loads unconditional
      // per-lane offsets are derived here from an opaque copy of the lane index, so that the
      // compiler recomputes them per group instead of holding them across steps 1 and 2
      int ol = lane;
      asm volatile("" : "+v"(ol));
      const int h = ol / 32, col = ol % 32;
      int offa[2], offb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        int I, J;
        gram_tile(t == 0 ? wave : 8 + (wave & 1), I, J);
        const int ca = 32 * I + col, cb = 32 * J + col;
        offa[t] = ca < 64 ? ca : m * 64 + (ca - 64);
        offb[t] = cb < 64 ? cb : m * 64 + (cb - 64);
      }
      const bool t2 = nt2 == 2;
      const int par = wave >> 1;
      for (int q = 0; q < pg; ++q) {
        const float* qb = smf + q * SL;
        const bool two = t2 && (q & 1) == par;
        for (int a0 = 0; a0 < m; a0 += 4) {
          const int ra = a0 + h, rb2 = a0 + 2 + h;
          const float sa = ra < m ? 1.f : 0.f, sb = rb2 < m ? 1.f : 0.f;
          const float* p0 = qb + min(ra, m - 1) * 64;
          const float* p1 = qb + min(rb2, m - 1) * 64;
          if (two) {
            const float x00 = p0[offa[0]], y00 = p0[offb[0]], x01 = p0[offa[1]], y01 = p0[offb[1]];
            const float x10 = p1[offa[0]], y10 = p1[offb[0]], x11 = p1[offa[1]], y11 = p1[offb[1]];
            gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa * x00, y00, gacc[0], 0, 0, 0);
            gacc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa * x01, y01, gacc[1], 0, 0, 0);
            gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(sb * x10, y10, gacc[0], 0, 0, 0);
            gacc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(sb * x11, y11, gacc[1], 0, 0, 0);
          } else {
            const float x00 = p0[offa[0]], y00 = p0[offb[0]];
            const float x10 = p1[offa[0]], y10 = p1[offb[0]];
            gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa * x00, y00, gacc[0], 0, 0, 0);
            gacc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(sb * x10, y10, gacc[0], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  // waves 2 and 3 hand their odd-q parts of tiles 8 and 9 to waves 0 and 1 through LDS
  if (wave == 2 || wave == 3)
#pragma unroll
    for (int r = 0; r < 16; ++r) smf[(wave - 2) * 1024 + lane * 16 + r] = gacc[1][r];
  __syncthreads();
  if (wave < 2)
#pragma unroll
    for (int r = 0; r < 16; ++r) gacc[1][r] += smf[wave * 1024 + lane * 16 + r];
  float* P = reinterpret_cast<float*>(ws + ch.w_S2p) + (int64_t)split * 128 * 128;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    if (t == 0 || wave < 2) {
      int I, J;
      gram_tile(t == 0 ? wave : 8 + wave, I, J);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * I + 8 * (r / 4) + 4 * h + (r % 4);
        P[row * 128 + 32 * J + col] = gacc[t][r];
      }
    }
  }
}

// Mode-2 Gram of long row stacks for any nt <= 256: rows of X (which = 0: (s, i) rows of the
// channel tensor) or of W (which = 1: (g, q, a) rows from the B-step), each a contiguous row of
// nt complex values.  With R = [Re rows | Im rows] (real column c < nt: Re of column c, else
// Im of column c - nt), R^T R is accumulated on its upper 32 x 32 tiles (T = ceil(2 nt / 32)
// tile rows, T (T + 1) / 2 tiles), eight tiles per 256-thread block (two per wave), one block
// per (tile octet, row split, channel); operands straight from the rows in memory.
__device__ __forceinline__ void upper_tile(int k, int T, int& I, int& J) {
  I = 0;
  while (k >= T - I) {
    k -= T - I;
    ++I;
  }
  J = I + k;
}

// Mode-2 Gram for wide arrays from the rows of X (which = 0: rows (s, i)) or of W (which = 1:
// rows (g, q, a)), each row nt complex read as 2 nt interleaved reals (re, im).  The real Gram
// P = R^T R of the rows r0..r1 of one split is accumulated in 128 x 128 super-tiles of the
// upper triangle, one per block; wave w computes the 2 x 2 tiles of 32 at rows 2 (w / 2) + {0, 1}
// and columns 2 (w % 2) + {0, 1} of its super-tile.  Chunks of 16 rows are staged in LDS
// column-major ([128 columns][16 rows + pad], double-buffered) so that a lane reads four
// consecutive rows at once: step 4 u + v takes row 8 u + 4 h + v in lane half h.  The next
// chunk's global loads (clamped, zeroed past the split or the row end) are in flight during
// the current chunk's products.
constexpr int kGK = 16, kGP = 20;  // rows per chunk, LDS column stride (conflict-free b128 reads)

__global__ void __launch_bounds__(256) k_gram_rows_st(const DevChan* __restrict__ chans,
                                                      const int32_t* __restrict__ toff,
                                                      int n_channels, const float2* __restrict__ X,
                                                      char* ws, int which) {
  __shared__ float4 sbuf4[2 * 2 * 128 * kGP / 4];  // [buffer][A, B][column][row]
  float* sbuf = reinterpret_cast<float*>(sbuf4);
  const int bt = xcd_tile(blockIdx.x, toff[n_channels]);  // the super-tiles of a split together
  if (bt < 0) return;
  const int cidx = tile_channel(toff, n_channels, bt);
  const int local = bt - toff[cidx];
  const DevChan& ch = chans[cidx];
  const int nt = ch.nt, nc = 2 * nt;
  const int S = (nc + 127) / 128, nst = S * (S + 1) / 2;
  const int st = local % nst, split = local / nst;
  int SI, SJ;
  upper_tile(st, S, SI, SJ);
  const float* M;
  int64_t nrows;
  if (which == 0) {
    M = reinterpret_cast<const float*>(X + ch.x);
    nrows = (int64_t)ch.nsc * ch.nr;
  } else {
    M = reinterpret_cast<const float*>(ws + ch.w_W);
    nrows = (int64_t)ch.ngroups * ch.p * ch.m;
  }
  const int64_t r0 = split * nrows / ch.nsplit, r1 = (split + 1) * nrows / ch.nsplit;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, h = lane / 32, col = lane % 32;
  const bool vec = (nt % 2) == 0 && ((reinterpret_cast<uintptr_t>(M) & 15) == 0);
  // staging role of this thread: element e = tid + 256 k, matrix e / 512 (A rows of SI, B of
  // SJ), row e % 16 of the chunk, columns 4 ((e / 16) % 32) .. + 3 of the 128 (consecutive
  // threads take consecutive rows, so that their column-major LDS writes hit distinct banks)
  int cb[4], lds[4], rowk[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = tid + 256 * k, mat = e >> 9, cq = (e >> 4) & 31;
    rowk[k] = e & 15;
    cb[k] = 128 * (mat ? SJ : SI) + 4 * cq;
    lds[k] = mat * 128 * kGP + 4 * cq * kGP + rowk[k];
  }
  float4 pf[4];
  auto load = [&](int64_t rc) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t rr = rc + rowk[k];
      const bool ok = rr < r1;
      const float* rp = M + min(rr, r1 - 1) * nc;
      const int c = cb[k];
      float4 v;
      if (vec) {  // nc % 4 == 0: the quad is wholly inside or wholly outside the row
        v = *reinterpret_cast<const float4*>(rp + min(c, nc - 4));
        if (c >= nc) v = make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        const float x0 = rp[min(c, nc - 1)], x1 = rp[min(c + 1, nc - 1)];
        const float x2 = rp[min(c + 2, nc - 1)], x3 = rp[min(c + 3, nc - 1)];
        v = make_float4(c < nc ? x0 : 0.f, c + 1 < nc ? x1 : 0.f, c + 2 < nc ? x2 : 0.f,
                        c + 3 < nc ? x3 : 0.f);
      }
      pf[k] = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store = [&](int buf) {
    float* d = sbuf + buf * 2 * 128 * kGP;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      d[lds[k]] = pf[k].x;
      d[lds[k] + kGP] = pf[k].y;
      d[lds[k] + 2 * kGP] = pf[k].z;
      d[lds[k] + 3 * kGP] = pf[k].w;
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;
  const int ti0 = 2 * (wave >> 1), tj0 = 2 * (wave & 1);
  const int nchunk = (int)((r1 - r0 + kGK - 1) / kGK);
  if (nchunk > 0) {
    load(r0);
    store(0);
  }
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    if (c + 1 < nchunk) load(r0 + (int64_t)(c + 1) * kGK);
    const float* sA = sbuf + (c & 1) * 2 * 128 * kGP;
    const float* sB = sA + 128 * kGP;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      float4 av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        av[a] = *reinterpret_cast<const float4*>(sA + (32 * (ti0 + a) + col) * kGP + 8 * u + 4 * h);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        bv[b] = *reinterpret_cast<const float4*>(sB + (32 * (tj0 + b) + col) * kGP + 8 * u + 4 * h);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].x, bv[b].x, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].y, bv[b].y, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].z, bv[b].z, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].w, bv[b].w, acc[a][b], 0, 0, 0);
        }
    }
    if (c + 1 < nchunk) store((c + 1) & 1);
    __syncthreads();
  }
  const int W = 128 * S;
  float* P = reinterpret_cast<float*>(ws + ch.w_S2p) + (int64_t)split * W * W;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 128 * SI + 32 * (ti0 + a) + 8 * (r / 4) + 4 * h + (r % 4);
        P[(int64_t)row * W + 128 * SJ + 32 * (tj0 + b) + col] = acc[a][b][r];
      }
}

// S2 (nt x nt complex) = sum over splits of the interleaved real Gram above:
// Re S2[j][k] = P[2j][2k] + P[2j+1][2k+1], Im S2[j][k] = P[2j][2k+1] - P[2j+1][2k].  Only
// entries whose real rows lie in a super-tile row at or above their columns' are read (the
// computed part of P, row-contiguous); the entries below are written as the conjugates.
__global__ void k_reduce_S2_st(const DevChan* __restrict__ chans, const int32_t* __restrict__ toff,
                               int n_channels, char* ws) {
  const int cidx = tile_channel(toff, n_channels, blockIdx.x);
  const DevChan& ch = chans[cidx];
  const int nt = ch.nt;
  const int e = (blockIdx.x - toff[cidx]) * blockDim.x + threadIdx.x;
  if (e >= nt * nt) return;
  const int j = e / nt, k = e % nt;
  if ((j >> 6) > (k >> 6)) return;  // super-tile row of 2 j below that of 2 k
  const int W = 128 * ((2 * nt + 127) / 128);
  const float* P = reinterpret_cast<const float*>(ws + ch.w_S2p);
  float re = 0.f, im = 0.f;
  for (int sp = 0; sp < ch.nsplit; ++sp) {
    const float* Q = P + (int64_t)sp * W * W;
    const float2 r0 = *reinterpret_cast<const float2*>(Q + (int64_t)(2 * j) * W + 2 * k);
    const float2 r1 = *reinterpret_cast<const float2*>(Q + (int64_t)(2 * j + 1) * W + 2 * k);
    re += r0.x + r1.y;
    im += r0.y - r1.x;
  }
  float2* S2 = reinterpret_cast<float2*>(ws + ch.w_S2);
  S2[e] = make_float2(re, im);
  if ((j >> 6) < (k >> 6)) S2[(int64_t)k * nt + j] = make_float2(re, -im);
}

// T_s = H_s B (nr x n) for all subcarriers, as a product over the rows (s, i) of X, each row
// nt complex.  Real form as in the T pass, K index k' = 2 j + part of the interleaved row; one
// 32-wide tile of the 2 n real output columns ([Re | Im]) per block with its real-form B slice
// in LDS ([2 nt][32] floats, k'-major); each wave takes 32-row tiles.  With nt % 8 == 0 and
// 16-byte aligned rows, step 4 u + v takes k' = 8 u + 4 half + v in lane half (16 contiguous
// bytes per lane per four steps); otherwise step t takes k' = 2 t + half.
__global__ void __launch_bounds__(256) k_rows_times_b(const DevChan* __restrict__ chans,
                                                      const int32_t* __restrict__ toff,
                                                      int n_channels, const float2* __restrict__ X,
                                                      const float2* __restrict__ B, char* ws) {
  extern __shared__ float bts[];  // [2 nt][32]
  constexpr int tiles_per_block = kTRowTiles;
  const int bt = xcd_tile(blockIdx.x, toff[n_channels]);  // column tiles of a row block together
  if (bt < 0) return;
  const int cidx = tile_channel(toff, n_channels, bt);
  const int local = bt - toff[cidx];
  const DevChan& ch = chans[cidx];
  const int nt = ch.nt, n = ch.n;
  const int nct = (2 * n + 31) / 32;
  const int ctile = local % nct;
  const int64_t nrows = (int64_t)ch.nsc * ch.nr;
  const int64_t rtiles = (nrows + 31) / 32;
  const int64_t t0 = (int64_t)(local / nct) * tiles_per_block;
  const float* in = reinterpret_cast<const float*>(X + ch.x);
  float2* out = reinterpret_cast<float2*>(ws + ch.w_T);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, half = lane / 32, col = lane % 32;
  for (int e = tid; e < 2 * nt * 32; e += 256) {
    const int kk = e / 32, c = 32 * ctile + e % 32, j = kk / 2, part = kk % 2;
    float v = 0.f;
    if (c < 2 * n) {
      const float2 b = B[ch.b + (int64_t)j * n + (c < n ? c : c - n)];
      v = (part == 0) ? (c < n ? b.x : b.y) : (c < n ? -b.y : b.x);
    }
    bts[e] = v;
  }
  __syncthreads();
  const int oc = 32 * ctile + col;  // real output column of this lane
  const bool ocv = oc < 2 * n;
  const int ob = oc < n ? oc : oc - n, opart = oc < n ? 0 : 1;
  const bool vec8 = (nt % 8) == 0 && ((reinterpret_cast<uintptr_t>(in) & 15) == 0);
  const int64_t tend = min(rtiles, t0 + tiles_per_block);
  for (int64_t rt = t0 + wave; rt < tend; rt += 4) {
    const int64_t row = min(rt * 32 + col, nrows - 1);
    const float* xr = in + row * 2 * nt;
    f32x16 acc, accb;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = accb[r] = 0.f;
    if (vec8) {
      // batches of eight 16-byte loads (32 products); the next batch is requested before the
      // current one's products (clamped to the row at its end)
      const float4* xr4 = reinterpret_cast<const float4*>(xr);
      const float* bcol = bts + 4 * half * 32 + col;
      const int nw = nt / 4;
      float4 xa[8];
#pragma unroll
      for (int d = 0; d < 8; ++d) xa[d] = xr4[2 * min(d, nw - 1) + half];
      for (int w0 = 0; w0 < nw; w0 += 8) {
        float4 xn[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) xn[d] = xr4[2 * min(w0 + 8 + d, nw - 1) + half];
#pragma unroll
        for (int d = 0; d < 8; d += 2)
          if (w0 + d < nw) {
            const float4 x0 = xa[d], x1 = xa[d + 1];
            const float* bw = bcol + 8 * (w0 + d) * 32;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, bw[0], acc, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.x, bw[256], accb, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.y, bw[32], acc, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.y, bw[288], accb, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.z, bw[64], acc, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.z, bw[320], accb, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.w, bw[96], acc, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.w, bw[352], accb, 0, 0, 0);
          }
#pragma unroll
        for (int d = 0; d < 8; ++d) xa[d] = xn[d];
      }
    } else {
      for (int t = 0; t < nt; ++t)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xr[2 * t + half], bts[(2 * t + half) * 32 + col],
                                                   acc, 0, 0, 0);
    }
    if (ocv)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t orow = rt * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        if (orow < nrows)
          reinterpret_cast<float*>(out + orow * n + ob)[opart] = acc[r] + accb[r];
      }
  }
}

// Precision form of the generic T pass: T = H B on 16-bit operands from the 16-bit copy of X
// (nt % 4 == 0).  B's real-form slice for one 32-wide output tile is staged in LDS as
// [32 c][2 nt + 4] 16-bit values (hi, then lo for the split form; the pad keeps the lanes'
// 8-byte reads on distinct banks).  K steps of 8 real indices; pairs of steps 2 u, 2 u + 1 take
// k' = 16 u + 8 h + 4 w + v in lane half h (16 contiguous bytes of the row per lane), a last
// single step (nt % 8 == 4) takes k' = 8 t + 4 h + v.
template <int PREC>
__global__ void __launch_bounds__(256) k_rows_times_b_lp(const DevChan* __restrict__ chans,
                                                         const int32_t* __restrict__ toff,
                                                         int n_channels,
                                                         const float2* __restrict__ B, char* ws) {
  extern __shared__ unsigned short bq[];  // [NQ][32][2 nt + 4]
  constexpr int NQ = PREC == 3 ? 2 : 1;
  constexpr int tiles_per_block = kTRowTiles;
  const int bt = xcd_tile(blockIdx.x, toff[n_channels]);  // column tiles of a row block together
  if (bt < 0) return;
  const int cidx = tile_channel(toff, n_channels, bt);
  const int local = bt - toff[cidx];
  const DevChan& ch = chans[cidx];
  const int nt = ch.nt, n = ch.n, nc = 2 * nt, sd = nc + 4;
  const int nct = (2 * n + 31) / 32;
  const int ctile = local % nct;
  const int64_t nrows = (int64_t)ch.nsc * ch.nr;
  const int64_t rtiles = (nrows + 31) / 32;
  const int64_t t0 = (int64_t)(local / nct) * tiles_per_block;
  const unsigned short* Xh = reinterpret_cast<const unsigned short*>(ws + ch.w_Xq);
  const int64_t xtot = nrows * nt;
  float2* out = reinterpret_cast<float2*>(ws + ch.w_T);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, half = lane / 32, col = lane % 32;
  for (int e = tid; e < 32 * nc; e += 256) {
    const int c = e / nc, kk = e % nc, j = kk / 2, part = kk % 2;
    const int oc = 32 * ctile + c;
    float v = 0.f;
    if (oc < 2 * n) {
      const float2 b = B[ch.b + (int64_t)j * n + (oc < n ? oc : oc - n)];
      v = (part == 0) ? (oc < n ? b.x : b.y) : (oc < n ? -b.y : b.x);
    }
    bq[c * sd + kk] = q_hi<PREC>(v);
    if (PREC == 3) bq[32 * sd + c * sd + kk] = q_lo<PREC>(v);
  }
  __syncthreads();
  const int oc = 32 * ctile + col;
  const bool ocv = oc < 2 * n;
  const int ob = oc < n ? oc : oc - n, opart = oc < n ? 0 : 1;
  const unsigned short* bh = bq + col * sd;
  const unsigned short* bl = bq + 32 * sd + col * sd;
  const int K16 = nt / 8;          // pairs of steps
  const bool tail = (nt % 8) != 0;  // one more step of 8
  const int64_t tend = min(rtiles, t0 + tiles_per_block);
  for (int64_t rt = t0 + wave; rt < tend; rt += 4) {
    const int64_t row = min(rt * 32 + col, nrows - 1);
    const unsigned short* xr = Xh + 2 * row * nt;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int u0 = 0; u0 < K16; u0 += 4) {
      uint4 a[4], al[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int u = min(u0 + d, K16 - 1);
        a[d] = *reinterpret_cast<const uint4*>(xr + 16 * u + 8 * half);
        if (PREC == 3) al[d] = *reinterpret_cast<const uint4*>(xr + 2 * xtot + 16 * u + 8 * half);
      }
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (u0 + d < K16) {
          const int u = u0 + d;
#pragma unroll
          for (int w = 0; w < 2; ++w) {
            const uint2 a2 = w == 0 ? make_uint2(a[d].x, a[d].y) : make_uint2(a[d].z, a[d].w);
            const uint2 b2 = *reinterpret_cast<const uint2*>(bh + 16 * u + 8 * half + 4 * w);
            const s16x4 av = __builtin_bit_cast(s16x4, a2), bv = __builtin_bit_cast(s16x4, b2);
            acc = mfma16<PREC>(av, bv, acc);
            if (PREC == 3) {
              const uint2 a2l = w == 0 ? make_uint2(al[d].x, al[d].y) : make_uint2(al[d].z, al[d].w);
              const uint2 b2l = *reinterpret_cast<const uint2*>(bl + 16 * u + 8 * half + 4 * w);
              acc = mfma16<PREC>(av, __builtin_bit_cast(s16x4, b2l), acc);
              acc = mfma16<PREC>(__builtin_bit_cast(s16x4, a2l), bv, acc);
            }
          }
        }
    }
    if (tail) {
      const int k0 = 16 * K16 + 4 * half;
      const s16x4 av = __builtin_bit_cast(s16x4, *reinterpret_cast<const uint2*>(xr + k0));
      const s16x4 bv = __builtin_bit_cast(s16x4, *reinterpret_cast<const uint2*>(bh + k0));
      acc = mfma16<PREC>(av, bv, acc);
      if (PREC == 3) {
        const s16x4 avl = __builtin_bit_cast(s16x4, *reinterpret_cast<const uint2*>(xr + 2 * xtot + k0));
        const s16x4 bvl = __builtin_bit_cast(s16x4, *reinterpret_cast<const uint2*>(bl + k0));
        acc = mfma16<PREC>(av, bvl, acc);
        acc = mfma16<PREC>(avl, bv, acc);
      }
    }
    if (ocv)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t orow = rt * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        if (orow < nrows) reinterpret_cast<float*>(out + orow * n + ob)[opart] = acc[r];
      }
  }
}

// B-step rows for wide arrays: W_q = A^H (sum_s conj(C[s,q]) H_s) for one group and a chunk of
// 32 transmit columns per block, written to the workspace as rows (g, q, a) of nt complex for
// the mode-2 Gram.  Step 1 contracts the subcarriers first, Hc_q = sum_s conj(C[s,q]) H_s,
// for up to 16 q at a time (one 32-row real tile (q, re/im) x K (s, re/im) x 32 columns j
// per antenna i), into LDS as separate re and im planes [q][i][32]; step 2 takes per q the
// product with A^H (rows (a, re/im), K (i, re/im)).  Rows q >= p_g of a short group come out
// zero through zero coefficients.
template <int SMAX, int PREC>
__global__ void __launch_bounds__(256) k_w_rows(const DevChan* __restrict__ chans,
                                                const float2* __restrict__ X,
                                                const float2* __restrict__ A,
                                                const float2* __restrict__ C, char* ws,
                                                const int32_t* __restrict__ toff, int n_channels,
                                                int qcap) {
  extern __shared__ float hcs[];  // [2][qcap][nr][32]
  const int cidx = tile_channel(toff, n_channels, blockIdx.x);
  const int local = blockIdx.x - toff[cidx];
  const DevChan& ch = chans[cidx];
  const int nr = ch.nr, nt = ch.nt, m = ch.m, p = ch.p;
  const int nchunk = (nt + 31) / 32;
  const int g = local / nchunk, jc = local % nchunk;
  const int s0 = g * ch.gs, sz = min(ch.gs, ch.nsc - s0), pg = min(p, sz);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, h = lane / 32, col = lane % 32;
  const int j = 32 * jc + col;
  const bool jv = j < nt;
  const int jcl = min(j, nt - 1);
  const int plane = qcap * nr * 32;
  const int rq = col >> 1, po = col & 1;  // MFMA row of this lane: (q or a, re/im)
  // step-2 A operand for K step i: po 0: (Re, Im)[h] of A[i][a], po 1: (-Im, Re)[h]
  float aco[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float2 av = A[ch.a + min(i, nr - 1) * m + min(rq, m - 1)];
    const float v = po == 0 ? (h == 0 ? av.x : av.y) : (h == 0 ? -av.y : av.x);
    aco[i] = (i < nr && rq < m) ? v : 0.f;
  }
  const float2* xg = X + ch.x + (int64_t)s0 * nr * nt;
  float2* Wg = reinterpret_cast<float2*>(ws + ch.w_W) + (int64_t)g * p * m * nt;
  // FP32 step 1 in K steps of 4: step 4 u + v takes k = (s, re/im) with s = 4 u + 2 h + v / 2
  // and part v % 2 in lane half h, so that a lane reads whole complex entries of two
  // subcarriers
  constexpr int SU = (SMAX + 3) / 4;
  for (int q0 = 0; q0 < p; q0 += qcap) {
    const int q = q0 + rq;
    const bool qv = q < pg && rq < qcap;
    float cpp[PREC == 0 ? SU : 1][4];
    if constexpr (PREC == 0)
#pragma unroll
      for (int u = 0; u < SU; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          const int sc = 4 * u + 2 * h + w;
          const float2 c = C[ch.c + (int64_t)(s0 + min(sc, sz - 1)) * p + min(q, p - 1)];
          const bool ok = qv && sc < sz;
          // row po 0: (Re C, Im C)[pi]; row po 1: (-Im C, Re C)[pi]
          cpp[u][2 * w] = ok ? (po == 0 ? c.x : -c.y) : 0.f;
          cpp[u][2 * w + 1] = ok ? (po == 0 ? c.y : c.x) : 0.f;
        }
    if (q0 > 0) __syncthreads();  // the previous q tile's step 2 has read the planes
    if constexpr (PREC != 0) {
      // 1. on 16-bit operands: K step t covers subcarriers 4 t .. 4 t + 3, lane half h holding
      // k = (s, re/im) for s = 4 t + 2 h and 4 t + 2 h + 1 (the v order re, im, re, im)
      constexpr int SQ = (SMAX + 3) / 4;
      constexpr int NQ = PREC == 3 ? 2 : 1;
      uint2 aq[NQ][SQ];
#pragma unroll
      for (int t = 0; t < SQ; ++t) {
        const int sa = 4 * t + 2 * h, sb = sa + 1;
        const float sga = (po == 1) ? -1.f : 1.f;  // sign of the pi = 0 entry of row po
        const float2 cva = C[ch.c + (int64_t)(s0 + min(sa, sz - 1)) * p + min(q, p - 1)];
        const float2 cvb = C[ch.c + (int64_t)(s0 + min(sb, sz - 1)) * p + min(q, p - 1)];
        const bool va = qv && sa < sz, vb = qv && sb < sz;
        // row po 0: (Re C, Im C)[pi]; row po 1: (-Im C, Re C)[pi]
        const float a0 = va ? (po == 0 ? cva.x : sga * cva.y) : 0.f;
        const float a1 = va ? (po == 0 ? cva.y : cva.x) : 0.f;
        const float b0 = vb ? (po == 0 ? cvb.x : sga * cvb.y) : 0.f;
        const float b1 = vb ? (po == 0 ? cvb.y : cvb.x) : 0.f;
        aq[0][t] = __builtin_bit_cast(uint2, pack4(q_hi<PREC>(a0), q_hi<PREC>(a1), q_hi<PREC>(b0), q_hi<PREC>(b1)));
        if (PREC == 3)
          aq[NQ - 1][t] = __builtin_bit_cast(uint2, pack4(q_lo<PREC>(a0), q_lo<PREC>(a1), q_lo<PREC>(b0), q_lo<PREC>(b1)));
      }
      const int64_t xtot = (int64_t)ch.nsc * nr * nt;
      const unsigned* xq = reinterpret_cast<const unsigned*>(ws + ch.w_Xq) + (int64_t)s0 * nr * nt;
      for (int i = wave; i < nr; i += 4) {
        uint2 xv[NQ][SQ];
#pragma unroll
        for (int t = 0; t < SQ; ++t) {
          const int64_t sa = min(4 * t + 2 * h, sz - 1), sb = min(4 * t + 2 * h + 1, sz - 1);
          const int64_t oa = (sa * nr + i) * nt + jcl, ob = (sb * nr + i) * nt + jcl;
          xv[0][t] = make_uint2(xq[oa], xq[ob]);
          if (PREC == 3) xv[NQ - 1][t] = make_uint2(xq[xtot + oa], xq[xtot + ob]);
        }
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
        for (int t = 0; t < SQ; ++t)
          if (4 * t < sz) {
            const s16x4 a = __builtin_bit_cast(s16x4, aq[0][t]), b = __builtin_bit_cast(s16x4, xv[0][t]);
            acc = mfma16<PREC>(a, b, acc);
            if (PREC == 3) {
              acc = mfma16<PREC>(a, __builtin_bit_cast(s16x4, xv[NQ - 1][t]), acc);
              acc = mfma16<PREC>(__builtin_bit_cast(s16x4, aq[NQ - 1][t]), b, acc);
            }
          }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 8 * (r / 4) + 4 * h + (r % 4), ql = row >> 1;
          if (ql < qcap) hcs[(row & 1) * plane + (ql * nr + i) * 32 + col] = acc[r];
        }
      }
    } else {
    // 1. NI antenna tiles i0 + 4 k per pass, all loads issued before the products
    constexpr int NI = SMAX <= 12 ? 2 : 1;
    for (int i0 = wave; i0 < nr; i0 += 4 * NI) {
      float2 xa[NI][SU][2];
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const int ic = min(i0 + 4 * k, nr - 1);
#pragma unroll
        for (int u = 0; u < SU; ++u)
#pragma unroll
          for (int w = 0; w < 2; ++w) {
            const int64_t sc = min(4 * u + 2 * h + w, sz - 1);
            xa[k][u][w] = xg[(sc * nr + ic) * nt + jcl];
          }
      }
      f32x16 acc[NI];
#pragma unroll
      for (int k = 0; k < NI; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;
#pragma unroll
      for (int u = 0; u < SU; ++u)
        if (4 * u < sz)
#pragma unroll
          for (int k = 0; k < NI; ++k) {
            acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(cpp[u][0], xa[k][u][0].x, acc[k], 0, 0, 0);
            acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(cpp[u][1], xa[k][u][0].y, acc[k], 0, 0, 0);
            acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(cpp[u][2], xa[k][u][1].x, acc[k], 0, 0, 0);
            acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(cpp[u][3], xa[k][u][1].y, acc[k], 0, 0, 0);
          }
      // accumulator (lane, r): row 8 (r / 4) + 4 h + r % 4 = (q - q0, re/im), column j
#pragma unroll
      for (int k = 0; k < NI; ++k)
        if (i0 + 4 * k < nr)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r / 4) + 4 * h + (r % 4), ql = row >> 1;
            if (ql < qcap) hcs[(row & 1) * plane + (ql * nr + i0 + 4 * k) * 32 + col] = acc[k][r];
          }
    }
    }
    __syncthreads();
    // 2. W_q = A^H Hc_q: rows (a, re/im), K = (i, re/im) with the lane half choosing the plane
    for (int ql = wave; ql < min(qcap, p - q0); ql += 4) {
      const float* hq = hcs + h * plane + ql * nr * 32 + col;
      f32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i < nr) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(aco[i], hq[i * 32], acc, 0, 0, 0);
      float2* wq = Wg + (int64_t)(q0 + ql) * m * nt + j;
      if (jv)
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const int a = (8 * (r / 4) + 4 * h + (r % 4)) >> 1;
          if (a < m) wq[(int64_t)a * nt] = make_float2(acc[r], acc[r + 1]);
        }
    }
  }
}

// Yh_s = A^H T_s (m x n) from T = H B: a thread owns column b of one T_s (nr entries, read
// once) and forms the m entries of that column of Yh_s.
__global__ void __launch_bounds__(256) k_yh_from_t(const DevChan* __restrict__ chans,
                                                   const int32_t* __restrict__ toff, int n_channels,
                                                   const float2* __restrict__ A, char* ws) {
  const int cidx = tile_channel(toff, n_channels, blockIdx.x);
  const DevChan& ch = chans[cidx];
  const int nr = ch.nr, m = ch.m, n = ch.n;
  const int64_t o = (int64_t)(blockIdx.x - toff[cidx]) * blockDim.x + threadIdx.x;
  if (o >= (int64_t)ch.nsc * n) return;
  const int b = (int)(o % n);
  const int64_t s = o / n;
  const float2* T = reinterpret_cast<const float2*>(ws + ch.w_T) + s * nr * n + b;
  float2 tc[kMaxNr];
#pragma unroll
  for (int i = 0; i < kMaxNr; ++i) tc[i] = T[(int64_t)min(i, nr - 1) * n];
  float2* Y = reinterpret_cast<float2*>(ws + ch.w_Yh) + s * m * n + b;
  const float2* Ac = A + ch.a;
  for (int a = 0; a < m; ++a) {
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int i = 0; i < kMaxNr; ++i)
      if (i < nr) {
        const float2 x = Ac[i * m + a];
        re += x.x * tc[i].x + x.y * tc[i].y;
        im += x.x * tc[i].y - x.y * tc[i].x;
      }
    Y[(int64_t)a * n] = make_float2(re, im);
  }
}

// S2 = sum over splits of the complex Gram assembled from the real blocks of R^T R
// (upper 32 x 32 tiles stored; lower entries by symmetry).
__global__ void __launch_bounds__(256) k_reduce_S2_mfma(const DevChan* __restrict__ chans, char* ws) {
  // One block per upper 32 x 32 tile (J, K) of S2 (J <= K) and channel.  With UL, UR, LR the
  // quadrants of the real Gram of [Re W | Im W] (stored as its upper 32 x 32 tiles):
  //   Re S2[j][k] = UL[j][k] + LR[j][k],  Im S2[j][k] = UR[j][k] - UR[k][j].
  // Every partial is read in its stored orientation (coalesced); the UR[k][j] sums and the
  // mirrored lower tile go through an LDS transpose.
  const DevChan& ch = chans[blockIdx.y];
  const int nt = ch.nt;
  const int t = blockIdx.x;
  const int J = t == 2 ? 1 : 0, K = t == 0 ? 0 : 1;
  if (32 * K >= nt) return;
  __shared__ float tra[32][33], trb[32][33];
  const float* P = reinterpret_cast<const float*>(ws + ch.w_S2p);
  const int tid = threadIdx.x, col = tid % 32, r0 = tid / 32;
  float re[4], ia[4], ib[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) re[u] = ia[u] = ib[u] = 0.f;
  for (int sp = 0; sp < ch.nsplit; ++sp) {
    const float* Q = P + (int64_t)sp * 128 * 128;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int row = r0 + 8 * u;
      re[u] += Q[(32 * J + row) * 128 + 32 * K + col] + Q[(64 + 32 * J + row) * 128 + 64 + 32 * K + col];
      ia[u] += Q[(32 * J + row) * 128 + 64 + 32 * K + col];  // UR[32 J + row][32 K + col]
      ib[u] += Q[(32 * K + row) * 128 + 64 + 32 * J + col];  // UR[32 K + row][32 J + col]
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) trb[r0 + 8 * u][col] = ib[u];
  __syncthreads();
  float2* S2 = reinterpret_cast<float2*>(ws + ch.w_S2);
  float im[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int row = r0 + 8 * u;
    im[u] = ia[u] - trb[col][row];  // UR[k][j] for j = 32 J + row, k = 32 K + col
    const int j = 32 * J + row, k = 32 * K + col;
    if (j < nt && k < nt) S2[j * nt + k] = make_float2(re[u], im[u]);
  }
  if (J == K) return;
  // lower tile: S2[k][j] = conj(S2[j][k]), written row-major through a transpose (after every
  // thread has read trb above)
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    tra[r0 + 8 * u][col] = re[u];
    trb[r0 + 8 * u][col] = im[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int row = r0 + 8 * u;  // k - 32 K
    const int k = 32 * K + row, j = 32 * J + col;
    if (j < nt && k < nt) S2[k * nt + j] = make_float2(tra[col][row], -trb[col][row]);
  }
}

// ---------------------------------------------------------------------------------------
// host side

static const int32_t* tiles_of(const LaunchCtx& L, TileKind k) {
  return L.d_tiles + (size_t)k * (L.n_channels + 1);
}

#define GT_LAUNCH_SH(name, grid, block, shm, ...)                       \
  do {                                                                  \
    prof_begin(#name, L.stream);                                        \
    hipLaunchKernelGGL(name, grid, block, shm, L.stream, __VA_ARGS__);  \
    prof_end(L.stream);                                                 \
    hipError_t e_ = hipGetLastError();                                  \
    if (e_ != hipSuccess) {                                             \
      set_error_detail(#name, e_);                                      \
      return GT_ERR_HIP;                                                \
    }                                                                   \
  } while (0)

static size_t t_bytes(const LaunchCtx& L) {
  return sizeof(float2) * ((size_t)L.max_nt * L.max_n + (size_t)L.max_nr * L.max_m +
                           (size_t)L.max_gs * L.max_nr * L.max_n + (size_t)L.max_gs * L.max_m * L.max_n +
                           (size_t)L.max_nr * L.max_nt);
}
static size_t z_bytes(const LaunchCtx& L) {
  return sizeof(float2) * ((size_t)L.max_gs * L.max_p + (size_t)L.max_p * L.max_nr * L.max_n);
}
static size_t b_bytes(const LaunchCtx& L) {
  return sizeof(float2) * ((size_t)L.max_p * L.max_m * L.max_nt + (size_t)L.max_nr * L.max_m +
                           (size_t)L.max_gs * L.max_p);
}

bool fused_fit_ok(const LaunchCtx& L) {
  return L.max_nt <= 64 && L.max_gs <= 32 && L.max_nr * L.max_nt <= 1024 && t_bytes(L) <= 64 * 1024 &&
         z_bytes(L) <= 64 * 1024 && b_bytes(L) <= 64 * 1024;
}

static size_t tm_bytes(const LaunchCtx& L) {
  return sizeof(float2) * (std::max<size_t>((size_t)L.max_nt * 32, (size_t)L.max_gs * (L.max_m * L.max_n + 2)) +
                           (size_t)L.max_nr * L.max_m + (size_t)L.max_gs * L.max_nr * L.max_n);
}

static size_t tlp_bytes(const LaunchCtx& L) {
  const size_t nq = L.ttm_prec == GT_TTM_SPLIT_BF16 ? 2 : 1;
  return nq * 32 * 2 * L.max_nt * sizeof(unsigned short) +
         sizeof(float2) * ((size_t)L.max_nr * L.max_m + (size_t)L.max_gs * L.max_nr * L.max_n +
                           (size_t)L.max_gs * (L.max_m * L.max_n + 2));
}

static int bmm_variant(const LaunchCtx& L);
bool fused_b_mfma_ok(const LaunchCtx& L);

// The precision form runs on the fused passes with the matrix-core B-step kernel and one
// 32-row tile per wave in the T pass (every channel's nt a multiple of 4, checked by the plan).
bool fused_lowp_ok(const LaunchCtx& L) {
  return fused_fit_ok(L) && bmm_variant(L) != 0 && L.max_gs * L.max_nr <= 128 &&
         tlp_bytes(L) <= 64 * 1024;
}

// T = H B over all rows of X (generic path).
gt_status launch_rows_times_b(const LaunchCtx& L, const float2* X, const float2* B) {
  if (L.tiles_total[TK_TROWS] == 0) return GT_OK;
  const dim3 grid(8 * ((L.tiles_total[TK_TROWS] + 7) / 8));
  const int32_t* toff = tiles_of(L, TK_TROWS);
  if (L.ttm_prec == GT_TTM_FP32) {
    GT_LAUNCH_SH(k_rows_times_b, grid, dim3(256), sizeof(float) * 2 * L.max_nt * 32, L.d_chans,
                 toff, L.n_channels, X, B, L.ws);
    return GT_OK;
  }
  const int nq = L.ttm_prec == GT_TTM_SPLIT_BF16 ? 2 : 1;
  const size_t sh = sizeof(unsigned short) * nq * 32 * (2 * L.max_nt + 4);
  switch (L.ttm_prec) {
    case GT_TTM_BF16:
      GT_LAUNCH_SH((k_rows_times_b_lp<1>), grid, dim3(256), sh, L.d_chans, toff, L.n_channels, B, L.ws);
      break;
    case GT_TTM_FP16:
      GT_LAUNCH_SH((k_rows_times_b_lp<2>), grid, dim3(256), sh, L.d_chans, toff, L.n_channels, B, L.ws);
      break;
    default:
      GT_LAUNCH_SH((k_rows_times_b_lp<3>), grid, dim3(256), sh, L.d_chans, toff, L.n_channels, B, L.ws);
      break;
  }
  return GT_OK;
}

// W rows of the B-step for plans with some nt > 64.
gt_status launch_w_rows(const LaunchCtx& L, const float2* X, const float2* A, const float2* C) {
  const int qcap = std::min(16, L.max_p);
  const dim3 grid(L.tiles_total[TK_WROWS]);
  if (grid.x == 0) return GT_OK;
  const int32_t* toff = tiles_of(L, TK_WROWS);
  const size_t sh = sizeof(float) * 2 * qcap * L.max_nr * 32;
#define GT_WROWS(SM, PR)                                                                       \
  GT_LAUNCH_SH((k_w_rows<SM, PR>), grid, dim3(256), sh, L.d_chans, X, A, C, L.ws, toff, \
               L.n_channels, qcap)
#define GT_WROWS_P(SM)                                     \
  switch (L.ttm_prec) {                                    \
    case GT_TTM_FP32: GT_WROWS(SM, 0); break;              \
    case GT_TTM_BF16: GT_WROWS(SM, 1); break;              \
    case GT_TTM_FP16: GT_WROWS(SM, 2); break;              \
    default: GT_WROWS(SM, 3); break;                       \
  }
  if (L.max_gs <= 12) {
    GT_WROWS_P(12)
  } else if (L.max_gs <= 24) {
    GT_WROWS_P(24)
  } else {
    GT_WROWS_P(32)
  }
#undef GT_WROWS_P
#undef GT_WROWS
  return GT_OK;
}

gt_status launch_yh_from_t(const LaunchCtx& L, const float2* A) {
  if (L.tiles_total[TK_YH] > 0)
    GT_LAUNCH_SH(k_yh_from_t, dim3(L.tiles_total[TK_YH]), dim3(256), 0, L.d_chans,
                 tiles_of(L, TK_YH), L.n_channels, A, L.ws);
  return GT_OK;
}

// Mode-2 Gram of X rows (which = 0) or W rows (which = 1) for plans with some nt > 64.
gt_status launch_gram_rows_big(const LaunchCtx& L, const float2* X, int which) {
  if (L.tiles_total[TK_GRAM] > 0)
    GT_LAUNCH_SH(k_gram_rows_st, dim3(8 * ((L.tiles_total[TK_GRAM] + 7) / 8)), dim3(256), 0, L.d_chans,
                 tiles_of(L, TK_GRAM), L.n_channels, X, L.ws, which);
  if (L.tiles_total[TK_RED2] > 0)
    GT_LAUNCH_SH(k_reduce_S2_st, dim3(L.tiles_total[TK_RED2]), dim3(256), 0, L.d_chans,
                 tiles_of(L, TK_RED2), L.n_channels, L.ws);
  return GT_OK;
}

gt_status launch_convert_x(const LaunchCtx& L, const float2* X) {
  const int64_t per = (int64_t)L.max_nsc * L.max_nr * L.max_nt;
  const dim3 grid((unsigned)std::min<int64_t>((per + 255) / 256, 2048), L.n_channels);
  switch (L.ttm_prec) {
    case GT_TTM_BF16: GT_LAUNCH_SH((k_convert_x<1>), grid, dim3(256), 0, L.d_chans, X, L.ws); break;
    case GT_TTM_FP16: GT_LAUNCH_SH((k_convert_x<2>), grid, dim3(256), 0, L.d_chans, X, L.ws); break;
    default: GT_LAUNCH_SH((k_convert_x<3>), grid, dim3(256), 0, L.d_chans, X, L.ws); break;
  }
  return GT_OK;
}

gt_status launch_fused_t(const LaunchCtx& L, const float2* X, const float2* A, const float2* B,
                         int do_c) {
  if (L.ttm_prec != GT_TTM_FP32) {
    const dim3 grid(L.total_groups);
    const size_t sh = tlp_bytes(L);
    switch (L.ttm_prec) {
      case GT_TTM_BF16:
        GT_LAUNCH_SH((k_fused_t_lp<1>), grid, dim3(256), sh, L.d_chans, L.d_groups, A, B, L.ws, do_c);
        break;
      case GT_TTM_FP16:
        GT_LAUNCH_SH((k_fused_t_lp<2>), grid, dim3(256), sh, L.d_chans, L.d_groups, A, B, L.ws, do_c);
        break;
      default:
        GT_LAUNCH_SH((k_fused_t_lp<3>), grid, dim3(256), sh, L.d_chans, L.d_groups, A, B, L.ws, do_c);
        break;
    }
    return GT_OK;
  }
  // matrix cores when the real output fits one column tile and at most 8 row tiles (unless
  // the tuned choice is the vector ALU kernel)
  if (L.tune_tpass == 0 && L.max_n <= 16 && L.max_gs * L.max_nr <= 256 && tm_bytes(L) <= 64 * 1024) {
    if (L.max_gs * L.max_nr <= 128)
      GT_LAUNCH_SH((k_fused_t_mfma<1>), dim3(L.total_groups), dim3(256), tm_bytes(L), L.d_chans,
                   L.d_groups, X, A, B, L.ws, do_c);
    else
      GT_LAUNCH_SH((k_fused_t_mfma<2>), dim3(L.total_groups), dim3(256), tm_bytes(L), L.d_chans,
                   L.d_groups, X, A, B, L.ws, do_c);
    return GT_OK;
  }
  GT_LAUNCH_SH(k_fused_t, dim3(L.total_groups), dim3(256), t_bytes(L), L.d_chans, L.d_groups, X, A, B,
               L.ws, do_c & T_MODE);
  return GT_OK;
}

gt_status launch_fused_z(const LaunchCtx& L, const float2* C, float2* G, int do_a, int do_core) {
  GT_LAUNCH_SH(k_fused_z, dim3(L.total_groups), dim3(256), z_bytes(L), L.d_chans, L.d_groups, C, G,
               L.ws, do_a, do_core);
  return GT_OK;
}

static size_t bm_bytes(const LaunchCtx& L) {
  return sizeof(float) * 2 * 64 * ((size_t)L.max_p * L.max_m + 1) +
         sizeof(float2) * ((size_t)L.max_nr * L.max_nt + (size_t)L.max_nr * L.max_m +
                           (size_t)L.max_gs * L.max_p);
}

// The matrix-core variant holds W (p m x 64, planar) and one subcarrier slice in LDS and keeps
// APER (a, j) pairs x PMAX group factors per thread in registers.
bool fused_b_mfma_ok(const LaunchCtx& L) {
  return L.max_nt <= 64 && L.max_p <= 16 && L.max_m * L.max_nt <= 512 && L.max_nr * L.max_nt <= 1024 &&
         bm_bytes(L) <= 64 * 1024;
}

// compile-time slot stride of the launch (0: per channel)
static int bmm_slc(const LaunchCtx& L) { return bmm_slot(L.max_nr, L.max_nt, L.max_m) <= 1024 ? 1024 : 0; }

static size_t bmm_bytes(const LaunchCtx& L) {
  // + 128 floats: step-2 operand reads run up to 127 floats past a slot's last row
  const size_t slots = bmm_slc(L) ? (size_t)16 * bmm_slc(L)
                                  : std::max<size_t>((size_t)L.max_p * bmm_slot(L.max_nr, L.max_nt, L.max_m), 2048);
  return sizeof(float) * (slots + (size_t)L.max_nr * 64 + 128);
}

// All-matrix-core variant: p, m <= 16 (32 real rows of steps 1 and 2), nt <= 64, a group's
// step-1 operands of this wave's column tiles (32 NT1W per wave) held in SMAX x NT1W registers.
static int bmm_variant(const LaunchCtx& L) {
  if (!(L.max_nt <= 64 && L.max_nr <= 16 && L.max_p <= 16 && L.max_m <= 16 &&
        bmm_bytes(L) <= 72 * 1024))
    return 0;
  const int n1 = (L.max_nr * L.max_nt + 31) / 32;
  if (L.max_gs <= 12) return n1 <= 8 ? 1 : (n1 <= 16 ? 2 : 0);
  if (L.max_gs <= 24) return n1 <= 8 ? 3 : 0;
  return 0;
}

gt_status launch_fused_b(const LaunchCtx& L, const float2* X, const float2* A, const float2* C,
                         hipEvent_t pre_reduce, hipEvent_t after_pass) {
  // after_pass, when set, is recorded behind the pass over X; the reduction overwrites the
  // channel's mode-2 Gram, so with pre_reduce set it first waits for that event (an eigensolve
  // of the previous Gram still running on another stream)
  auto wait_pre = [&]() {
    return (!after_pass || hipEventRecord(after_pass, L.stream) == hipSuccess) &&
           (!pre_reduce || hipStreamWaitEvent(L.stream, pre_reduce, 0) == hipSuccess);
  };
  const int v = (L.tune_bstep == 2 && fused_b_mfma_ok(L)) ? 0 : bmm_variant(L);
  if (v) {
    const dim3 grid(L.max_nsplit, L.n_channels);
    const size_t sh = bmm_bytes(L);
    const bool pf = L.tune_bstep == 1 && L.ttm_prec == GT_TTM_FP32;
    const bool slc = bmm_slc(L) != 0;
    // row-quad layout: every channel m == nr <= 8 (one 8 x 128 slot per q)
    const bool ql = slc && L.full_mode1 && L.max_nr <= 8;
#define GT_BMM_S(NT1W, SMAX, PF, PREC)                                                                           \
  if (ql)                                                                                                        \
    GT_LAUNCH_SH((k_fused_b_mm<NT1W, SMAX, PF, PREC, 1024, true>), grid, dim3(512), sh, L.d_chans, X, A, C, L.ws); \
  else if (slc)                                                                                                  \
    GT_LAUNCH_SH((k_fused_b_mm<NT1W, SMAX, PF, PREC, 1024>), grid, dim3(512), sh, L.d_chans, X, A, C, L.ws);       \
  else                                                                                                           \
    GT_LAUNCH_SH((k_fused_b_mm<NT1W, SMAX, PF, PREC, 0>), grid, dim3(512), sh, L.d_chans, X, A, C, L.ws)
#define GT_BMM(NT1W, SMAX, PREC)   \
  if (PREC == 0 && pf) {           \
    GT_BMM_S(NT1W, SMAX, true, 0); \
  } else {                         \
    GT_BMM_S(NT1W, SMAX, false, PREC); \
  }
#define GT_BMM_PREC(NT1W, SMAX)                          \
  switch (L.ttm_prec) {                                  \
    case GT_TTM_BF16: GT_BMM(NT1W, SMAX, 1); break;      \
    case GT_TTM_FP16: GT_BMM(NT1W, SMAX, 2); break;      \
    case GT_TTM_SPLIT_BF16: GT_BMM(NT1W, SMAX, 3); break; \
    default: GT_BMM(NT1W, SMAX, 0); break;               \
  }
    switch (v) {
      case 1: GT_BMM_PREC(1, 12); break;
      case 2: GT_BMM_PREC(2, 12); break;
      default: GT_BMM_PREC(1, 24); break;
    }
#undef GT_BMM_PREC
#undef GT_BMM
#undef GT_BMM_S
    if (!wait_pre()) return GT_ERR_HIP;
    GT_LAUNCH_SH(k_reduce_S2_mfma, dim3(3, L.n_channels), dim3(256), 0,
                 L.d_chans, L.ws);
    return GT_OK;
  }
  if (fused_b_mfma_ok(L)) {
    if (L.max_p <= 4)
      GT_LAUNCH_SH((k_fused_b_mfma<2, 4>), dim3(L.max_nsplit, L.n_channels), dim3(256), bm_bytes(L),
                   L.d_chans, X, A, C, L.ws);
    else if (L.max_p <= 8)
      GT_LAUNCH_SH((k_fused_b_mfma<2, 8>), dim3(L.max_nsplit, L.n_channels), dim3(256), bm_bytes(L),
                   L.d_chans, X, A, C, L.ws);
    else if (L.max_p <= 12)
      GT_LAUNCH_SH((k_fused_b_mfma<2, 12>), dim3(L.max_nsplit, L.n_channels), dim3(256), bm_bytes(L),
                   L.d_chans, X, A, C, L.ws);
    else
      GT_LAUNCH_SH((k_fused_b_mfma<2, 16>), dim3(L.max_nsplit, L.n_channels), dim3(256), bm_bytes(L),
                   L.d_chans, X, A, C, L.ws);
    if (!wait_pre()) return GT_ERR_HIP;
    GT_LAUNCH_SH(k_reduce_S2_mfma, dim3(3, L.n_channels), dim3(256), 0,
                 L.d_chans, L.ws);
    return GT_OK;
  }
  GT_LAUNCH_SH(k_fused_b, dim3(L.max_nsplit, L.n_channels), dim3(256), b_bytes(L), L.d_chans, X, A, C,
               L.ws);
  if (!wait_pre()) return GT_ERR_HIP;
  GT_LAUNCH_SH(k_reduce_S2, dim3((L.max_nt * L.max_nt + 255) / 256, L.n_channels), dim3(256), 0,
               L.d_chans, L.ws);
  return GT_OK;
}

}  // namespace gt
