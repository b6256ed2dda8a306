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
    Yg[o] = v;
  }
  __syncthreads();
  group_gram_s3(Yh, wsp2(ws, ch.w_S3) + (int64_t)it.g * ch.gs * ch.gs, ch.gs, sz, m * n, tid);
}

// Matrix-core variant of k_fused_t.  Stacking the group's rows (s, i) of H gives
// T = H B as one complex (sz nr) x nt by nt x n product.  In real form the K index runs over
// (j, re/im) pairs, k' = 2 j + part, which matches the interleaved storage of H, and
//   A[(s,i)][k'] = (part 0: Re H, part 1: Im H)[s][i][j]
//   Bt[k'][c]    = part 0: (c < n: Re B[j][c], else Im B[j][c - n])
//                  part 1: (c < n: -Im B[j][c], else Re B[j][c - n])
// so that the real product A Bt is [Re T | Im T].  Output tiles are 32 x 32 over rows
// (s, i) and the 2 n real columns (n <= 16: one column tile); tile r goes to wave r % 4.
template <int TPW>
__global__ void __launch_bounds__(256) k_fused_t_mfma(const DevChan* __restrict__ chans,
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
  float* Bt = reinterpret_cast<float*>(smem);        // [2 nt][32]
  float2* As = smem + nt * 32;                        // nr x m
  float2* Ts = As + nr * m;                           // sz x nr x n
  float2* Yh = Ts + ch.gs * nr * n;                   // sz x m x n
  for (int e = tid; e < 2 * nt * 32; e += 256) {
    const int kk = e / 32, c = e % 32, j = kk / 2, part = kk % 2;
    float v = 0.f;
    if (c < 2 * n) {
      const float2 b = B[ch.b + j * n + (c < n ? c : c - n)];
      v = (part == 0) ? (c < n ? b.x : b.y) : (c < n ? -b.y : b.x);
    }
    Bt[e] = v;
  }
  for (int e = tid; e < nr * m; e += 256) As[e] = A[ch.a + e];
  __syncthreads();
  const int rows = sz * nr;
  const int ntile = (rows + 31) / 32;
  const float* Xf = reinterpret_cast<const float*>(X + ch.x + (int64_t)s0 * nr * nt);
  f32x16 acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[u][r] = 0.f;
  const int half = lane / 32, col = lane % 32;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int tile = wave + 4 * u;
    if (tile < ntile) {
      const int row = tile * 32 + col;
      const bool rv = row < rows;
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
  // accumulator element (row 8 (r / 4) + 4 half + r % 4, column col) of tile -> T
  float2* Tg = wsp2(ws, ch.w_T) + (int64_t)s0 * nr * n;
  float* Tsf = reinterpret_cast<float*>(Ts);
  float* Tgf = reinterpret_cast<float*>(Tg);
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
          Tgf[2 * (row * n + c) + part] = acc[u][r];
        }
      }
    }
  }
  if (!do_c) return;
  __syncthreads();
  float2* Yg = wsp2(ws, ch.w_Yh) + (int64_t)s0 * m * n;
  for (int o = tid; o < sz * m * n; o += 256) {
    const int b = o % n;
    const int a = (o / n) % m;
    const int s = o / (m * n);
    Cx<float> acc2{0.f, 0.f};
    for (int i = 0; i < nr; ++i) cfmac(acc2, ld(As + i * m + a), ld(Ts + (s * nr + i) * n + b));
    const float2 v = make_float2(acc2.re, acc2.im);
    Yh[o] = v;
    Yg[o] = v;
  }
  __syncthreads();
  group_gram_s3(Yh, wsp2(ws, ch.w_S3) + (int64_t)it.g * ch.gs * ch.gs, ch.gs, sz, m * n, tid);
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
    const float2* Tg = wsp2(ws, ch.w_T) + (int64_t)s0 * nr * n;
    for (int o = tid; o < pg * nr * n; o += 256) {
      const int q = o / (nr * n), e = o % (nr * n);
      Cx<float> z{0.f, 0.f};
      for (int s = 0; s < sz; ++s) cfmac(z, ld(Cs + s * p + q), ld(Tg + s * nr * n + e));
      Zs[o] = make_float2(z.re, z.im);
    }
    __syncthreads();
    // S1[i][k] = sum_{q, b} Z_q[i][b] conj(Z_q[k][b]); four threads per output split b
    {
      const int o = tid / 4, part = tid % 4;
      float ar = 0.f, ai = 0.f;
      if (o < nr * nr) {
        const int i = o / nr, k = o % nr;
        for (int q = 0; q < pg; ++q) {
          const float2* zq = Zs + q * nr * n;
          for (int b = part; b < n; b += 4) {
            float2 zi = zq[i * n + b], zk = zq[k * n + b];
            ar += zi.x * zk.x + zi.y * zk.y;
            ai += zi.y * zk.x - zi.x * zk.y;
          }
        }
      }
      ar += __shfl_xor(ar, 1, 64);
      ai += __shfl_xor(ai, 1, 64);
      ar += __shfl_xor(ar, 2, 64);
      ai += __shfl_xor(ai, 2, 64);
      if (o < nr * nr && part == 0)
        wsp2(ws, ch.w_S1p)[(int64_t)it.g * nr * nr + o] = make_float2(ar, ai);
    }
  }
  if (do_core) {
    const int mn = m * n;
    const float2* Yg = wsp2(ws, ch.w_Yh) + (int64_t)s0 * mn;
    for (int o = tid; o < p * mn; o += 256) {
      const int q = o / mn, e = o % mn;
      Cx<float> acc{0.f, 0.f};
      if (q < pg)
        for (int s = 0; s < sz; ++s) cfmac(acc, ld(Cs + s * p + q), ld(Yg + s * mn + e));
      G[ch.g + (int64_t)it.g * p * mn + o] = make_float2(acc.re, acc.im);
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

// S2 = sum over splits of the complex Gram assembled from the real blocks of R^T R
// (upper 32 x 32 tiles stored; lower entries by symmetry).
__global__ void k_reduce_S2_mfma(const DevChan* __restrict__ chans, char* ws) {
  const DevChan& ch = chans[blockIdx.y];
  const int nt = ch.nt;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt * nt) return;
  const int j = e / nt, k = e % nt;
  const float* P = reinterpret_cast<const float*>(ws + ch.w_S2p);
  auto at = [&](const float* Q, int a, int b) {
    return ((a >> 5) <= (b >> 5)) ? Q[a * 128 + b] : Q[b * 128 + a];
  };
  float re = 0.f, im = 0.f;
  for (int sp = 0; sp < ch.nsplit; ++sp) {
    const float* Q = P + (int64_t)sp * 128 * 128;
    re += at(Q, j, k) + at(Q, 64 + j, 64 + k);
    im += at(Q, j, 64 + k) - at(Q, 64 + j, k);
  }
  reinterpret_cast<float2*>(ws + ch.w_S2)[e] = make_float2(re, im);
}

// ---------------------------------------------------------------------------------------
// host side

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
  return sizeof(float2) * ((size_t)L.max_nt * 32 + (size_t)L.max_nr * L.max_m +
                           (size_t)L.max_gs * L.max_nr * L.max_n + (size_t)L.max_gs * L.max_m * L.max_n);
}

gt_status launch_fused_t(const LaunchCtx& L, const float2* X, const float2* A, const float2* B,
                         int do_c) {
  // matrix cores when the real output fits one column tile and at most 8 row tiles
  if (L.max_n <= 16 && L.max_gs * L.max_nr <= 256 && tm_bytes(L) <= 64 * 1024) {
    if (L.max_gs * L.max_nr <= 128)
      GT_LAUNCH_SH((k_fused_t_mfma<1>), dim3(L.total_groups), dim3(256), tm_bytes(L), L.d_chans,
                   L.d_groups, X, A, B, L.ws, do_c);
    else
      GT_LAUNCH_SH((k_fused_t_mfma<2>), dim3(L.total_groups), dim3(256), tm_bytes(L), L.d_chans,
                   L.d_groups, X, A, B, L.ws, do_c);
    return GT_OK;
  }
  GT_LAUNCH_SH(k_fused_t, dim3(L.total_groups), dim3(256), t_bytes(L), L.d_chans, L.d_groups, X, A, B,
               L.ws, do_c);
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

gt_status launch_fused_b(const LaunchCtx& L, const float2* X, const float2* A, const float2* C) {
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
    GT_LAUNCH_SH(k_reduce_S2_mfma, dim3((L.max_nt * L.max_nt + 255) / 256, L.n_channels), dim3(256), 0,
                 L.d_chans, L.ws);
    return GT_OK;
  }
  GT_LAUNCH_SH(k_fused_b, dim3(L.max_nsplit, L.n_channels), dim3(256), b_bytes(L), L.d_chans, X, A, C,
               L.ws);
  GT_LAUNCH_SH(k_reduce_S2, dim3((L.max_nt * L.max_nt + 255) / 256, L.n_channels), dim3(256), 0,
               L.d_chans, L.ws);
  return GT_OK;
}

}  // namespace gt
