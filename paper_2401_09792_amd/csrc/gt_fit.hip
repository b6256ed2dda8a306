// Groupwise Tucker fit on the GPU: HOSVD initialisation, alternating (Gauss-Seidel) factor
// updates and the final cores (Section 3.2: equations "update A", "update B", "update C",
// "kernel" and the groupwise compression algorithm).
//
// Matrix forms used by the kernels, for the subcarrier slices H_s of one group g:
//   A-step   Z_q = sum_s conj(C[s,q]) H_s B,      S1 = sum_{g,q} Z_q Z_q^H        (nr x nr)
//   B-step   Y_s = A^H H_s, W_q = sum_s conj(C[s,q]) Y_s,  S2 = sum_{g,q} W_q^H W_q (nt x nt)
//   C-step   Yh_s = Y_s B,  S3_g[s,s'] = <Yh_s, Yh_s'>                          (gs x gs)
//   core     G_g[q] = sum_s conj(C[s,q]) Yh_s
// These are the unfolded Grams of the paper's tensor expressions with the mode-2 factor in
// matrix form (B = conj of the tensor-form factor).  After each half-step the objective is
// f = ||X||^2 - (sum of the kept eigenvalues), since ||G||^2 = tr(U^H S U) at the maximiser.
#include <hip/hip_runtime.h>

#include "gt_device.h"
#include "gt_internal.h"
#include "gt_rows.h"

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace gt {

#define CH_BEGIN(ch_index)                   \
  const DevChan& ch = chans[(ch_index)];     \
  (void)ch;

__device__ __forceinline__ float2* wsp(char* ws, int64_t off) {
  return reinterpret_cast<float2*>(ws + off);
}
__device__ __forceinline__ double* wsd(char* ws, int64_t off) {
  return reinterpret_cast<double*>(ws + off);
}

// ---------------------------------------------------------------------------------------
// Initial Grams of one group: S1 partial = sum_s H_s H_s^H (want_s1), S3_g[s,s'] = <H_s, H_s'>,
// and the group's squared norm.  The group's slices are staged through LDS in chunks.
__global__ void __launch_bounds__(256) k_init_group(const DevChan* __restrict__ chans,
                                                    const GroupItem* __restrict__ items,
                                                    const float2* __restrict__ X, char* ws,
                                                    int want_s1) {
  constexpr int CHUNK = 4096;  // complex elements staged at a time (32 KB)
  __shared__ float2 xs[CHUNK];
  __shared__ double red[256];
  const GroupItem it = items[blockIdx.x];
  CH_BEGIN(it.ch);
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  const int nr = ch.nr, nt = ch.nt, gs = ch.gs;
  const int slice = nr * nt;
  const float2* Xg = X + ch.x + (int64_t)s0 * slice;
  const int tid = threadIdx.x;
  // outputs of this thread: S1 entries o1 = tid (nr*nr <= 256) and S3 entries tid, tid+256, ...
  Cx<float> a1{0.f, 0.f};
  Cx<float> a3[4] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
  double nrm = 0.0;
  // columns j are chunked so that sz * nr * jc <= CHUNK
  const int jc = max(1, min(nt, CHUNK / (sz * nr)));
  for (int j0 = 0; j0 < nt; j0 += jc) {
    const int jw = min(jc, nt - j0);
    __syncthreads();
    for (int e = tid; e < sz * nr * jw; e += 256) {
      const int j = e % jw, si = e / jw;
      const float2 v = Xg[(int64_t)si * nt + j0 + j];
      xs[e] = v;
      nrm += (double)v.x * v.x + (double)v.y * v.y;
    }
    __syncthreads();
    if (want_s1 && tid < nr * nr) {
      const int i = tid / nr, k = tid % nr;
      for (int s = 0; s < sz; ++s)
        for (int j = 0; j < jw; ++j)  // H[i][j] conj(H[k][j])
          cfmac(a1, ld(xs + (s * nr + k) * jw + j), ld(xs + (s * nr + i) * jw + j));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = tid + 256 * u;
      if (o < gs * gs) {
        const int s = o / gs, t = o % gs;
        if (s < sz && t < sz)
          for (int e = 0; e < nr * jw; ++e)  // H_s conj(H_t)
            cfmac(a3[u], ld(xs + t * nr * jw + e), ld(xs + s * nr * jw + e));
      }
    }
  }
  if (want_s1 && tid < nr * nr) st(wsp(ws, ch.w_S1p) + (int64_t)it.g * nr * nr + tid, a1);
  float2* S3 = wsp(ws, ch.w_S3) + (int64_t)it.g * gs * gs;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int o = tid + 256 * u;
    if (o < gs * gs) st(S3 + o, a3[u]);
  }
  red[tid] = nrm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) wsd(ws, ch.w_lamg)[it.g] = red[0];
}

// The same for groups of at most 8192 complex entries, staged whole: 16 lanes per output over
// the upper triangles of S1 (over (s, j)) and S3 (over (i, j)), mirrored below; 512 threads, so
// that the two blocks per CU that the 64 KB stage allows keep 16 waves busy.
__global__ void __launch_bounds__(512) k_init_group_lds(const DevChan* __restrict__ chans,
                                                        const GroupItem* __restrict__ items,
                                                        const float2* __restrict__ X, char* ws,
                                                        int want_s1) {
  __shared__ float2 xs[8192];
  __shared__ double red[512];
  const GroupItem it = items[blockIdx.x];
  CH_BEGIN(it.ch);
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  const int nr = ch.nr, nt = ch.nt, gs = ch.gs;
  const int slice = nr * nt, tot = sz * slice;
  const float2* Xg = X + ch.x + (int64_t)s0 * slice;
  const int tid = threadIdx.x, l16 = tid % 16;
  double nrm = 0.0;
  // each thread issues up to 12 loads before its LDS stores: one memory latency per pass
  constexpr int B = 12;
  for (int e0 = tid; e0 < tot; e0 += B * 512) {
    float2 v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + 512 * u;
      v[u] = e < tot ? Xg[e] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + 512 * u;
      if (e < tot) {
        xs[e] = v[u];
        nrm += (double)v[u].x * v[u].x + (double)v[u].y * v[u].y;
      }
    }
  }
  __syncthreads();
  const int n1 = want_s1 ? nr * (nr + 1) / 2 : 0, n3 = gs * (gs + 1) / 2;
  float2* S1 = wsp(ws, ch.w_S1p) + (int64_t)it.g * nr * nr;
  float2* S3 = wsp(ws, ch.w_S3) + (int64_t)it.g * gs * gs;
  for (int k = tid / 16; k < n1 + n3; k += 32) {
    const bool one = k < n1;
    const int dim = one ? nr : gs;
    int a = 0, rem = one ? k : k - n1;
    while (rem >= dim - a) {
      rem -= dim - a;
      ++a;
    }
    const int b = a + rem;
    float ar = 0.f, ai = 0.f;
    if (one) {
      // S1[a][b] = sum_{s, j} H_s[a][j] conj(H_s[b][j])
      for (int s = 0; s < sz; ++s)
#pragma unroll 8
        for (int j = l16; j < nt; j += 16) {
          const float2 x = xs[s * slice + a * nt + j], y = xs[s * slice + b * nt + j];
          ar += x.x * y.x + x.y * y.y;
          ai += x.y * y.x - x.x * y.y;
        }
    } else if (b < sz) {
      // S3[a][b] = <H_a, H_b> = sum_e H_a[e] conj(H_b[e])
#pragma unroll 8
      for (int e = l16; e < slice; e += 16) {
        const float2 x = xs[a * slice + e], y = xs[b * slice + e];
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
      float2* S = one ? S1 : S3;
      S[a * dim + b] = make_float2(ar, ai);
      if (a != b) S[b * dim + a] = make_float2(ar, -ai);
    }
  }
  red[tid] = nrm;
  __syncthreads();
  for (int o = 256; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) wsd(ws, ch.w_lamg)[it.g] = red[0];
}

// Sum of the per-group norms: scal[0] = ||X||^2.
__global__ void k_norm_total(const DevChan* __restrict__ chans, int n_channels, char* ws) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_channels) return;
  CH_BEGIN(c);
  const double* lg = wsd(ws, ch.w_lamg);
  double s = 0.0;
  for (int g = 0; g < ch.ngroups; ++g) s += lg[g];
  wsd(ws, ch.w_scal)[0] = s;
}

// ---------------------------------------------------------------------------------------
// Split-row Gram: partial[split][j][k] = sum over the split's rows of conj(M[row][j]) M[row][k].
// which = 0: rows of X (nsc*nr rows of length nt).  which = 1: rows of W.
__global__ void __launch_bounds__(256) k_gram_rows(const DevChan* __restrict__ chans,
                                                   const float2* __restrict__ X, char* ws,
                                                   int which) {
  CH_BEGIN(blockIdx.z);
  const int nt = ch.nt;
  const int tiles = (nt + 15) / 16;
  const int tj = blockIdx.x / tiles, tk = blockIdx.x % tiles;
  if (tj >= tiles) return;
  const int split = blockIdx.y;
  if (split >= ch.nsplit) return;
  const float2* M;
  int64_t nrows;
  if (which == 0) {
    M = X + ch.x;
    nrows = (int64_t)ch.nsc * ch.nr;
  } else {
    M = wsp(ws, ch.w_W);
    nrows = (int64_t)ch.ngroups * ch.p * ch.m;
  }
  const int64_t chunk = (nrows + ch.nsplit - 1) / ch.nsplit;
  const int64_t r0 = split * chunk;
  const int64_t r1 = min(nrows, r0 + chunk);
  __shared__ float2 a_t[16][17];
  __shared__ float2 b_t[16][17];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int j = tj * 16 + ty, k = tk * 16 + tx;
  Cx<float> acc{0.f, 0.f};
  for (int64_t rb = r0; rb < r1; rb += 16) {
    // load 16 rows x 16 cols for both column blocks
    {
      const int lr = threadIdx.x / 16, lc = threadIdx.x % 16;
      const int64_t row = rb + lr;
      float2 va = make_float2(0.f, 0.f), vb = make_float2(0.f, 0.f);
      if (row < r1) {
        if (tj * 16 + lc < nt) va = M[row * nt + tj * 16 + lc];
        if (tk * 16 + lc < nt) vb = M[row * nt + tk * 16 + lc];
      }
      a_t[lr][lc] = va;
      b_t[lr][lc] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      float2 a = a_t[rr][ty], b = b_t[rr][tx];
      cfmac(acc, Cx<float>{a.x, a.y}, Cx<float>{b.x, b.y});
    }
    __syncthreads();
  }
  if (j < nt && k < nt) st(wsp(ws, ch.w_S2p) + ((int64_t)split * nt + j) * nt + k, acc);
}

// S1 = sum of the per-group partials (fixed order, four independent accumulators).
// S1 = sum of the per-group partials: the four waves of the block each sum a quarter of the
// groups (four interleaved accumulators per entry), then the quarters are added in order.
__global__ void __launch_bounds__(256) k_reduce_S1(const DevChan* __restrict__ chans, char* ws) {
  CH_BEGIN(blockIdx.y);
  __shared__ float2 part[4][kMaxNr * kMaxNr];
  const int nn = ch.nr * ch.nr;
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  const int g0 = (int)((int64_t)w * ch.ngroups / 4), g1 = (int)((int64_t)(w + 1) * ch.ngroups / 4);
  const float2* P = wsp(ws, ch.w_S1p);
  for (int e = l; e < nn; e += 64) {
    float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
    int g = g0;
    for (; g + 4 <= g1; g += 4)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float2 v = P[(int64_t)(g + u) * nn + e];
        ar[u] += v.x;
        ai[u] += v.y;
      }
    for (; g < g1; ++g) {
      float2 v = P[(int64_t)g * nn + e];
      ar[0] += v.x;
      ai[0] += v.y;
    }
    part[w][e] = make_float2((ar[0] + ar[1]) + (ar[2] + ar[3]), (ai[0] + ai[1]) + (ai[2] + ai[3]));
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += 256) {
    const float2 a0 = part[0][e], a1 = part[1][e], a2 = part[2][e], a3 = part[3][e];
    st(wsp(ws, ch.w_S1) + e, Cx<float>{(a0.x + a1.x) + (a2.x + a3.x), (a0.y + a1.y) + (a2.y + a3.y)});
  }
}

// S2 = sum of the split partials (fixed order).
__global__ void k_reduce_S2(const DevChan* __restrict__ chans, char* ws) {
  CH_BEGIN(blockIdx.y);
  const int nt = ch.nt;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt * nt) return;
  const float2* P = wsp(ws, ch.w_S2p);
  Cx<float> acc{0.f, 0.f};
  for (int sp = 0; sp < ch.nsplit; ++sp) {
    float2 v = P[(int64_t)sp * nt * nt + e];
    acc.re += v.x;
    acc.im += v.y;
  }
  st(wsp(ws, ch.w_S2) + e, acc);
}

// ---------------------------------------------------------------------------------------
// Eigen kernels: top eigenvectors (descending, canonical phase) of the mode-1 Gram (sum of
// the per-group partials), the mode-2 Gram, and each group's mode-3 Gram.

template <typename T, int MP>
__device__ __forceinline__ void eig_finish(EigLds<T, MP>& L, int r, int d, int rk, float2* dst, int ld,
                           int rpad, double* lamsum, int32_t* status, bool conv) {
  eig_sort_desc<T, MP>(L, r, d);
  double ls = 0.0;
  for (int j = 0; j < rpad; ++j) {
    if (j < rk) {
      const int col = L.src[j];
      Cx<T> ph = canonical_phase<T, MP>(L, r, d, col);
      if (r < d && dst) {
        Cx<T> v{L.vr[r][col], L.vi[r][col]};
        Cx<T> o = cmul(v, ph);
        dst[(int64_t)r * ld + j] = make_float2((float)o.re, (float)o.im);
      }
      ls += (double)L.lam[col];
    } else if (r < d && dst) {
      dst[(int64_t)r * ld + j] = make_float2(0.f, 0.f);
    }
  }
  if (r == 0) {
    if (lamsum) *lamsum = ls;
    if (status) {
      uint32_t bits = conv ? 0u : GT_DEV_EIG_SWEEPS;
      if (!(ls == ls) || ls > 1e300 || ls < -1e300) bits |= GT_DEV_NONFINITE;
      if (bits) atomicOr(reinterpret_cast<unsigned int*>(status), bits);
    }
  }
}

// Warm starts (FP32 eigensolves only): every eigen kernel stores its full eigenbasis in the
// workspace; the next call on the same Gram family rotates the new Gram into that basis
// before the sweeps, so only the change since the last call remains to be diagonalised.

template <typename T, int MP>
__device__ __forceinline__ void load_basis(EigLds<T, MP>& L, const float2* V, int r) {
  for (int j = 0; j < MP; ++j) {
    float2 v = V[r * MP + j];
    L.vr[r][j] = (T)v.x;
    L.vi[r][j] = (T)v.y;
  }
}

template <typename T, int MP>
__device__ __forceinline__ void store_basis(const EigLds<T, MP>& L, float2* V, int r) {
  for (int j = 0; j < MP; ++j) V[r * MP + j] = make_float2((float)L.vr[r][j], (float)L.vi[r][j]);
}

// mode-1: one MP-lane group per channel
template <typename T, int MP>
__global__ void __launch_bounds__(64, (sizeof(T) == 4 && MP == 16) ? 2 : 1) k_eigA(const DevChan* __restrict__ chans, int n_channels,
                                              char* ws, float2* A, int32_t* status, int warm) {
  constexpr int GPW = 64 / MP;
  __shared__ EigLds<T, MP> lds[GPW];
  const int grp = threadIdx.x / MP, r = threadIdx.x % MP;
  const int c = blockIdx.x * GPW + grp;
  EigLds<T, MP>& L = lds[grp];
  const bool valid = c < n_channels;
  const DevChan* chp = valid ? &chans[c] : nullptr;
  const int d = valid ? chp->nr : 0;
  const bool use_warm = warm && sizeof(T) == 4;
  if (use_warm) {
    if (valid)
      load_basis<T, MP>(L, wsp(ws, chp->w_VA), r);
    else
      for (int j = 0; j < MP; ++j) {
        L.vr[r][j] = (j == r) ? T(1) : T(0);
        L.vi[r][j] = T(0);
      }
    wave_sync();
    reorthonormalize_r<T, MP>(L, r);
  }
  for (int j = 0; j < MP; ++j) {
    T sr = 0, si = 0;
    if (r < d && j < d) {
      float2 v = wsp(ws, chp->w_S1)[(int64_t)r * d + j];
      sr = (T)v.x;
      si = (T)v.y;
    }
    L.kr[r][j] = sr;
    L.ki[r][j] = si;
  }
  wave_sync();
  if (use_warm) rotate_into_basis_r<T, MP>(L, r);
  wave_sync();
  bool conv = jacobi_herm<T, MP, 1>(L, r, 0, sizeof(T) == 4 ? 12 : 20, use_warm);
  if (valid) {
    if (sizeof(T) == 4) store_basis<T, MP>(L, wsp(ws, chp->w_VA), r);
    double* ls = wsd(ws, chp->w_scal) + 1;
    eig_finish<T, MP>(L, r, d, chp->m, A + chp->a, chp->m, chp->m, ls,
                      status ? status + c : nullptr, conv);
  } else {
    eig_sort_desc<T, MP>(L, r, 0);
  }
}

// Mode-2 solve by Rayleigh-Ritz (FP32, nt <= 64, n <= 16), one 256-thread block per channel, on
// the previous call's top-n basis (warm: Bp the current B, the last solve's n leading
// eigenvectors of this channel's Gram family) or on an orthonormal basis of S2 Omega (cold, see
// eigB_cold_block): Y = S2 Bp, H = Bp^H Y, H = U diag(theta) U^H, the
// residual R = Y - Bp H.  The Ritz pairs (Bp U, theta) are the n leading eigenpairs of S2 to FP32
// accuracy when every Ritz vector z_j = Bp U[:, j] has ||S2 z_j - theta_j z_j|| <= 1e-5 theta_max
// (Bp spans an invariant subspace of a Gram within that distance of S2, which is about the
// rounding S2 itself carries after its FP32 accumulation over every subcarrier; the residual of
// z_j is the norm of R U[:, j]) and the complement's
// trace tr(S2) - sum(theta) does not exceed theta_min + 1e-5 tr(S2) (no eigenvalue outside that
// subspace lies above the kept ones, up to the Gram's rounding); then B = Bp U (descending, each
// column's largest-modulus entry real positive) and the call returns true.  Otherwise it returns
// false and the caller runs the full Jacobi.  Run by the 256 threads of k_eigB's block, in its
// LDS (before the Jacobi's own use of it).
constexpr int kRitzN = 16;
struct RitzLds {
  float2 s[64][65];               // S2 (zero past nt)
  float2 b[64][kRitzN];           // the previous basis
  float2 y[64][kRitzN];           // S2 Bp
  float2 h[kRitzN][kRitzN + 1];   // Bp^H Y, then U (rows)
  float2 g[kRitzN][kRitzN + 1];   // R^H R
  float res[kRitzN];              // ||S2 z_j - theta_j z_j||^2 per Ritz vector
  float4 rot[kRitzN];
  float lam[kRitzN];
  int src[kRitzN];
  float red[4];
  int cold_ok;
};

// Cold start of the Rayleigh-Ritz step: Bp = an orthonormal basis of S2 (S2 Omega), two steps
// of subspace iteration from a fixed pseudo-random d x n block Omega of (+-1) + i (+-1)
// entries.  When S2 has rank r <= n (a channel with at most n paths), S2 Omega already spans
// its range, but the rounding of Y = S2 Omega leaves the directions of the smallest nonzero
// eigenvalues tilted by about eps theta_max / theta_r; the second product removes that tilt.
// A column that vanishes under the orthogonalisation (rank below n) is replaced by a unit
// vector made orthogonal to the others, which then lies in the numerical null space.  Channels
// of higher rank fail the Ritz acceptance test and go to the Jacobi.
//
// Wave 0 orthonormalises the rows in L.y (row i in lane i) into L.b by classical Gram-Schmidt
// applied twice per column; returns false (in every thread) if a column could not be completed.
__device__ __forceinline__ bool eigB_cold_orth(RitzLds& L, int d, int n) {
  constexpr int NB = kRitzN;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  if (wave == 0) {
    float br[NB], bi[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      br[j] = lane < d ? L.y[lane][j].x : 0.f;
      bi[j] = lane < d ? L.y[lane][j].y : 0.f;
    }
    float scale = 0.f;
#pragma unroll
    for (int j = 0; j < NB; ++j) scale = fmaxf(scale, group_sum<64>(br[j] * br[j] + bi[j] * bi[j]));
    // a column is kept when its norm after the projections is above 1e-6 of the largest column's:
    // directions of eigenvalues down to about 1e-6 theta_max survive the products, rounding noise
    // does not
    const float tol2 = 1e-12f * scale;
    int u = 0;  // next unit-vector candidate
    bool good = scale > 0.f;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (k < n) {
        float nrm2 = 0.f;
        bool found = false;
        for (int attempt = 0; attempt <= d; ++attempt) {
#pragma unroll
          for (int pass = 0; pass < 2; ++pass) {
            // classical Gram-Schmidt, twice: the k projections b_j^H b_k reduce independently
            float dr[NB], di[NB];
#pragma unroll
            for (int j = 0; j < k; ++j) {
              dr[j] = group_sum<64>(br[j] * br[k] + bi[j] * bi[k]);
              di[j] = group_sum<64>(br[j] * bi[k] - bi[j] * br[k]);
            }
#pragma unroll
            for (int j = 0; j < k; ++j) {
              br[k] -= dr[j] * br[j] - di[j] * bi[j];
              bi[k] -= dr[j] * bi[j] + di[j] * br[j];
            }
          }
          nrm2 = group_sum<64>(br[k] * br[k] + bi[k] * bi[k]);
          if (nrm2 > (attempt == 0 ? tol2 : 0.05f)) {
            found = true;
            break;
          }
          if (u >= d) break;
          br[k] = lane == u ? 1.f : 0.f;  // replace by e_u, orthogonalised on the next pass
          bi[k] = 0.f;
          ++u;
        }
        good = good && found;
        const float inv = found ? __builtin_amdgcn_rsqf(nrm2) : 0.f;
        br[k] *= inv;
        bi[k] *= inv;
      } else {
        br[k] = bi[k] = 0.f;
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) L.b[lane][j] = make_float2(lane < d ? br[j] : 0.f, lane < d ? bi[j] : 0.f);
    if (lane == 0) L.cold_ok = good ? 1 : 0;
  }
  __syncthreads();
  return L.cold_ok != 0;
}

// Y = S2 Bp into L.y: thread (row i, four columns)
__device__ __forceinline__ void eigB_s_times_b(RitzLds& L) {
  const int t = threadIdx.x, i = t / 4, j0 = 4 * (t % 4);
  float yr[4] = {0.f, 0.f, 0.f, 0.f}, yi[4] = {0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < 64; ++k) {
    const float2 a = L.s[i][k];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const float2 bv = L.b[k][j0 + jj];
      yr[jj] += a.x * bv.x - a.y * bv.y;
      yi[jj] += a.x * bv.y + a.y * bv.x;
    }
  }
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) L.y[i][j0 + jj] = make_float2(yr[jj], yi[jj]);
}

__device__ __forceinline__ bool eigB_cold_block(RitzLds& L, int d, int n) {
  {
    // Y = S2 Omega, Omega[k][j] = (+-1) + i (+-1), the signs two bits of a multiplicative hash
    // of (k, j)
    const int t = threadIdx.x, i = t / 4, j0 = 4 * (t % 4);
    float yr[4] = {0.f, 0.f, 0.f, 0.f}, yi[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < d; ++k) {
      const float2 a = L.s[i][k];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const unsigned hsh = ((unsigned)k * 2654435761u) ^ ((unsigned)(j0 + jj + 1) * 40503u);
        const float cs = (hsh & 0x10000u) ? 1.f : -1.f, sn = (hsh & 0x20000u) ? 1.f : -1.f;
        yr[jj] += a.x * cs - a.y * sn;
        yi[jj] += a.x * sn + a.y * cs;
      }
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      L.y[i][j0 + jj] = (j0 + jj < n) ? make_float2(yr[jj], yi[jj]) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  if (!eigB_cold_orth(L, d, n)) return false;
  eigB_s_times_b(L);
  __syncthreads();
  return eigB_cold_orth(L, d, n);
}

__device__ __forceinline__ bool eigB_ritz(RitzLds& L, const DevChan& ch, int c, char* ws, float2* B,
                                          int32_t* status, bool cold) {
  constexpr int NB = kRitzN;
  const int t = threadIdx.x, lane = t % 64, wave = t / 64;
  const int d = ch.nt, n = ch.n;
  double* sc = wsd(ws, ch.w_scal);
  if (d > 64 || n > NB) return false;
  const float2* S = wsp(ws, ch.w_S2);
  for (int e = t; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    L.s[i][j] = (i < d && j < d) ? S[(int64_t)i * d + j] : make_float2(0.f, 0.f);
  }
  if (!cold)
    for (int e = t; e < 64 * NB; e += 256) {
      const int i = e / NB, j = e % NB;
      L.b[i][j] = (i < d && j < n) ? B[ch.b + (int64_t)i * n + j] : make_float2(0.f, 0.f);
    }
  __syncthreads();
  // a starting block that is not orthonormal (a column could not be completed) goes to the
  // Jacobi; the barrier keeps every read of cold_ok before the LDS is reused
  if (cold && !eigB_cold_block(L, d, n)) {
    __syncthreads();
    return false;
  }
  // Y = S2 Bp
  eigB_s_times_b(L);
  __syncthreads();
  // H = Bp^H Y: thread (a, b)
  {
    const int a = t / NB, b = t % NB;
    float hr = 0.f, hi = 0.f;
    for (int k = 0; k < 64; ++k) {
      const float2 x = L.b[k][a], y = L.y[k][b];
      hr += x.x * y.x + x.y * y.y;
      hi += x.x * y.y - x.y * y.x;
    }
    L.h[a][b] = make_float2(hr, hi);
  }
  __syncthreads();
  // residual R = Y - Bp H into L.y (all threads), then its Gram R^H R (waves 1-3) while wave 0
  // diagonalises H on 16 lanes
  {
    const int i = t / 4, j0 = 4 * (t % 4);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      float xr = L.y[i][j0 + jj].x, xi = L.y[i][j0 + jj].y;
      for (int k = 0; k < NB; ++k) {
        const float2 bv = L.b[i][k], hv = L.h[k][j0 + jj];
        xr -= bv.x * hv.x - bv.y * hv.y;
        xi -= bv.x * hv.y + bv.y * hv.x;
      }
      L.y[i][j0 + jj] = make_float2(xr, xi);
    }
  }
  float trs = (t < 64 && t < d) ? L.s[t][t].x : 0.f;
  bool conv = true;
  float ur[NB], ui[NB];
  __syncthreads();  // every read of H and every entry of R are done
  if (wave > 0) {
    for (int e = t - 64; e < NB * NB; e += 192) {
      const int a = e / NB, b = e % NB;
      float gr = 0.f, gi = 0.f;
      for (int k = 0; k < 64; ++k) {
        const float2 x = L.y[k][a], y = L.y[k][b];
        gr += x.x * y.x + x.y * y.y;
        gi += x.x * y.y - x.y * y.x;
      }
      L.g[a][b] = make_float2(gr, gi);
    }
  }
  if (wave == 0 && lane < NB) {
    float kr[NB], ki[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const bool on = lane < n && j < n;
      kr[j] = on ? L.h[lane][j].x : 0.f;
      ki[j] = on ? L.h[lane][j].y : 0.f;
    }
    conv = rows_eig<NB>(L.rot, lane, kr, ki, ur, ui, false, 64.f, 12);
    float me = 0.f;
#pragma unroll
    for (int j = 0; j < NB; ++j) me = (j == lane) ? kr[j] : me;
    L.lam[lane] = lane < n ? me : -__builtin_huge_valf();
  }
  // block sum: tr(S2)
  trs = group_sum<64>(trs);
  __syncthreads();
  if (lane == 0) L.red[wave] = trs;
  if (wave == 0 && lane < NB) {
    // U rows to LDS (row lane of U), and the descending order of theta
#pragma unroll
    for (int j = 0; j < NB; ++j) L.h[lane][j] = make_float2(ur[j], ui[j]);
    const float mine = L.lam[lane];
    int rank = 0;
    for (int j = 0; j < NB; ++j) {
      const float o = L.lam[j];
      rank += (o > mine || (o == mine && j < lane)) ? 1 : 0;
    }
    L.src[rank] = lane;
  }
  __syncthreads();
  if (t < NB) {
    // residual of Ritz vector z_t = Bp U[:, t]: U[:, t]^H (R^H R) U[:, t]
    float acc = 0.f;
    if (t < n)
      for (int a = 0; a < NB; ++a) {
        float vr = 0.f, vi = 0.f;  // (G U[:, t])_a
        for (int b = 0; b < NB; ++b) {
          const float2 gv = L.g[a][b], uv = L.h[b][t];
          vr += gv.x * uv.x - gv.y * uv.y;
          vi += gv.x * uv.y + gv.y * uv.x;
        }
        const float2 ua = L.h[a][t];
        acc += ua.x * vr + ua.y * vi;
      }
    L.res[t] = acc;
  }
  const float tr_s = (L.red[0] + L.red[1]) + (L.red[2] + L.red[3]);
  float th_max = L.lam[L.src[0]], th_min = L.lam[L.src[n - 1]];
  float th_sum = 0.f;
  for (int j = 0; j < n; ++j) th_sum += L.lam[j];
  const int conv_all = __syncthreads_and(conv ? 1 : 0);
  float r2 = 0.f;
  for (int j = 0; j < n; ++j) r2 = fmaxf(r2, L.res[j]);
  const bool ok = conv_all && th_max > 0.f && r2 <= 1.0e-10f * th_max * th_max &&
                  tr_s - th_sum <= th_min + 1.0e-5f * tr_s;
  if (!ok) {
    __syncthreads();  // every read of the Ritz data is done before the Jacobi reuses the LDS
    return false;
  }
  // B = Bp U, column j from Ritz vector src[j], with its phase: thread (column j = t / 16, rows
  // (t % 16) + 16 k)
  {
    const int j = t / 16, l16 = t % 16;
    const int col = L.src[j < n ? j : 0];
    float vr[4], vi[4], mag = -1.f;
    int idx = 1 << 30;
    float pr = 0.f, pi = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = l16 + 16 * k;
      float ar = 0.f, ai = 0.f;
      for (int q = 0; q < NB; ++q) {
        const float2 bv = L.b[i][q], u = L.h[q][col];
        ar += bv.x * u.x - bv.y * u.y;
        ai += bv.x * u.y + bv.y * u.x;
      }
      vr[k] = ar;
      vi[k] = ai;
      const float mg = (i < d) ? ar * ar + ai * ai : -1.f;
      if (mg > mag) {  // rows ascend with k: the first maximum is the lowest row
        mag = mg;
        idx = i;
        pr = ar;
        pi = ai;
      }
    }
    rows_argmax<16>(mag, idx, pr, pi);
    const float mod = __builtin_sqrtf(pr * pr + pi * pi);
    float phr = 1.f, phi = 0.f;
    if (mod > 0.f) {
      phr = pr / mod;
      phi = -pi / mod;
    }
    if (j < n) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = l16 + 16 * k;
        if (i < d) B[ch.b + (int64_t)i * n + j] = make_float2(vr[k] * phr - vi[k] * phi, vr[k] * phi + vi[k] * phr);
      }
    }
  }
  if (t == 0) {
    double ls = 0.0;
    for (int j = 0; j < n; ++j) ls += (double)L.lam[L.src[j]];
    sc[2] = ls;
    uint32_t bits = 0u;
    if (!(ls == ls) || ls > 1e300 || ls < -1e300) bits |= GT_DEV_NONFINITE;
    if (bits && status) atomicOr(reinterpret_cast<unsigned int*>(status + c), bits);
  }
  return true;
}

// mode-2: one block of NW waves per channel, nt <= 64
template <typename T, int NW>
__global__ void __launch_bounds__(64 * NW) k_eigB(const DevChan* __restrict__ chans, char* ws,
                                                  float2* B, int32_t* status, int warm, int ritz) {
  constexpr int MP = 64;
  constexpr bool kWarmOk = sizeof(T) == 4 && NW == 4;
  __shared__ EigLds<T, MP> L;
  const int r = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int c = blockIdx.x;
  const DevChan& ch = chans[c];
  const int d = ch.nt;
  if (d > MP) return;  // wide arrays: subspace-iteration kernel
  if (kWarmOk && ritz) {
    // FP32 solve: the Rayleigh-Ritz step first, in this block's LDS, on the previous basis
    // (warm) or on a basis of S2 Omega (cold)
    static_assert(sizeof(RitzLds) <= sizeof(EigLds<float, 64>), "Ritz data must fit the Jacobi LDS");
    if (eigB_ritz(*reinterpret_cast<RitzLds*>(&L), ch, c, ws, B, status, !warm)) {
      // after a cold start the stored basis is set to the identity, a valid start for a later
      // warm Jacobi that the Ritz step cannot settle
      if (!warm) {
        float2* VBw = wsp(ws, ch.w_VB);
        for (int e = threadIdx.x; e < MP * MP; e += 64 * NW)
          VBw[e] = make_float2(e / MP == e % MP ? 1.f : 0.f, 0.f);
      }
      return;
    }
  }
  const float2* S = wsp(ws, ch.w_S2);
  float2* VB = wsp(ws, ch.w_VB);
  const bool use_warm = kWarmOk && warm;
  if (use_warm) {
    for (int e = threadIdx.x; e < MP * MP; e += 64 * NW) {
      float2 v = VB[e];
      L.vr[e / MP][e % MP] = (T)v.x;
      L.vi[e / MP][e % MP] = (T)v.y;
    }
    __syncthreads();
    if (kWarmOk) reorthonormalize64<T>(L);
  }
  for (int e = threadIdx.x; e < MP * MP; e += 64 * NW) {
    const int i = e / MP, j = e % MP;
    T sr = 0, si = 0;
    if (i < d && j < d) {
      float2 v = S[(int64_t)i * d + j];
      sr = (T)v.x;
      si = (T)v.y;
    }
    L.kr[i][j] = sr;
    L.ki[i][j] = si;
  }
  __syncthreads();
  if (kWarmOk && use_warm) rotate_into_basis64<T>(L);
  bool conv = jacobi_herm<T, MP, NW>(L, r, wave, sizeof(T) == 4 ? 12 : 20, use_warm);
  if (sizeof(T) == 4)
    for (int e = threadIdx.x; e < MP * MP; e += 64 * NW)
      VB[e] = make_float2((float)L.vr[e / MP][e % MP], (float)L.vi[e / MP][e % MP]);
  if (wave == 0)
    eig_finish<T, MP>(L, r, d, ch.n, B + ch.b, ch.n, ch.n, wsd(ws, ch.w_scal) + 2,
                      status ? status + c : nullptr, conv);
}

// mode-3: one MP-lane group per subcarrier group
template <typename T, int MP>
__global__ void __launch_bounds__(64, (sizeof(T) == 4 && MP == 16) ? 2 : 1) k_eigC(const DevChan* __restrict__ chans,
                                              const GroupItem* __restrict__ items,
                                              int total_groups, char* ws, float2* C,
                                              int32_t* status, int warm) {
  constexpr int GPW = 64 / MP;
  __shared__ EigLds<T, MP> lds[GPW];
  const int grp = threadIdx.x / MP, r = threadIdx.x % MP;
  const int gi = blockIdx.x * GPW + grp;
  EigLds<T, MP>& L = lds[grp];
  const bool valid = gi < total_groups;
  GroupItem it{0, 0};
  if (valid) it = items[gi];
  const DevChan& ch = chans[it.ch];
  const int s0 = it.g * ch.gs;
  const int d = valid ? min(ch.gs, ch.nsc - s0) : 0;
  const float2* S = wsp(ws, ch.w_S3) + (int64_t)it.g * ch.gs * ch.gs;
  float2* VC = wsp(ws, ch.w_VC) + (int64_t)it.g * MP * MP;
  const bool use_warm = warm && sizeof(T) == 4;
  if (use_warm) {
    if (valid)
      load_basis<T, MP>(L, VC, r);
    else
      for (int j = 0; j < MP; ++j) {
        L.vr[r][j] = (j == r) ? T(1) : T(0);
        L.vi[r][j] = T(0);
      }
    wave_sync();
    reorthonormalize_r<T, MP>(L, r);
  }
  for (int j = 0; j < MP; ++j) {
    T sr = 0, si = 0;
    if (r < d && j < d) {
      float2 v = S[r * ch.gs + j];
      sr = (T)v.x;
      si = (T)v.y;
    }
    L.kr[r][j] = sr;
    L.ki[r][j] = si;
  }
  wave_sync();
  if (use_warm) rotate_into_basis_r<T, MP>(L, r);
  wave_sync();
  bool conv = jacobi_herm<T, MP, 1>(L, r, 0, sizeof(T) == 4 ? 12 : 20, use_warm);
  if (valid) {
    if (sizeof(T) == 4) store_basis<T, MP>(L, VC, r);
    const int pg = min(ch.p, d);
    eig_finish<T, MP>(L, r, d, pg, C + ch.c + (int64_t)s0 * ch.p, ch.p, ch.p,
                      wsd(ws, ch.w_lamg) + it.g, status ? status + it.ch : nullptr, conv);
  } else {
    eig_sort_desc<T, MP>(L, r, 0);
  }
}

// FP32 register-row variants of the two kernels above (MP lanes per matrix, row r of the Gram
// and of the eigenvector matrix in lane r; Jacobi pairs r with r xor t, as in the SINR kernels):
// the same outputs, warm starts and convergence test (squared off-diagonal norm below 64 eps^2
// times the squared diagonal norm, at most 12 sweeps) without the LDS round trips of every
// rotation step.

// mode-1: one MP-lane group per channel (nr <= MP)
template <int MP>
__global__ void __launch_bounds__(64) k_eigA_rows(const DevChan* __restrict__ chans, int n_channels,
                                                  char* ws, float2* A, int32_t* status, int warm) {
  constexpr int GPW = 64 / MP;
  __shared__ RowsEigLds<MP> lds[GPW];
  const int grp = threadIdx.x / MP, r = threadIdx.x % MP;
  const int c = blockIdx.x * GPW + grp;
  RowsEigLds<MP>& S = lds[grp];
  const bool live = c < n_channels;
  const DevChan* chp = live ? &chans[c] : nullptr;
  const int d = live ? chp->nr : 0;
  float kr[MP], ki[MP], vr[MP], vi[MP];
  const float2* Sg = live ? wsp(ws, chp->w_S1) : nullptr;
  const float2* VA = live ? wsp(ws, chp->w_VA) : nullptr;
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    float2 v = make_float2(0.f, 0.f);
    if (r < d && j < d) v = Sg[(int64_t)r * d + j];
    kr[j] = v.x;
    ki[j] = v.y;
    float2 b = make_float2(j == r ? 1.f : 0.f, 0.f);
    if (live && warm) b = VA[r * MP + j];
    vr[j] = b.x;
    vi[j] = b.y;
  }
  if (warm) rows_warm<MP>(S, r, kr, ki, vr, vi);
  const bool conv = rows_eig<MP>(S.rot, r, kr, ki, vr, vi, true, 64.f, 12);
  if (live) {
    float2* VAw = wsp(ws, chp->w_VA);
#pragma unroll
    for (int j = 0; j < MP; ++j) VAw[r * MP + j] = make_float2(vr[j], vi[j]);
  }
  rows_eig_finish<MP>(S, r, live, d, live ? chp->m : 0, live ? A + chp->a : nullptr,
                      live ? chp->m : 0, live ? chp->m : 0,
                      live ? wsd(ws, chp->w_scal) + 1 : nullptr, live && status ? status + c : nullptr,
                      conv, kr, vr, vi);
}

// mode-3: one 16-lane group per subcarrier group of up to 16 subcarriers
__global__ void __launch_bounds__(64) k_eigC_rows(const DevChan* __restrict__ chans,
                                                  const GroupItem* __restrict__ items,
                                                  int total_groups, char* ws, float2* C,
                                                  int32_t* status, int warm) {
  constexpr int MP = 16, GPW = 4;
  __shared__ RowsEigLds<MP> lds[GPW];
  const int grp = threadIdx.x / MP, r = threadIdx.x % MP;
  const int gi = blockIdx.x * GPW + grp;
  RowsEigLds<MP>& S = lds[grp];
  const bool live = gi < total_groups;
  GroupItem it{0, 0};
  if (live) it = items[gi];
  const DevChan& ch = chans[it.ch];
  const int s0 = it.g * ch.gs;
  const int d = live ? min(ch.gs, ch.nsc - s0) : 0;
  const float2* Sg = wsp(ws, ch.w_S3) + (int64_t)it.g * ch.gs * ch.gs;
  float2* VC = wsp(ws, ch.w_VC) + (int64_t)it.g * MP * MP;
  float kr[MP], ki[MP], vr[MP], vi[MP];
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    float2 v = make_float2(0.f, 0.f);
    if (r < d && j < d) v = Sg[r * ch.gs + j];
    kr[j] = v.x;
    ki[j] = v.y;
    float2 b = make_float2(j == r ? 1.f : 0.f, 0.f);
    if (live && warm) b = VC[r * MP + j];
    vr[j] = b.x;
    vi[j] = b.y;
  }
  if (warm) rows_warm<MP>(S, r, kr, ki, vr, vi);
  const bool conv = rows_eig<MP>(S.rot, r, kr, ki, vr, vi, true, 64.f, 12);
  if (live) {
#pragma unroll
    for (int j = 0; j < MP; ++j) VC[r * MP + j] = make_float2(vr[j], vi[j]);
  }
  const int pg = min(ch.p, d);
  rows_eig_finish<MP>(S, r, live, d, pg, C + ch.c + (int64_t)s0 * ch.p, ch.p, ch.p,
                      wsd(ws, ch.w_lamg) + it.g, live && status ? status + it.ch : nullptr, conv,
                      kr, vr, vi);
}

// ---------------------------------------------------------------------------------------
// Mode-n products of the sweep.

// Per group: Z_q = sum_s conj(C[s,q]) T_s for a chunk of q at once (a thread owns entries
// (i, b) and reads each T_s entry once per chunk), then the S1 partial sum_q Z_q Z_q^H with
// thr threads per output (i, k) splitting the (q, b) sum.  Dynamic LDS: C_g [gs][p], then Z
// [qc][nr][n] with qc nr n <= kZLds.
constexpr int kZLds = 8192;  // complex entries of Z held at once (64 KB)

template <int SMAX>
__global__ void __launch_bounds__(256) k_stepA_group(const DevChan* __restrict__ chans,
                                                     const GroupItem* __restrict__ items,
                                                     const float2* __restrict__ C, char* ws) {
  extern __shared__ float2 sa_lds[];
  const GroupItem it = items[blockIdx.x];
  CH_BEGIN(it.ch);
  const int nr = ch.nr, n = ch.n, p = ch.p;
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  const int pg = min(p, sz);
  const int ne = nr * n;
  const int qc = max(1, min(pg, kZLds / ne));
  float2* Cs = sa_lds;               // [gs][p]
  float2* Z = sa_lds + ch.gs * p;    // [qc][nr][n]
  for (int e = threadIdx.x; e < sz * p; e += blockDim.x) Cs[e] = C[ch.c + (int64_t)s0 * p + e];
  const float2* T = wsp(ws, ch.w_T) + (int64_t)s0 * ne;
  int thr = 1;
  while (thr * 2 * nr * nr <= 256 && thr < 64) thr *= 2;
  const int o = threadIdx.x / thr, part = threadIdx.x % thr;
  float ar = 0.f, ai = 0.f;
  for (int q0 = 0; q0 < pg; q0 += qc) {
    const int q1 = min(pg, q0 + qc);
    __syncthreads();  // C staged; the previous chunk's Z read
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
      float2 tv[SMAX];
#pragma unroll
      for (int s = 0; s < SMAX; ++s) tv[s] = T[(int64_t)min(s, sz - 1) * ne + e];
      for (int q = q0; q < q1; ++q) {
        float zr = 0.f, zi = 0.f;
#pragma unroll
        for (int s = 0; s < SMAX; ++s)
          if (s < sz) {
            const float2 c = Cs[s * p + q];  // conj(c) t
            zr += c.x * tv[s].x + c.y * tv[s].y;
            zi += c.x * tv[s].y - c.y * tv[s].x;
          }
        Z[(q - q0) * ne + e] = make_float2(zr, zi);
      }
    }
    __syncthreads();
    // S1[i][k] += sum_{q in chunk, b} Z_q[i][b] conj(Z_q[k][b])
    if (o < nr * nr) {
      const int i = o / nr, k = o % nr;
      for (int q = 0; q < q1 - q0; ++q)
        for (int b = part; b < n; b += thr) {
          const float2 zi = Z[q * ne + i * n + b], zk = Z[q * ne + k * n + b];
          ar += zk.x * zi.x + zk.y * zi.y;
          ai += zk.x * zi.y - zk.y * zi.x;
        }
    }
  }
  for (int d = thr / 2; d > 0; d >>= 1) {
    ar += __shfl_xor(ar, d, 64);
    ai += __shfl_xor(ai, d, 64);
  }
  if (o < nr * nr && part == 0)
    wsp(ws, ch.w_S1p)[(int64_t)it.g * nr * nr + o] = make_float2(ar, ai);
}

// S3_g[s][t] = sum_e conj(Yh_t[e]) Yh_s[e] over the subcarriers of each group, on matrix cores:
// rows s (one 32-row tile), columns (t, re/im) in one or two 32-wide tiles, K = (e, re/im)
// with e over the m n entries; the K range is split over the four waves and their partial
// tiles are summed in a fixed order.  Row s, column (t, 0) takes Re, (t, 1) Im: B operand
// (Re, Im)[k] of Yh_t[e] for part 0 and (-Im, Re)[k] for part 1.
__global__ void __launch_bounds__(256) k_S3(const DevChan* __restrict__ chans,
                                            const GroupItem* __restrict__ items, char* ws) {
  __shared__ float part[4][2][1024];
  const GroupItem it = items[blockIdx.x];
  const DevChan& ch = chans[it.ch];
  const int gs = ch.gs;
  const int s0 = it.g * gs;
  const int sz = min(gs, ch.nsc - s0);
  const int mn = ch.m * ch.n;
  const float* Yh = reinterpret_cast<const float*>(wsp(ws, ch.w_Yh) + (int64_t)s0 * mn);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, h = lane / 32, c32 = lane % 32;
  const int nct = gs <= 16 ? 1 : 2;
  const bool rv = c32 < sz;
  const float* ya = Yh + (int64_t)min(c32, sz - 1) * 2 * mn + h;
  const float* yb[2];
  float bsgn[2];
  bool bv[2];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int c = 32 * ct + c32, t = c >> 1, pt = c & 1;
    bv[ct] = t < sz;
    bsgn[ct] = (pt == 1 && h == 0) ? -1.f : 1.f;
    yb[ct] = Yh + (int64_t)min(t, sz - 1) * 2 * mn + (pt ^ h);
  }
  f32x16 acc[2];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[ct][r] = 0.f;
  const int kq = (mn + 3) / 4, e0 = wave * kq, e1 = min(mn, e0 + kq);
  for (int e = e0; e < e1; e += 4) {
    float av[4], b0[4], b1[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int ee = min(e + d, e1 - 1);
      const bool ok = e + d < e1;
      const float x = ya[2 * ee], y0 = yb[0][2 * ee], y1 = yb[1][2 * ee];
      av[d] = (ok && rv) ? x : 0.f;
      b0[d] = (ok && bv[0]) ? bsgn[0] * y0 : 0.f;
      b1[d] = (ok && bv[1]) ? bsgn[1] * y1 : 0.f;
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[d], b0[d], acc[0], 0, 0, 0);
      if (nct == 2) acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[d], b1[d], acc[1], 0, 0, 0);
    }
  }
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
    if (ct < nct)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        part[wave][ct][(8 * (r / 4) + 4 * h + (r % 4)) * 32 + c32] = acc[ct][r];
  __syncthreads();
  float2* S3 = wsp(ws, ch.w_S3) + (int64_t)it.g * gs * gs;
  for (int o = tid; o < gs * gs; o += 256) {
    const int si = o / gs, t = o % gs, ct = t >> 4, col = (2 * t) & 31;
    const int ix = si * 32 + col;
    const float re = (part[0][ct][ix] + part[1][ct][ix]) + (part[2][ct][ix] + part[3][ct][ix]);
    const float im = (part[0][ct][ix + 1] + part[1][ct][ix + 1]) + (part[2][ct][ix + 1] + part[3][ct][ix + 1]);
    S3[o] = make_float2(re, im);
  }
}

// per group: sum_q c_q^H S3_g c_q with the current C (objective of given factors)
__global__ void __launch_bounds__(64) k_objC(const DevChan* __restrict__ chans,
                                             const GroupItem* __restrict__ items,
                                             const float2* __restrict__ C, char* ws) {
  const GroupItem it = items[blockIdx.x];
  CH_BEGIN(it.ch);
  const int gs = ch.gs;
  const int s0 = it.g * gs;
  const int sz = min(gs, ch.nsc - s0);
  const int pg = min(ch.p, sz);
  const float2* S3 = wsp(ws, ch.w_S3) + (int64_t)it.g * gs * gs;
  __shared__ double red[64];
  double acc = 0.0;
  for (int o = threadIdx.x; o < pg * sz; o += blockDim.x) {
    const int q = o / sz, s = o % sz;
    // (S3 c)_s conj(c_s)
    double re = 0.0, im = 0.0;
    for (int t = 0; t < sz; ++t) {
      float2 a = S3[s * gs + t];
      float2 c = C[ch.c + (int64_t)(s0 + t) * ch.p + q];
      re += (double)a.x * c.x - (double)a.y * c.y;
      im += (double)a.x * c.y + (double)a.y * c.x;
    }
    float2 cs = C[ch.c + (int64_t)(s0 + s) * ch.p + q];
    acc += (double)cs.x * re + (double)cs.y * im;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) wsd(ws, ch.w_lamg)[it.g] = red[0];
}

// objective entry: mode 0 = scal[1] (A step), 1 = scal[2] (B step), 2 = sum of group sums
__global__ void k_trace(const DevChan* __restrict__ chans, int n_channels, char* ws,
                        double* trace, int stride, int idx, int mode) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_channels) return;
  CH_BEGIN(c);
  const double* sc = wsd(ws, ch.w_scal);
  double kept;
  if (mode == 0)
    kept = sc[1];
  else if (mode == 1)
    kept = sc[2];
  else {
    kept = 0.0;
    const double* lg = wsd(ws, ch.w_lamg);
    for (int g = 0; g < ch.ngroups; ++g) kept += lg[g];
  }
  trace[(int64_t)c * stride + idx] = sc[0] - kept;
}

// G_g[q] = sum_s conj(C[s,q]) Yh_s; zero for q >= p_g
__global__ void __launch_bounds__(256) k_core(const DevChan* __restrict__ chans,
                                              const float2* __restrict__ C, float2* G, char* ws) {
  CH_BEGIN(blockIdx.y);
  const int mn = ch.m * ch.n;
  const int64_t per_g = (int64_t)ch.p * mn;
  const int64_t total = per_g * ch.ngroups;
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= total) return;
  const int g = (int)(o / per_g);
  const int q = (int)((o % per_g) / mn);
  const int e = (int)(o % mn);
  const int s0 = g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  Cx<float> acc{0.f, 0.f};
  if (q < min(ch.p, sz)) {
    const float2* Yh = wsp(ws, ch.w_Yh);
    for (int i = 0; i < sz; ++i)
      cfmac(acc, ld(C + ch.c + (int64_t)(s0 + i) * ch.p + q), ld(Yh + (int64_t)(s0 + i) * mn + e));
  }
  st(G + ch.g + o, acc);
}

// ---------------------------------------------------------------------------------------
// Host side

#define GT_LAUNCH(name, grid, block, ...)                        \
  do {                                                           \
    prof_begin(#name, L.stream);                                 \
    hipLaunchKernelGGL(name, grid, block, 0, L.stream, __VA_ARGS__); \
    prof_end(L.stream);                                          \
    hipError_t e_ = hipGetLastError();                           \
    if (e_ != hipSuccess) {                                      \
      set_error_detail(#name, e_);                               \
      return GT_ERR_HIP;                                         \
    }                                                            \
  } while (0)

// the same with dynamic LDS
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

// the same on the stream of another context
#define GT_LAUNCH2(ctx, name, grid, block, ...)                      \
  do {                                                               \
    prof_begin(#name, (ctx).stream);                                 \
    hipLaunchKernelGGL(name, grid, block, 0, (ctx).stream, __VA_ARGS__); \
    prof_end((ctx).stream);                                          \
    hipError_t e_ = hipGetLastError();                               \
    if (e_ != hipSuccess) {                                          \
      set_error_detail(#name, e_);                                   \
      return GT_ERR_HIP;                                             \
    }                                                                \
  } while (0)

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

gt_status launch_eigB_sub(const LaunchCtx& L, float2* B, int32_t* status, int warm);
gt_status launch_share_gram(const LaunchCtx& L, int which);

// The eigensolves of one half-step.  Channels that share a factor get the Gram summed over the
// sharing channels first (equations "update A" and "update B" over the shared index sets).
template <typename T>
static gt_status eig_all(const LaunchCtx& L, int which, float2* A, float2* B, float2* C,
                         int32_t* status, int warm) {
  if (which == 0) {
    GT_LAUNCH(k_reduce_S1, dim3(1, L.n_channels), dim3(256), L.d_chans,
              L.ws);
    gt_status st = launch_share_gram(L, 0);
    if (st != GT_OK) return st;
    if (sizeof(T) == 4 && L.max_nr <= 8)
      GT_LAUNCH((k_eigA_rows<8>), dim3(cdiv(L.n_channels, 8)), dim3(64), L.d_chans, L.n_channels,
                L.ws, A, status, warm);
    else if (sizeof(T) == 4)
      GT_LAUNCH((k_eigA_rows<16>), dim3(cdiv(L.n_channels, 4)), dim3(64), L.d_chans,
                L.n_channels, L.ws, A, status, warm);
    else
      GT_LAUNCH((k_eigA<T, 16>), dim3(cdiv(L.n_channels, 4)), dim3(64), L.d_chans, L.n_channels,
                L.ws, A, status, warm);
  } else if (which == 1) {
    gt_status sst = launch_share_gram(L, 1);
    if (sst != GT_OK) return sst;
    constexpr int NW = sizeof(T) == 4 ? 4 : 8;
    if (L.min_nt <= 64) {
      // FP32 solves try the Rayleigh-Ritz step first (on the previous basis, or cold on S2 Omega)
      // and run the Jacobi only for the channels it cannot settle
      const int ritz = sizeof(T) == 4 ? 1 : 0;
      GT_LAUNCH((k_eigB<T, NW>), dim3(L.n_channels), dim3(64 * NW), L.d_chans, L.ws, B, status, warm,
                ritz);
    }
    if (L.max_nt > 64) {
      gt_status st = launch_eigB_sub(L, B, status, warm);
      if (st != GT_OK) return st;
    }
  } else {
    // groups of up to 16 subcarriers on 16-lane solvers, larger ones on 32-lane solvers
    const int ns = L.n_small_groups, nl = L.total_groups - L.n_small_groups;
    if (ns > 0 && sizeof(T) == 4)
      GT_LAUNCH(k_eigC_rows, dim3(cdiv(ns, 4)), dim3(64), L.d_chans, L.d_groups_by_size, ns,
                L.ws, C, status, warm);
    else if (ns > 0)
      GT_LAUNCH((k_eigC<T, 16>), dim3(cdiv(ns, 4)), dim3(64), L.d_chans, L.d_groups_by_size, ns,
                L.ws, C, status, warm);
    if (nl > 0)
      GT_LAUNCH((k_eigC<T, 32>), dim3(cdiv(nl, 2)), dim3(64), L.d_chans, L.d_groups_by_size + ns, nl,
                L.ws, C, status, warm);
  }
  return GT_OK;
}

static gt_status eig_dispatch(const LaunchCtx& L, int which, float2* A, float2* B, float2* C,
                              int32_t* status, int warm) {
  return L.eig_fp64 ? eig_all<double>(L, which, A, B, C, status, warm)
                    : eig_all<float>(L, which, A, B, C, status, warm);
}

bool fused_fit_ok(const LaunchCtx& L);
bool fused_lowp_ok(const LaunchCtx& L);
gt_status launch_convert_x(const LaunchCtx& L, const float2* X);
gt_status launch_gram_rows_big(const LaunchCtx& L, const float2* X, int which);
gt_status launch_rows_times_b(const LaunchCtx& L, const float2* X, const float2* B);
gt_status launch_w_rows(const LaunchCtx& L, const float2* X, const float2* A, const float2* C);
gt_status launch_yh_from_t(const LaunchCtx& L, const float2* A);
gt_status launch_eigB_sub(const LaunchCtx& L, float2* B, int32_t* status, int warm);
gt_status launch_fused_t(const LaunchCtx& L, const float2* X, const float2* A, const float2* B,
                         int do_c);
gt_status launch_fused_z(const LaunchCtx& L, const float2* C, float2* G, int do_a, int do_core);
gt_status launch_fused_b(const LaunchCtx& L, const float2* X, const float2* A, const float2* C,
                         hipEvent_t pre_reduce = nullptr, hipEvent_t after_pass = nullptr);

static gt_status split_fork(const LaunchCtx& L, const SplitCtx& S) {
  if (hipEventRecord(S.fork, L.stream) != hipSuccess) return GT_ERR_HIP;
  for (int k = 1; k < S.n; ++k)
    if (hipStreamWaitEvent(S.parts[k].stream, S.fork, 0) != hipSuccess) return GT_ERR_HIP;
  return GT_OK;
}

static gt_status split_join(const LaunchCtx& L, const SplitCtx& S) {
  for (int k = 1; k < S.n; ++k) {
    if (hipEventRecord(S.join[k - 1], S.parts[k].stream) != hipSuccess) return GT_ERR_HIP;
    if (hipStreamWaitEvent(L.stream, S.join[k - 1], 0) != hipSuccess) return GT_ERR_HIP;
  }
  return GT_OK;
}

gt_status launch_fit(const LaunchCtx& L, const SplitCtx* split, const float2* X, float2* A,
                     float2* B, float2* C, float2* G, double* trace, int32_t* status, int iters,
                     bool warm) {
  const int nch = L.n_channels;
  const int stride = 1 + 3 * iters;
  const dim3 b256(256);
  const unsigned gCore = cdiv((int64_t)L.max_groups * L.max_p * L.max_m * L.max_n, 256);
  const int tiles = (L.max_nt + 15) / 16;
  const dim3 gGram(tiles * tiles, L.max_nsplit, nch);
  const dim3 gRed(cdiv((int64_t)L.max_nt * L.max_nt, 256), nch);

  // the fused per-group passes need their own limits for 16-bit contractions; the generic
  // row passes take any shape
  const bool fused = fused_fit_ok(L) && (L.ttm_prec == GT_TTM_FP32 || fused_lowp_ok(L));
  // With m == nr in every channel A is square and unitary once an eigensolve has made it,
  // so the B- and C-step Grams do not depend on it (W^H W = Hc^H A A^H Hc = Hc^H Hc, and
  // likewise for Yh): only the last A-step, whose A the outputs and cores use, runs (and the
  // first one when A comes from the caller), unless the objective trace asks for every
  // half-step.
  const bool skip_a = L.full_mode1 && !trace;
  auto a_step = [&](int na) { return !skip_a || na == iters - 1 || (warm && na == 0); };
  // Pipelined parts whose first use of the starting B is the warm start of their first mode-2
  // eigensolve (no A-step and no objective before it): the mode-2 Gram of X and its cold
  // eigensolve run on the last part's stream, beside the other initial passes and the parts'
  // first B-steps.  Those B-steps write the Gram's partials, so the caller's stream waits for
  // the Gram before the parts start; each part's first B-step reduction overwrites the Gram,
  // so it waits for the eigensolve.  Every cross-stream wait is on an event of the caller's
  // stream or made by it, as for the fork and join of the parts: part 0 (the caller's stream)
  // waits for the eigensolve and relays it to the middle parts through init[3]; the last part
  // runs behind the eigensolve on its own stream.
  const bool side_b0 = !warm && fused && split && split->mode == 2 && split->n > 1 && iters > 0 &&
                       !a_step(0);
  // Without the objective trace, with m == nr everywhere and no caller factors, the starting A
  // is read by nothing (the B- and C-step Grams do not depend on it, and the last A-step, the
  // only one that runs, forms its own Gram): its HOSVD Gram and eigensolve are skipped and that
  // A-step starts cold.
  const bool no_a0 = fused && !warm && skip_a && iters >= 1;
  LaunchCtx LQ = L;
  if (side_b0) {
    LQ.stream = split->parts[split->n - 1].stream;
    if (hipEventRecord(split->init[0], L.stream) != hipSuccess ||
        hipStreamWaitEvent(LQ.stream, split->init[0], 0) != hipSuccess)
      return GT_ERR_HIP;
  }

  // initialisation: Grams of the unfoldings, norms
  const int want_s1 = no_a0 ? 0 : 1;
  if ((int64_t)L.max_gs * L.max_nr * L.max_nt <= 8192)
    GT_LAUNCH(k_init_group_lds, dim3(L.total_groups), dim3(512), L.d_chans, L.d_groups, X, L.ws,
              want_s1);
  else
    GT_LAUNCH(k_init_group, dim3(L.total_groups), b256, L.d_chans, L.d_groups, X, L.ws, want_s1);
  GT_LAUNCH(k_norm_total, dim3(cdiv(nch, 64)), dim3(64), L.d_chans, nch, L.ws);
  if (!warm) {
    gt_status st;
    // mode-2 Gram of the rows of X in 128 x 128 super-tiles (LDS-staged row chunks); for
    // nt <= 64 one super-tile holds the whole real Gram
    if ((st = launch_gram_rows_big(LQ, X, 0)) != GT_OK) return st;
    if (side_b0 && hipEventRecord(split->init[1], LQ.stream) != hipSuccess) return GT_ERR_HIP;
    if (!no_a0 && (st = eig_dispatch(L, 0, A, B, C, status, 0)) != GT_OK) return st;
    if ((st = eig_dispatch(LQ, 1, A, B, C, status, 0)) != GT_OK) return st;
    if (side_b0 && hipEventRecord(split->init[2], LQ.stream) != hipSuccess) return GT_ERR_HIP;
    if ((st = eig_dispatch(L, 2, A, B, C, status, 0)) != GT_OK) return st;
    if (side_b0 && hipStreamWaitEvent(L.stream, split->init[1], 0) != hipSuccess)
      return GT_ERR_HIP;
  }
  // objective of the starting factors (the generic path also needs Yh for the cores)
  if (L.ttm_prec != GT_TTM_FP32) {  // 16-bit copy of X for the contractions below
    gt_status st;
    if ((st = launch_convert_x(L, X)) != GT_OK) return st;
  }
  if (trace || !fused) {
    // T = H B (kept for the first A-step of the generic path), Yh = A^H T
    gt_status st;
    if ((st = launch_rows_times_b(L, X, B)) != GT_OK) return st;
    if ((st = launch_yh_from_t(L, A)) != GT_OK) return st;
  }
  if (trace) {
    GT_LAUNCH(k_S3, dim3(L.total_groups), b256, L.d_chans, L.d_groups, L.ws);
    GT_LAUNCH(k_objC, dim3(L.total_groups), dim3(64), L.d_chans, L.d_groups, C, L.ws);
    GT_LAUNCH(k_trace, dim3(cdiv(nch, 64)), dim3(64), L.d_chans, nch, L.ws, trace, stride, 0, 2);
  }
  if (fused) {
    // per sweep: eigA, [W + Gram], eigB, [T, Yh, S3], eigC, [Z + S1 or cores]; the first
    // A-step Gram comes from [T] and [Z] with the starting factors
    gt_status st;
    // T pass of sweep it: T is stored only for a following A-step; channels with m == nr take
    // the mode-3 Gram of T
    auto t_flags = [&](int it) {
      const bool last = it == iters - 1;
      return (last ? 2 : 1) | ((!last && a_step(it + 1)) ? 0 : T_NO_STORE) | T_GRAM_OF_T;
    };
    if (iters == 0 || a_step(0)) {
      if ((st = launch_fused_t(L, X, A, B, 0)) != GT_OK) return st;
      if ((st = launch_fused_z(L, C, G, iters > 0 ? 1 : 0, 0)) != GT_OK) return st;
    }
    if (iters == 0) {
      if ((st = launch_fused_t(L, X, A, B, 2)) != GT_OK) return st;
      return launch_fused_z(L, C, G, 0, 1);
    }
    if (split) {
      // The B-step pass runs over the whole batch; the rest of each sweep (mode-2 eigensolve,
      // T pass, mode-3 eigensolves, Z pass, next mode-1 eigensolve) runs per part on its own
      // stream, so that the small eigensolve launches of one part overlap the other parts'
      // passes.
      auto part_sweep = [&](int it, bool with_bc) -> gt_status {
        gt_status s2;
        if ((s2 = split_fork(L, *split)) != GT_OK) return s2;
        for (int k = 0; k < split->n; ++k) {
          const LaunchCtx& P = split->parts[k];
          const int pn = P.n_channels;
          int32_t* ps = status ? status + P.c0 : nullptr;
          double* pt = trace ? trace + (int64_t)P.c0 * stride : nullptr;
          const bool last = it == iters - 1;
          const int w = (warm && it == 0) ? 0 : 1;
          if (with_bc) {
            if ((s2 = eig_dispatch(P, 1, A, B, C, ps, w)) != GT_OK) return s2;
            if (pt)
              GT_LAUNCH2(P, k_trace, dim3(cdiv(pn, 64)), dim3(64), P.d_chans, pn, P.ws, pt,
                         stride, 2 + 3 * it, 1);
            if ((s2 = launch_fused_t(P, X, A, B, t_flags(it))) != GT_OK) return s2;
            if ((s2 = eig_dispatch(P, 2, A, B, C, ps, w)) != GT_OK) return s2;
            if (pt)
              GT_LAUNCH2(P, k_trace, dim3(cdiv(pn, 64)), dim3(64), P.d_chans, pn, P.ws, pt,
                         stride, 3 + 3 * it, 2);
            const int za = (!last && a_step(it + 1)) ? 1 : 0;
            if ((za || last) && (s2 = launch_fused_z(P, C, G, za, last ? 1 : 0)) != GT_OK)
              return s2;
          }
          // mode-1 eigensolve of the next sweep (of sweep 0 when called before the loop)
          const int na = with_bc ? it + 1 : 0;
          if (na < iters && a_step(na)) {
            const int wa = ((warm && na == 0) || no_a0) ? 0 : 1;
            if ((s2 = eig_dispatch(P, 0, A, B, C, ps, wa)) != GT_OK) return s2;
            if (pt)
              GT_LAUNCH2(P, k_trace, dim3(cdiv(pn, 64)), dim3(64), P.d_chans, pn, P.ws, pt,
                         stride, 1 + 3 * na, 0);
          }
        }
        return split_join(L, *split);
      };
      if (split->mode == 2) {
        // pipelined parts: every part runs its own sweeps, B-step included, so that one part's
        // matrix-core passes overlap another part's eigensolves; the parts only meet at the end
        if ((st = split_fork(L, *split)) != GT_OK) return st;
        for (int it = -1; it < iters; ++it) {
          for (int k = 0; k < split->n; ++k) {
            const LaunchCtx& P = split->parts[k];
            const int pn = P.n_channels;
            int32_t* ps = status ? status + P.c0 : nullptr;
            double* pt = trace ? trace + (int64_t)P.c0 * stride : nullptr;
            const int w = (warm && it <= 0) ? 0 : 1;
            if (it >= 0) {
              const bool last = it == iters - 1;
              if (it == 0 && k > 0 &&
                  hipStreamWaitEvent(P.stream, split->stag[k - 1], 0) != hipSuccess)
                return GT_ERR_HIP;
              // the next part's first B-step follows this one's B-step kernel
              hipEvent_t mm = (it == 0 && k + 1 < split->n) ? split->stag[k] : nullptr;
              hipEvent_t pre = nullptr;
              if (side_b0 && it == 0 && k + 1 < split->n) pre = split->init[k == 0 ? 2 : 3];
              if ((st = launch_fused_b(P, X, A, C, pre, mm)) != GT_OK) return st;
              if (side_b0 && it == 0 && k == 0 &&
                  hipEventRecord(split->init[3], P.stream) != hipSuccess)
                return GT_ERR_HIP;
              if ((st = eig_dispatch(P, 1, A, B, C, ps, w)) != GT_OK) return st;
              if (pt)
                GT_LAUNCH2(P, k_trace, dim3(cdiv(pn, 64)), dim3(64), P.d_chans, pn, P.ws, pt,
                           stride, 2 + 3 * it, 1);
              if ((st = launch_fused_t(P, X, A, B, t_flags(it))) != GT_OK) return st;
              if ((st = eig_dispatch(P, 2, A, B, C, ps, w)) != GT_OK) return st;
              if (pt)
                GT_LAUNCH2(P, k_trace, dim3(cdiv(pn, 64)), dim3(64), P.d_chans, pn, P.ws, pt,
                           stride, 3 + 3 * it, 2);
              const int za = (!last && a_step(it + 1)) ? 1 : 0;
              if ((za || last) && (st = launch_fused_z(P, C, G, za, last ? 1 : 0)) != GT_OK)
                return st;
            }
            const int na = it + 1;  // mode-1 eigensolve of the next sweep
            if (na < iters && a_step(na)) {
              const int wa = ((warm && na == 0) || no_a0) ? 0 : 1;
              if ((st = eig_dispatch(P, 0, A, B, C, ps, wa)) != GT_OK) return st;
              if (pt)
                GT_LAUNCH2(P, k_trace, dim3(cdiv(pn, 64)), dim3(64), P.d_chans, pn, P.ws, pt,
                           stride, 1 + 3 * na, 0);
            }
          }
        }
        return split_join(L, *split);
      }
      if ((st = part_sweep(0, false)) != GT_OK) return st;
      for (int it = 0; it < iters; ++it) {
        if ((st = launch_fused_b(L, X, A, C)) != GT_OK) return st;
        if ((st = part_sweep(it, true)) != GT_OK) return st;
      }
      return GT_OK;
    }
    for (int it = 0; it < iters; ++it) {
      const int w = (warm && it == 0) ? 0 : 1;
      if (a_step(it) && (st = eig_dispatch(L, 0, A, B, C, status, no_a0 ? 0 : w)) != GT_OK)
        return st;
      if (trace)
        GT_LAUNCH(k_trace, dim3(cdiv(nch, 64)), dim3(64), L.d_chans, nch, L.ws, trace, stride,
                  1 + 3 * it, 0);
      if ((st = launch_fused_b(L, X, A, C)) != GT_OK) return st;
      if ((st = eig_dispatch(L, 1, A, B, C, status, w)) != GT_OK) return st;
      if (trace)
        GT_LAUNCH(k_trace, dim3(cdiv(nch, 64)), dim3(64), L.d_chans, nch, L.ws, trace, stride,
                  2 + 3 * it, 1);
      const bool last = it == iters - 1;
      // the C-step pass of the last sweep also keeps Yh for the cores
      if ((st = launch_fused_t(L, X, A, B, t_flags(it))) != GT_OK) return st;
      if ((st = eig_dispatch(L, 2, A, B, C, status, w)) != GT_OK) return st;
      if (trace)
        GT_LAUNCH(k_trace, dim3(cdiv(nch, 64)), dim3(64), L.d_chans, nch, L.ws, trace, stride,
                  3 + 3 * it, 2);
      const int za = (!last && a_step(it + 1)) ? 1 : 0;
      if ((za || last) && (st = launch_fused_z(L, C, G, za, last ? 1 : 0)) != GT_OK) return st;
    }
    return GT_OK;
  }
  // per sweep: [Z + S1] from T = H B of the previous C-step, eigA, [W rows, Gram], eigB,
  // [T = H B, Yh = A^H T, S3], eigC
  for (int it = 0; it < iters; ++it) {
    gt_status st;
    // A-step (B, C of the previous sweep)
    {
      const size_t sh = sizeof(float2) * ((size_t)L.max_gs * L.max_p +
                                          std::min<size_t>(kZLds, (size_t)L.max_p * L.max_nr * L.max_n));
      if (L.max_gs <= 12)
        GT_LAUNCH_SH((k_stepA_group<12>), dim3(L.total_groups), b256, sh, L.d_chans, L.d_groups, C, L.ws);
      else if (L.max_gs <= 24)
        GT_LAUNCH_SH((k_stepA_group<24>), dim3(L.total_groups), b256, sh, L.d_chans, L.d_groups, C, L.ws);
      else
        GT_LAUNCH_SH((k_stepA_group<32>), dim3(L.total_groups), b256, sh, L.d_chans, L.d_groups, C, L.ws);
    }
    if ((st = eig_dispatch(L, 0, A, B, C, status, (warm && it == 0) ? 0 : 1)) != GT_OK) return st;
    if (trace)
      GT_LAUNCH(k_trace, dim3(cdiv(nch, 64)), dim3(64), L.d_chans, nch, L.ws, trace, stride,
                1 + 3 * it, 0);
    // B-step (new A, C of the previous sweep)
    if ((st = launch_w_rows(L, X, A, C)) != GT_OK) return st;
    if (L.max_nt > 64) {
      if ((st = launch_gram_rows_big(L, X, 1)) != GT_OK) return st;
    } else {
      GT_LAUNCH(k_gram_rows, gGram, b256, L.d_chans, X, L.ws, 1);
      GT_LAUNCH(k_reduce_S2, gRed, b256, L.d_chans, L.ws);
    }
    if ((st = eig_dispatch(L, 1, A, B, C, status, (warm && it == 0) ? 0 : 1)) != GT_OK) return st;
    if (trace)
      GT_LAUNCH(k_trace, dim3(cdiv(nch, 64)), dim3(64), L.d_chans, nch, L.ws, trace, stride,
                2 + 3 * it, 1);
    // C-step (new A, B); T = H B also serves the next sweep's A-step
    if ((st = launch_rows_times_b(L, X, B)) != GT_OK) return st;
    if ((st = launch_yh_from_t(L, A)) != GT_OK) return st;
    GT_LAUNCH(k_S3, dim3(L.total_groups), b256, L.d_chans, L.d_groups, L.ws);
    if ((st = eig_dispatch(L, 2, A, B, C, status, (warm && it == 0) ? 0 : 1)) != GT_OK) return st;
    if (trace)
      GT_LAUNCH(k_trace, dim3(cdiv(nch, 64)), dim3(64), L.d_chans, nch, L.ws, trace, stride,
                3 + 3 * it, 2);
  }
  // cores from the last Yh (computed with the final A and B)
  GT_LAUNCH(k_core, dim3(gCore, nch), b256, L.d_chans, C, G, L.ws);
  return GT_OK;
}

}  // namespace gt
