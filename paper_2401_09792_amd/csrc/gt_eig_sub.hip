// Mode-2 eigensolve for wide transmit arrays (nt > 64): the n leading eigenvectors of the
// nt x nt Hermitian Gram S2 of equation "update B" (and of the HOSVD initialisation,
// Section 2.3) by subspace iteration with Rayleigh-Ritz projection on a block of 64 vectors:
//
//   Y = S2 V,  H = V^H Y,  H = U diag(theta) U^H  (parallel Jacobi, theta descending),
//   V <- V U,  Y <- Y U                           (Ritz vectors and S2 times them),
//   stop once ||Y_j - theta_j V_j|| <= tol theta_0 for every kept column j < n,
//   otherwise V <- orth(Y) by classical Gram-Schmidt applied twice, and repeat.
//
// One 256-thread block per channel, in FP32 or (the FP64 eigensolve option) FP64 throughout:
// the Gram itself is the FP32-accumulated S2, promoted on load.  V, Y and a third buffer live
// in the workspace as column blocks [64][nt] (column k contiguous), so the passes over them
// read whole rows.
// The final Ritz basis stays in the workspace and starts the next call on the same channel
// (warm start inside the alternating sweeps); a cold start uses V = orth(S2 Omega) with a
// fixed pseudo-random unimodular Omega.
#include <hip/hip_runtime.h>

#include "gt_device.h"
#include "gt_internal.h"

namespace gt {

namespace {

constexpr int KB = 64;    // Ritz block size
constexpr int NTH = 256;  // threads per block; nt <= NTH so each thread owns one row

template <typename T>
struct V2T;
template <>
struct V2T<float> {
  using type = float2;
};
template <>
struct V2T<double> {
  using type = double2;
};
template <typename T>
using V2 = typename V2T<T>::type;

template <typename T>
__device__ __forceinline__ V2<T> mk(T a, T b) {
  V2<T> v;
  v.x = a;
  v.y = b;
  return v;
}

// Per-precision constants: staging chunk width, stopping tolerance on the relative residual,
// eigenvalue floor (relative to the largest) below which a kept pair is not held to the
// tolerance, Cholesky pivot floor, Gram-Schmidt survival threshold (squared norm ratio) and
// floor.  The Gram is accumulated in FP32, so in the FP64 form eigenpairs below about 1e-6 of
// the largest eigenvalue lie in its rounding noise: their vectors are any orthonormal
// completion and are not iterated to the FP64 tolerance.
template <typename T>
struct SubP;
template <>
struct SubP<float> {
  static constexpr int KC = 32;
  static constexpr float tol = 5.0e-6f, floor = 0.0f, piv = 1.0e-5f, keep = 1.0e-8f, tiny = 1.0e-36f;
};
template <>
struct SubP<double> {
  static constexpr int KC = 8;
  static constexpr double tol = 1.0e-8, floor = 1.0e-6, piv = 1.0e-10, keep = 1.0e-16, tiny = 1.0e-300;
};

__device__ __forceinline__ float rsqrt_t(float x) { return 1.0f / __builtin_sqrtf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / __builtin_sqrt(x); }
__device__ __forceinline__ float sqrt_t(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return __builtin_sqrt(x); }

// Fixed pseudo-random start entries in {1, i, -1, -i} (integer hash of the position).
template <typename T>
__device__ __forceinline__ V2<T> omega(int k, int j) {
  uint32_t h = (uint32_t)k * 0x9E3779B1u ^ (uint32_t)j * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  switch (h & 3u) {
    case 0: return mk<T>(1, 0);
    case 1: return mk<T>(0, 1);
    case 2: return mk<T>(-1, 0);
    default: return mk<T>(0, -1);
  }
}

template <typename T>
struct SubLds {
  static constexpr int KC = SubP<T>::KC;
  EigLds<T, KB> e;        // Rayleigh quotient, Cholesky factor and their eigenvectors / inverse
  V2<T> sa[64][KC + 1];   // staging tile: 64 rows x KC
  V2<T> sb[KC][65];       // staging tile: KC x 64 columns
  T red[4][KB][2];        // per-wave partial sums of the Gram-Schmidt coefficients
  T rs[KB];               // residual norms of the Ritz pairs / Gram diagonal
  T ph[KB][2];            // output phases
  T bsum[4];
};

// Sum of v over the block (every thread gets the result).
template <typename T>
__device__ T block_sum(SubLds<T>& L, T v) {
  v = group_sum<64>(v);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) L.bsum[wave] = v;
  __syncthreads();
  return (L.bsum[0] + L.bsum[1]) + (L.bsum[2] + L.bsum[3]);
}

// Y[k][i] = sum_j S[i][j] Vin[k][j]  (Vin == nullptr: the start block Omega)
template <typename T>
__device__ void apply_gram(SubLds<T>& L, const float2* __restrict__ S, const V2<T>* Vin, V2<T>* Y,
                           int nt, int i_lo = 0, int i_hi = 1 << 30) {
  constexpr int KC = SubP<T>::KC;
  const int t = threadIdx.x;
  const int bi = (t / 16) * 4, bk = (t % 16) * 4;
  for (int i0 = i_lo; i0 < min(nt, i_hi); i0 += 64) {
    T ar[4][4], ai[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) ar[a][b] = ai[a][b] = 0;
    for (int j0 = 0; j0 < nt; j0 += KC) {
      __syncthreads();
      for (int e = t; e < 64 * KC; e += NTH) {
        const int r = e / KC, c = e % KC, i = i0 + r, j = j0 + c;
        const float2 v = (i < nt && j < nt) ? S[(int64_t)i * nt + j] : make_float2(0.f, 0.f);
        L.sa[r][c] = mk<T>((T)v.x, (T)v.y);
      }
      for (int e = t; e < 64 * KC; e += NTH) {
        const int k = e / KC, c = e % KC, j = j0 + c;
        V2<T> v = mk<T>(0, 0);
        if (j < nt) v = Vin ? Vin[(int64_t)k * nt + j] : omega<T>(k, j);
        L.sb[c][k] = v;
      }
      __syncthreads();
#pragma unroll 4
      for (int c = 0; c < KC; ++c) {
        V2<T> x[4], y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = L.sa[bi + a][c];
#pragma unroll
        for (int b = 0; b < 4; ++b) y[b] = L.sb[c][bk + b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            ar[a][b] += x[a].x * y[b].x - x[a].y * y[b].y;
            ai[a][b] += x[a].x * y[b].y + x[a].y * y[b].x;
          }
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + bi + a;
      if (i < nt)
#pragma unroll
        for (int b = 0; b < 4; ++b) Y[(int64_t)(bk + b) * nt + i] = mk<T>(ar[a][b], ai[a][b]);
    }
  }
  __syncthreads();
}

// H = V^H Y into L.e.kr/ki (Hermitian part)
template <typename T>
__device__ void rayleigh(SubLds<T>& L, const V2<T>* V, const V2<T>* Y, int nt, int i_lo = 0,
                         int i_hi = 1 << 30) {
  constexpr int KC = SubP<T>::KC;
  const int t = threadIdx.x;
  const int ba = (t / 16) * 4, bb = (t % 16) * 4;
  T ar[4][4], ai[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) ar[a][b] = ai[a][b] = 0;
  const int iend = min(nt, i_hi);
  for (int i0 = i_lo; i0 < iend; i0 += KC) {
    __syncthreads();
    for (int e = t; e < 64 * KC; e += NTH) {
      const int k = e / KC, c = e % KC, i = i0 + c;
      const bool ok = i < iend;
      L.sa[k][c] = ok ? V[(int64_t)k * nt + i] : mk<T>(0, 0);
      L.sb[c][k] = ok ? Y[(int64_t)k * nt + i] : mk<T>(0, 0);
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < KC; ++c) {
      V2<T> x[4], y[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) x[a] = L.sa[ba + a][c];
#pragma unroll
      for (int b = 0; b < 4; ++b) y[b] = L.sb[c][bb + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {  // conj(x) y
          ar[a][b] += x[a].x * y[b].x + x[a].y * y[b].y;
          ai[a][b] += x[a].x * y[b].y - x[a].y * y[b].x;
        }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      L.e.kr[ba + a][bb + b] = ar[a][b];
      L.e.ki[ba + a][bb + b] = ai[a][b];
    }
  __syncthreads();
  // Hermitian part: (H + H^H) / 2
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      ar[a][b] = T(0.5) * (ar[a][b] + L.e.kr[bb + b][ba + a]);
      ai[a][b] = T(0.5) * (ai[a][b] - L.e.ki[bb + b][ba + a]);
    }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      L.e.kr[ba + a][bb + b] = ar[a][b];
      L.e.ki[ba + a][bb + b] = ai[a][b];
    }
  __syncthreads();
}

// Out[j][i] = sum_a In[a][i] U[a][src[j]]  (U = L.e.vr/vi: eigenvectors or R^{-1}); In may
// equal Out (every row block is read completely before it is written)
template <typename T>
__device__ void rotate_block(SubLds<T>& L, const V2<T>* In, V2<T>* Out, int nt, int i_lo = 0,
                             int i_hi = 1 << 30) {
  constexpr int KC = SubP<T>::KC;
  const int t = threadIdx.x;
  const int bi = (t / 16) * 4, bj = (t % 16) * 4;
  int cj[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) cj[b] = L.e.src[bj + b];
  for (int i0 = i_lo; i0 < min(nt, i_hi); i0 += 64) {
    T ar[4][4], ai[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) ar[a][b] = ai[a][b] = 0;
    for (int a0 = 0; a0 < KB; a0 += KC) {
      __syncthreads();
      for (int e = t; e < 64 * KC; e += NTH) {
        const int c = e / 64, r = e % 64, i = i0 + r;
        L.sa[r][c] = (i < nt) ? In[(int64_t)(a0 + c) * nt + i] : mk<T>(0, 0);
      }
      __syncthreads();
#pragma unroll 4
      for (int c = 0; c < KC; ++c) {
        V2<T> x[4];
        T ur[4], ui[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = L.sa[bi + a][c];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          ur[b] = L.e.vr[a0 + c][cj[b]];
          ui[b] = L.e.vi[a0 + c][cj[b]];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            ar[a][b] += x[a].x * ur[b] - x[a].y * ui[b];
            ai[a][b] += x[a].x * ui[b] + x[a].y * ur[b];
          }
      }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + bi + a;
      if (i < nt)
#pragma unroll
        for (int b = 0; b < 4; ++b) Out[(int64_t)(bj + b) * nt + i] = mk<T>(ar[a][b], ai[a][b]);
    }
  }
  __syncthreads();
}

// Dst = orthonormal basis of the columns of Src, column by column (classical Gram-Schmidt,
// two passes).  A column that keeps too little of its norm is replaced by the matching
// column of Fb (or of Omega when Fb is null), then by unit vectors, until one survives.
template <typename T>
__device__ void orthonormalize(SubLds<T>& L, const V2<T>* Src, const V2<T>* Fb, V2<T>* Dst,
                               int nt) {
  const int i = threadIdx.x, wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const bool live = i < nt;
  for (int j = 0; j < KB; ++j) {
    V2<T> y = live ? Src[(int64_t)j * nt + i] : mk<T>(0, 0);
    T n0 = block_sum<T>(L, y.x * y.x + y.y * y.y);
    T n1 = 0;
    for (int attempt = 0;; ++attempt) {
      for (int pass = 0; pass < 2; ++pass) {
        if (j > 0) {
          for (int k = 0; k < j; ++k) {
            V2<T> q = live ? Dst[(int64_t)k * nt + i] : mk<T>(0, 0);
            T pr = q.x * y.x + q.y * y.y, pi = q.x * y.y - q.y * y.x;  // conj(q) y
            pr = group_sum<64>(pr);
            pi = group_sum<64>(pi);
            if (lane == 0) {
              L.red[wave][k][0] = pr;
              L.red[wave][k][1] = pi;
            }
          }
          __syncthreads();
          for (int k = 0; k < j; ++k) {
            const T cr = (L.red[0][k][0] + L.red[1][k][0]) + (L.red[2][k][0] + L.red[3][k][0]);
            const T ci = (L.red[0][k][1] + L.red[1][k][1]) + (L.red[2][k][1] + L.red[3][k][1]);
            if (live) {
              V2<T> q = Dst[(int64_t)k * nt + i];
              y.x -= q.x * cr - q.y * ci;
              y.y -= q.x * ci + q.y * cr;
            }
          }
          __syncthreads();
        }
      }
      n1 = block_sum<T>(L, y.x * y.x + y.y * y.y);
      if ((n1 > SubP<T>::keep * n0 && n1 > SubP<T>::tiny) || attempt > nt + 1) break;
      // replacement candidate
      if (attempt == 0)
        y = live ? (Fb ? Fb[(int64_t)j * nt + i] : omega<T>(j, i)) : mk<T>(0, 0);
      else
        y = (i == (j + attempt - 1) % nt) ? mk<T>(1, 0) : mk<T>(0, 0);
      n0 = block_sum<T>(L, y.x * y.x + y.y * y.y);
    }
    const T s = (n1 > 0) ? rsqrt_t(n1) : T(0);
    if (live) Dst[(int64_t)j * nt + i] = mk<T>(y.x * s, y.y * s);
  }
  __syncthreads();
}

// Cholesky factorisation Src^H Src = R^H R of the Gram block in L.e.kr/ki (upper triangle,
// overwritten by R, on wave 0), then R^{-1} column by column (lane j solves R x = e_j by back
// substitution) into L.e.vr/vi with the identity column order in L.e.src, so that
// rotate_block applies R^{-1}.  Returns false in every thread when a pivot falls below the
// pivot floor times its diagonal entry of the Gram (a column nearly dependent on the ones
// before).
template <typename T>
__device__ bool chol_inv(SubLds<T>& L) {
  const int t = threadIdx.x;
  if (t < KB) {
    const int j = t;
    L.rs[j] = L.e.kr[j][j];
    wave_sync();
    bool ok = true;
    for (int k = 0; k < KB; ++k) {
      const T d = L.e.kr[k][k];
      const bool good = d > SubP<T>::piv * L.rs[k] && d > SubP<T>::tiny;
      ok = ok && good;
      const T rinv = good ? rsqrt_t(d) : T(1);
      wave_sync();
      T gr = 0, gi = 0;
      if (j >= k) {
        gr = (j == k) ? d * rinv : L.e.kr[k][j] * rinv;
        gi = (j == k) ? T(0) : L.e.ki[k][j] * rinv;
        L.e.kr[k][j] = gr;
        L.e.ki[k][j] = gi;
      }
      wave_sync();
      // G[i][j] -= conj(R[k][i]) R[k][j] for k < i <= j
      for (int i = k + 1; i <= j; ++i) {
        const T ar = L.e.kr[k][i], ai = L.e.ki[k][i];
        L.e.kr[i][j] -= ar * gr + ai * gi;
        L.e.ki[i][j] -= ar * gi - ai * gr;
      }
      wave_sync();
    }
    // column j of R^{-1}: x_j = 1 / R_jj, x_i = -(sum_{i < k <= j} R_ik x_k) / R_ii
    for (int i = KB - 1; i > j; --i) {
      L.e.vr[i][j] = 0;
      L.e.vi[i][j] = 0;
    }
    L.e.vr[j][j] = T(1) / L.e.kr[j][j];
    L.e.vi[j][j] = 0;
    for (int i = j - 1; i >= 0; --i) {
      T sr = 0, si = 0;
      for (int k = i + 1; k <= j; ++k) {
        const T rr = L.e.kr[i][k], ri = L.e.ki[i][k];
        const T xr = L.e.vr[k][j], xi = L.e.vi[k][j];
        sr += rr * xr - ri * xi;
        si += rr * xi + ri * xr;
      }
      const T dinv = T(-1) / L.e.kr[i][i];
      L.e.vr[i][j] = sr * dinv;
      L.e.vi[i][j] = si * dinv;
    }
    L.e.src[j] = j;
    if (j == 0) L.bsum[0] = ok ? T(1) : T(0);
  }
  __syncthreads();
  return L.bsum[0] != T(0);
}

// Dst = orthonormal basis of the columns of Src: Cholesky-QR (passes 1 or 2, the second
// in place on Dst), falling back to Gram-Schmidt with column replacement when the block is
// too close to rank deficient for the Cholesky factorisation.
template <typename T>
__device__ void orth_block(SubLds<T>& L, const V2<T>* Src, const V2<T>* Fb, V2<T>* Dst, int nt,
                           int passes) {
  rayleigh<T>(L, Src, Src, nt);
  bool ok = chol_inv<T>(L);
  if (ok) {
    rotate_block<T>(L, Src, Dst, nt);
    if (passes > 1) {
      rayleigh<T>(L, Dst, Dst, nt);
      ok = chol_inv<T>(L);
      if (ok) rotate_block<T>(L, Dst, Dst, nt);
    }
  }
  if (!ok) orthonormalize<T>(L, Src, Fb, Dst, nt);
}

// Largest relative residual ||W_j - theta_j Z_j|| / theta_0 over the kept columns j < n with
// theta_j above the eigenvalue floor.
template <typename T>
__device__ T max_residual(SubLds<T>& L, const V2<T>* Z, const V2<T>* W, int nt, int n) {
  const int t = threadIdx.x;
  const int j = t / 4, part = t % 4;
  const T th = L.e.lam[L.e.src[j]];
  T acc = 0;
  for (int i = part; i < nt; i += 4) {
    V2<T> z = Z[(int64_t)j * nt + i], w = W[(int64_t)j * nt + i];
    const T dr = w.x - th * z.x, di = w.y - th * z.y;
    acc += dr * dr + di * di;
  }
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  __syncthreads();
  if (part == 0) L.rs[j] = acc;
  __syncthreads();
  const T th0 = L.e.lam[L.e.src[0]];
  T m = 0;
  for (int k = 0; k < n; ++k)
    if (!(L.e.lam[L.e.src[k]] <= SubP<T>::floor * th0)) m = fmax(m, L.rs[k]);
  // NaN propagates: comparisons below fail and the caller stops at the cap
  const T den = th0 * th0;
  return (den > 0) ? sqrt_t(m / den) : (m > 0 ? T(1) : T(0));
}

}  // namespace

// Workspace of the multi-block first step (offsets in elements of the eigensolve's precision
// from w_SP, wide channels): slice
// partials of H = V^H S2 V and M = V^H V, then Q = R^{-1} U (M = R^H R, U the eigenvectors of
// R^{-H} H R^{-1}), the sorted Ritz values, the slice partials of the residual norms, and the
// flags (Cholesky accepted, Jacobi converged).
constexpr int kSlices = 4;  // 64-row slices of nt <= 256
struct SubWs {
  static constexpr int part = 0;                        // [4][2][64][64] complex
  static constexpr int q = kSlices * 2 * 64 * 64 * 2;   // [64][64] complex, column-major order
  static constexpr int lam = q + 64 * 64 * 2;           // [64]
  static constexpr int res = lam + 64;                  // [4][64]
  static constexpr int flags = res + kSlices * 64;      // [2]
  static constexpr int total = flags + 2;
};

template <typename T>
__global__ void __launch_bounds__(NTH) k_eigB_sub(const DevChan* __restrict__ chans, char* ws,
                                                   float2* B, int32_t* status, int warm,
                                                   int max_iter, int resume) {
  __shared__ SubLds<T> L;
  const DevChan& ch = chans[blockIdx.x];
  const int nt = ch.nt, n = ch.n;
  if (nt <= 64) return;  // handled by the in-LDS Jacobi kernel
  const int t = threadIdx.x, r = t % 64, wave = t / 64;
  const float2* S = reinterpret_cast<const float2*>(ws + ch.w_S2);
  V2<T>* P0 = reinterpret_cast<V2<T>*>(ws + ch.w_VB);
  V2<T>* P1 = reinterpret_cast<V2<T>*>(ws + ch.w_VS);
  V2<T>* P2 = P1 + (int64_t)KB * nt;

  bool conv = false, jconv = true, done = false;
  T res = 0;
  V2<T>* Z = P1;
  V2<T> *V, *Y, *F;
  if (resume) {
    // the multi-block first step left Ritz vectors Z in P1, S2 Z in P2, the Ritz values and
    // the residual partials
    const T* sp = reinterpret_cast<const T*>(ws + ch.w_SP);
    const bool chol_ok = sp[SubWs::flags] != T(0);
    jconv = sp[SubWs::flags + 1] != T(0);
    if (t < KB) {
      L.e.lam[t] = sp[SubWs::lam + t];
      L.e.src[t] = t;
      T acc = 0;
      for (int sl = 0; sl < (nt + 63) / 64; ++sl) acc += sp[SubWs::res + 64 * sl + t];
      L.rs[t] = acc;
    }
    __syncthreads();
    if (chol_ok) {
      const T th0 = L.e.lam[0];
      T m = 0;
      for (int k = 0; k < n; ++k)
        if (!(L.e.lam[k] <= SubP<T>::floor * th0)) m = fmax(m, L.rs[k]);
      const T den = th0 * th0;
      res = (den > 0) ? sqrt_t(m / den) : (m > 0 ? T(1) : T(0));
      if (res <= SubP<T>::tol) {
        conv = done = true;
        Z = P1;
      } else {
        orth_block<T>(L, P2, P1, P0, nt, 2);  // next block from S2 Z
        V = P0;
        Y = P2;
        F = P1;
      }
    } else {  // the old basis was not accepted: the single-block warm start
      jconv = true;
      orth_block<T>(L, P0, nullptr, P1, nt, 1);
      V = P1;
      Y = P2;
      F = P0;
    }
  } else if (warm) {
    // starting orthonormal block in V
    orth_block<T>(L, P0, nullptr, P1, nt, 1);  // the previous Ritz basis, orthonormal to rounding
    V = P1;
    Y = P2;
    F = P0;
  } else {
    apply_gram<T>(L, S, nullptr, P1, nt);
    orth_block<T>(L, P1, nullptr, P0, nt, 2);
    V = P0;
    Y = P1;
    F = P2;
  }
  if (!done) Z = F;
  for (int it = 0; it < (done ? 0 : max_iter); ++it) {
    apply_gram<T>(L, S, V, Y, nt);
    rayleigh<T>(L, V, Y, nt);
    jconv = jacobi_herm<T, KB, 4>(L.e, r, wave, sizeof(T) == 4 ? 12 : 20, false) && jconv;
    __syncthreads();
    if (wave == 0) eig_sort_desc<T, KB>(L.e, r, KB);
    __syncthreads();
    Z = F;
    rotate_block<T>(L, V, Z, nt);  // Ritz vectors
    rotate_block<T>(L, Y, V, nt);  // S2 times the Ritz vectors (V's storage is free now)
    res = max_residual<T>(L, Z, V, nt, n);
    if (res <= SubP<T>::tol) {
      conv = true;
      break;
    }
    if (it == max_iter - 1) break;
    orth_block<T>(L, V, Z, Y, nt, 2);  // next block, in Y's storage
    V2<T>* nv = Y;
    Y = V;
    F = Z;
    V = nv;
  }

  // keep the Ritz basis for the next call
  if (Z != P0) {
    for (int e = t; e < KB * nt; e += NTH) P0[e] = Z[e];
    __syncthreads();
    Z = P0;
  }
  // canonical phase of each kept column: its largest-modulus entry (lowest row on ties)
  // becomes real positive
  if (t < n) {
    T best = -1;
    V2<T> bv = mk<T>(1, 0);
    for (int i = 0; i < nt; ++i) {
      const V2<T> v = Z[(int64_t)t * nt + i];
      const T mag = v.x * v.x + v.y * v.y;
      if (mag > best) {
        best = mag;
        bv = v;
      }
    }
    const T a = sqrt_t(bv.x * bv.x + bv.y * bv.y);
    L.ph[t][0] = (a > 0) ? bv.x / a : T(1);
    L.ph[t][1] = (a > 0) ? -bv.y / a : T(0);
  }
  __syncthreads();
  float2* Bc = B + ch.b;
  for (int e = t; e < nt * n; e += NTH) {
    const int i = e / n, j = e % n;
    const V2<T> v = Z[(int64_t)j * nt + i];
    const T pr = L.ph[j][0], pi = L.ph[j][1];
    Bc[e] = make_float2((float)(v.x * pr - v.y * pi), (float)(v.x * pi + v.y * pr));
  }
  if (t == 0) {
    double ls = 0.0;
    for (int j = 0; j < n; ++j) ls += (double)L.e.lam[L.e.src[j]];
    reinterpret_cast<double*>(ws + ch.w_scal)[2] = ls;
    uint32_t bits = (conv && jconv) ? 0u : GT_DEV_EIG_SWEEPS;
    if (!(ls == ls) || !(res == res) || ls > 1e300 || ls < -1e300) bits |= GT_DEV_NONFINITE;
    if (bits && status) atomicOr(reinterpret_cast<unsigned int*>(status + blockIdx.x), bits);
  }
}

// Multi-block first step of a warm call (four blocks per wide channel, one per 64-row
// slice): Rayleigh-Ritz on the previous Ritz basis V without orthonormalising it first, as the
// generalised problem H x = theta M x with M = V^H V = R^H R (so that V R^{-1} is the
// orthonormal basis), then the Ritz vectors Z = V Q and S2 Z with Q = R^{-1} U.

// Block (channel, slice): Y = S2 V on the slice's rows into P2, then the slice's partials of H
// and M.
template <typename T>
__global__ void __launch_bounds__(NTH) k_sub_prod(const DevChan* __restrict__ chans, char* ws) {
  __shared__ SubLds<T> L;
  const DevChan& ch = chans[blockIdx.x / kSlices];
  const int slice = blockIdx.x % kSlices, nt = ch.nt;
  if (nt <= 64 || 64 * slice >= nt) return;
  const float2* S = reinterpret_cast<const float2*>(ws + ch.w_S2);
  const V2<T>* P0 = reinterpret_cast<const V2<T>*>(ws + ch.w_VB);
  V2<T>* P2 = reinterpret_cast<V2<T>*>(ws + ch.w_VS) + (int64_t)KB * nt;
  T* part = reinterpret_cast<T*>(ws + ch.w_SP) + SubWs::part + slice * 2 * 64 * 64 * 2;
  const int lo = 64 * slice, hi = lo + 64;
  apply_gram<T>(L, S, P0, P2, nt, lo, hi);
  for (int w = 0; w < 2; ++w) {
    rayleigh<T>(L, P0, w == 0 ? P2 : P0, nt, lo, hi);
    T* dst = part + w * 64 * 64 * 2;
    for (int e = threadIdx.x; e < 64 * 64; e += NTH) {
      dst[2 * e] = L.e.kr[e / 64][e % 64];
      dst[2 * e + 1] = L.e.ki[e / 64][e % 64];
    }
  }
}

// One block per wide channel: sums the partials, factors M = R^H R, forms H' = R^{-H} H R^{-1},
// diagonalises it (Jacobi, eigenvalues descending) and stores Q = R^{-1} U, the Ritz values
// and the flags.
template <typename T>
__global__ void __launch_bounds__(NTH) k_sub_rr(const DevChan* __restrict__ chans, char* ws) {
  __shared__ SubLds<T> L;
  const DevChan& ch = chans[blockIdx.x];
  if (ch.nt <= 64) return;
  const int t = threadIdx.x, r = t % 64, wave = t / 64;
  T* sp = reinterpret_cast<T*>(ws + ch.w_SP);
  const int nsl = (ch.nt + 63) / 64;
  // M into kr/ki, H kept in registers: thread t owns entries e = t + 256 u
  T hr[16], hi[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    T ar = 0, ai = 0, mr = 0, mi = 0;
    for (int sl = 0; sl < nsl; ++sl) {
      const T* pp = sp + SubWs::part + sl * 2 * 64 * 64 * 2;
      ar += pp[2 * e];
      ai += pp[2 * e + 1];
      mr += pp[64 * 64 * 2 + 2 * e];
      mi += pp[64 * 64 * 2 + 2 * e + 1];
    }
    hr[u] = ar;
    hi[u] = ai;
    L.e.kr[e / 64][e % 64] = mr;
    L.e.ki[e / 64][e % 64] = mi;
  }
  __syncthreads();
  const bool chol_ok = chol_inv<T>(L);  // R^{-1} in vr/vi (R in kr/ki is not needed again)
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    L.e.kr[e / 64][e % 64] = hr[u];
    L.e.ki[e / 64][e % 64] = hi[u];
  }
  __syncthreads();
  // X = H R^{-1} (R^{-1} upper triangular), into kr/ki once H is read
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u, a = e / 64, b = e % 64;
    T xr = 0, xi = 0;
    for (int k = 0; k <= b; ++k) {
      const T h1 = L.e.kr[a][k], h2 = L.e.ki[a][k], q1 = L.e.vr[k][b], q2 = L.e.vi[k][b];
      xr += h1 * q1 - h2 * q2;
      xi += h1 * q2 + h2 * q1;
    }
    hr[u] = xr;
    hi[u] = xi;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    L.e.kr[e / 64][e % 64] = hr[u];
    L.e.ki[e / 64][e % 64] = hi[u];
  }
  __syncthreads();
  // H' = R^{-H} X, then its Hermitian part, into kr/ki
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u, a = e / 64, b = e % 64;
    T xr = 0, xi = 0;
    for (int k = 0; k <= a; ++k) {  // conj(R^{-1}[k][a]) X[k][b]
      const T q1 = L.e.vr[k][a], q2 = L.e.vi[k][a], x1 = L.e.kr[k][b], x2 = L.e.ki[k][b];
      xr += q1 * x1 + q2 * x2;
      xi += q1 * x2 - q2 * x1;
    }
    hr[u] = xr;
    hi[u] = xi;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    L.e.kr[e / 64][e % 64] = hr[u];
    L.e.ki[e / 64][e % 64] = hi[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u, a = e / 64, b = e % 64;
    hr[u] = T(0.5) * (hr[u] + L.e.kr[b][a]);
    hi[u] = T(0.5) * (hi[u] - L.e.ki[b][a]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u;
    L.e.kr[e / 64][e % 64] = hr[u];
    L.e.ki[e / 64][e % 64] = hi[u];
  }
  __syncthreads();
  // Jacobi with its rotations accumulated onto R^{-1}: the eigenvector matrix it leaves is
  // Q = R^{-1} U
  const bool jc = jacobi_herm<T, KB, 4>(L.e, r, wave, sizeof(T) == 4 ? 12 : 20, true);
  __syncthreads();
  if (wave == 0) eig_sort_desc<T, KB>(L.e, r, KB);
  __syncthreads();
  // Q[:, j] = column src[j], stored column-major ([j][a])
  T* q = sp + SubWs::q;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = t + 256 * u, j = e / 64, a = e % 64, cj = L.e.src[j];
    q[2 * e] = L.e.vr[a][cj];
    q[2 * e + 1] = L.e.vi[a][cj];
  }
  if (t < KB) sp[SubWs::lam + t] = L.e.lam[L.e.src[t]];
  if (t == 0) {
    sp[SubWs::flags] = chol_ok ? T(1) : T(0);
    sp[SubWs::flags + 1] = jc ? T(1) : T(0);
  }
}

// Block (channel, slice): Z = V Q into P1 and S2 Z = Y Q in place in P2 on the slice's rows,
// and the slice's partial residual norms ||S2 z_j - theta_j z_j||^2.
template <typename T>
__global__ void __launch_bounds__(NTH) k_sub_rot(const DevChan* __restrict__ chans, char* ws) {
  __shared__ SubLds<T> L;
  const DevChan& ch = chans[blockIdx.x / kSlices];
  const int slice = blockIdx.x % kSlices, nt = ch.nt;
  if (nt <= 64 || 64 * slice >= nt) return;
  const int t = threadIdx.x;
  T* sp = reinterpret_cast<T*>(ws + ch.w_SP);
  if (sp[SubWs::flags] == T(0)) return;  // the resume kernel redoes the step on one block
  const T* q = sp + SubWs::q;
  for (int e = t; e < 64 * 64; e += NTH) {
    L.e.vr[e % 64][e / 64] = q[2 * e];  // vr[a][j]
    L.e.vi[e % 64][e / 64] = q[2 * e + 1];
  }
  if (t < KB) {
    L.e.src[t] = t;
    L.e.lam[t] = sp[SubWs::lam + t];
  }
  __syncthreads();
  const V2<T>* P0 = reinterpret_cast<const V2<T>*>(ws + ch.w_VB);
  V2<T>* P1 = reinterpret_cast<V2<T>*>(ws + ch.w_VS);
  V2<T>* P2 = P1 + (int64_t)KB * nt;
  const int lo = 64 * slice, hi = min(nt, lo + 64);
  rotate_block<T>(L, P0, P1, nt, lo, hi);
  rotate_block<T>(L, P2, P2, nt, lo, hi);
  const int j = t / 4, pt = t % 4;
  const T th = L.e.lam[j];
  T acc = 0;
  for (int i = lo + pt; i < hi; i += 4) {
    const V2<T> z = P1[(int64_t)j * nt + i], w = P2[(int64_t)j * nt + i];
    const T dr = w.x - th * z.x, di = w.y - th * z.y;
    acc += dr * dr + di * di;
  }
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  if (pt == 0) sp[SubWs::res + 64 * slice + j] = acc;
}

gt_status launch_eigB_sub(const LaunchCtx& L, float2* B, int32_t* status, int warm) {
  const int max_iter = warm ? 40 : 100;
  const bool multi = warm != 0;
  if (multi) {
    const dim3 gs(kSlices * L.n_channels), gc(L.n_channels), b(NTH);
    prof_begin("k_sub_prod", L.stream);
    if (L.eig_fp64)
      hipLaunchKernelGGL(k_sub_prod<double>, gs, b, 0, L.stream, L.d_chans, L.ws);
    else
      hipLaunchKernelGGL(k_sub_prod<float>, gs, b, 0, L.stream, L.d_chans, L.ws);
    prof_end(L.stream);
    prof_begin("k_sub_rr", L.stream);
    if (L.eig_fp64)
      hipLaunchKernelGGL(k_sub_rr<double>, gc, b, 0, L.stream, L.d_chans, L.ws);
    else
      hipLaunchKernelGGL(k_sub_rr<float>, gc, b, 0, L.stream, L.d_chans, L.ws);
    prof_end(L.stream);
    prof_begin("k_sub_rot", L.stream);
    if (L.eig_fp64)
      hipLaunchKernelGGL(k_sub_rot<double>, gs, b, 0, L.stream, L.d_chans, L.ws);
    else
      hipLaunchKernelGGL(k_sub_rot<float>, gs, b, 0, L.stream, L.d_chans, L.ws);
    prof_end(L.stream);
  }
  prof_begin("k_eigB_sub", L.stream);
  if (L.eig_fp64)
    hipLaunchKernelGGL(k_eigB_sub<double>, dim3(L.n_channels), dim3(NTH), 0, L.stream, L.d_chans,
                       L.ws, B, status, warm, max_iter, multi ? 1 : 0);
  else
    hipLaunchKernelGGL(k_eigB_sub<float>, dim3(L.n_channels), dim3(NTH), 0, L.stream, L.d_chans,
                       L.ws, B, status, warm, max_iter, multi ? 1 : 0);
  prof_end(L.stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error_detail("k_eigB_sub", e);
    return GT_ERR_HIP;
  }
  return GT_OK;
}

}  // namespace gt
