// Device-side helpers: complex arithmetic on (re, im) pairs, wave-level synchronisation and
// reductions, and a wave-synchronous parallel Jacobi eigensolver for small Hermitian
// matrices held in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt {

template <typename T>
struct Cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ void cfma(Cx<T>& acc, Cx<T> a, Cx<T> b) {  // acc += a*b
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}
template <typename T>
__device__ __forceinline__ void cfmac(Cx<T>& acc, Cx<T> a, Cx<T> b) {  // acc += conj(a)*b
  acc.re += a.re * b.re + a.im * b.im;
  acc.im += a.re * b.im - a.im * b.re;
}

__device__ __forceinline__ Cx<float> ld(const float2* p) {
  float2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ void st(float2* p, Cx<float> v) { *p = make_float2(v.re, v.im); }

template <typename T>
__device__ __forceinline__ T dsqrt(T x);
template <>
__device__ __forceinline__ float dsqrt<float>(float x) {
  return __builtin_sqrtf(x);
}
template <>
__device__ __forceinline__ double dsqrt<double>(double x) {
  return __builtin_sqrt(x);
}

template <typename T>
struct Num;
template <>
struct Num<float> {
  static __device__ __forceinline__ float eps() { return 5.9604645e-08f; }
  static __device__ __forceinline__ float big() { return 1.0e18f; }
  static __device__ __forceinline__ float ninf() { return -__builtin_huge_valf(); }
  // smallest sigma_r / sigma_1 a Gram-based FP32 SVD resolves (about sqrt(eps))
  static __device__ __forceinline__ float zero_stream() { return 1.0e-3f; }
};
template <>
struct Num<double> {
  static __device__ __forceinline__ double eps() { return 1.1102230246251565e-16; }
  static __device__ __forceinline__ double big() { return 1.0e150; }
  static __device__ __forceinline__ double ninf() { return -__builtin_huge_val(); }
  static __device__ __forceinline__ double zero_stream() { return 1.0e-6; }
};

// Channel of block b in a compact grid: the c with off[c] <= b < off[c + 1] (off holds the
// prefix sums of the channels' block counts, off[0] = 0).
__device__ __forceinline__ int tile_channel(const int32_t* __restrict__ off, int n_channels, int b) {
  int lo = 0, hi = n_channels;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Workgroups are dealt to the chip's 8 XCDs round-robin by block index; this order hands each
// XCD a contiguous range of logical tiles (total of them, grid 8 ceil(total / 8)), so that
// neighbouring tiles sharing input rows meet in one XCD's L2.  Returns -1 for the padding.
__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int per = (total + 7) / 8;
  const int t = (b % 8) * per + b / 8;
  return t < total ? t : -1;
}

// Orders the wave's LDS accesses: everything before is visible to every lane after.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over an aligned group of G lanes (G a power of two <= 64).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ bool wave_all(bool p) { return __all(p ? 1 : 0) != 0; }

// ---------------------------------------------------------------------------------------
// Parallel cyclic Jacobi for Hermitian matrices of dimension d <= MP held in LDS.
//
// MP lanes (an aligned group inside one wave) cooperate on one matrix; lane r owns row r of
// the matrix and of the eigenvector matrix.  A wave may hold 64/MP independent problems;
// all of them follow the same rotation schedule (round-robin pairing: in step t the lanes
// are paired so that every pair of indices meets once per sweep), which keeps the wave in
// lockstep.  Rows and columns >= d must be zero; they stay zero.
template <typename T, int MP>
struct EigLds {
  T kr[MP][MP + 1];
  T ki[MP][MP + 1];
  T vr[MP][MP + 1];
  T vi[MP][MP + 1];
  T rc[MP / 2], rsr[MP / 2], rsi[MP / 2];
  int rp[MP / 2], rq[MP / 2];
  T lam[MP];
  int src[MP];
};

template <int MP>
__device__ __forceinline__ void rr_pair(int t, int r, int& pos, int& partner) {
  if (MP == 1) {
    pos = 0;
    partner = 0;
    return;
  }
  constexpr int N1 = MP - 1;
  pos = (r == 0) ? 0 : ((r - 1 - t + 2 * N1 * MP) % N1) + 1;
  int ppos = MP - 1 - pos;
  partner = (ppos == 0) ? 0 : ((ppos - 1 + t) % N1) + 1;
}

// Synchronisation for the Jacobi step: a wave-level fence when one wave owns the matrix, a
// block barrier when NW waves share it.
template <int NW>
__device__ __forceinline__ void jsync() {
  if (NW == 1)
    wave_sync();
  else
    __syncthreads();
}

// Cyclic Jacobi sweeps on L.kr/ki.  Lane r (0 <= r < MP) of every cooperating wave owns row
// r.  With NW > 1 (MP == 64 only) the NW waves of the block share one matrix: wave w applies
// the rotations of pairs k = w, w + NW, ... to both the matrix and the eigenvectors; the
// column sets of different pairs are disjoint, so waves only meet at two barriers per step.
// With NW == 1 a wave may hold 64/MP matrices.  If `preset_v` is false V starts as the
// identity, otherwise the caller has stored a starting basis in vr/vi (the rotations are then
// accumulated onto it).  Returns true once the off-diagonal Frobenius norm is below
// 8 eps times the diagonal norm for every matrix of the wave (or block).
template <typename T, int MP, int NW>
__device__ __forceinline__ bool jacobi_herm(EigLds<T, MP>& L, int r, int wave, int max_sweeps,
                            bool preset_v = false) {
  static_assert(NW == 1 || MP == 64, "multi-wave Jacobi needs MP == 64");
  constexpr int KP = MP / 2;
  constexpr int KW = KP / NW;
  constexpr int KC = (sizeof(T) == 4) ? (KW < 8 ? KW : 8) : (KW < 4 ? KW : 4);
  static_assert(KW % KC == 0, "chunk must divide the pairs per wave");
  if (!preset_v && wave == 0) {
    for (int j = 0; j < MP; ++j) {
      L.vr[r][j] = (j == r) ? T(1) : T(0);
      L.vi[r][j] = T(0);
    }
  }
  jsync<NW>();
  const T eps = Num<T>::eps();
  bool conv = false;
  for (int sw = 0; sw <= max_sweeps; ++sw) {
    // done: every matrix of the wave (block) has converged; gdone: this lane's matrix has.  A
    // converged matrix takes identity rotations while the others finish, so that its result
    // does not depend on the matrices it shares a wave with.
    bool done, gdone;
    if (NW == 1) {
      T off = 0, dg = 0;
      for (int j = 0; j < MP; ++j) {
        T a = L.kr[r][j], b = L.ki[r][j];
        T v = a * a + b * b;
        if (j == r)
          dg += v;
        else
          off += v;
      }
      off = group_sum<MP>(off);
      dg = group_sum<MP>(dg);
      gdone = off <= T(64) * eps * eps * dg;  // the same in every lane of the group
      done = wave_all(gdone);
    } else {
      if (wave == 0) {
        T off = 0, dg = 0;
        for (int j = 0; j < MP; ++j) {
          T a = L.kr[r][j], b = L.ki[r][j];
          T v = a * a + b * b;
          if (j == r)
            dg += v;
          else
            off += v;
        }
        off = group_sum<MP>(off);
        dg = group_sum<MP>(dg);
        if (r == 0) L.src[0] = (off <= T(64) * eps * eps * dg) ? 1 : 0;
      }
      __syncthreads();
      done = L.src[0] != 0;
      gdone = done;
      __syncthreads();
    }
    if (done) {
      conv = true;
      break;
    }
    if (sw == max_sweeps) {
      conv = gdone;
      break;
    }
    for (int t = 0; t < MP - 1; ++t) {
      int pos, partner;
      rr_pair<MP>(t, r, pos, partner);
      const bool first = pos < MP / 2;
      if (first && wave == 0) {
        T a = L.kr[r][r], b = L.kr[partner][partner];
        T cre = L.kr[r][partner], cim = L.ki[r][partner];
        T ac = dsqrt(cre * cre + cim * cim);
        T cs = 1, sre = 0, sim = 0;
        if (!gdone && ac > T(0) && ac > eps * T(0.5) * (__builtin_fabs(a) + __builtin_fabs(b))) {
          T z = (b - a) / (T(2) * ac);
          T az = __builtin_fabs(z);
          T tt = (az > Num<T>::big()) ? T(0.5) / az : T(1) / (az + dsqrt(T(1) + az * az));
          if (z >= T(0)) tt = -tt;
          cs = T(1) / dsqrt(T(1) + tt * tt);
          T sn = tt * cs;
          sre = sn * cre / ac;
          sim = sn * cim / ac;
        }
        L.rc[pos] = cs;
        L.rsr[pos] = sre;
        L.rsi[pos] = sim;
        L.rp[pos] = r;
        L.rq[pos] = partner;
      }
      jsync<NW>();
      const int slot = first ? pos : (MP - 1 - pos);
      const T csr = L.rc[slot];
      const Cx<T> sv{L.rsr[slot], L.rsi[slot]};
#pragma unroll
      for (int kb = 0; kb < KW; kb += KC) {
        Cx<T> x[KC], y[KC], xp[KC], yp[KC], vp[KC], vq[KC];
        int pk[KC], qk[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          const int k = wave + NW * (kb + c);
          const int p = L.rp[k], q = L.rq[k];
          pk[c] = p;
          qk[c] = q;
          x[c] = {L.kr[r][p], L.ki[r][p]};
          y[c] = {L.kr[r][q], L.ki[r][q]};
          xp[c] = {L.kr[partner][p], L.ki[partner][p]};
          yp[c] = {L.kr[partner][q], L.ki[partner][q]};
          vp[c] = {L.vr[r][p], L.vi[r][p]};
          vq[c] = {L.vr[r][q], L.vi[r][q]};
        }
        wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          const int k = wave + NW * (kb + c);
          const int p = pk[c], q = qk[c];
          const T cs = L.rc[k];
          const Cx<T> s{L.rsr[k], L.rsi[k]};
          Cx<T> Rx, Ry;
          if (first) {  // row r = p of its pair: cs*row_p + s*row_q
            Cx<T> a1 = cmul(sv, xp[c]), a2 = cmul(sv, yp[c]);
            Rx = {csr * x[c].re + a1.re, csr * x[c].im + a1.im};
            Ry = {csr * y[c].re + a2.re, csr * y[c].im + a2.im};
          } else {      // row r = q of its pair: -conj(s)*row_p + cs*row_q
            Cx<T> a1 = cmulc(sv, xp[c]), a2 = cmulc(sv, yp[c]);
            Rx = {csr * x[c].re - a1.re, csr * x[c].im - a1.im};
            Ry = {csr * y[c].re - a2.re, csr * y[c].im - a2.im};
          }
          // (K J)[:,p] = K[:,p] cs + K[:,q] conj(s);  (K J)[:,q] = -K[:,p] s + K[:,q] cs
          Cx<T> b1 = cmulc(s, Ry), b2 = cmul(Rx, s);
          Cx<T> nx{Rx.re * cs + b1.re, Rx.im * cs + b1.im};
          Cx<T> ny{Ry.re * cs - b2.re, Ry.im * cs - b2.im};
          if (r == p) ny = {T(0), T(0)};
          if (r == q) nx = {T(0), T(0)};
          Cx<T> c1 = cmulc(s, vq[c]), c2 = cmul(vp[c], s);
          L.kr[r][p] = nx.re;
          L.ki[r][p] = nx.im;
          L.kr[r][q] = ny.re;
          L.ki[r][q] = ny.im;
          L.vr[r][p] = vp[c].re * cs + c1.re;
          L.vi[r][p] = vp[c].im * cs + c1.im;
          L.vr[r][q] = vq[c].re * cs - c2.re;
          L.vi[r][q] = vq[c].im * cs - c2.im;
        }
      }
      jsync<NW>();
    }
  }
  return conv;
}

// Warm start: K <- V^H K V, with the starting basis V already in L.vr/vi (one MP-lane group
// per matrix, lane r owns row r).  tr/ti is scratch of the matrix's shape.  After this the
// Jacobi sweeps run with preset_v = true and accumulate their rotations onto V.
template <typename T, int MP>
__device__ __forceinline__ void rotate_into_basis(EigLds<T, MP>& L, T (*tr)[MP + 1], T (*ti)[MP + 1], int r) {
  for (int j = 0; j < MP; ++j) {  // (K V)[r][j]
    T ar = 0, ai = 0;
    for (int k = 0; k < MP; ++k) {
      T kr = L.kr[r][k], ki = L.ki[r][k], vr = L.vr[k][j], vi = L.vi[k][j];
      ar += kr * vr - ki * vi;
      ai += kr * vi + ki * vr;
    }
    tr[r][j] = ar;
    ti[r][j] = ai;
  }
  wave_sync();
  for (int j = 0; j < MP; ++j) {  // (V^H (K V))[r][j]
    T ar = 0, ai = 0;
    for (int k = 0; k < MP; ++k) {
      T vr = L.vr[k][r], vi = L.vi[k][r], xr = tr[k][j], xi = ti[k][j];
      ar += vr * xr + vi * xi;
      ai += vr * xi - vi * xr;
    }
    L.kr[r][j] = ar;
    L.ki[r][j] = ai;
  }
  wave_sync();
}

// One Newton-Schulz step V <- V (3 I - V^H V) / 2 on the starting basis in L.vr/vi: bases
// carried from call to call in FP32 slowly lose orthonormality under many rotations, and the
// step squares that error.  Uses L.kr/ki and tr/ti as scratch, so it runs before the matrix
// is loaded.
template <typename T, int MP>
__device__ __forceinline__ void reorthonormalize(EigLds<T, MP>& L, T (*tr)[MP + 1], T (*ti)[MP + 1], int r) {
  for (int j = 0; j < MP; ++j) {  // E = V^H V, row r
    T ar = 0, ai = 0;
    for (int k = 0; k < MP; ++k) {
      T xr = L.vr[k][r], xi = L.vi[k][r], yr = L.vr[k][j], yi = L.vi[k][j];
      ar += xr * yr + xi * yi;
      ai += xr * yi - xi * yr;
    }
    tr[r][j] = ar;
    ti[r][j] = ai;
  }
  wave_sync();
  for (int j = 0; j < MP; ++j) {  // row r of 1.5 V - 0.5 V E
    T ar = 0, ai = 0;
    for (int k = 0; k < MP; ++k) {
      T xr = L.vr[r][k], xi = L.vi[r][k], yr = tr[k][j], yi = ti[k][j];
      ar += xr * yr - xi * yi;
      ai += xr * yi + xi * yr;
    }
    L.kr[r][j] = T(1.5) * L.vr[r][j] - T(0.5) * ar;
    L.ki[r][j] = T(1.5) * L.vi[r][j] - T(0.5) * ai;
  }
  wave_sync();
  for (int j = 0; j < MP; ++j) {
    L.vr[r][j] = L.kr[r][j];
    L.vi[r][j] = L.ki[r][j];
  }
  wave_sync();
}

// Register-row variants of the two warm-start steps above for one MP-lane group: the
// intermediate rows live in registers and in the matrix arrays, so no scratch matrix is needed.
template <typename T, int MP>
__device__ __forceinline__ void rotate_into_basis_r(EigLds<T, MP>& L, int r) {
  T xr[MP], xi[MP];
#pragma unroll
  for (int j = 0; j < MP; ++j) {  // (K V)[r][j]; only row r of K is read by lane r
    T ar = 0, ai = 0;
    for (int k = 0; k < MP; ++k) {
      T kr = L.kr[r][k], ki = L.ki[r][k], vr = L.vr[k][j], vi = L.vi[k][j];
      ar += kr * vr - ki * vi;
      ai += kr * vi + ki * vr;
    }
    xr[j] = ar;
    xi[j] = ai;
  }
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    L.kr[r][j] = xr[j];
    L.ki[r][j] = xi[j];
  }
  wave_sync();
#pragma unroll
  for (int j = 0; j < MP; ++j) {  // (V^H (K V))[r][j]
    T ar = 0, ai = 0;
    for (int k = 0; k < MP; ++k) {
      T vr = L.vr[k][r], vi = L.vi[k][r], yr = L.kr[k][j], yi = L.ki[k][j];
      ar += vr * yr + vi * yi;
      ai += vr * yi - vi * yr;
    }
    xr[j] = ar;
    xi[j] = ai;
  }
  wave_sync();
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    L.kr[r][j] = xr[j];
    L.ki[r][j] = xi[j];
  }
  wave_sync();
}

// Newton-Schulz step with E = V^H V held in the (still unused) matrix arrays.
template <typename T, int MP>
__device__ __forceinline__ void reorthonormalize_r(EigLds<T, MP>& L, int r) {
  T xr[MP], xi[MP];
#pragma unroll
  for (int j = 0; j < MP; ++j) {  // E = V^H V, row r
    T ar = 0, ai = 0;
    for (int k = 0; k < MP; ++k) {
      T yr = L.vr[k][r], yi = L.vi[k][r], zr = L.vr[k][j], zi = L.vi[k][j];
      ar += yr * zr + yi * zi;
      ai += yr * zi - yi * zr;
    }
    L.kr[r][j] = ar;
    L.ki[r][j] = ai;
  }
  wave_sync();
#pragma unroll
  for (int j = 0; j < MP; ++j) {  // row r of 1.5 V - 0.5 V E
    T ar = 0, ai = 0;
    for (int k = 0; k < MP; ++k) {
      T yr = L.vr[r][k], yi = L.vi[r][k], zr = L.kr[k][j], zi = L.ki[k][j];
      ar += yr * zr - yi * zi;
      ai += yr * zi + yi * zr;
    }
    xr[j] = T(1.5) * L.vr[r][j] - T(0.5) * ar;
    xi[j] = T(1.5) * L.vi[r][j] - T(0.5) * ai;
  }
  wave_sync();
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    L.vr[r][j] = xr[j];
    L.vi[r][j] = xi[j];
  }
  wave_sync();
}

// Block versions for MP = 64 and 256 threads (a 4 x 4 output tile per thread).  Each product is
// formed in registers and written back over an operand after a barrier, so no scratch matrix is
// needed: the kernel's LDS is the Jacobi's own K and V.
template <typename T>
__device__ __forceinline__ void tile_product64(const T (*xr)[65], const T (*xi)[65], bool xh,
                                               const T (*yr)[65], const T (*yi)[65], int bi, int bj,
                                               T (&ar)[4][4], T (&ai)[4][4]) {
  // (X Y) or (X^H Y) on rows bi.., columns bj..
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) ar[a][b] = ai[a][b] = 0;
  for (int k = 0; k < 64; ++k) {
    T pr[4], pi[4], qr[4], qi[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      pr[a] = xh ? xr[k][bi + a] : xr[bi + a][k];
      pi[a] = xh ? -xi[k][bi + a] : xi[bi + a][k];
      qr[a] = yr[k][bj + a];
      qi[a] = yi[k][bj + a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        ar[a][b] += pr[a] * qr[b] - pi[a] * qi[b];
        ai[a][b] += pr[a] * qi[b] + pi[a] * qr[b];
      }
  }
}

// V <- V (3 I - V^H V) / 2 with E = V^H V held in K's arrays (K is loaded afterwards).
template <typename T>
__device__ __forceinline__ void reorthonormalize64(EigLds<T, 64>& L) {
  const int t = threadIdx.x;
  const int bi = (t / 16) * 4, bj = (t % 16) * 4;
  T ar[4][4], ai[4][4];
  tile_product64<T>(L.vr, L.vi, true, L.vr, L.vi, bi, bj, ar, ai);  // E = V^H V
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      L.kr[bi + a][bj + b] = ar[a][b];
      L.ki[bi + a][bj + b] = ai[a][b];
    }
  __syncthreads();
  tile_product64<T>(L.vr, L.vi, false, L.kr, L.ki, bi, bj, ar, ai);  // V E
  __syncthreads();  // every read of V and E is done
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      L.vr[bi + a][bj + b] = T(1.5) * L.vr[bi + a][bj + b] - T(0.5) * ar[a][b];
      L.vi[bi + a][bj + b] = T(1.5) * L.vi[bi + a][bj + b] - T(0.5) * ai[a][b];
    }
  __syncthreads();
}

// K <- V^H K V, the intermediate K V held in K's arrays.
template <typename T>
__device__ __forceinline__ void rotate_into_basis64(EigLds<T, 64>& L) {
  const int t = threadIdx.x;
  const int bi = (t / 16) * 4, bj = (t % 16) * 4;
  T ar[4][4], ai[4][4];
  tile_product64<T>(L.kr, L.ki, false, L.vr, L.vi, bi, bj, ar, ai);  // K V
  __syncthreads();  // every read of K is done
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      L.kr[bi + a][bj + b] = ar[a][b];
      L.ki[bi + a][bj + b] = ai[a][b];
    }
  __syncthreads();
  tile_product64<T>(L.vr, L.vi, true, L.kr, L.ki, bi, bj, ar, ai);  // V^H (K V)
  __syncthreads();  // every read of K V is done
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      L.kr[bi + a][bj + b] = ar[a][b];
      L.ki[bi + a][bj + b] = ai[a][b];
    }
  __syncthreads();
}

// After jacobi_herm: eigenvalues sorted descending over the first d indices (padding last).
// L.src[j] = index of the j-th largest eigenvalue; L.lam[i] = eigenvalue i.
template <typename T, int MP>
__device__ __forceinline__ void eig_sort_desc(EigLds<T, MP>& L, int r, int d) {
  L.lam[r] = (r < d) ? L.kr[r][r] : Num<T>::ninf();
  wave_sync();
  const T me = L.lam[r];
  int rank = 0;
  for (int j = 0; j < MP; ++j) {
    T o = L.lam[j];
    rank += (o > me || (o == me && j < r)) ? 1 : 0;
  }
  L.src[rank] = r;
  wave_sync();
}

// Phase of output column j (eigenvector src[j]) so that its largest-modulus entry among the
// first d rows (lowest row on ties) becomes real positive.  Returns the multiplier
// conj(v_k)/|v_k| in every lane of the group.
template <typename T, int MP>
__device__ __forceinline__ Cx<T> canonical_phase(EigLds<T, MP>& L, int r, int d, int col) {
  T vr = L.vr[r][col], vi = L.vi[r][col];
  T mag = (r < d) ? vr * vr + vi * vi : T(-1);
  int idx = r;
#pragma unroll
  for (int o = MP / 2; o > 0; o >>= 1) {
    T om = __shfl_xor(mag, o, 64);
    int oi = __shfl_xor(idx, o, 64);
    if (om > mag || (om == mag && oi < idx)) {
      mag = om;
      idx = oi;
    }
  }
  T pr = L.vr[idx][col], pi = L.vi[idx][col];
  T a = dsqrt(pr * pr + pi * pi);
  if (a > T(0)) return {pr / a, -pi / a};
  return {T(1), T(0)};
}

}  // namespace gt
