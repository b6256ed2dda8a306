// Row-parallel building blocks for per-subcarrier m x m problems: MP lanes of one wave (an
// aligned group, MP = 4 or 8 >= m) handle one subcarrier and lane r owns row r of every
// matrix, in registers.  Used by the SINR kernels and their adjoint, and by the multi-cell SINR.
//   rows_gram   K = Ht Ht^H from Ht rows formed kRowsChunk columns at a time and staged in LDS;
//   rows_eig    parallel two-sided Jacobi pairing lane r with r xor t (t = 1 .. MP-1), rows
//               exchanged with ds_swizzle, column rotations from (c, s) published in LDS;
//   rows_hv     descending order, singular values, U_ns and HV = U_ns Sigma_ns rows;
//   rows_chol   left-looking Cholesky with row c published at step c;
//   rows_solve  forward and back substitution, one row's values published per step;
//   rows_inner  products of two row-distributed matrices summed over the group.
#pragma once

#include <hip/hip_runtime.h>

#include "gt_device.h"
#include "gt_internal.h"

namespace gt {

struct RowsSnr {
  float s2[kMaxSnr];
  int n;
};

// Channels of a compact subcarrier range (channels ordered by SINR kernel class).
struct RowsRange {
  const int32_t* ch;
  const int64_t* off;
  int n;
  int64_t base;
  int64_t count;
};

__device__ __forceinline__ int rows_locate(const RowsRange& R, const DevChan* chans, int64_t i,
                                           int64_t& gsc) {
  const int64_t pos = R.base + i;
  int lo = 0, hi = R.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (R.off[mid] <= pos)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int c = R.ch[lo];
  gsc = chans[c].sc + (pos - R.off[lo]);
  return c;
}

// Value of lane (this lane xor T) within the same 32 lanes (ds_swizzle bitmask mode: and
// mask 0x1F, xor mask T).
template <int T>
__device__ __forceinline__ float xswz(float v) {
  static_assert(T > 0 && T < 32, "xor distance");
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (T << 10)));
}

template <int MP>
__device__ __forceinline__ float rows_sum(float v) {
  if (MP > 1) v += xswz<1>(v);
  if (MP > 2) v += xswz<2>(v);
  if (MP > 4) v += xswz<4>(v);
  if (MP > 8) v += xswz<8>(v);
  return v;
}

template <int MP>
__device__ __forceinline__ uint32_t rows_or(uint32_t v) {
  if (MP > 1) v |= (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (1 << 10));
  if (MP > 2) v |= (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (2 << 10));
  if (MP > 4) v |= (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (4 << 10));
  if (MP > 8) v |= (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (8 << 10));
  return v;
}

constexpr int kRowsChunk = 8;  // default Ht columns staged per pass (CH)

// Groups a wave's 64 / MP consecutive subcarriers may span and still have their cores staged:
// two for 8 subcarriers (groups of 8 or more), four for 16.
template <int MP>
constexpr int kRowsMaxG = MP >= 8 ? 2 : 4;

template <int MP, int NS, int CH = kRowsChunk>
struct RowsLds {
  static constexpr int kChunk = CH;
  union {
    float2 ht[MP][CH];          // chunk of the Ht rows (Gram stage)
    struct {
      float2 hv[MP][NS];        // rows of HV = U_ns Sigma_ns
      float2 l[MP][MP];         // rows of the Cholesky factor
      float2 y[MP][NS];         // rows of the substitution results
    } m;
  } u;
  float4 rot[MP];               // (c, Re s, Im s, -) of lane r's Jacobi pair in this step
  float lam[MP];                // eigenvalues (K's diagonal after the sweeps)
};

// Jacobi rotation of the pair (p, q) zeroing K[p][q] = (kr, ki), with a = K[p][p] and
// b = K[q][q]: rows p' = cs p + s q and q' = -conj(s) p + cs q, columns likewise from the right;
// the new diagonal entries are a + tac and b - tac.  Identity when !live (a converged matrix) or
// when the entry is already negligible.
__device__ __forceinline__ void rows_rot_params(float a, float b, float kr, float ki, bool live,
                                                float& cs, float& sr, float& si, float& tac) {
  const float eps = 5.9604645e-08f;
  const float ac = __builtin_sqrtf(kr * kr + ki * ki);
  cs = 1.f;
  sr = si = tac = 0.f;
  if (live && ac > 0.f && ac > eps * 0.5f * (__builtin_fabsf(a) + __builtin_fabsf(b))) {
    const float z = (b - a) / (2.f * ac);
    const float az = __builtin_fabsf(z);
    float tt = (az > 1.0e18f) ? 0.5f / az : 1.f / (az + __builtin_sqrtf(1.f + az * az));
    if (z >= 0.f) tt = -tt;
    cs = 1.f / __builtin_sqrtf(1.f + tt * tt);
    const float sn = tt * cs;
    sr = sn * kr / ac;
    si = sn * ki / ac;
    tac = tt * ac;
  }
}

// Step T of a sweep: pair (r, r ^ T).  Rows (kr, ki) of K and (vr, vi) of V in this lane.
template <int MP, int T>
__device__ __forceinline__ void rows_jacobi_step(float4* rot, int r, bool live, float (&kr)[MP],
                                                 float (&ki)[MP], float (&vr)[MP],
                                                 float (&vi)[MP]) {
  const int partner = r ^ T;
  const bool lo = r < partner;
  float d_me = 0.f, e_r = 0.f, e_i = 0.f;
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    d_me = (j == r) ? kr[j] : d_me;
    e_r = (j == partner) ? kr[j] : e_r;
    e_i = (j == partner) ? ki[j] : e_i;
  }
  const float d_pa = xswz<T>(d_me);
  const float f_r = xswz<T>(e_r), f_i = xswz<T>(e_i);
  // both lanes of the pair use K[p][p], K[q][q] and K[p][q] as the lower lane p holds them
  const float a = lo ? d_me : d_pa, b = lo ? d_pa : d_me;
  const float pr = lo ? e_r : f_r, pi = lo ? e_i : f_i;
  float cs, sr, si, tac;
  rows_rot_params(a, b, pr, pi, live, cs, sr, si, tac);
  rot[r] = make_float4(cs, sr, si, 0.f);
  wave_sync();
  // K <- K J and V <- V J on the columns (j, j ^ T) of every pair, j < (j ^ T):
  // column j' = c col_j + conj(s) col_jq, column jq' = -s col_j + c col_jq
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    constexpr int unused = 0;
    (void)unused;
    if (j < (j ^ T)) {
      const int jq = j ^ T;
      const float4 pj = rot[j];
      const float c = pj.x, s_r = pj.y, s_i = pj.z;
      float xr = kr[j], xi = ki[j], yr = kr[jq], yi = ki[jq];
      kr[j] = c * xr + (s_r * yr + s_i * yi);
      ki[j] = c * xi + (s_r * yi - s_i * yr);
      kr[jq] = c * yr - (s_r * xr - s_i * xi);
      ki[jq] = c * yi - (s_r * xi + s_i * xr);
      xr = vr[j];
      xi = vi[j];
      yr = vr[jq];
      yi = vi[jq];
      vr[j] = c * xr + (s_r * yr + s_i * yi);
      vi[j] = c * xi + (s_r * yi - s_i * yr);
      vr[jq] = c * yr - (s_r * xr - s_i * xi);
      vi[jq] = c * yi - (s_r * xi + s_i * xr);
    }
  }
  // K <- J^H K: the lower lane takes cs x + s y, the upper one cs x - conj(s) y (y the
  // partner's row after the column rotations)
  const float tr = lo ? sr : -sr;
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    const float yr = xswz<T>(kr[j]), yi = xswz<T>(ki[j]);
    kr[j] = cs * kr[j] + (tr * yr - si * yi);
    ki[j] = cs * ki[j] + (tr * yi + si * yr);
  }
  if (tac != 0.f || sr != 0.f || si != 0.f) {
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      if (j == partner) {
        kr[j] = 0.f;
        ki[j] = 0.f;
      }
      if (j == r) {
        kr[j] = lo ? a + tac : b - tac;
        ki[j] = 0.f;
      }
    }
  }
  wave_sync();
  // V's rotations feed nothing but later rotations of V, so the compiler would otherwise sink
  // them to the end of the sweep and keep every step's (c, s) live (about 3 MP/2 registers per
  // step); an empty asm that takes and returns the rows makes each step's V final here.
#pragma unroll
  for (int j = 0; j < MP; ++j) asm volatile("" : "+v"(vr[j]), "+v"(vi[j]));
}

template <int MP, int T>
struct RowsSweep {
  static __device__ __forceinline__ void run(float4* rot, int r, bool live, float (&kr)[MP],
                                             float (&ki)[MP], float (&vr)[MP], float (&vi)[MP]) {
    rows_jacobi_step<MP, T>(rot, r, live, kr, ki, vr, vi);
    RowsSweep<MP, T + 1>::run(rot, r, live, kr, ki, vr, vi);
  }
};
template <int MP>
struct RowsSweep<MP, MP> {
  static __device__ __forceinline__ void run(float4*, int, bool, float (&)[MP], float (&)[MP],
                                             float (&)[MP], float (&)[MP]) {}
};

// ---- Jacobi on K rows in xor-relative order ------------------------------------------------
// Lane r holds row r of K with column r ^ k at position k: the diagonal sits at position 0 and,
// in step t of a sweep, the entry K[r][r ^ t] of the lane's own pair at position t, so the
// rotation parameters, the partner's entries of the row rotation (position k ^ t of lane
// r ^ t) and the fix of the rotated pair all have compile-time positions.  V keeps the natural
// column order.

// Rotation zeroing K[p][q] = (kr, ki) with a = K[p][p], b = K[q][q] (as rows_rot_params), with
// hardware reciprocals and reciprocal square roots and no branch.
__device__ __forceinline__ void rows_rot_params_fast(float a, float b, float kr, float ki, bool live,
                                                     float& cs, float& sr, float& si,
                                                     float& tac) {
  const float eps = 5.9604645e-08f;
  const float ac = __builtin_sqrtf(kr * kr + ki * ki);
  const bool on = live && ac > 0.f && ac > eps * 0.5f * (__builtin_fabsf(a) + __builtin_fabsf(b));
  const float inv = on ? __builtin_amdgcn_rcpf(ac) : 0.f;
  const float z = 0.5f * (b - a) * inv;
  const float az = __builtin_fabsf(z);
  float tt = az > 1.0e18f ? 0.5f * __builtin_amdgcn_rcpf(az)
                          : __builtin_amdgcn_rcpf(az + __builtin_sqrtf(1.f + az * az));
  tt = z >= 0.f ? -tt : tt;
  tt = on ? tt : 0.f;
  cs = __builtin_amdgcn_rsqf(1.f + tt * tt);
  const float sn = tt * cs * inv;
  sr = sn * kr;
  si = sn * ki;
  tac = tt * ac;
}

template <int MP, int T>
__device__ __forceinline__ void rows_jacobi_step_x(float4* rot, int r, bool live, float (&kr)[MP],
                                                   float (&ki)[MP], float (&vr)[MP],
                                                   float (&vi)[MP]) {
  const bool lo = (r ^ T) > r;
  const float d_pa = xswz<T>(kr[0]);
  const float f_r = xswz<T>(kr[T]), f_i = xswz<T>(ki[T]);
  // both lanes of the pair use K[p][p], K[q][q] and K[p][q] as the lower lane p holds them
  const float a = lo ? kr[0] : d_pa, b = lo ? d_pa : kr[0];
  const float pr = lo ? kr[T] : f_r, pi = lo ? ki[T] : f_i;
  float cs, sr, si, tac;
  rows_rot_params_fast(a, b, pr, pi, live, cs, sr, si, tac);
  rot[r] = make_float4(cs, sr, si, 0.f);
  wave_sync();
  // K <- K J: positions (k, k ^ T), k < k ^ T, hold columns j1 = k ^ r and j2 = j1 ^ T; j1 is
  // the lower column of its pair exactly when bit b of r is clear (b the top bit of T), so with
  // t = s-bar for a lower j1 and -s otherwise: x' = c x + t y, y' = c y - conj(t) x
  constexpr int TB = T >= 8 ? 8 : (T >= 4 ? 4 : (T >= 2 ? 2 : 1));
  const float sg = (r & TB) ? -1.f : 1.f;
#pragma unroll
  for (int k = 0; k < MP; ++k) {
    if (k < (k ^ T)) {
      const int kq = k ^ T;
      const float4 pj = rot[k ^ r];
      const float c = pj.x, tr = sg * pj.y, ti = -pj.z;
      const float xr = kr[k], xi = ki[k], yr = kr[kq], yi = ki[kq];
      kr[k] = c * xr + (tr * yr - ti * yi);
      ki[k] = c * xi + (tr * yi + ti * yr);
      kr[kq] = c * yr - (tr * xr + ti * xi);
      ki[kq] = c * yi - (tr * xi - ti * xr);
    }
  }
  // V <- V J in natural order: column j' = c col_j + conj(s) col_jq, jq' = -s col_j + c col_jq
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    if (j < (j ^ T)) {
      const int jq = j ^ T;
      const float4 pj = rot[j];
      const float c = pj.x, s_r = pj.y, s_i = pj.z;
      const float xr = vr[j], xi = vi[j], yr = vr[jq], yi = vi[jq];
      vr[j] = c * xr + (s_r * yr + s_i * yi);
      vi[j] = c * xi + (s_r * yi - s_i * yr);
      vr[jq] = c * yr - (s_r * xr - s_i * xi);
      vi[jq] = c * yi - (s_r * xi + s_i * xr);
    }
  }
  // K <- J^H K: the lower lane takes c x + s y, the upper one c x - conj(s) y, y the partner's
  // entry of the same column (its position k ^ T)
  // (positions k and k ^ T read each other's partner entries: both are exchanged before either
  // is overwritten)
  const float ur = lo ? sr : -sr;
#pragma unroll
  for (int k = 0; k < MP; ++k) {
    if (k < (k ^ T)) {
      const int kq = k ^ T;
      const float y1r = xswz<T>(kr[kq]), y1i = xswz<T>(ki[kq]);
      const float y2r = xswz<T>(kr[k]), y2i = xswz<T>(ki[k]);
      kr[k] = cs * kr[k] + (ur * y1r - si * y1i);
      ki[k] = cs * ki[k] + (ur * y1i + si * y1r);
      kr[kq] = cs * kr[kq] + (ur * y2r - si * y2i);
      ki[kq] = cs * ki[kq] + (ur * y2i + si * y2r);
    }
  }
  const bool rotd = tac != 0.f || sr != 0.f || si != 0.f;
  kr[0] = rotd ? (lo ? a + tac : b - tac) : kr[0];
  ki[0] = rotd ? 0.f : ki[0];
  kr[T] = rotd ? 0.f : kr[T];
  ki[T] = rotd ? 0.f : ki[T];
  wave_sync();
  // the V rotations feed nothing but later rotations of V: keep each step's V final here (the
  // compiler would otherwise sink them and hold every step's (c, s) live)
#pragma unroll
  for (int j = 0; j < MP; ++j) asm volatile("" : "+v"(vr[j]), "+v"(vi[j]));
}

template <int MP, int T>
struct RowsSweepX {
  static __device__ __forceinline__ void run(float4* rot, int r, bool live, float (&kr)[MP],
                                             float (&ki)[MP], float (&vr)[MP], float (&vi)[MP]) {
    rows_jacobi_step_x<MP, T>(rot, r, live, kr, ki, vr, vi);
    RowsSweepX<MP, T + 1>::run(rot, r, live, kr, ki, vr, vi);
  }
};
template <int MP>
struct RowsSweepX<MP, MP> {
  static __device__ __forceinline__ void run(float4*, int, bool, float (&)[MP], float (&)[MP],
                                             float (&)[MP], float (&)[MP]) {}
};

// rows_eig on K in xor-relative order (the eigenvalue of index r ends at position 0 of lane r).
template <int MP>
__device__ __forceinline__ bool rows_eig_x(float4* rot, int r, float (&kr)[MP], float (&ki)[MP],
                                           float (&vr)[MP], float (&vi)[MP], bool preset = false,
                                           float tol = 4.f, int max_sweeps = 10) {
  if (!preset) {
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      vr[j] = (j == r) ? 1.f : 0.f;
      vi[j] = 0.f;
    }
  }
  const float eps = 5.9604645e-08f;
  for (int sw = 0; sw <= max_sweeps; ++sw) {
    float off = 0.f;
#pragma unroll
    for (int k = 1; k < MP; ++k) off += kr[k] * kr[k] + ki[k] * ki[k];
    const float dg = rows_sum<MP>(kr[0] * kr[0] + ki[0] * ki[0]);
    off = rows_sum<MP>(off);
    const bool gdone = off <= tol * eps * eps * dg;  // the same in every lane of the group
    if (__all(gdone ? 1 : 0)) return true;
    if (sw == max_sweeps) return gdone;
    RowsSweepX<MP, 1>::run(rot, r, !gdone, kr, ki, vr, vi);
  }
  return false;
}

// ---- stages shared by the forward kernel and its adjoint ----------------------------------

// Chunk [j0, j0 + kRowsChunk) of row r of Ht = sum_q C[s,q] G_g[q] (zero past n and for the
// padding rows r >= m).
template <int MP, int CH>
__device__ __forceinline__ void rows_ht_chunk(bool row, int j0, int n, int pg,
                                              const float2* __restrict__ Cs,
                                              const float2* __restrict__ Gr, int64_t gq,
                                              float (&hr)[CH], float (&hi)[CH]) {
#pragma unroll
  for (int jj = 0; jj < CH; ++jj) hr[jj] = hi[jj] = 0.f;
  if (j0 + CH <= n && (gq & 1) == 0 && (reinterpret_cast<uintptr_t>(Gr + j0) & 15) == 0) {
    // whole chunk, rows 16-byte aligned: two entries per load
    for (int q = 0; q < pg; ++q) {
      const float2 cq = Cs[q];
      const float4* Gq = reinterpret_cast<const float4*>(Gr + q * gq + j0);
#pragma unroll
      for (int jj = 0; jj < CH; jj += 2) {
        const float4 gv = Gq[jj / 2];
        hr[jj] += cq.x * gv.x - cq.y * gv.y;
        hi[jj] += cq.x * gv.y + cq.y * gv.x;
        hr[jj + 1] += cq.x * gv.z - cq.y * gv.w;
        hi[jj + 1] += cq.x * gv.w + cq.y * gv.z;
      }
    }
  } else {
    for (int q = 0; q < pg; ++q) {
      const float2 cq = Cs[q];
      const float2* Gq = Gr + q * gq;
#pragma unroll
      for (int jj = 0; jj < CH; ++jj) {
        const int j = min(j0 + jj, n - 1);
        const float2 gv = Gq[j];
        hr[jj] += cq.x * gv.x - cq.y * gv.y;
        hi[jj] += cq.x * gv.y + cq.y * gv.x;
      }
    }
  }
#pragma unroll
  for (int jj = 0; jj < CH; ++jj) {
    const bool on = row && (j0 + jj < n);
    hr[jj] = on ? hr[jj] : 0.f;
    hi[jj] = on ? hi[jj] : 0.f;
  }
}

// The groups of a wave's subcarriers, for staging their cores in LDS: the 64 / MP subcarriers
// of a wave are consecutive, so they fall in a few groups; slot k holds the k-th distinct
// (channel, group) of the wave with the offset of G_g's first row, m, n and p_g (the same in
// every lane), and gidx is the slot of this lane's subcarrier.  ngrp > MAXG: not staged.
template <int MAXG>
struct RowsWave {
  int gidx, ngrp;
  int64_t base[MAXG];
  int mk[MAXG], nk[MAXG], pgk[MAXG];
};

template <int MP, int MAXG>
__device__ __forceinline__ RowsWave<MAXG> rows_wave_groups(bool valid, int c, int g, int64_t goff,
                                                          int m, int n, int pg) {
  constexpr int MPW = 64 / MP;
  RowsWave<MAXG> W;
  const int lane = threadIdx.x % 64, me = lane / MP;
  const int key = valid ? (c << 16) + g : -1;
  int prev = -1, first[MAXG];
  W.ngrp = 0;
  W.gidx = 0;
#pragma unroll
  for (int k = 0; k < MAXG; ++k) first[k] = 0;
#pragma unroll
  for (int t = 0; t < MPW; ++t) {
    const int kt = __shfl(key, t * MP, 64);
    if (kt >= 0 && kt != prev) {
#pragma unroll
      for (int k = 0; k < MAXG; ++k)
        if (k == W.ngrp) first[k] = t;
      ++W.ngrp;
      prev = kt;
    }
    if (t == me) W.gidx = W.ngrp > 0 ? W.ngrp - 1 : 0;
  }
  const int lo = (int)(goff & 0xffffffff), hi = (int)(goff >> 32);
  // the slot values are the same in every lane: readfirstlane keeps them in scalar registers
  W.ngrp = __builtin_amdgcn_readfirstlane(W.ngrp);
#pragma unroll
  for (int k = 0; k < MAXG; ++k) {
    const int src = first[k] * MP;
    const uint32_t blo = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl(lo, src, 64));
    const int bhi = __builtin_amdgcn_readfirstlane(__shfl(hi, src, 64));
    W.base[k] = ((int64_t)bhi << 32) | blo;
    W.mk[k] = __builtin_amdgcn_readfirstlane(__shfl(m, src, 64));
    W.nk[k] = __builtin_amdgcn_readfirstlane(__shfl(n, src, 64));
    W.pgk[k] = (k < W.ngrp) ? __builtin_amdgcn_readfirstlane(__shfl(pg, src, 64)) : 0;
  }
  return W;
}

// rows_ht_chunk with the wave's group cores staged in LDS (stage: [MAXG][MP][CH] complex, free
// for the wave): per q, the wave loads columns [j0, j0 + CH) of G_g[q] of each of its groups
// with consecutive lanes on consecutive entries (one q ahead, in registers), then every lane
// forms its row from LDS.
template <int MP, int CH, int MAXG>
__device__ __forceinline__ void rows_ht_chunk_staged(float2* stage, const RowsWave<MAXG>& W,
                                                     const float2* __restrict__ G, int r, bool row,
                                                     int j0, int n, int pg,
                                                     const float2* __restrict__ Cs,
                                                     float (&hr)[CH], float (&hi)[CH]) {
  const int lane = threadIdx.x % 64;
  int pgmax = 0;
#pragma unroll
  for (int k = 0; k < MAXG; ++k) pgmax = max(pgmax, W.pgk[k]);
#pragma unroll
  for (int jj = 0; jj < CH; ++jj) hr[jj] = hi[jj] = 0.f;
  const float2* my = stage + (W.gidx * MP + r) * CH;
  // software pipeline: the entries (and the C entry) of q + 1 are loaded into registers while
  // the wave forms its rows from those of q in LDS
  constexpr int NE = (MP * CH + 63) / 64;
  float2 nxt[MAXG][NE];
  auto fetch = [&](int q) {
#pragma unroll
    for (int k = 0; k < MAXG; ++k) {
      const int mk = W.mk[k], nk = W.nk[k];
      const float2* Gq = G + W.base[k] + (int64_t)q * mk * nk;
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = 64 * u + lane, rw = e / CH, j = j0 + e % CH;
        float2 v = make_float2(0.f, 0.f);
        if (k < W.ngrp && e < MP * CH && rw < mk && j < nk && q < W.pgk[k]) v = Gq[rw * nk + j];
        nxt[k][u] = v;
      }
    }
  };
  if (pgmax > 0) fetch(0);
  float2 cn = 0 < pg ? Cs[0] : make_float2(0.f, 0.f);
  for (int q = 0; q < pgmax; ++q) {
#pragma unroll
    for (int k = 0; k < MAXG; ++k)
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = 64 * u + lane;
        if (k < W.ngrp && e < MP * CH) stage[k * MP * CH + e] = nxt[k][u];
      }
    const float2 cq = cn;
    if (q + 1 < pgmax) {
      fetch(q + 1);
      cn = q + 1 < pg ? Cs[q + 1] : make_float2(0.f, 0.f);
    }
    wave_sync();
#pragma unroll
    for (int jj = 0; jj < CH; jj += 2) {
      const float4 gv = *reinterpret_cast<const float4*>(my + jj);
      hr[jj] += cq.x * gv.x - cq.y * gv.y;
      hi[jj] += cq.x * gv.y + cq.y * gv.x;
      hr[jj + 1] += cq.x * gv.z - cq.y * gv.w;
      hi[jj + 1] += cq.x * gv.w + cq.y * gv.z;
    }
    wave_sync();
  }
#pragma unroll
  for (int jj = 0; jj < CH; ++jj) {
    const bool on = row && (j0 + jj < n);
    hr[jj] = on ? hr[jj] : 0.f;
    hi[jj] = on ? hi[jj] : 0.f;
  }
}

// Row r of K = Ht Ht^H (XOR: in xor-relative order, column r ^ k at position k).  With W (and
// its stage) the Ht rows come from the staged cores when the wave's subcarriers fall in at
// most MAXG groups.
template <int MP, int NS, int CH, int MAXG = 1, bool XOR = false>
__device__ __forceinline__ void rows_gram(RowsLds<MP, NS, CH>& S, int r, bool row, int n, int pg,
                                          const float2* __restrict__ Cs,
                                          const float2* __restrict__ Gr, int64_t gq,
                                          float (&kr)[MP], float (&ki)[MP],
                                          const RowsWave<MAXG>* W = nullptr,
                                          float2* stage = nullptr,
                                          const float2* __restrict__ G = nullptr) {
#pragma unroll
  for (int j = 0; j < MP; ++j) kr[j] = ki[j] = 0.f;
  const bool staged = W && W->ngrp <= MAXG;  // the same in every lane of the wave
  int jend = n;
  if (staged) {  // chunks over the widest group of the wave
    jend = 0;
#pragma unroll
    for (int k = 0; k < MAXG; ++k)
      if (k < W->ngrp) jend = max(jend, W->nk[k]);
  }
  for (int j0 = 0; j0 < jend; j0 += CH) {
    float hr[CH], hi[CH];
    if (staged)
      rows_ht_chunk_staged<MP, CH, MAXG>(stage, *W, G, r, row, j0, n, pg, Cs, hr, hi);
    else
      rows_ht_chunk<MP, CH>(row, j0, n, pg, Cs, Gr, gq, hr, hi);
#pragma unroll
    for (int jj = 0; jj < CH; ++jj) S.u.ht[r][jj] = make_float2(hr[jj], hi[jj]);
    wave_sync();
#pragma unroll
    for (int k = 0; k < MP; ++k) {
#pragma unroll
      for (int jj = 0; jj < CH; jj += 2) {
        const float4 b = *reinterpret_cast<const float4*>(&S.u.ht[XOR ? (k ^ r) : k][jj]);
        // h_r conj(h_k)
        kr[k] += hr[jj] * b.x + hi[jj] * b.y + (hr[jj + 1] * b.z + hi[jj + 1] * b.w);
        ki[k] += hi[jj] * b.x - hr[jj] * b.y + (hi[jj + 1] * b.z - hr[jj + 1] * b.w);
      }
    }
    wave_sync();
  }
}

// Jacobi sweeps on K until the squared off-diagonal norm is below tol eps^2 times the squared
// diagonal norm (per matrix; converged matrices take identity rotations while the others of the
// wave finish), at most max_sweeps.  V starts as the identity, or, with preset, as the basis the
// caller holds in (vr, vi); the rotations accumulate onto it.  Leaves the eigenvalues on K's
// diagonal and the eigenvectors in the columns of V (row r in this lane).  Returns false if
// the sweep cap was reached.
template <int MP>
__device__ __forceinline__ bool rows_eig(float4* rot, int r, float (&kr)[MP], float (&ki)[MP],
                                         float (&vr)[MP], float (&vi)[MP], bool preset = false,
                                         float tol = 4.f, int max_sweeps = 10) {
  if (!preset) {
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      vr[j] = (j == r) ? 1.f : 0.f;
      vi[j] = 0.f;
    }
  }
  const float eps = 5.9604645e-08f;
  for (int sw = 0; sw <= max_sweeps; ++sw) {
    float off = 0.f, dg = 0.f;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      const float v = kr[j] * kr[j] + ki[j] * ki[j];
      if (j == r)
        dg += v;
      else
        off += v;
    }
    off = rows_sum<MP>(off);
    dg = rows_sum<MP>(dg);
    const bool gdone = off <= tol * eps * eps * dg;  // the same in every lane of the group
    if (__all(gdone ? 1 : 0)) return true;
    if (sw == max_sweeps) return gdone;
    RowsSweep<MP, 1>::run(rot, r, !gdone, kr, ki, vr, vi);
  }
  return false;
}

// Descending eigenvalues over the first m indices; singular values sig[k] and, in this lane,
// row r of U_ns (ur, ui) and of HV = U_ns Sigma_ns (hvr, hvi), zero past ns and for padding
// rows.  Publishes the HV rows to LDS.
template <int MP, int NS, int CH, bool XOR = false>
__device__ __forceinline__ void rows_hv(RowsLds<MP, NS, CH>& S, int r, bool row, int ns,
                                        const float (&kr)[MP], const float (&vr)[MP],
                                        const float (&vi)[MP], float (&sig)[NS],
                                        float (&ur)[NS], float (&ui)[NS], float (&hvr)[NS],
                                        float (&hvi)[NS], uint32_t& bits) {
  float lam_me = XOR ? kr[0] : 0.f;
  if (!XOR) {
#pragma unroll
    for (int j = 0; j < MP; ++j) lam_me = (j == r) ? kr[j] : lam_me;
  }
  S.lam[r] = row ? lam_me : -3.0e38f;
  wave_sync();
  float lam[MP];
#pragma unroll
  for (int j = 0; j < MP; ++j) lam[j] = S.lam[j];
  int src[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) src[k] = 0;
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    int rk = 0;
#pragma unroll
    for (int i = 0; i < MP; ++i) rk += (lam[i] > lam[j] || (lam[i] == lam[j] && i < j)) ? 1 : 0;
#pragma unroll
    for (int k = 0; k < NS; ++k) src[k] = (rk == k) ? j : src[k];
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    float l = 0.f, a = 0.f, b = 0.f;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      l = (src[k] == j) ? lam[j] : l;
      a = (src[k] == j) ? vr[j] : a;
      b = (src[k] == j) ? vi[j] : b;
    }
    sig[k] = __builtin_sqrtf(l > 0.f ? l : 0.f);
    const bool on = row && k < ns;
    ur[k] = on ? a : 0.f;
    ui[k] = on ? b : 0.f;
    hvr[k] = sig[k] * ur[k];
    hvi[k] = sig[k] * ui[k];
  }
#pragma unroll
  for (int k = 0; k < NS; ++k)
    if (k < ns && !(sig[k] > 1.0e-3f * sig[0])) bits |= GT_DEV_ZERO_STREAM;
#pragma unroll
  for (int k = 0; k < NS; ++k) S.u.m.hv[r][k] = make_float2(hvr[k], hvi[k]);
  wave_sync();
}

// Row r of the Cholesky factor of Q, left-looking, with row c of L published to LDS at step c;
// (lr, li) hold row r of Q on entry (padding rows: the identity).  ok is false if this lane's
// pivot was not positive; rd receives 1 / L[r][r] (hardware reciprocal), which the published
// diagonal entry carries in its imaginary slot (L's diagonal is real) for the rows below.
template <int MP, int NS, int CH>
__device__ __forceinline__ void rows_chol_factor(RowsLds<MP, NS, CH>& S, int r, float (&lr)[MP],
                                                 float (&li)[MP], bool& ok, float& rd) {
  ok = true;
  rd = 1.f;
#pragma unroll
  for (int cc = 0; cc < MP; ++cc) {
    if (r == cc) {
      float d = lr[cc];
#pragma unroll
      for (int k = 0; k < cc; ++k) d -= lr[k] * lr[k] + li[k] * li[k];
      ok = d > 0.f;
      lr[cc] = __builtin_sqrtf(d > 0.f ? d : 1.f);
      li[cc] = 0.f;
      rd = __builtin_amdgcn_rcpf(lr[cc]);
#pragma unroll
      for (int k = 0; k < cc; ++k) S.u.m.l[cc][k] = make_float2(lr[k], li[k]);
      S.u.m.l[cc][cc] = make_float2(lr[cc], rd);
    }
    wave_sync();
    if (r > cc) {
      float ar = lr[cc], ai = li[cc];
#pragma unroll
      for (int k = 0; k < cc; ++k) {  // L[r][k] conj(L[cc][k])
        const float2 y = S.u.m.l[cc][k];
        ar -= lr[k] * y.x + li[k] * y.y;
        ai -= li[k] * y.x - lr[k] * y.y;
      }
      const float inv = S.u.m.l[cc][cc].y;
      lr[cc] = ar * inv;
      li[cc] = ai * inv;
    }
  }
}

// Row r of the Cholesky factor of Q = HV HV^H + s2 I (single link), from the HV rows in LDS.
template <int MP, int NS, int CH>
__device__ __forceinline__ void rows_chol(RowsLds<MP, NS, CH>& S, int r, bool row, float s2,
                                          const float (&hvr)[NS], const float (&hvi)[NS],
                                          float (&lr)[MP], float (&li)[MP], bool& ok, float& rd) {
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    float ar = 0.f, ai = 0.f;
#pragma unroll
    for (int k = 0; k < NS; ++k) {  // hv_r conj(hv_j)
      const float2 h = S.u.m.hv[j][k];
      ar += hvr[k] * h.x + hvi[k] * h.y;
      ai += hvi[k] * h.x - hvr[k] * h.y;
    }
    lr[j] = row ? ar + ((j == r) ? s2 : 0.f) : ((j == r) ? 1.f : 0.f);
    li[j] = row ? ai : 0.f;
  }
  rows_chol_factor<MP, NS, CH>(S, r, lr, li, ok, rd);
}

// In place: row r of X <- row r of Q^{-1} X (NS columns) with Q = L L^H: forward substitution
// (row i final at step i, published), then back substitution (row i final at step i,
// descending; the rows j < i subtract conj(L[i][j]) x_i with L[i][j] from the published rows).
// rd is 1 / L[r][r] from rows_chol_factor.
template <int MP, int NS, int CH>
__device__ __forceinline__ void rows_solve(RowsLds<MP, NS, CH>& S, int r, const float (&lr)[MP],
                                           const float (&li)[MP], float rd, float (&xr)[NS],
                                           float (&xi)[NS]) {
#pragma unroll
  for (int i = 0; i < MP; ++i) {
    if (r == i) {
      const float inv = rd;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        xr[k] *= inv;
        xi[k] *= inv;
        S.u.m.y[i][k] = make_float2(xr[k], xi[k]);
      }
    }
    wave_sync();
    if (r > i) {
      const float ar = lr[i], ai = li[i];  // L[r][i]
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const float2 y = S.u.m.y[i][k];
        xr[k] -= ar * y.x - ai * y.y;
        xi[k] -= ar * y.y + ai * y.x;
      }
    }
  }
  wave_sync();
#pragma unroll
  for (int i = MP - 1; i >= 0; --i) {
    if (r == i) {
      const float inv = rd;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        xr[k] *= inv;
        xi[k] *= inv;
        S.u.m.y[i][k] = make_float2(xr[k], xi[k]);
      }
    }
    wave_sync();
    if (r < i) {
      const float2 l = S.u.m.l[i][r];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const float2 w = S.u.m.y[i][k];
        xr[k] -= l.x * w.x + l.y * w.y;
        xi[k] -= l.x * w.y - l.y * w.x;
      }
    }
  }
  wave_sync();
}

// P[j][k] = sum over the group's rows i of conj(A[i][j]) B[i][k] (the same in every lane).
template <int MP, int NS>
__device__ __forceinline__ void rows_inner(const float (&ar)[NS], const float (&ai)[NS],
                                           const float (&br)[NS], const float (&bi)[NS],
                                           float (&pr)[NS][NS], float (&pi)[NS][NS]) {
#pragma unroll
  for (int j = 0; j < NS; ++j)
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      pr[j][k] = rows_sum<MP>(ar[j] * br[k] + ai[j] * bi[k]);
      pi[j][k] = rows_sum<MP>(ar[j] * bi[k] - ai[j] * br[k]);
    }
}

// ---- Hermitian eigensolves of the fit (mode-1 and mode-3 Grams) -----------------------------

template <int MP>
struct RowsEigLds {
  float2 w0[MP][MP];  // published rows of V, then of V after re-orthonormalisation
  float2 w1[MP][MP];  // published rows of V^H V, then of K V
  float4 rot[MP];
  float lam[MP];
  int src[MP];
};

template <int MP>
__device__ __forceinline__ void rows_put(float2 (*W)[MP], int r, const float (&xr)[MP],
                                         const float (&xi)[MP]) {
#pragma unroll
  for (int j = 0; j < MP; j += 2)
    *reinterpret_cast<float4*>(&W[r][j]) = make_float4(xr[j], xi[j], xr[j + 1], xi[j + 1]);
}

// Row r of X^H Y for X, Y published in LDS: sum_k conj(X[k][r]) Y[k][j].
template <int MP>
__device__ __forceinline__ void rows_ah_b(const float2 (*X)[MP], const float2 (*Y)[MP], int r,
                                          float (&o_r)[MP], float (&o_i)[MP]) {
#pragma unroll
  for (int j = 0; j < MP; ++j) o_r[j] = o_i[j] = 0.f;
#pragma unroll
  for (int k = 0; k < MP; ++k) {
    const float2 a = X[k][r];
#pragma unroll
    for (int j = 0; j < MP; j += 2) {
      const float4 b = *reinterpret_cast<const float4*>(&Y[k][j]);
      o_r[j] += a.x * b.x + a.y * b.y;
      o_i[j] += a.x * b.y - a.y * b.x;
      o_r[j + 1] += a.x * b.z + a.y * b.w;
      o_i[j + 1] += a.x * b.w - a.y * b.z;
    }
  }
}

// Row r of A Y with row r of A in registers and Y published in LDS: sum_k A[r][k] Y[k][j].
template <int MP>
__device__ __forceinline__ void rows_a_b(const float (&ar)[MP], const float (&ai)[MP],
                                         const float2 (*Y)[MP], float (&o_r)[MP],
                                         float (&o_i)[MP]) {
#pragma unroll
  for (int j = 0; j < MP; ++j) o_r[j] = o_i[j] = 0.f;
#pragma unroll
  for (int k = 0; k < MP; ++k) {
    const float xr = ar[k], xi = ai[k];
#pragma unroll
    for (int j = 0; j < MP; j += 2) {
      const float4 b = *reinterpret_cast<const float4*>(&Y[k][j]);
      o_r[j] += xr * b.x - xi * b.y;
      o_i[j] += xr * b.y + xi * b.x;
      o_r[j + 1] += xr * b.z - xi * b.w;
      o_i[j + 1] += xr * b.w + xi * b.z;
    }
  }
}

// Warm start of a Jacobi eigensolve from the basis V of an earlier solve on the same Gram
// family: one Newton-Schulz step V <- V (3 I - V^H V) / 2 restores orthonormality lost to FP32
// rounding, then K <- V^H K V, so that only the change since the earlier solve is left for the
// sweeps (which then run with preset = true and accumulate onto V).
template <int MP>
__device__ __forceinline__ void rows_warm(RowsEigLds<MP>& S, int r, float (&kr)[MP],
                                          float (&ki)[MP], float (&vr)[MP], float (&vi)[MP]) {
  float tr[MP], ti[MP], er[MP], ei[MP];
  rows_put<MP>(S.w0, r, vr, vi);
  wave_sync();
  rows_ah_b<MP>(S.w0, S.w0, r, er, ei);  // E = V^H V
  rows_put<MP>(S.w1, r, er, ei);
  wave_sync();
  rows_a_b<MP>(vr, vi, S.w1, tr, ti);  // V E
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    vr[j] = 1.5f * vr[j] - 0.5f * tr[j];
    vi[j] = 1.5f * vi[j] - 0.5f * ti[j];
  }
  rows_put<MP>(S.w0, r, vr, vi);  // every read of the old V ended before E was published
  wave_sync();
  rows_a_b<MP>(kr, ki, S.w0, tr, ti);  // K V
  rows_put<MP>(S.w1, r, tr, ti);      // every read of E ended before V was republished
  wave_sync();
  rows_ah_b<MP>(S.w0, S.w1, r, kr, ki);  // V^H (K V)
  wave_sync();
}

// Lane (of the group) holding the largest m (lowest index on ties), with its (a, b).
template <int MP>
__device__ __forceinline__ void rows_argmax(float& m, int& idx, float& a, float& b) {
#define GT_ROWS_MAXSTEP(T)                                         \
  if (MP > T) {                                                    \
    const float om = xswz<T>(m), oa = xswz<T>(a), ob = xswz<T>(b); \
    const int oi = __builtin_amdgcn_ds_swizzle(idx, 0x1F | (T << 10)); \
    if (om > m || (om == m && oi < idx)) {                         \
      m = om;                                                      \
      idx = oi;                                                    \
      a = oa;                                                      \
      b = ob;                                                      \
    }                                                              \
  }
  GT_ROWS_MAXSTEP(8)
  GT_ROWS_MAXSTEP(4)
  GT_ROWS_MAXSTEP(2)
  GT_ROWS_MAXSTEP(1)
#undef GT_ROWS_MAXSTEP
}

// Output of an eigensolve: the rk eigenvectors of the largest eigenvalues among the first d
// indices, descending (lowest index on ties), each with the phase that makes its
// largest-modulus entry (lowest row on ties) real positive, into rows r < d of dst (leading
// dimension ld); columns rk .. rpad-1 are zeroed.  lamsum (if not NULL) receives the sum of
// the rk eigenvalues in double; status (if not NULL) gets GT_DEV_EIG_SWEEPS when the sweeps
// did not converge and GT_DEV_NONFINITE for a non-finite sum.  live: this group holds a matrix.
template <int MP>
__device__ __forceinline__ void rows_eig_finish(RowsEigLds<MP>& S, int r, bool live, int d, int rk,
                                                float2* dst, int ld, int rpad, double* lamsum,
                                                int32_t* status, bool conv, const float (&kr)[MP],
                                                const float (&vr)[MP], const float (&vi)[MP]) {
  float me = 0.f;
#pragma unroll
  for (int j = 0; j < MP; ++j) me = (j == r) ? kr[j] : me;
  S.lam[r] = (r < d) ? me : -__builtin_huge_valf();
  wave_sync();
  {
    const float mine = S.lam[r];
    int rank = 0;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      const float o = S.lam[j];
      rank += (o > mine || (o == mine && j < r)) ? 1 : 0;
    }
    S.src[rank] = r;
  }
  wave_sync();
  double ls = 0.0;
  for (int jo = 0; jo < rpad; ++jo) {
    if (jo < rk) {
      const int col = S.src[jo] & (MP - 1);
      float a = 0.f, b = 0.f;
#pragma unroll
      for (int j = 0; j < MP; ++j) {
        a = (j == col) ? vr[j] : a;
        b = (j == col) ? vi[j] : b;
      }
      float m = (r < d) ? a * a + b * b : -1.f, pa = a, pb = b;
      int idx = r;
      rows_argmax<MP>(m, idx, pa, pb);
      const float mod = __builtin_sqrtf(pa * pa + pb * pb);
      float phr = 1.f, phi = 0.f;
      if (mod > 0.f) {
        phr = pa / mod;
        phi = -pb / mod;
      }
      if (live && r < d) dst[(int64_t)r * ld + jo] = make_float2(a * phr - b * phi, a * phi + b * phr);
      ls += (double)S.lam[col];
    } else if (live && r < d) {
      dst[(int64_t)r * ld + jo] = make_float2(0.f, 0.f);
    }
  }
  if (live && r == 0) {
    if (lamsum) *lamsum = ls;
    if (status) {
      uint32_t bits = conv ? 0u : GT_DEV_EIG_SWEEPS;
      if (!(ls == ls) || ls > 1e300 || ls < -1e300) bits |= GT_DEV_NONFINITE;
      if (bits) atomicOr(reinterpret_cast<unsigned int*>(status), bits);
    }
  }
}

}  // namespace gt
