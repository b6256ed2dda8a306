// Per-subcarrier SINR from the compressed form (Section 3.3) or from the full channel
// (Section 2.2), and its adjoint: the LDS-cooperative kernels (the full-channel SINR, compressed
// channels with m > 8 or with more than 4 streams in the adjoint, and every FP64 call), the
// per-group reduction of the adjoint, and the launchers of every SINR class (compressed channels
// with m <= 8 run on the register-resident row-parallel kernels of gt_sinr_rows.hip).
//
// One aligned group of MP lanes handles one subcarrier; lane i owns row i of every small
// matrix.  Chain for a channel matrix H (M x N; M = m, N = n for the compressed form):
//   K = H H^H, eigendecomposition K = U diag(sigma^2) U^H (Jacobi)          SVD of H
//   precoder P = V_ns (first ns right singular vectors, equation "precoding matrix");
//   HV = H P = U_ns Sigma_ns  (the form the paper states for W = Q^{-1} U Sigma)
//   Q = HV HV^H + s2 I_M               (equation "covariance matrix", single link)
//   Q = L L^H (Cholesky), W = Q^{-1} HV (equation "MMSE receive filter")
//   s_r = |w_r^H hv_r|^2              (equation "s_r^ij")
//   SINR_r = s_r / (w_r^H Q w_r - s_r) (equation "SINR formula")
// The denominator is evaluated as s2 ||w_r||^2 + sum_{k != r} |w_r^H hv_k|^2: Q expanded
// into its noise and per-stream terms.  This equals w_r^H Q w_r - s_r exactly and is the
// interference-plus-noise power the paper names, but avoids subtracting two numbers close
// to one at high SNR.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gt_device.h"
#include "gt_internal.h"

namespace gt {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct SnrArgs {
  float s2[kMaxSnr];
  int n;
};

// Element storage of the complex buffers: interleaved FP32 (float2) for c64 plans, FP64
// (double2) for c128 plans.  Loads convert to the arithmetic type T.
template <typename E>
struct Elem;
template <>
struct Elem<float2> {
  using R = float;
  static __device__ __forceinline__ float2 make(float re, float im) { return make_float2(re, im); }
};
template <>
struct Elem<double2> {
  using R = double;
  static __device__ __forceinline__ double2 make(double re, double im) { return make_double2(re, im); }
};
template <typename T, typename E>
__device__ __forceinline__ Cx<T> ldc(const E* p) {
  const E v = *p;
  return {(T)v.x, (T)v.y};
}

template <typename T, int MP, int NMAX>
struct SinrLds {
  EigLds<T, MP> e;
  T hr[MP][NMAX + 1], hi[MP][NMAX + 1];  // compressed channel rows (when staged)
  T hvr[MP][MP + 1], hvi[MP][MP + 1];    // HV = U_ns Sigma_ns (columns r < ns)
  T wr[MP][MP + 1], wi[MP][MP + 1];      // W (columns r < ns)
  T sig[MP];
  // backward only
  T gr[MP][MP + 1], gi[MP][MP + 1];      // adjoint of HV
  T vr[MP][NMAX + 1], vi[MP][NMAX + 1];  // right singular vectors v_r as rows
};

// The forward chain's LDS: the staged channel rows are read only while the Gram is formed,
// so HV and W take their place afterwards (less LDS per subcarrier, more waves per CU).
template <typename T, int MP, int NMAX>
struct SinrFwdLds {
  EigLds<T, MP> e;
  union {
    struct {
      T hr[MP][NMAX + 1], hi[MP][NMAX + 1];
    };
    struct {
      T hvr[MP][MP + 1], hvi[MP][MP + 1];
      T wr[MP][MP + 1], wi[MP][MP + 1];
    };
  };
  T sig[MP];
};

// A compact range of subcarriers: the channels of one or more consecutive SINR kernel classes
// (channels ordered by class, subcarriers numbered through that order).
struct ScRange {
  const int32_t* ch;   // channels of the range
  const int64_t* off;  // first position of each in the class order (ascending)
  int n;               // channels in the range (>= 1)
  int64_t base;        // position of the range's first subcarrier in the class order
  int64_t count;       // subcarriers in the range
};

// Channel and global subcarrier index of item i < R.count of the range.
__device__ __forceinline__ int locate_sc(const ScRange& R, const DevChan* chans, int64_t i,
                                         int64_t& gsc) {
  const int64_t pos = R.base + i;
  int lo = 0, hi = R.n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (R.off[mid] <= pos)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int c = R.ch[lo];
  gsc = chans[c].sc + (pos - R.off[lo]);
  return c;
}

// Fills S.e.kr/ki with K = H H^H (padded) and, for the compressed form, stages Ht in S.hr/hi.
template <typename T, int MP, int NMAX, bool FULL, typename Lds, typename E>
__device__ void build_gram(Lds& S, int r, bool valid, const DevChan& ch, int64_t s,
                           const E* __restrict__ X, const E* __restrict__ C,
                           const E* __restrict__ G, int& M, int& N) {
  M = valid ? (FULL ? ch.nr : ch.m) : 0;
  N = valid ? (FULL ? ch.nt : ch.n) : 0;
  if (!FULL) {
    if (r < M) {
      const int g = (int)(s / ch.gs);
      const E* Cs = C + ch.c + s * ch.p;
      const E* Gg = G + ch.g + (int64_t)g * ch.p * ch.m * ch.n;
      const int pg = min(ch.p, min(ch.gs, ch.nsc - g * ch.gs));
      for (int j = 0; j < N; ++j) {
        Cx<T> acc{T(0), T(0)};
        for (int q = 0; q < pg; ++q)
          cfma(acc, ldc<T>(Cs + q), ldc<T>(Gg + ((int64_t)q * ch.m + r) * ch.n + j));
        S.hr[r][j] = (T)acc.re;
        S.hi[r][j] = (T)acc.im;
      }
    }
    wave_sync();
  }
  for (int k = 0; k < MP; ++k) {
    T ar = 0, ai = 0;
    if (r < M && k < M) {
      if (FULL) {
        const E* Hi = X + ch.x + (s * ch.nr + r) * ch.nt;
        const E* Hk = X + ch.x + (s * ch.nr + k) * ch.nt;
        for (int j = 0; j < N; ++j) {
          E a = Hi[j], b = Hk[j];
          ar += (T)a.x * (T)b.x + (T)a.y * (T)b.y;
          ai += (T)a.y * (T)b.x - (T)a.x * (T)b.y;
        }
      } else {
        for (int j = 0; j < N; ++j) {
          T xr = S.hr[r][j], xi = S.hi[r][j], yr = S.hr[k][j], yi = S.hi[k][j];
          ar += xr * yr + xi * yi;
          ai += xi * yr - xr * yi;
        }
      }
    }
    S.e.kr[r][k] = ar;
    S.e.ki[r][k] = ai;
  }
  wave_sync();
}

// After the eigensolve: singular values and HV = U_ns Sigma_ns.  Returns the number of
// streams of this subcarrier (0 if invalid) and flags zero streams.
template <typename T, int MP, int NMAX, typename Lds>
__device__ int singular_setup(Lds& S, int r, int M, int ns, uint32_t& bits) {
  eig_sort_desc<T, MP>(S.e, r, M);
  if (r < ns) {
    T l = S.e.lam[S.e.src[r]];
    S.sig[r] = dsqrt(l > T(0) ? l : T(0));
  }
  wave_sync();
  const T sig1 = ns > 0 ? S.sig[0] : T(0);
  for (int k = 0; k < ns; ++k) {
    const int col = S.e.src[k];
    T sk = S.sig[k];
    if (r < M) {
      S.hvr[r][k] = sk * S.e.vr[r][col];
      S.hvi[r][k] = sk * S.e.vi[r][col];
    }
  }
  if (r == 0)
    for (int k = 0; k < ns; ++k)
      if (!(S.sig[k] > Num<T>::zero_stream() * sig1)) bits |= GT_DEV_ZERO_STREAM;
  wave_sync();
  return ns;
}

// Cholesky of Q = HV HV^H + s2 I (lower, in S.e.kr/ki), then W = Q^{-1} HV by two triangular
// solves (column r in lane r).  Returns false if Q is not numerically positive definite.
template <typename T, int MP, int NMAX, typename Lds>
__device__ bool mmse_filter(Lds& S, int r, int M, int ns, T s2) {
  for (int j = 0; j < MP; ++j) {
    T qr = 0, qi = 0;
    if (r < M && j < M) {
      for (int k = 0; k < ns; ++k) {  // hv[r][k] conj(hv[j][k])
        T ar = S.hvr[r][k], ai = S.hvi[r][k], br = S.hvr[j][k], bi = S.hvi[j][k];
        qr += ar * br + ai * bi;
        qi += ai * br - ar * bi;
      }
      if (j == r) qr += s2;
    }
    S.e.kr[r][j] = qr;
    S.e.ki[r][j] = qi;
  }
  wave_sync();
  bool ok = true;
  for (int c = 0; c < M; ++c) {
    if (r == c) {
      T d = S.e.kr[c][c];
      for (int j = 0; j < c; ++j) d -= S.e.kr[c][j] * S.e.kr[c][j] + S.e.ki[c][j] * S.e.ki[c][j];
      S.e.lam[c] = d;  // radicand, checked below by every lane
      S.e.kr[c][c] = dsqrt(d > T(0) ? d : T(1));
      S.e.ki[c][c] = 0;
    }
    wave_sync();
    const T piv = S.e.lam[c];
    ok = ok && (piv > T(0));
    if (r > c && r < M) {
      T ar = S.e.kr[r][c], ai = S.e.ki[r][c];
      for (int j = 0; j < c; ++j) {  // L[r][j] conj(L[c][j])
        T xr = S.e.kr[r][j], xi = S.e.ki[r][j], yr = S.e.kr[c][j], yi = S.e.ki[c][j];
        ar -= xr * yr + xi * yi;
        ai -= xi * yr - xr * yi;
      }
      T inv = T(1) / S.e.kr[c][c];
      S.e.kr[r][c] = ar * inv;
      S.e.ki[r][c] = ai * inv;
    }
    wave_sync();
  }
  if (r < ns) {
    // L y = hv_r
    for (int i = 0; i < M; ++i) {
      T ar = S.hvr[i][r], ai = S.hvi[i][r];
      for (int j = 0; j < i; ++j) {
        T lr = S.e.kr[i][j], li = S.e.ki[i][j], yr = S.wr[j][r], yi = S.wi[j][r];
        ar -= lr * yr - li * yi;
        ai -= lr * yi + li * yr;
      }
      T inv = T(1) / S.e.kr[i][i];
      S.wr[i][r] = ar * inv;
      S.wi[i][r] = ai * inv;
    }
    // L^H w = y
    for (int i = M - 1; i >= 0; --i) {
      T ar = S.wr[i][r], ai = S.wi[i][r];
      for (int j = i + 1; j < M; ++j) {  // conj(L[j][i]) w_j
        T lr = S.e.kr[j][i], li = S.e.ki[j][i], wr = S.wr[j][r], wi = S.wi[j][r];
        ar -= lr * wr + li * wi;
        ai -= lr * wi - li * wr;
      }
      T inv = T(1) / S.e.kr[i][i];
      S.wr[i][r] = ar * inv;
      S.wi[i][r] = ai * inv;
    }
  }
  wave_sync();
  return ok;
}

// SINR of stream r from W and HV; also returns s_r, d_r and the products c_rk = w_r^H hv_k
template <typename T, int MP, int NMAX, typename Lds>
__device__ T stream_sinr(Lds& S, int r, int M, int ns, T s2, T& sr_out, T& dr_out) {
  T sig = 0, den = 0, nw = 0;
  for (int k = 0; k < ns; ++k) {
    T cr = 0, ci = 0;
    for (int i = 0; i < M; ++i) {  // conj(w[i][r]) hv[i][k]
      T wr = S.wr[i][r], wi = S.wi[i][r], hr = S.hvr[i][k], hi = S.hvi[i][k];
      cr += wr * hr + wi * hi;
      ci += wr * hi - wi * hr;
    }
    T p = cr * cr + ci * ci;
    if (k == r)
      sig = p;
    else
      den += p;
  }
  for (int i = 0; i < M; ++i) nw += S.wr[i][r] * S.wr[i][r] + S.wi[i][r] * S.wi[i][r];
  den += s2 * nw;
  sr_out = sig;
  dr_out = den;
  return sig / den;
}

// SPB subcarriers per block of SPB * MP lanes (64 / MP for FP32; FP64 blocks hold one
// subcarrier so that their LDS fits).
template <typename T, int MP, int NMAX, bool FULL, typename E = float2, typename O = float,
          int SPB = 64 / MP>
__global__ void __launch_bounds__(64) k_sinr(const DevChan* __restrict__ chans, ScRange R,
                                              int64_t total_sc, const E* __restrict__ X,
                                              const E* __restrict__ C,
                                              const E* __restrict__ G, SnrArgs snr,
                                              O* __restrict__ out, int ns_max,
                                              int32_t* status) {
  __shared__ SinrFwdLds<T, MP, NMAX> lds[SPB];
  const int grp = threadIdx.x / MP, r = threadIdx.x % MP;
  SinrFwdLds<T, MP, NMAX>& S = lds[grp];
  const int64_t it = (int64_t)blockIdx.x * SPB + grp;
  const bool valid = it < R.count;
  int64_t gsc = 0;
  const int c = valid ? locate_sc(R, chans, it, gsc) : 0;
  const DevChan& ch = chans[c];
  const int64_t s = gsc - ch.sc;
  int M, N;
  build_gram<T, MP, NMAX, FULL>(S, r, valid, ch, s, X, C, G, M, N);
  bool conv = jacobi_herm<T, MP, 1>(S.e, r, 0, sizeof(T) == 4 ? 12 : 20);
  uint32_t bits = conv ? 0u : GT_DEV_EIG_SWEEPS;
  const int ns = valid ? ch.ns : 0;
  singular_setup<T, MP, NMAX>(S, r, M, ns, bits);
  for (int k = 0; k < snr.n; ++k) {
    const T s2 = (T)snr.s2[k];
    bool ok = mmse_filter<T, MP, NMAX>(S, r, M, ns, s2);
    T sv, dv;
    T val = T(0);
    if (r < ns) {
      val = stream_sinr<T, MP, NMAX>(S, r, M, ns, s2, sv, dv);
      if (!ok) val = T(0);
      if (!(S.sig[r] > Num<T>::zero_stream() * S.sig[0])) val = T(0);
      if (!(val == val) || val > T(3e38)) {
        val = T(0);
        bits |= GT_DEV_NONFINITE;
      }
    }
    if (!ok && r == 0) bits |= GT_DEV_CHOLESKY;
    if (valid && r < ns_max) out[((int64_t)k * total_sc + gsc) * ns_max + r] = (O)val;
  }
  if (valid && status && bits && r == 0) atomicOr(reinterpret_cast<unsigned int*>(status + c), bits);
}

// ---------------------------------------------------------------------------------------
// Adjoint.  Per subcarrier: recompute Ht, its SVD and, per noise level, the Cholesky factor
// and W; back-propagate dl/dSINR through SINR = s/d, s_r = |c_rr|^2, d_r = s2 ||w_r||^2 +
// sum_{k != r} |c_rk|^2 (c = W^H HV), W = Q^{-1} HV and Q = HV HV^H + s2 I to dl/dHV; then
// through HV = U_ns Sigma_ns to dl/dHt with the singular-vector adjoint restricted to the
// kept block:
//   P = U_ns^H (dl/dHV),  D_aa = Re P_aa,
//   D_ab = (sigma_b^2 P_ab - sigma_a sigma_b conj(P_ba)) / (sigma_b^2 - sigma_a^2)  (a != b),
//   dl/dHt = U_ns D V_ns^H.
// The chain depends on HV only through HV^H HV, so dl/dHV = HV S with S Hermitian; its
// component outside span(U_ns) is zero and no out-of-block terms arise.  D_ab is set to 0
// when sigma_a and sigma_b are numerically equal (the exact value for such S).
// dl/dHt per subcarrier goes to the workspace; k_sinr_bwd_reduce forms dl/dG and dl/dC.

template <typename T, int MP, int NMAX, typename E = float2, typename O = float, int SPB = 64 / MP>
__global__ void __launch_bounds__(64) k_sinr_bwd(const DevChan* __restrict__ chans, ScRange R,
                                                  int64_t total_sc, const E* __restrict__ C,
                                                  const E* __restrict__ G, SnrArgs snr,
                                                  const O* __restrict__ gsinr, int ns_max,
                                                  char* ws, int32_t* status) {
  __shared__ SinrLds<T, MP, NMAX> lds[SPB];
  const int grp = threadIdx.x / MP, r = threadIdx.x % MP;
  SinrLds<T, MP, NMAX>& S = lds[grp];
  const int64_t it = (int64_t)blockIdx.x * SPB + grp;
  const bool valid = it < R.count;
  int64_t gsc = 0;
  const int c = valid ? locate_sc(R, chans, it, gsc) : 0;
  const DevChan& ch = chans[c];
  const int64_t s = gsc - ch.sc;
  int M, N;
  build_gram<T, MP, NMAX, false>(S, r, valid, ch, s, (const E*)nullptr, C, G, M, N);
  bool conv = jacobi_herm<T, MP, 1>(S.e, r, 0, sizeof(T) == 4 ? 12 : 20);
  uint32_t bits = conv ? 0u : GT_DEV_EIG_SWEEPS;
  const int ns = valid ? ch.ns : 0;
  singular_setup<T, MP, NMAX>(S, r, M, ns, bits);
  // right singular vectors v_k = Ht^H u_k / sigma_k, rows of S.vr/vi (lanes stride over n)
  for (int k = 0; k < ns; ++k) {
    const int col = S.e.src[k];
    const T inv = S.sig[k] > T(0) ? T(1) / S.sig[k] : T(0);
    for (int j = r; j < N; j += MP) {
      T ar = 0, ai = 0;
      for (int i = 0; i < M; ++i) {  // conj(Ht[i][j]) u[i]
        T hr = S.hr[i][j], hi = S.hi[i][j], ur = S.e.vr[i][col], ui = S.e.vi[i][col];
        ar += hr * ur + hi * ui;
        ai += hr * ui - hi * ur;
      }
      S.vr[k][j] = ar * inv;
      S.vi[k][j] = ai * inv;
    }
  }
  // dl/dHV accumulated over noise levels (row r, columns k < ns)
  for (int k = 0; k < MP; ++k) {
    S.gr[r][k] = 0;
    S.gi[r][k] = 0;
  }
  wave_sync();
  // per-lane scratch for stream r: C-bar row and N-bar
  for (int kk = 0; kk < snr.n; ++kk) {
    const T s2 = (T)snr.s2[kk];
    bool ok = mmse_filter<T, MP, NMAX>(S, r, M, ns, s2);
    if (!ok && r == 0) bits |= GT_DEV_CHOLESKY;
    // stage 1 (lane r < ns): s_r, d_r, the row C-bar[r][.] and N-bar_r; W-bar column r
    T cbr[MP], cbi[MP];
    T nbar = 0;
    if (r < ns && ok) {
      T sv, dv;
      stream_sinr<T, MP, NMAX>(S, r, M, ns, s2, sv, dv);
      const T g = valid ? (T)gsinr[((int64_t)kk * total_sc + gsc) * ns_max + r] : T(0);
      const T sbar = g / dv;
      const T dbar = -g * sv / (dv * dv);
      nbar = s2 * dbar;
#pragma unroll
      for (int k = 0; k < MP; ++k) {
        T cr = 0, ci = 0;
        if (k < ns)
          for (int i = 0; i < M; ++i) {
            T wr = S.wr[i][r], wi = S.wi[i][r], hr = S.hvr[i][k], hi = S.hvi[i][k];
            cr += wr * hr + wi * hi;
            ci += wr * hi - wi * hr;
          }
        const T f = (k == r) ? T(2) * sbar : T(2) * dbar;
        cbr[k] = f * cr;
        cbi[k] = f * ci;
      }
    } else {
#pragma unroll
      for (int k = 0; k < MP; ++k) cbr[k] = cbi[k] = 0;
    }
    // publish C-bar (row r) through the e.vr/vi rows >= MP/?  -> use S.e.lam/src free space:
    // store C-bar in the (now unused) eigenvector storage of columns >= MP/2 would alias;
    // use the dedicated rows of hr/hi beyond N instead: keep it simple with shuffles below.
    // W-bar[i][r] = sum_k hv[i][k] conj(Cbar[r][k]) + 2 nbar w[i][r]  -> stored in S.hr? no:
    // Lambda = Q^{-1} W-bar computed column r in lane r, kept in registers lr/li[].
    T lr_[MP], li_[MP];
#pragma unroll
    for (int i = 0; i < MP; ++i) {
      T ar = 0, ai = 0;
      if (r < ns && ok && i < M) {
#pragma unroll
        for (int k = 0; k < MP; ++k) {
          if (k < ns) {  // hv[i][k] conj(cb[k])
            T hr = S.hvr[i][k], hi = S.hvi[i][k];
            ar += hr * cbr[k] + hi * cbi[k];
            ai += hi * cbr[k] - hr * cbi[k];
          }
        }
        ar += T(2) * nbar * S.wr[i][r];
        ai += T(2) * nbar * S.wi[i][r];
      }
      lr_[i] = ar;
      li_[i] = ai;
    }
    if (r < ns && ok) {
      // forward solve L y = wbar, back solve L^H lambda = y (in registers, unrolled)
#pragma unroll
      for (int i = 0; i < MP; ++i) {
        if (i < M) {
          T ar = lr_[i], ai = li_[i];
#pragma unroll
          for (int j = 0; j < MP; ++j)
            if (j < i) {
              T l_r = S.e.kr[i][j], l_i = S.e.ki[i][j];
              ar -= l_r * lr_[j] - l_i * li_[j];
              ai -= l_r * li_[j] + l_i * lr_[j];
            }
          T inv = T(1) / S.e.kr[i][i];
          lr_[i] = ar * inv;
          li_[i] = ai * inv;
        }
      }
#pragma unroll
      for (int i = MP - 1; i >= 0; --i) {
        if (i < M) {
          T ar = lr_[i], ai = li_[i];
#pragma unroll
          for (int j = 0; j < MP; ++j)
            if (j > i && j < M) {
              T l_r = S.e.kr[j][i], l_i = S.e.ki[j][i];
              ar -= l_r * lr_[j] + l_i * li_[j];
              ai -= l_r * li_[j] - l_i * lr_[j];
            }
          T inv = T(1) / S.e.kr[i][i];
          lr_[i] = ar * inv;
          li_[i] = ai * inv;
        }
      }
    }
    // publish Lambda (column r) and C-bar (row r) to LDS: Lambda -> S.hvr/hvi is in use;
    // reuse S.e.vr/vi columns? They hold U which is still needed.  Use S.vr/vi rows from
    // MP/2? They hold v_k (k < ns).  So stage in the dedicated adjoint buffers:
    //   Lambda[i][r] in S.wr/wi is not possible (W still needed) -> use gr/gi as temporary?
    // gr/gi accumulates dl/dHV, so stage Lambda in the eigen K storage (Cholesky no longer
    // needed after this point) and C-bar in S.e.vr? no: in S.e.lam/src cannot hold MP^2.
    wave_sync();
    if (r < MP) {
#pragma unroll
      for (int i = 0; i < MP; ++i) {
        S.e.kr[i][r] = (r < ns && ok) ? lr_[i] : T(0);  // Lambda column r
        S.e.ki[i][r] = (r < ns && ok) ? li_[i] : T(0);
      }
    }
    // C-bar row r into S.hr/hi rows beyond the compressed channel? hr has MP rows of NMAX;
    // it still holds Ht (needed later only for v, already computed), so reuse it.
#pragma unroll
    for (int k = 0; k < MP; ++k) {
      if (k <= NMAX) {
        S.hr[r][k] = cbr[k];
        S.hi[r][k] = cbi[k];
      }
    }
    wave_sync();
    // dl/dHV[i][k] += (W Cbar)[i][k] + Lambda[i][k] - (Lambda W^H HV + W Lambda^H HV)[i][k]
    if (r < M && ok) {
      for (int k = 0; k < ns; ++k) {
        T ar = S.e.kr[r][k], ai = S.e.ki[r][k];  // Lambda[r][k]
        for (int j = 0; j < ns; ++j) {
          // W[r][j] Cbar[j][k]
          T wr = S.wr[r][j], wi = S.wi[r][j], cr = S.hr[j][k], ci = S.hi[j][k];
          ar += wr * cr - wi * ci;
          ai += wr * ci + wi * cr;
          // c_jk = w_j^H hv_k ;  (Lambda W^H HV)[r][k] = sum_j Lambda[r][j] c_jk
          T xr = 0, xi = 0, yr = 0, yi = 0;
          for (int i = 0; i < M; ++i) {
            T w_r = S.wr[i][j], w_i = S.wi[i][j], l_r = S.e.kr[i][j], l_i = S.e.ki[i][j];
            T h_r = S.hvr[i][k], h_i = S.hvi[i][k];
            xr += w_r * h_r + w_i * h_i;  // conj(w) hv
            xi += w_r * h_i - w_i * h_r;
            yr += l_r * h_r + l_i * h_i;  // conj(lambda) hv
            yi += l_r * h_i - l_i * h_r;
          }
          T Lr = S.e.kr[r][j], Li = S.e.ki[r][j];
          ar -= Lr * xr - Li * xi;
          ai -= Lr * xi + Li * xr;
          ar -= wr * yr - wi * yi;
          ai -= wr * yi + wi * yr;
        }
        S.gr[r][k] += ar;
        S.gi[r][k] += ai;
      }
    }
    wave_sync();
  }
  // singular-vector stage: P = U_ns^H dl/dHV (ns x ns), then D, then dl/dHt = U_ns D V_ns^H
  // lane a < ns computes row a of P then of D
  T dr_[MP], di_[MP];
#pragma unroll
  for (int b = 0; b < MP; ++b) dr_[b] = di_[b] = 0;
  if (r < ns) {
    const int cola = S.e.src[r];
#pragma unroll
    for (int b = 0; b < MP; ++b) {
      if (b < ns) {
        T pr = 0, pi = 0;
        for (int i = 0; i < M; ++i) {
          T ur = S.e.vr[i][cola], ui = S.e.vi[i][cola], gr = S.gr[i][b], gi = S.gi[i][b];
          pr += ur * gr + ui * gi;
          pi += ur * gi - ui * gr;
        }
        dr_[b] = pr;
        di_[b] = pi;
      }
    }
  }
  wave_sync();
  // publish P rows into S.hr/hi (rows a < ns)
  if (r < ns) {
#pragma unroll
    for (int b = 0; b < MP; ++b)
      if (b <= NMAX) {
        S.hr[r][b] = dr_[b];
        S.hi[r][b] = di_[b];
      }
  }
  wave_sync();
  if (r < ns) {
    const T sa = S.sig[r];
    const T la = sa * sa;
    const T lam1 = S.sig[0] * S.sig[0];
#pragma unroll
    for (int b = 0; b < MP; ++b) {
      if (b < ns) {
        if (b == r) {
          dr_[b] = S.hr[r][r];
          di_[b] = 0;
        } else {
          const T sb = S.sig[b];
          const T lb = sb * sb;
          const T gap = lb - la;
          if (__builtin_fabs(gap) > T(1e-5) * lam1) {
            T pab_r = S.hr[r][b], pab_i = S.hi[r][b];
            T pba_r = S.hr[b][r], pba_i = S.hi[b][r];
            dr_[b] = (lb * pab_r - sa * sb * pba_r) / gap;
            di_[b] = (lb * pab_i + sa * sb * pba_i) / gap;
          } else {
            dr_[b] = di_[b] = 0;
          }
        }
      }
    }
  }
  wave_sync();
  if (r < ns) {
#pragma unroll
    for (int b = 0; b < MP; ++b)
      if (b <= NMAX) {
        S.hr[r][b] = dr_[b];
        S.hi[r][b] = di_[b];
      }
  }
  wave_sync();
  // dl/dHt[i][j] = sum_{a,b} u_a[i] D[a][b] conj(v_b[j]); lane i = row
  if (valid && r < M) {
    E* gH = reinterpret_cast<E*>(ws + ch.w_gH) + s * ch.m * ch.n;
    for (int j = 0; j < N; ++j) {
      T ar = 0, ai = 0;
      for (int a = 0; a < ns; ++a) {
        const int cola = S.e.src[a];
        T ur = S.e.vr[r][cola], ui = S.e.vi[r][cola];
        T tr = 0, ti = 0;  // sum_b D[a][b] conj(v_b[j])
        for (int b = 0; b < ns; ++b) {
          T dr = S.hr[a][b], di = S.hi[a][b], vr = S.vr[b][j], vi = -S.vi[b][j];
          tr += dr * vr - di * vi;
          ti += dr * vi + di * vr;
        }
        ar += ur * tr - ui * ti;
        ai += ur * ti + ui * tr;
      }
      gH[(int64_t)r * ch.n + j] = Elem<E>::make((typename Elem<E>::R)ar, (typename Elem<E>::R)ai);
    }
  }
  if (valid && status && bits && r == 0) atomicOr(reinterpret_cast<unsigned int*>(status + c), bits);
}

// dl/dG_g[q] = sum_{s in g} conj(C[s,q]) dl/dHt_s ;  dl/dC[s,q] = <dl/dHt_s, G_g[q]>
// STAGE: dl/dHt_s of the group and G_g are first copied to LDS (when they fit), so that the two
// contractions read them from LDS rather than through the caches once per q or per entry.
template <bool STAGE, typename E = float2>
__global__ void __launch_bounds__(256) k_sinr_bwd_reduce(const DevChan* __restrict__ chans,
                                                         const GroupItem* __restrict__ items,
                                                         const E* __restrict__ C,
                                                         const E* __restrict__ G,
                                                         E* gC, E* gG, char* ws) {
  using R = typename Elem<E>::R;
  extern __shared__ __align__(16) char sm_raw[];
  E* sm = reinterpret_cast<E*>(sm_raw);
  const GroupItem it = items[blockIdx.x];
  const DevChan& ch = chans[it.ch];
  const int s0 = it.g * ch.gs;
  const int sz = min(ch.gs, ch.nsc - s0);
  const int pg = min(ch.p, sz);
  const int mn = ch.m * ch.n;
  const E* gHm = reinterpret_cast<const E*>(ws + ch.w_gH) + (int64_t)s0 * mn;
  const E* Ggm = G + ch.g + (int64_t)it.g * ch.p * mn;
  E* gGg = gG + ch.g + (int64_t)it.g * ch.p * mn;
  const E* gH = gHm;
  const E* Gg = Ggm;
  const E* Cg = C + ch.c + (int64_t)s0 * ch.p;  // the group's C rows (stride p)
  // matrix-core form (FP32, groups of at most 16 subcarriers, p <= 16, m n a multiple of 16):
  // the staged rows of dl/dHt and of the cores take a stride of m n + 1 so that the 16 rows a
  // product operand spans fall in distinct LDS banks
  const bool mf = STAGE && sizeof(E) == 8 && ch.gs <= 16 && ch.p <= 16 && (mn % 16) == 0;
  const int ld = mf ? mn + 1 : mn;
  if (STAGE) {
    // dl/dHt, the cores and the C rows of the group in LDS (every product below reads them
    // many times)
    E* sH = sm;
    E* sG = sm + sz * ld;
    E* sC = sG + pg * ld;
    // every thread issues its loads of the three arrays (up to B of each) before its LDS
    // stores, so one memory latency covers the copy of a group
    constexpr int B = 8;
    const int nH = sz * mn, nG = pg * mn, nC = sz * ch.p;
    const int nmax = max(nH, max(nG, nC));
    for (int e0 = threadIdx.x; e0 < nmax; e0 += B * blockDim.x) {
      E vh[B], vg[B], vc[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int e = e0 + u * (int)blockDim.x;
        if (e < nH) vh[u] = gHm[e];
        if (e < nG) vg[u] = Ggm[e];
        if (e < nC) vc[u] = Cg[e];
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int e = e0 + u * (int)blockDim.x;
        if (e < nH) sH[mf ? (e / mn) * ld + e % mn : e] = vh[u];
        if (e < nG) sG[mf ? (e / mn) * ld + e % mn : e] = vg[u];
        if (e < nC) sC[e] = vc[u];
      }
    }
    __syncthreads();
    gH = sH;
    Gg = sG;
    Cg = sC;
  }
  if constexpr (sizeof(E) == 8) {
    if (mf) {
      // 16 x 16 x 4 FP32 matrix-core products on the real forms, lane l holding operand row
      // (or column) l % 16 and K index 4 t + l / 16; K runs over (subcarrier or entry, re/im):
      //   dl/dG[q][e] = sum_s conj(C[s,q]) dHt_s[e]: Re = sum (cr hr + ci hi), Im = sum (cr hi - ci hr)
      //   dl/dC[s][q] = sum_e conj(G_q[e]) dHt_s[e]: Re = sum (hr gr + hi gi), Im = sum (hi gr - hr gi)
      const float* sHf = reinterpret_cast<const float*>(gH);
      const float* sGf = reinterpret_cast<const float*>(Gg);
      const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, l16 = lane % 16, kq = lane / 16;
      const int ksteps = (2 * sz + 3) / 4;
      for (int Et = wave; Et < mn / 16; Et += 4) {
        const int e = 16 * Et + l16;
        f32x4 are = {0.f, 0.f, 0.f, 0.f}, aim = {0.f, 0.f, 0.f, 0.f};
        for (int t = 0; t < ksteps; ++t) {
          const int k = 4 * t + kq, sk = k >> 1, part = k & 1;
          float cr = 0.f, ci = 0.f, hr = 0.f, hi = 0.f;
          if (sk < sz) {
            if (l16 < pg) {
              const E cv = Cg[sk * ch.p + l16];
              cr = cv.x;
              ci = cv.y;
            }
            hr = sHf[2 * (sk * ld + e)];
            hi = sHf[2 * (sk * ld + e) + 1];
          }
          are = __builtin_amdgcn_mfma_f32_16x16x4f32(part ? ci : cr, part ? hi : hr, are, 0, 0, 0);
          aim = __builtin_amdgcn_mfma_f32_16x16x4f32(part ? -ci : cr, part ? hr : hi, aim, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int q = 4 * kq + v;
          if (q < ch.p) gGg[(int64_t)q * mn + e] = Elem<E>::make(are[v], aim[v]);
        }
      }
      // dl/dC: the four waves split the entries, then their 16 x 16 partial tiles are summed
      f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
      {
        const int ew = mn / 4, e0w = wave * ew;  // this wave's entries
        for (int t = 0; t < ew / 2; ++t) {
          const int k = 4 * t + kq, e = e0w + (k >> 1), part = k & 1;
          float hr = 0.f, hi = 0.f, gr = 0.f, gi = 0.f;
          if (l16 < sz) {
            hr = sHf[2 * (l16 * ld + e)];
            hi = sHf[2 * (l16 * ld + e) + 1];
          }
          if (l16 < pg) {
            gr = sGf[2 * (l16 * ld + e)];
            gi = sGf[2 * (l16 * ld + e) + 1];
          }
          cre = __builtin_amdgcn_mfma_f32_16x16x4f32(part ? hi : hr, part ? gi : gr, cre, 0, 0, 0);
          cim = __builtin_amdgcn_mfma_f32_16x16x4f32(part ? hr : hi, part ? -gi : gr, cim, 0, 0, 0);
        }
      }
      __syncthreads();  // every read of the staged rows is done: the partials reuse that LDS
      float* red = reinterpret_cast<float*>(sm);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        red[(wave * 4 + v) * 128 + lane] = cre[v];
        red[(wave * 4 + v) * 128 + 64 + lane] = cim[v];
      }
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float xr = 0.f, xi = 0.f;
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            xr += red[(w * 4 + v) * 128 + lane];
            xi += red[(w * 4 + v) * 128 + 64 + lane];
          }
          const int si = 4 * kq + v;  // output row (subcarrier), column q = l16
          if (si < sz && l16 < ch.p)
            gC[ch.c + (int64_t)(s0 + si) * ch.p + l16] = Elem<E>::make(xr, xi);
        }
      }
      return;
    }
  }
  // dl/dG: a thread owns entry e for QC consecutive q, so each dl/dHt entry is read once per
  // chunk of q (rows q >= p_g are written as zero)
  constexpr int QC = 8;
  const int nqc = (ch.p + QC - 1) / QC;
  // (with FP32 elements, an even p and the C rows 16-byte aligned, the C entries are read two
  // per 16-byte load)
  const bool c_pairs =
      sizeof(E) == 8 && (ch.p % 2) == 0 && (reinterpret_cast<uintptr_t>(Cg) & 15) == 0;
  for (int o = threadIdx.x; o < nqc * mn; o += blockDim.x) {
    const int qc = o / mn, e = o - qc * mn;
    Cx<R> acc[QC];
#pragma unroll
    for (int j = 0; j < QC; ++j) acc[j] = Cx<R>{R(0), R(0)};
    for (int i = 0; i < sz; ++i) {
      const Cx<R> h = ldc<R>(gH + (int64_t)i * mn + e);
      const E* Ci = Cg + (int64_t)i * ch.p + qc * QC;
      if (c_pairs) {
#pragma unroll
        for (int j = 0; j < QC; j += 2) {
          if (qc * QC + j < pg) {
            const float4 cv = *reinterpret_cast<const float4*>(Ci + j);
            cfmac(acc[j], Cx<R>{R(cv.x), R(cv.y)}, h);
            if (qc * QC + j + 1 < pg) cfmac(acc[j + 1], Cx<R>{R(cv.z), R(cv.w)}, h);
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < QC; ++j)
          if (qc * QC + j < pg) cfmac(acc[j], ldc<R>(Ci + j), h);
      }
    }
#pragma unroll
    for (int j = 0; j < QC; ++j)
      if (qc * QC + j < ch.p) gGg[(int64_t)(qc * QC + j) * mn + e] = Elem<E>::make(acc[j].re, acc[j].im);
  }
  // dl/dC: 16 lanes per 2 x 2 tile of (s, q) split the m n entries and reduce by shuffles (each
  // loaded entry of dl/dHt and of a core serves two outputs); the 16 lanes of a tile are aligned
  // and run the same passes
  const int l16 = threadIdx.x % 16;
  const int ti = (sz + 1) / 2, tq = (ch.p + 1) / 2;
  for (int o = threadIdx.x / 16; o < ti * tq; o += blockDim.x / 16) {
    const int i0 = 2 * (o / tq), q0 = 2 * (o % tq);
    const bool i1 = i0 + 1 < sz, g0 = q0 < pg, g1 = q0 + 1 < pg;
    R ar[2][2], ai[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) ar[a][b] = ai[a][b] = R(0);
    const E zero = Elem<E>::make(R(0), R(0));
#pragma unroll 4
    for (int e = l16; e < mn; e += 16) {
      E h[2], g[2];
      h[0] = gH[(int64_t)i0 * mn + e];
      h[1] = i1 ? gH[(int64_t)(i0 + 1) * mn + e] : zero;
      g[0] = g0 ? Gg[(int64_t)q0 * mn + e] : zero;
      g[1] = g1 ? Gg[(int64_t)(q0 + 1) * mn + e] : zero;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {  // conj(g_b) h_a
          ar[a][b] += g[b].x * h[a].x + g[b].y * h[a].y;
          ai[a][b] += g[b].x * h[a].y - g[b].y * h[a].x;
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int d = 8; d > 0; d >>= 1) {
          ar[a][b] += __shfl_xor(ar[a][b], d, 64);
          ai[a][b] += __shfl_xor(ai[a][b], d, 64);
        }
    if (l16 == 0) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (i0 + a < sz && q0 + b < ch.p)
            gC[ch.c + (int64_t)(s0 + i0 + a) * ch.p + q0 + b] = Elem<E>::make(ar[a][b], ai[a][b]);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Host launchers

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

// Range of SINR classes [k0, k1) of the plan; count 0 when they hold no channel.
static ScRange sc_range(const LaunchCtx& L, int k0, int k1) {
  ScRange R;
  const int j0 = L.sc_j[k0], j1 = L.sc_j[k1];
  R.ch = L.d_sc_ch + j0;
  R.off = L.d_sc_off + j0;
  R.n = j1 - j0;
  R.base = L.sc_base[k0];
  R.count = L.sc_base[k1] - L.sc_base[k0];
  return R;
}

static int sc_maxn(const LaunchCtx& L, int k0, int k1) {
  int v = 0;
  for (int k = k0; k < k1; ++k) v = std::max(v, L.sc_maxn[k]);
  return v;
}

template <int MP, int NMAX, bool FULL>
static gt_status sinr_launch_t(const LaunchCtx& L, const ScRange& R, int64_t total_sc,
                               const float2* X, const float2* C, const float2* G, const SnrArgs& a,
                               float* out, int ns_max, int32_t* status) {
  constexpr int SPB = 64 / MP;
  const unsigned grid = (unsigned)((R.count + SPB - 1) / SPB);
  GT_LAUNCH((k_sinr<float, MP, NMAX, FULL>), dim3(grid), dim3(64), L.d_chans, R, total_sc, X, C, G,
            a, out, ns_max, status);
  return GT_OK;
}

gt_status launch_sinr_rows(const LaunchCtx& L, int k0, int k1, int mp, int nsm, int64_t total_sc,
                           const float2* C, const float2* G, const float* s2, int n_snr,
                           float* out, int ns_max, int32_t* status);

// One launch per non-empty SINR class: the row-parallel kernel for m <= 8, the cooperative
// one for larger m; the full-channel form runs one cooperative launch over every channel.
gt_status launch_sinr(const LaunchCtx& L, int64_t total_sc, bool full, const float2* X,
                      const float2* C, const float2* G, const float* s2, int n_snr, float* out,
                      int ns_max, int32_t* status) {
  SnrArgs a{};
  a.n = n_snr;
  for (int k = 0; k < n_snr; ++k) a.s2[k] = s2[k];
  if (full) {
    const ScRange R = sc_range(L, 0, SC_COUNT);
    const int M = L.max_nr;
    if (M <= 4) return sinr_launch_t<4, 1, true>(L, R, total_sc, X, C, G, a, out, ns_max, status);
    if (M <= 8) return sinr_launch_t<8, 1, true>(L, R, total_sc, X, C, G, a, out, ns_max, status);
    return sinr_launch_t<16, 1, true>(L, R, total_sc, X, C, G, a, out, ns_max, status);
  }
  for (int k = 0; k < SC_COUNT; ++k) {
    const ScRange R = sc_range(L, k, k + 1);
    if (R.count == 0) continue;
    gt_status st = GT_OK;
    switch (k) {
      case SC_LANE4_2: st = launch_sinr_rows(L, k, k + 1, 4, 2, total_sc, C, G, s2, n_snr, out, ns_max, status); break;
      case SC_LANE4_4: st = launch_sinr_rows(L, k, k + 1, 4, 4, total_sc, C, G, s2, n_snr, out, ns_max, status); break;
      case SC_LANE8_4: st = launch_sinr_rows(L, k, k + 1, 8, 4, total_sc, C, G, s2, n_snr, out, ns_max, status); break;
      case SC_LANE8_8: st = launch_sinr_rows(L, k, k + 1, 8, 8, total_sc, C, G, s2, n_snr, out, ns_max, status); break;
      case SC_COOP_32:
        st = sinr_launch_t<16, 32, false>(L, R, total_sc, X, C, G, a, out, ns_max, status);
        break;
      default:
        st = sinr_launch_t<16, 64, false>(L, R, total_sc, X, C, G, a, out, ns_max, status);
        break;
    }
    if (st != GT_OK) return st;
  }
  return GT_OK;
}

gt_status launch_grad_cg(const LaunchCtx& L, const float2* C, const float2* G, float2* gC, float2* gG);

template <int MP, int NMAX>
static gt_status sinr_bwd_t(const LaunchCtx& L, const ScRange& R, int64_t total_sc, const float2* C,
                            const float2* G, const SnrArgs& a, const float* gs, int ns_max,
                            int32_t* status) {
  constexpr int SPB = 64 / MP;
  const unsigned grid = (unsigned)((R.count + SPB - 1) / SPB);
  GT_LAUNCH((k_sinr_bwd<float, MP, NMAX>), dim3(grid), dim3(64), L.d_chans, R, total_sc, C, G, a, gs,
            ns_max, L.ws, status);
  return GT_OK;
}

gt_status launch_sinr_bwd_rows(const LaunchCtx& L, int k0, int k1, int mp, int nsm,
                               int64_t total_sc, const float2* C, const float2* G, const float* s2,
                               int n_snr, const float* gsinr, int ns_max, int32_t* status);

// The adjoint: the row-parallel kernel for m <= 8 with ns <= 4, the cooperative one for the rest
// (m <= 8 with ns > 4 on 8-lane groups sized by n), one launch per non-empty class, then the
// per-group reduction into dl/dC and dl/dG.
gt_status launch_sinr_bwd(const LaunchCtx& L, int64_t total_sc, const float2* C, const float2* G,
                          const float* s2, int n_snr, const float* gsinr, float2* gC, float2* gG,
                          int ns_max, int32_t* status) {
  SnrArgs a{};
  a.n = n_snr;
  for (int k = 0; k < n_snr; ++k) a.s2[k] = s2[k];
  for (int k = 0; k < SC_COUNT; ++k) {
    const ScRange R = sc_range(L, k, k + 1);
    if (R.count == 0) continue;
    gt_status st = GT_OK;
    switch (k) {
      case SC_LANE4_2: st = launch_sinr_bwd_rows(L, k, k + 1, 4, 2, total_sc, C, G, s2, n_snr, gsinr, ns_max, status); break;
      case SC_LANE4_4: st = launch_sinr_bwd_rows(L, k, k + 1, 4, 4, total_sc, C, G, s2, n_snr, gsinr, ns_max, status); break;
      case SC_LANE8_4: st = launch_sinr_bwd_rows(L, k, k + 1, 8, 4, total_sc, C, G, s2, n_snr, gsinr, ns_max, status); break;
      case SC_LANE8_8: {
        const int N = sc_maxn(L, k, k + 1);
        st = N <= 16 ? sinr_bwd_t<8, 16>(L, R, total_sc, C, G, a, gsinr, ns_max, status)
                     : (N <= 32 ? sinr_bwd_t<8, 32>(L, R, total_sc, C, G, a, gsinr, ns_max, status)
                                : sinr_bwd_t<8, 64>(L, R, total_sc, C, G, a, gsinr, ns_max, status));
        break;
      }
      case SC_COOP_32: st = sinr_bwd_t<16, 32>(L, R, total_sc, C, G, a, gsinr, ns_max, status); break;
      default: st = sinr_bwd_t<16, 64>(L, R, total_sc, C, G, a, gsinr, ns_max, status); break;
    }
    if (st != GT_OK) return st;
  }
  return launch_grad_cg(L, C, G, gC, gG);
}

template <typename E>
static gt_status grad_cg_t(const LaunchCtx& L, const E* C, const E* G, E* gC, E* gG) {
  // (the staged rows may take a stride of m n + 1, and the matrix-core form reuses at least 8 KB
  // of the block's LDS for the four waves' partial dl/dC tiles)
  const size_t sh = std::max<size_t>(
      8192, sizeof(E) * (((size_t)L.max_gs + L.max_p) * ((size_t)L.max_m * L.max_n + 1) +
                         (size_t)L.max_gs * L.max_p));
  if (sh <= 64 * 1024) {
    prof_begin("k_sinr_bwd_reduce", L.stream);
    hipLaunchKernelGGL((k_sinr_bwd_reduce<true, E>), dim3(L.total_groups), dim3(256), sh, L.stream,
                       L.d_chans, L.d_groups, C, G, gC, gG, L.ws);
    prof_end(L.stream);
    hipError_t e_ = hipGetLastError();
    if (e_ != hipSuccess) {
      set_error_detail("k_sinr_bwd_reduce", e_);
      return GT_ERR_HIP;
    }
    return GT_OK;
  }
  GT_LAUNCH((k_sinr_bwd_reduce<false, E>), dim3(L.total_groups), dim3(256), L.d_chans, L.d_groups, C, G,
            gC, gG, L.ws);
  return GT_OK;
}

gt_status launch_grad_cg(const LaunchCtx& L, const float2* C, const float2* G, float2* gC, float2* gG) {
  return grad_cg_t<float2>(L, C, G, gC, gG);
}

// ---------------------------------------------------------------------------------------
// FP64 (c128 plans): every class on the cooperative kernels in double, one subcarrier per
// block of MP lanes (MP = 4, 8 or 16 by the class's m; staged rows sized by its largest n).
// This form exists for validation and gradient checks, not for throughput.

template <int MP, int NMAX, bool FULL>
static gt_status sinr64_t(const LaunchCtx& L, const ScRange& R, int64_t total_sc, const double2* X,
                          const double2* C, const double2* G, const SnrArgs& a, double* out,
                          int ns_max, int32_t* status) {
  GT_LAUNCH((k_sinr<double, MP, NMAX, FULL, double2, double, 1>), dim3((unsigned)R.count), dim3(MP),
            L.d_chans, R, total_sc, X, C, G, a, out, ns_max, status);
  return GT_OK;
}

template <int MP>
static gt_status sinr64_by_n(const LaunchCtx& L, const ScRange& R, int N, int64_t total_sc,
                             const double2* C, const double2* G, const SnrArgs& a, double* out,
                             int ns_max, int32_t* status) {
  if (N <= 16) return sinr64_t<MP, 16, false>(L, R, total_sc, nullptr, C, G, a, out, ns_max, status);
  if (N <= 32) return sinr64_t<MP, 32, false>(L, R, total_sc, nullptr, C, G, a, out, ns_max, status);
  return sinr64_t<MP, 64, false>(L, R, total_sc, nullptr, C, G, a, out, ns_max, status);
}

static int class_mp(int k) {
  return (k == SC_LANE4_2 || k == SC_LANE4_4) ? 4 : ((k == SC_LANE8_4 || k == SC_LANE8_8) ? 8 : 16);
}

gt_status launch_sinr_c128(const LaunchCtx& L, int64_t total_sc, bool full, const double2* X,
                           const double2* C, const double2* G, const float* s2, int n_snr,
                           double* out, int ns_max, int32_t* status) {
  SnrArgs a{};
  a.n = n_snr;
  for (int k = 0; k < n_snr; ++k) a.s2[k] = s2[k];
  if (full) {
    const ScRange R = sc_range(L, 0, SC_COUNT);
    if (R.count == 0) return GT_OK;
    const int M = L.max_nr;
    if (M <= 4) return sinr64_t<4, 1, true>(L, R, total_sc, X, C, G, a, out, ns_max, status);
    if (M <= 8) return sinr64_t<8, 1, true>(L, R, total_sc, X, C, G, a, out, ns_max, status);
    return sinr64_t<16, 1, true>(L, R, total_sc, X, C, G, a, out, ns_max, status);
  }
  for (int k = 0; k < SC_COUNT; ++k) {
    const ScRange R = sc_range(L, k, k + 1);
    if (R.count == 0) continue;
    const int N = sc_maxn(L, k, k + 1);
    const int mp = class_mp(k);
    gt_status st = mp == 4 ? sinr64_by_n<4>(L, R, N, total_sc, C, G, a, out, ns_max, status)
                 : mp == 8 ? sinr64_by_n<8>(L, R, N, total_sc, C, G, a, out, ns_max, status)
                           : sinr64_by_n<16>(L, R, N, total_sc, C, G, a, out, ns_max, status);
    if (st != GT_OK) return st;
  }
  return GT_OK;
}

template <int MP, int NMAX>
static gt_status sinr64_bwd_t(const LaunchCtx& L, const ScRange& R, int64_t total_sc, const double2* C,
                              const double2* G, const SnrArgs& a, const double* gs, int ns_max,
                              int32_t* status) {
  GT_LAUNCH((k_sinr_bwd<double, MP, NMAX, double2, double, 1>), dim3((unsigned)R.count), dim3(MP),
            L.d_chans, R, total_sc, C, G, a, gs, ns_max, L.ws, status);
  return GT_OK;
}

template <int MP>
static gt_status sinr64_bwd_by_n(const LaunchCtx& L, const ScRange& R, int N, int64_t total_sc,
                                 const double2* C, const double2* G, const SnrArgs& a,
                                 const double* gs, int ns_max, int32_t* status) {
  if (N <= 16) return sinr64_bwd_t<MP, 16>(L, R, total_sc, C, G, a, gs, ns_max, status);
  if (N <= 32) return sinr64_bwd_t<MP, 32>(L, R, total_sc, C, G, a, gs, ns_max, status);
  return sinr64_bwd_t<MP, 64>(L, R, total_sc, C, G, a, gs, ns_max, status);
}

gt_status launch_sinr_bwd_c128(const LaunchCtx& L, int64_t total_sc, const double2* C,
                               const double2* G, const float* s2, int n_snr, const double* gsinr,
                               double2* gC, double2* gG, int ns_max, int32_t* status) {
  SnrArgs a{};
  a.n = n_snr;
  for (int k = 0; k < n_snr; ++k) a.s2[k] = s2[k];
  for (int k = 0; k < SC_COUNT; ++k) {
    const ScRange R = sc_range(L, k, k + 1);
    if (R.count == 0) continue;
    const int N = sc_maxn(L, k, k + 1);
    const int mp = class_mp(k);
    gt_status st = mp == 4 ? sinr64_bwd_by_n<4>(L, R, N, total_sc, C, G, a, gsinr, ns_max, status)
                 : mp == 8 ? sinr64_bwd_by_n<8>(L, R, N, total_sc, C, G, a, gsinr, ns_max, status)
                           : sinr64_bwd_by_n<16>(L, R, N, total_sc, C, G, a, gsinr, ns_max, status);
    if (st != GT_OK) return st;
  }
  return grad_cg_t<double2>(L, C, G, gC, gG);
}

}  // namespace gt
