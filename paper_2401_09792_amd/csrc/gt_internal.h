// Internal types shared by the host plan code and the HIP kernels of libgtucker.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gtucker.h"

namespace gt {

// Upper bounds on shapes (checked at plan creation; the kernels size LDS by them).
constexpr int kMaxNr = 16;        // receive antennas, also bounds m
constexpr int kMaxNt = 64;        // transmit antennas handled by the Jacobi mode-2 eigensolver
constexpr int kMaxGroup = 32;     // subcarriers per group, also bounds p
constexpr int kMaxSnr = 16;
constexpr int kMaxCombinePts = 1 << 20;  // points per call of the coefficient-vector combinations

// Per-channel descriptor as the kernels see it (lives in the workspace).
struct DevChan {
  int32_t nr, nt, nsc, gs, m, n, p, ns;
  int32_t ngroups, nsplit;         // groups; row splits of the mode-2 Gram reduction
  int32_t gfirst, pad0;            // index of the channel's first group in the group table
  int64_t x, a, b, c, g, ht, sc;   // data offsets (complex elements; sc in subcarriers)
  // workspace byte offsets of this channel's scratch
  int64_t w_W;     // [ngroups][p][m][nt] c64   A^H sum_s conj(C[s,q]) H_s
  int64_t w_T;     // [nsc][nr][n]        c64   H_s B
  int64_t w_Yh;    // [nsc][m][n]         c64   A^H H_s B
  int64_t w_S1p;   // [ngroups][nr][nr]   c64   per-group mode-1 Gram
  int64_t w_S1;    // [nr][nr]            c64   mode-1 Gram
  int64_t w_S2p;   // [nsplit][nt][nt]    c64   split partials of the mode-2 Gram
  int64_t w_S2;    // [nt][nt]            c64   mode-2 Gram
  int64_t w_S3;    // [ngroups][gs][gs]   c64   per-group mode-3 Gram
  int64_t w_VA;    // [16][16]            c64   last mode-1 eigenbasis (padded)
  int64_t w_VB;    // [64][max(64,nt)]    c64   last mode-2 eigenbasis (padded; for nt > 64 the
                   //                           64-column Ritz block, column-major, c128 under
                   //                           the FP64 eigensolve)
  int64_t w_VS;    // [2][64][nt]         c64   subspace-iteration buffers (nt > 64 only; c128
                   //                           under the FP64 eigensolve)
  int64_t w_SP;    // f32 partials and small matrices of the multi-block subspace step
                   //                           (nt > 64 only)
  int64_t w_Xq;    // [2][nsc][nr][nt][2] u16   16-bit copy of X (hi, lo) for the precision form
  int64_t w_VC;    // [ngroups][32][32]   c64   last mode-3 eigenbases (padded)
  int64_t w_lamg;  // [ngroups] double          per-group sums (norms, eigenvalue sums)
  int64_t w_scal;  // [8] double                ||X||^2, eigenvalue sums of the A and B steps
  int64_t w_gH;    // [nsc][m][n]         c64   per-subcarrier gradient of Ht
  int64_t w_gAp;   // [ngroups][nr][m]    c64   per-group partial gradient of A
  int64_t w_gBp;   // [ngroups][nt][n]    c64   per-group partial gradient of B
  // prefix sums over the preceding channels of m n and nr nt: a channel's block in the
  // combined-matrix layouts starts at n_pts times these
  int64_t mn_off, rt_off;
};

struct GroupItem {
  int32_t ch, g;
};

// Compact launch grids for the generic row passes: block b of a pass belongs to the channel c
// with tiles[kind][c] <= b < tiles[kind][c + 1] (prefix sums of the channel's block counts),
// so that uneven batches launch no empty blocks.
enum TileKind {
  TK_WROWS = 0,  // W rows: ngroups x ceil(nt / 32)
  TK_TROWS,      // T = H B: ceil(ceil(nsc nr / 32) / kTRowTiles) x ceil(2 n / 32)
  TK_GRAM,       // mode-2 Gram super-tiles: S (S + 1) / 2 x nsplit, S = ceil(2 nt / 128)
  TK_RED2,       // Gram reduction: ceil(nt^2 / 256)
  TK_YH,         // Yh = A^H T: ceil(nsc n / 256)
  TK_COUNT
};
constexpr int kTRowTiles = 16;  // 32-row tiles per block of the T pass

// SINR kernel classes of a channel, by its compressed shape: the per-lane kernel for
// m <= 4 / 8 and ns <= 2 / 4 / 8, the cooperative kernel for m > 8 by n.  A batch that
// mixes classes runs one launch per class over a compact subcarrier range.
enum ScClass {
  SC_LANE4_2 = 0,  // m <= 4, ns <= 2
  SC_LANE4_4,      // m <= 4, ns <= 4
  SC_LANE8_4,      // m <= 8, ns <= 4
  SC_LANE8_8,      // m <= 8, ns <= 8
  SC_COOP_32,      // m <= 16, n <= 32
  SC_COOP_64,      // m <= 16, n <= 64
  SC_COUNT
};

// Workspace header: where the tables sit.
struct WsLayout {
  int64_t share_off[2] = {0, 0};  // int32[groups + 1] per shared factor
  int64_t share_ch[2] = {0, 0};   // int32[members]
  int64_t sys_serving = 0;        // int32[n_channels]
  int64_t sys_terms_off[3] = {0, 0, 0};  // int32[n_channels + 1] per interference mode
  int64_t sys_terms[3] = {0, 0, 0};      // int32[2 terms] per interference mode
  int64_t chans;   // DevChan[n_channels]
  int64_t groups;  // GroupItem[total_groups]
  int64_t groups_by_size;  // GroupItem[total_groups]: groups of size <= 16 first, then the rest
  int64_t tiles;   // int32[TK_COUNT][n_channels + 1]
  int64_t sc_ch;   // int32[n_channels]: channels ordered by SINR kernel class
  int64_t sc_off;  // int64[n_channels + 1]: subcarrier prefix sums in that order
  int64_t total;   // bytes
};

// Host-side launch helpers implemented in gt_plan.cpp.
struct LaunchCtx {
  hipStream_t stream;
  char* ws;
  const DevChan* d_chans;     // device pointer into ws
  const GroupItem* d_groups;  // device pointer into ws
  const GroupItem* d_groups_by_size;  // groups of size <= 16, then larger ones
  const int32_t* d_tiles;     // [TK_COUNT][n_channels + 1] block prefix sums
  int tiles_total[TK_COUNT];
  int n_channels;
  int total_groups;
  int n_small_groups;         // groups of size <= 16
  int max_nr, max_nt, max_nsc, max_gs, max_m, max_n, max_p, max_ns, max_groups, max_nsplit;
  int min_nt;
  // every channel has m == nr: A is square and unitary, so A A^H = I and the B- and C-step
  // Grams do not depend on it (the fit then runs only the last A-step, see launch_fit)
  int full_mode1 = 0;
  int eig_fp64;
  int ttm_prec;  // gt_ttm_prec of the plan
  int c0 = 0;    // first channel of this context in the caller's channel numbering
  int tune_bstep = 0;  // B-step pass variant (see gt_plan_autotune)
  int tune_tpass = 0;  // T pass variant
  // SINR classes: channels in class order, subcarrier prefix sums in that order, and per class
  // its first position, first subcarrier and largest n
  const int32_t* d_sc_ch = nullptr;
  const int64_t* d_sc_off = nullptr;
  int sc_j[SC_COUNT + 1] = {};
  int64_t sc_base[SC_COUNT + 1] = {};
  int sc_maxn[SC_COUNT] = {};
  // factor sharing (0: mode-1 factor A, 1: mode-2 factor B): groups of two or more channels
  // with the same label, members d_share_ch[d_share_off[g] .. d_share_off[g + 1])
  int n_share[2] = {0, 0};
  const int32_t* d_share_off[2] = {nullptr, nullptr};
  const int32_t* d_share_ch[2] = {nullptr, nullptr};
  // multi-cell system: 1 for each UE's serving channel
  const int32_t* d_sys_serving = nullptr;
};

// Bits of the T pass's do_c argument: the mode (0 = T only; 1 = also the group's mode-3 Gram;
// 2 = as 1 and Yh to the workspace for the cores), T_NO_STORE (T is not stored to the
// workspace: no A-step reads it) and T_GRAM_OF_T (a channel with m == nr has a square unitary
// A, so its Gram may be taken of T instead of Yh = A^H T).  The vector-ALU kernel uses the mode
// only.
constexpr int T_MODE = 3, T_NO_STORE = 4, T_GRAM_OF_T = 8;

// A fit whose batch is split into parts of consecutive channels: the parts' contexts (their
// own tables over the same per-channel workspace, part 0 on the caller's stream) and the
// events that fork the side streams from the caller's stream and join them back.
struct SplitCtx {
  int n;
  const LaunchCtx* parts;
  hipEvent_t fork;
  hipEvent_t join[3];
  // 1: the B-step pass runs over the whole batch and the parts meet after every sweep;
  // 2: every part runs whole sweeps on its own stream, part k starting its first B-step after
  //    part k-1's (stag[k-1])
  int mode;
  hipEvent_t stag[3];
  // mode 2 with the starting mode-2 factor made on the last part's stream: [0] the start of the
  // fit on the caller's stream, [1] the mode-2 Gram of X reduced, [2] its eigensolve done,
  // [3] the same passed on by the caller's stream
  hipEvent_t init[4];
};

// kernel timing hooks (no-ops unless profiling is on)
void prof_begin(const char* name, hipStream_t s);
void prof_end(hipStream_t s);
void set_error_detail(const char* where, hipError_t e);

}  // namespace gt
