// Host side of libgtucker: plan creation and validation, packed-buffer offsets, workspace
// layout, the C ABI entry points, status strings and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gt_internal.h"
#include "gtucker.h"

namespace gt {
gt_status launch_fit(const LaunchCtx& L, const SplitCtx* split, const float2* X, float2* A,
                     float2* B, float2* C, float2* G, double* trace, int32_t* status, int iters,
                     bool warm);
bool fused_lowp_ok(const LaunchCtx& L);
bool fused_fit_ok(const LaunchCtx& L);
gt_status launch_reconstruct(const LaunchCtx& L, int64_t total_sc, const float2* A, const float2* B,
                             const float2* C, const float2* G, float2* Ht, float2* Xhat);
gt_status launch_reconstruct_bwd(const LaunchCtx& L, int64_t total_sc, const float2* A,
                                 const float2* B, const float2* C, const float2* G,
                                 const float2* gHt, const float2* gX, float2* gA, float2* gB,
                                 float2* gC, float2* gG);
gt_status launch_sinr(const LaunchCtx& L, int64_t total_sc, bool full, const float2* X,
                      const float2* C, const float2* G, const float* s2, int n_snr, float* out,
                      int ns_max, int32_t* status);
gt_status launch_sinr_bwd(const LaunchCtx& L, int64_t total_sc, const float2* C, const float2* G,
                          const float* s2, int n_snr, const float* gsinr, float2* gC, float2* gG,
                          int ns_max, int32_t* status);
gt_status launch_sinr_system(const LaunchCtx& L, int64_t total_sc, const int32_t* terms_off,
                             const int32_t* terms, const float2* C, const float2* G,
                             const float* s2, int n_snr, float* out, int ns_max, int32_t* status);
gt_status launch_combine_core(const LaunchCtx& L, int n_pts, const float2* C, const float2* G,
                              const float2* U, float2* Ht);
gt_status launch_combine_full(const LaunchCtx& L, int n_pts, const float2* X, const float2* U,
                              float2* H);
gt_status launch_sinr_c128(const LaunchCtx& L, int64_t total_sc, bool full, const double2* X,
                           const double2* C, const double2* G, const float* s2, int n_snr,
                           double* out, int ns_max, int32_t* status);
gt_status launch_sinr_bwd_c128(const LaunchCtx& L, int64_t total_sc, const double2* C,
                               const double2* G, const float* s2, int n_snr, const double* gsinr,
                               double2* gC, double2* gG, int ns_max, int32_t* status);

// ---------------------------------------------------------------------------------------
// error detail and kernel timing

static thread_local std::string g_detail;

void set_error_detail(const char* where, hipError_t e) {
  g_detail = std::string(where) + ": " + hipGetErrorString(e);
}

struct ProfRec {
  std::string name;
  hipEvent_t start, stop;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;
static thread_local int g_prof_open = -1;

void prof_begin(const char* name, hipStream_t s) {
  if (!g_prof_on) return;
  ProfRec r;
  r.name = name;
  if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) return;
  hipEventRecord(r.start, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back(r);
  g_prof_open = (int)g_prof.size() - 1;
}

void prof_end(hipStream_t s) {
  if (!g_prof_on || g_prof_open < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEventRecord(g_prof[g_prof_open].stop, s);
  g_prof_open = -1;
}

static void prof_clear_locked() {
  for (auto& r : g_prof) {
    hipEventDestroy(r.start);
    hipEventDestroy(r.stop);
  }
  g_prof.clear();
}

}  // namespace gt

using namespace gt;

struct gt_plan {
  std::vector<gt_channel_desc> desc;
  std::vector<DevChan> chans;
  std::vector<GroupItem> groups;
  gt_fit_options opt;
  WsLayout lay;
  std::vector<char> blob;  // device tables, copied into the workspace by gt_workspace_init
  gt_offsets totals;
  int ns_max;
  int max_nr, max_nt, max_nsc, max_gs, max_m, max_n, max_p, max_ns, max_groups, max_nsplit;
  int full_mode1 = 1;  // every channel keeps its full mode-1 rank (m == nr)
  int min_nt;
  std::vector<GroupItem> groups_by_size;
  int n_small_groups;
  std::vector<int32_t> tiles;  // [TK_COUNT][n_channels + 1]
  // SINR classes: channels in class order, their subcarrier prefix sums, and per class its
  // first position, first subcarrier and largest n
  std::vector<int32_t> sc_ch;
  std::vector<int64_t> sc_off;
  int sc_j[SC_COUNT + 1] = {};
  int64_t sc_base[SC_COUNT + 1] = {};
  int sc_maxn[SC_COUNT] = {};
  // The fit of a batch of 8 or more channels on the fused per-group passes runs most of each
  // sweep as parts of consecutive channels on concurrent streams.  A part is a view: its own
  // tables (channels, groups, grids) in a workspace region after this plan's, over the same
  // per-channel workspace; side streams and events are made on the first fit.
  std::vector<gt_plan*> parts;
  std::vector<int32_t> part_c0;
  std::vector<int64_t> part_ws;
  int64_t ws_total = 0;
  std::mutex side_mu;
  bool side_tried = false, side_ok = false;
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_stag[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_init[4] = {nullptr, nullptr, nullptr, nullptr};
  // pass variants chosen by gt_plan_autotune
  int tune_bstep = 0, tune_tpass = 0, tune_split = 2;
  // compact layout of the SINR adjoint's scratch alone (tables and dl/dHt), for the entry point
  // that runs in the library's static scratch array; sblob holds its table bytes
  WsLayout slay{};
  std::vector<char> sblob;
  // factor sharing: groups of channels with the same nonzero a_id (0) or b_id (1)
  std::vector<int32_t> share_off[2], share_ch[2];
  bool sharing = false;
  // multi-cell system: serving flags and, per interference mode, each serving channel's
  // transmissions (channel Ht_{u,k}, serving channel of the precoder's UE)
  bool system = false;
  bool sys_uniform = false;
  std::vector<int32_t> sys_serving;
  std::vector<int32_t> sys_terms_off[3], sys_terms[3];
  ~gt_plan();
};

gt_plan::~gt_plan() {
  for (gt_plan* c : parts) delete c;
  for (hipStream_t& st : side)
    if (st) (void)hipStreamDestroy(st);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  for (hipEvent_t& e : ev_stag)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t& e : ev_init)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t& e : ev_join)
    if (e) (void)hipEventDestroy(e);
}

static int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

// SINR kernel class of a channel (compressed shape m x n, ns streams; ns <= m).
static int sc_class(const DevChan& ch) {
  if (ch.m <= 4) return ch.ns <= 2 ? SC_LANE4_2 : SC_LANE4_4;
  if (ch.m <= 8) return ch.ns <= 4 ? SC_LANE8_4 : SC_LANE8_8;
  return ch.n <= 32 ? SC_COOP_32 : SC_COOP_64;
}

extern "C" {

const char* gt_status_string(gt_status s) {
  switch (s) {
    case GT_OK: return "ok";
    case GT_ERR_ARG: return "invalid argument";
    case GT_ERR_SHAPE: return "unsupported or invalid shape";
    case GT_ERR_RANK: return "rank or stream count out of range";
    case GT_ERR_WORKSPACE: return "workspace missing or too small";
    case GT_ERR_UNSUPPORTED: return "operation not supported";
    case GT_ERR_HIP: return "HIP runtime error";
    case GT_ERR_NO_DEVICE: return "no GPU device";
  }
  return "unknown status";
}

const char* gt_last_error_detail(void) { return g_detail.c_str(); }

static gt_status validate(const gt_channel_desc& d) {
  if (d.nr < 1 || d.nt < 1 || d.nsc < 1 || d.group_size < 1) return GT_ERR_SHAPE;
  if (d.nr > kMaxNr || d.nt > 256 || d.group_size > kMaxGroup) return GT_ERR_SHAPE;
  if (d.m < 1 || d.m > d.nr || d.n < 1 || d.n > d.nt || d.n > 64) return GT_ERR_RANK;
  if (d.p < 1 || d.p > d.group_size) return GT_ERR_RANK;
  if (d.ns < 1 || d.ns > std::min(d.m, d.n)) return GT_ERR_RANK;
  if (d.a_id < 0 || d.b_id < 0 || d.serving < 0 || d.serving > 1) return GT_ERR_ARG;
  return GT_OK;
}

static LaunchCtx make_ctx(const gt_plan* p, void* ws, void* stream);
static gt_status plan_build(const gt_channel_desc* descs, int32_t n_channels,
                            const gt_fit_options* opt, bool allow_split, gt_plan** out);

gt_status gt_plan_create(const gt_channel_desc* descs, int32_t n_channels, const gt_fit_options* opt,
                         gt_plan** out) {
  return plan_build(descs, n_channels, opt, true, out);
}

static gt_status plan_build(const gt_channel_desc* descs, int32_t n_channels,
                            const gt_fit_options* opt, bool allow_split, gt_plan** out) {
  if (!descs || !out || n_channels < 1) return GT_ERR_ARG;
  *out = nullptr;
  gt_fit_options o{};
  if (opt) o = *opt;
  if (o.iters < 0 || o.eig_fp64 < 0 || o.eig_fp64 > 1) return GT_ERR_ARG;
  if (o.ttm_prec < GT_TTM_FP32 || o.ttm_prec > GT_TTM_SPLIT_BF16) return GT_ERR_ARG;
  if (o.flags & ~GT_FIT_WARM_START) return GT_ERR_ARG;
  if (o.dtype != GT_C64 && o.dtype != GT_C128) return GT_ERR_ARG;
  // c128 plans evaluate the SINR chain and its adjoint in FP64; the contraction precision
  // option belongs to the fit, which they do not run
  if (o.dtype == GT_C128 && o.ttm_prec != GT_TTM_FP32) return GT_ERR_UNSUPPORTED;
  for (int c = 0; c < n_channels; ++c) {
    gt_status st = validate(descs[c]);
    if (st != GT_OK) return st;
  }
  gt_plan* p = new (std::nothrow) gt_plan();
  if (!p) return GT_ERR_ARG;
  p->desc.assign(descs, descs + n_channels);
  p->opt = o;
  p->chans.resize(n_channels);
  int64_t ox = 0, oa = 0, ob = 0, oc = 0, og = 0, oht = 0, osc = 0, omn = 0, ort = 0;
  int gfirst = 0;
  p->max_nr = p->max_nt = p->max_nsc = p->max_gs = p->max_m = p->max_n = p->max_p = p->max_ns = 0;
  p->max_groups = p->max_nsplit = 0;
  p->min_nt = descs[0].nt;
  for (int c = 0; c < n_channels; ++c) {
    const gt_channel_desc& d = descs[c];
    DevChan& ch = p->chans[c];
    std::memset(&ch, 0, sizeof(ch));
    ch.nr = d.nr;
    ch.nt = d.nt;
    ch.nsc = d.nsc;
    ch.gs = d.group_size;
    ch.m = d.m;
    ch.n = d.n;
    ch.p = d.p;
    ch.ns = d.ns;
    ch.ngroups = (d.nsc + d.group_size - 1) / d.group_size;
    ch.nsplit = std::min(ch.ngroups, 16);
    ch.gfirst = gfirst;
    ch.x = ox;
    ch.a = oa;
    ch.b = ob;
    ch.c = oc;
    ch.g = og;
    ch.ht = oht;
    ch.sc = osc;
    ch.mn_off = omn;
    ch.rt_off = ort;
    omn += (int64_t)d.m * d.n;
    ort += (int64_t)d.nr * d.nt;
    ox += (int64_t)d.nsc * d.nr * d.nt;
    oa += (int64_t)d.nr * d.m;
    ob += (int64_t)d.nt * d.n;
    oc += (int64_t)d.nsc * d.p;
    og += (int64_t)ch.ngroups * d.p * d.m * d.n;
    oht += (int64_t)d.nsc * d.m * d.n;
    osc += d.nsc;
    for (int g = 0; g < ch.ngroups; ++g) p->groups.push_back(GroupItem{c, g});
    gfirst += ch.ngroups;
    p->max_nr = std::max(p->max_nr, d.nr);
    p->max_nt = std::max(p->max_nt, d.nt);
    p->min_nt = std::min(p->min_nt, d.nt);
    p->max_nsc = std::max(p->max_nsc, d.nsc);
    p->max_gs = std::max(p->max_gs, d.group_size);
    p->max_m = std::max(p->max_m, d.m);
    if (d.m != d.nr) p->full_mode1 = 0;
    p->max_n = std::max(p->max_n, d.n);
    p->max_p = std::max(p->max_p, d.p);
    p->max_ns = std::max(p->max_ns, d.ns);
    p->max_groups = std::max(p->max_groups, ch.ngroups);
    p->max_nsplit = std::max(p->max_nsplit, ch.nsplit);
  }
  p->totals = gt_offsets{ox, oa, ob, oc, og, oht, osc, gfirst, 0};
  {  // factor sharing: members of each label in channel order; groups of two or more
    for (int f = 0; f < 2; ++f) {
      std::vector<std::pair<int32_t, int32_t>> lab;
      for (int c = 0; c < n_channels; ++c) {
        const int32_t id = f == 0 ? descs[c].a_id : descs[c].b_id;
        if (id > 0) lab.push_back({id, c});
      }
      std::sort(lab.begin(), lab.end());
      p->share_off[f].assign(1, 0);
      p->share_ch[f].clear();
      for (size_t a = 0; a < lab.size();) {
        size_t b = a;
        while (b < lab.size() && lab[b].first == lab[a].first) ++b;
        if (b - a >= 2) {
          const gt_channel_desc& d0 = descs[lab[a].second];
          for (size_t k = a; k < b; ++k) {
            const gt_channel_desc& d = descs[lab[k].second];
            const bool same = f == 0 ? (d.nr == d0.nr && d.m == d0.m) : (d.nt == d0.nt && d.n == d0.n);
            if (!same) {
              delete p;
              return GT_ERR_SHAPE;
            }
            p->share_ch[f].push_back(lab[k].second);
          }
          p->share_off[f].push_back((int32_t)p->share_ch[f].size());
          p->sharing = true;
        }
        a = b;
      }
    }
    // a complete system: every channel labelled, one serving link per UE, at most one channel
    // per (UE, BS); the transmissions each UE sees under the three interference modes
    bool sys = true;
    std::vector<int> ue_serv;   // serving channel per UE label (index label - 1)
    int max_ue = 0, max_bs = 0;
    for (int c = 0; c < n_channels; ++c) {
      if (descs[c].a_id < 1 || descs[c].b_id < 1) sys = false;
      max_ue = std::max(max_ue, descs[c].a_id);
      max_bs = std::max(max_bs, descs[c].b_id);
    }
    std::vector<int> link;  // channel of (UE, BS), -1 if absent
    if (sys) {
      ue_serv.assign(max_ue, -1);
      link.assign((size_t)max_ue * max_bs, -1);
      for (int c = 0; c < n_channels; ++c) {
        const int u = descs[c].a_id - 1, k = descs[c].b_id - 1;
        if (link[(size_t)u * max_bs + k] >= 0) sys = false;
        link[(size_t)u * max_bs + k] = c;
        if (descs[c].serving) {
          if (ue_serv[u] >= 0) sys = false;
          ue_serv[u] = c;
        }
      }
      for (int u = 0; u < max_ue && sys; ++u)
        if (ue_serv[u] < 0 && std::any_of(link.begin() + (size_t)u * max_bs,
                                          link.begin() + (size_t)(u + 1) * max_bs,
                                          [](int v) { return v >= 0; }))
          sys = false;
    }
    p->system = sys;
    p->sys_serving.assign(n_channels, 0);
    for (int f = 0; f < 3; ++f) {
      p->sys_terms_off[f].assign(n_channels + 1, 0);
      p->sys_terms[f].clear();
    }
    if (sys) {
      bool uniform = true;
      for (int c = 0; c < n_channels; ++c) {
        p->sys_serving[c] = descs[c].serving;
        uniform = uniform && descs[c].nsc == descs[0].nsc && descs[c].ns == descs[0].ns &&
                  descs[c].m <= 8 && descs[c].ns <= 4;
      }
      // first UE of each cell: the lowest UE label among the serving links of that BS
      std::vector<int> first(max_bs, -1);
      for (int u = 0; u < max_ue; ++u)
        if (ue_serv[u] >= 0) {
          const int k = descs[ue_serv[u]].b_id - 1;
          if (first[k] < 0) first[k] = u;
        }
      for (int f = 0; f < 3; ++f) {
        for (int c = 0; c < n_channels; ++c) {
          if (descs[c].serving) {
            const int u = descs[c].a_id - 1, i = descs[c].b_id - 1;
            p->sys_terms[f].push_back(c);
            p->sys_terms[f].push_back(c);
            for (int v = 0; v < max_ue; ++v) {
              if (v == u || ue_serv[v] < 0) continue;
              const int k = descs[ue_serv[v]].b_id - 1;
              const bool seen = f == 2 || (f == 1 && k != i && first[k] == v);
              if (!seen) continue;
              const int ct = link[(size_t)u * max_bs + k];
              if (ct < 0) {
                uniform = false;  // the UE has no channel from that BS: this mode is not available
                continue;
              }
              p->sys_terms[f].push_back(ct);
              p->sys_terms[f].push_back(ue_serv[v]);
            }
          }
          p->sys_terms_off[f][c + 1] = (int32_t)(p->sys_terms[f].size() / 2);
        }
      }
      p->sys_uniform = uniform;
    }
  }
  p->ns_max = p->max_ns;
  // workspace: tables then per-channel scratch
  int64_t off = 0;
  p->lay.chans = off;
  off = align256(off + (int64_t)sizeof(DevChan) * n_channels);
  p->lay.groups = off;
  off = align256(off + (int64_t)sizeof(GroupItem) * gfirst);
  // groups ordered by size class (the mode-3 eigensolve takes 16- and 32-lane groups)
  p->groups_by_size.clear();
  for (const GroupItem& it : p->groups)
    if (p->chans[it.ch].gs <= 16) p->groups_by_size.push_back(it);
  p->n_small_groups = (int)p->groups_by_size.size();
  for (const GroupItem& it : p->groups)
    if (p->chans[it.ch].gs > 16) p->groups_by_size.push_back(it);
  p->lay.groups_by_size = off;
  off = align256(off + (int64_t)sizeof(GroupItem) * gfirst);
  // block prefix sums of the compact grids
  p->tiles.assign((size_t)TK_COUNT * (n_channels + 1), 0);
  for (int c = 0; c < n_channels; ++c) {
    const DevChan& ch = p->chans[c];
    const int64_t rtiles = ((int64_t)ch.nsc * ch.nr + 31) / 32;
    const int64_t S = (2 * (int64_t)ch.nt + 127) / 128;
    const int64_t cnt[TK_COUNT] = {
        (int64_t)ch.ngroups * ((ch.nt + 31) / 32),
        ((rtiles + kTRowTiles - 1) / kTRowTiles) * ((2 * ch.n + 31) / 32),
        S * (S + 1) / 2 * ch.nsplit,
        ((int64_t)ch.nt * ch.nt + 255) / 256,
        ((int64_t)ch.nsc * ch.n + 255) / 256};
    for (int k = 0; k < TK_COUNT; ++k) {
      const int64_t v = p->tiles[(size_t)k * (n_channels + 1) + c] + cnt[k];
      if (v > INT32_MAX) {
        delete p;
        return GT_ERR_SHAPE;
      }
      p->tiles[(size_t)k * (n_channels + 1) + c + 1] = (int32_t)v;
    }
  }
  p->lay.tiles = off;
  off = align256(off + (int64_t)sizeof(int32_t) * p->tiles.size());
  // channels ordered by SINR class (stable), subcarriers numbered through that order
  p->sc_ch.clear();
  p->sc_off.assign(1, 0);
  for (int k = 0; k < SC_COUNT; ++k) {
    p->sc_j[k] = (int)p->sc_ch.size();
    p->sc_base[k] = p->sc_off.back();
    p->sc_maxn[k] = 0;
    for (int c = 0; c < n_channels; ++c)
      if (sc_class(p->chans[c]) == k) {
        p->sc_ch.push_back(c);
        p->sc_off.push_back(p->sc_off.back() + p->chans[c].nsc);
        p->sc_maxn[k] = std::max(p->sc_maxn[k], p->chans[c].n);
      }
  }
  p->sc_j[SC_COUNT] = n_channels;
  p->sc_base[SC_COUNT] = p->sc_off.back();
  p->lay.sc_ch = off;
  off = align256(off + (int64_t)sizeof(int32_t) * n_channels);
  p->lay.sc_off = off;
  off = align256(off + (int64_t)sizeof(int64_t) * (n_channels + 1));
  for (int f = 0; f < 2; ++f) {
    p->lay.share_off[f] = off;
    off = align256(off + (int64_t)sizeof(int32_t) * p->share_off[f].size());
    p->lay.share_ch[f] = off;
    off = align256(off + (int64_t)sizeof(int32_t) * std::max<size_t>(p->share_ch[f].size(), 1));
  }
  p->lay.sys_serving = off;
  off = align256(off + (int64_t)sizeof(int32_t) * n_channels);
  for (int f = 0; f < 3; ++f) {
    p->lay.sys_terms_off[f] = off;
    off = align256(off + (int64_t)sizeof(int32_t) * (n_channels + 1));
    p->lay.sys_terms[f] = off;
    off = align256(off + (int64_t)sizeof(int32_t) * std::max<size_t>(p->sys_terms[f].size(), 1));
  }
  const int64_t tables_end = off;
  const int64_t c8 = 8;
  for (int c = 0; c < n_channels; ++c) {
    DevChan& ch = p->chans[c];
    auto take = [&](int64_t bytes) {
      int64_t at = off;
      off = align256(off + std::max<int64_t>(bytes, 8));
      return at;
    };
    ch.w_W = take(c8 * ch.ngroups * ch.p * ch.m * ch.nt);
    ch.w_T = take(c8 * ch.nsc * ch.nr * ch.n);
    ch.w_Yh = take(c8 * ch.nsc * ch.m * ch.n);
    ch.w_S1p = take(c8 * ch.ngroups * ch.nr * ch.nr);
    ch.w_S1 = take(c8 * ch.nr * ch.nr);
    {  // split partials: complex nt x nt (VALU Gram) or the real Gram in 128-wide super-tiles
      const int64_t wr = 128 * ((2 * (int64_t)std::max(ch.nt, 64) + 127) / 128);
      ch.w_S2p = take(std::max<int64_t>(c8 * ch.nsplit * ch.nt * ch.nt, 4LL * ch.nsplit * wr * wr));
    }
    ch.w_S2 = take(c8 * ch.nt * ch.nt);
    ch.w_S3 = take(c8 * ch.ngroups * ch.gs * ch.gs);
    ch.w_VA = take(c8 * 16 * 16);
    {  // eigenbasis buffers: complex FP32, or FP64 for the subspace iteration's FP64 form
      const int64_t cv = (ch.nt > 64 && o.eig_fp64) ? 16 : 8;
      ch.w_VB = take(cv * 64 * std::max(64, ch.nt));
      ch.w_VS = take(ch.nt > 64 ? cv * 2 * 64 * ch.nt : 8);
      // slice partials of two 64 x 64 complex blocks (4 slices), Q, Ritz values, residual
      // partials and two flags
      ch.w_SP = take(ch.nt > 64 ? (cv / 2) * (4 * 2 * 64 * 64 * 2 + 64 * 64 * 2 + 64 + 4 * 64 + 2) : 8);
    }
    ch.w_Xq = take(o.ttm_prec == GT_TTM_FP32 ? 8
                   : (o.ttm_prec == GT_TTM_SPLIT_BF16 ? 8 : 4) * (int64_t)ch.nsc * ch.nr * ch.nt);
    ch.w_VC = take(c8 * ch.ngroups * 32 * 32);
    ch.w_lamg = take(8 * (int64_t)ch.ngroups);
    ch.w_scal = take(8 * 8);
    ch.w_gH = take((o.dtype == GT_C128 ? 2 : 1) * c8 * ch.nsc * ch.m * ch.n);
    ch.w_gAp = take(c8 * ch.ngroups * ch.nr * ch.m);
    ch.w_gBp = take(c8 * ch.ngroups * ch.nt * ch.n);
  }
  p->lay.total = off;
  {  // the SINR adjoint's scratch alone: tables, then dl/dHt per channel
    int64_t so = 0;
    p->slay.chans = so;
    so = align256(so + (int64_t)sizeof(DevChan) * n_channels);
    p->slay.groups = so;
    so = align256(so + (int64_t)sizeof(GroupItem) * gfirst);
    p->slay.sc_ch = so;
    so = align256(so + (int64_t)sizeof(int32_t) * n_channels);
    p->slay.sc_off = so;
    so = align256(so + (int64_t)sizeof(int64_t) * (n_channels + 1));
    const int64_t tables = so;
    std::vector<DevChan> sc(p->chans);
    const int64_t ce = o.dtype == GT_C128 ? 16 : 8;
    for (int c = 0; c < n_channels; ++c) {
      DevChan& ch = sc[c];
      ch.w_W = ch.w_T = ch.w_Yh = ch.w_S1p = ch.w_S1 = ch.w_S2p = ch.w_S2 = ch.w_S3 = 0;
      ch.w_VA = ch.w_VB = ch.w_VS = ch.w_SP = ch.w_Xq = ch.w_VC = ch.w_lamg = ch.w_scal = 0;
      ch.w_gAp = ch.w_gBp = 0;
      ch.w_gH = so;
      so = align256(so + std::max<int64_t>(ce * ch.nsc * ch.m * ch.n, 8));
    }
    p->slay.groups_by_size = p->slay.groups;
    p->slay.tiles = 0;
    p->slay.total = so;
    p->sblob.assign((size_t)tables, 0);
    std::memcpy(p->sblob.data() + p->slay.chans, sc.data(), sizeof(DevChan) * n_channels);
    std::memcpy(p->sblob.data() + p->slay.groups, p->groups.data(), sizeof(GroupItem) * gfirst);
    std::memcpy(p->sblob.data() + p->slay.sc_ch, p->sc_ch.data(), sizeof(int32_t) * n_channels);
    std::memcpy(p->sblob.data() + p->slay.sc_off, p->sc_off.data(),
                sizeof(int64_t) * (n_channels + 1));
  }
  p->blob.assign((size_t)tables_end, 0);
  std::memcpy(p->blob.data() + p->lay.chans, p->chans.data(), sizeof(DevChan) * n_channels);
  std::memcpy(p->blob.data() + p->lay.groups, p->groups.data(), sizeof(GroupItem) * gfirst);
  std::memcpy(p->blob.data() + p->lay.groups_by_size, p->groups_by_size.data(),
              sizeof(GroupItem) * gfirst);
  std::memcpy(p->blob.data() + p->lay.tiles, p->tiles.data(), sizeof(int32_t) * p->tiles.size());
  std::memcpy(p->blob.data() + p->lay.sc_ch, p->sc_ch.data(), sizeof(int32_t) * n_channels);
  for (int f = 0; f < 2; ++f) {
    std::memcpy(p->blob.data() + p->lay.share_off[f], p->share_off[f].data(),
                sizeof(int32_t) * p->share_off[f].size());
    if (!p->share_ch[f].empty())
      std::memcpy(p->blob.data() + p->lay.share_ch[f], p->share_ch[f].data(),
                  sizeof(int32_t) * p->share_ch[f].size());
  }
  std::memcpy(p->blob.data() + p->lay.sys_serving, p->sys_serving.data(), sizeof(int32_t) * n_channels);
  for (int f = 0; f < 3; ++f) {
    std::memcpy(p->blob.data() + p->lay.sys_terms_off[f], p->sys_terms_off[f].data(),
                sizeof(int32_t) * (n_channels + 1));
    if (!p->sys_terms[f].empty())
      std::memcpy(p->blob.data() + p->lay.sys_terms[f], p->sys_terms[f].data(),
                  sizeof(int32_t) * p->sys_terms[f].size());
  }
  std::memcpy(p->blob.data() + p->lay.sc_off, p->sc_off.data(), sizeof(int64_t) * (n_channels + 1));
  p->ws_total = p->lay.total;
  // batch split of the fit (fused passes, 8 or more channels): views over parts
  if (allow_split && !p->sharing && n_channels >= 8 && fused_fit_ok(make_ctx(p, nullptr, nullptr))) {
    const int k = n_channels >= 16 ? 4 : 2;
    int64_t woff = align256(p->lay.total);
    for (int i = 0; i < k; ++i) {
      const int c0 = (int)((int64_t)i * n_channels / k), c1 = (int)((int64_t)(i + 1) * n_channels / k);
      const int nc = c1 - c0;
      gt_plan* v = new (std::nothrow) gt_plan();
      if (!v) {
        delete p;
        return GT_ERR_ARG;
      }
      v->desc.assign(descs + c0, descs + c1);
      v->opt = o;
      v->chans.assign(p->chans.begin() + c0, p->chans.begin() + c1);
      for (const GroupItem& it : p->groups)
        if (it.ch >= c0 && it.ch < c1) v->groups.push_back(GroupItem{it.ch - c0, it.g});
      for (const GroupItem& it : v->groups)
        if (v->chans[it.ch].gs <= 16) v->groups_by_size.push_back(it);
      v->n_small_groups = (int)v->groups_by_size.size();
      for (const GroupItem& it : v->groups)
        if (v->chans[it.ch].gs > 16) v->groups_by_size.push_back(it);
      v->tiles.assign((size_t)TK_COUNT * (nc + 1), 0);
      for (int t = 0; t < TK_COUNT; ++t)
        for (int c = 0; c <= nc; ++c)
          v->tiles[(size_t)t * (nc + 1) + c] = p->tiles[(size_t)t * (n_channels + 1) + c0 + c] -
                                               p->tiles[(size_t)t * (n_channels + 1) + c0];
      v->max_nr = p->max_nr;
      v->max_nt = p->max_nt;
      v->min_nt = p->min_nt;
      v->max_nsc = p->max_nsc;
      v->max_gs = p->max_gs;
      v->max_m = p->max_m;
      v->full_mode1 = p->full_mode1;
      v->max_n = p->max_n;
      v->max_p = p->max_p;
      v->max_ns = p->max_ns;
      v->max_groups = p->max_groups;
      v->max_nsplit = p->max_nsplit;
      v->ns_max = p->ns_max;
      v->totals = p->totals;
      // tables at absolute workspace offsets, one contiguous blob from lay.chans
      const int64_t ng = (int64_t)v->groups.size();
      v->lay.chans = woff;
      v->lay.groups = align256(v->lay.chans + (int64_t)sizeof(DevChan) * nc);
      v->lay.groups_by_size = align256(v->lay.groups + (int64_t)sizeof(GroupItem) * ng);
      v->lay.tiles = align256(v->lay.groups_by_size + (int64_t)sizeof(GroupItem) * ng);
      v->lay.total = v->lay.tiles + (int64_t)sizeof(int32_t) * v->tiles.size();
      v->blob.assign((size_t)(v->lay.total - woff), 0);
      std::memcpy(v->blob.data(), v->chans.data(), sizeof(DevChan) * nc);
      std::memcpy(v->blob.data() + (v->lay.groups - woff), v->groups.data(), sizeof(GroupItem) * ng);
      std::memcpy(v->blob.data() + (v->lay.groups_by_size - woff), v->groups_by_size.data(),
                  sizeof(GroupItem) * ng);
      std::memcpy(v->blob.data() + (v->lay.tiles - woff), v->tiles.data(),
                  sizeof(int32_t) * v->tiles.size());
      p->parts.push_back(v);
      p->part_c0.push_back(c0);
      p->part_ws.push_back(woff);
      woff = align256(v->lay.total);
    }
    p->ws_total = woff;
  }
  *out = p;
  return GT_OK;
}

void gt_plan_destroy(gt_plan* plan) { delete plan; }

gt_status gt_plan_offsets(const gt_plan* plan, int32_t channel, gt_offsets* out) {
  if (!plan || !out) return GT_ERR_ARG;
  if (channel < 0 || channel >= (int32_t)plan->chans.size()) return GT_ERR_ARG;
  const DevChan& ch = plan->chans[channel];
  *out = gt_offsets{ch.x, ch.a, ch.b, ch.c, ch.g, ch.ht, ch.sc, ch.ngroups, 0};
  return GT_OK;
}

gt_status gt_plan_totals(const gt_plan* plan, gt_offsets* totals, int32_t* ns_max) {
  if (!plan) return GT_ERR_ARG;
  if (totals) *totals = plan->totals;
  if (ns_max) *ns_max = plan->ns_max;
  return GT_OK;
}

gt_status gt_plan_workspace_bytes(const gt_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return GT_ERR_ARG;
  *bytes = (size_t)plan->ws_total;
  return GT_OK;
}

static gt_status check_ws(const gt_plan* plan, void* ws, size_t ws_bytes) {
  if (!plan) return GT_ERR_ARG;
  if (!ws || ws_bytes < (size_t)plan->ws_total) return GT_ERR_WORKSPACE;
  return GT_OK;
}

// Launch context over the tables of layout `lay` at device address `ws`.
static LaunchCtx make_ctx_at(const gt_plan* p, const WsLayout& lay, void* ws, void* stream) {
  LaunchCtx L;
  L.stream = reinterpret_cast<hipStream_t>(stream);
  L.ws = reinterpret_cast<char*>(ws);
  L.d_chans = reinterpret_cast<const DevChan*>(L.ws + lay.chans);
  L.d_groups = reinterpret_cast<const GroupItem*>(L.ws + lay.groups);
  L.d_groups_by_size = reinterpret_cast<const GroupItem*>(L.ws + lay.groups_by_size);
  L.d_tiles = reinterpret_cast<const int32_t*>(L.ws + lay.tiles);
  if (!p->sc_ch.empty()) {  // split views run no SINR and carry no class tables
    L.d_sc_ch = reinterpret_cast<const int32_t*>(L.ws + lay.sc_ch);
    L.d_sc_off = reinterpret_cast<const int64_t*>(L.ws + lay.sc_off);
  }
  for (int k = 0; k <= SC_COUNT; ++k) {
    L.sc_j[k] = p->sc_j[k];
    L.sc_base[k] = p->sc_base[k];
  }
  for (int k = 0; k < SC_COUNT; ++k) L.sc_maxn[k] = p->sc_maxn[k];
  L.n_channels = (int)p->chans.size();
  for (int k = 0; k < TK_COUNT; ++k)
    L.tiles_total[k] = p->tiles[(size_t)k * (L.n_channels + 1) + L.n_channels];
  L.total_groups = (int)p->groups.size();
  L.n_small_groups = p->n_small_groups;
  L.max_nr = p->max_nr;
  L.max_nt = p->max_nt;
  L.max_nsc = p->max_nsc;
  L.max_gs = p->max_gs;
  L.max_m = p->max_m;
  L.full_mode1 = p->full_mode1;
  L.max_n = p->max_n;
  L.max_p = p->max_p;
  L.max_ns = p->max_ns;
  L.max_groups = p->max_groups;
  L.max_nsplit = p->max_nsplit;
  L.min_nt = p->min_nt;
  L.ttm_prec = p->opt.ttm_prec;
  L.eig_fp64 = p->opt.eig_fp64;
  L.tune_bstep = p->tune_bstep;
  L.tune_tpass = p->tune_tpass;
  if (&lay == &p->lay && p->sharing) {
    for (int f = 0; f < 2; ++f) {
      L.n_share[f] = (int)p->share_off[f].size() - 1;
      L.d_share_off[f] = reinterpret_cast<const int32_t*>(L.ws + lay.share_off[f]);
      L.d_share_ch[f] = reinterpret_cast<const int32_t*>(L.ws + lay.share_ch[f]);
    }
  }
  if (&lay == &p->lay) L.d_sys_serving = reinterpret_cast<const int32_t*>(L.ws + lay.sys_serving);
  return L;
}

static LaunchCtx make_ctx(const gt_plan* p, void* ws, void* stream) {
  return make_ctx_at(p, p->lay, ws, stream);
}

gt_status gt_workspace_init(const gt_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  hipError_t e = hipMemcpyAsync(ws, plan->blob.data(), plan->blob.size(), hipMemcpyHostToDevice,
                                reinterpret_cast<hipStream_t>(stream));
  for (size_t i = 0; e == hipSuccess && i < plan->parts.size(); ++i)
    e = hipMemcpyAsync(reinterpret_cast<char*>(ws) + plan->part_ws[i], plan->parts[i]->blob.data(),
                       plan->parts[i]->blob.size(), hipMemcpyHostToDevice,
                       reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    set_error_detail("gt_workspace_init", e);
    return GT_ERR_HIP;
  }
  return GT_OK;
}

// Side streams (default priority) and events of a split plan, made once on the current device.
static bool side_ready(gt_plan* p) {
  std::lock_guard<std::mutex> lk(p->side_mu);
  if (p->side_tried) return p->side_ok;
  p->side_tried = true;
  const size_t ns = p->parts.size() - 1;
  bool ok = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) == hipSuccess;
  for (hipEvent_t& e : p->ev_init)
    ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  for (size_t i = 0; ok && i < ns; ++i)
    ok = hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&p->ev_join[i], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&p->ev_stag[i], hipEventDisableTiming) == hipSuccess;
  p->side_ok = ok;
  return ok;
}

// One fit of the plan's batch on `stream` with `iters` sweeps (split over the side streams when
// the plan has parts and the split is on).
static gt_status run_fit(const gt_plan* plan, const void* X, void* A, void* B, void* C, void* G,
                         double* obj_trace, int32_t* dev_status, void* ws, void* stream, int iters) {
  LaunchCtx L = make_ctx(plan, ws, stream);
  const bool warm = (plan->opt.flags & GT_FIT_WARM_START) != 0;
  gt_plan* mp = const_cast<gt_plan*>(plan);
  if (plan->parts.empty() || !plan->tune_split || !side_ready(mp))
    return launch_fit(L, nullptr, (const float2*)X, (float2*)A, (float2*)B, (float2*)C,
                      (float2*)G, obj_trace, dev_status, iters, warm);
  // split batch: part 0 on the caller's stream, the others on side streams
  LaunchCtx P[4];
  SplitCtx S;
  S.n = (int)plan->parts.size();
  S.parts = P;
  S.fork = mp->ev_fork;
  S.mode = plan->tune_split;
  for (int i = 0; i < 4; ++i) S.init[i] = mp->ev_init[i];
  for (int k = 0; k < S.n; ++k) {
    P[k] = make_ctx(plan->parts[k], ws, k == 0 ? stream : (void*)mp->side[k - 1]);
    P[k].c0 = plan->part_c0[k];
    P[k].tune_bstep = plan->tune_bstep;
    P[k].tune_tpass = plan->tune_tpass;
    if (k > 0) {
      S.join[k - 1] = mp->ev_join[k - 1];
      S.stag[k - 1] = mp->ev_stag[k - 1];
    }
  }
  return launch_fit(L, &S, (const float2*)X, (float2*)A, (float2*)B, (float2*)C, (float2*)G,
                    obj_trace, dev_status, iters, warm);
}

gt_status gt_tucker_fit(const gt_plan* plan, const void* X, void* A, void* B, void* C, void* G,
                        double* obj_trace, int32_t* dev_status, void* ws, size_t ws_bytes,
                        void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if (!X || !A || !B || !C || !G) return GT_ERR_ARG;
  if (plan->opt.dtype != GT_C64) return GT_ERR_UNSUPPORTED;
  if (plan->sharing && obj_trace) return GT_ERR_UNSUPPORTED;
  // 16-bit contractions take K steps of 8 reals: every nt a multiple of 4
  if (plan->opt.ttm_prec != GT_TTM_FP32) {
    for (const auto& d : plan->desc)
      if (d.nt % 4 != 0) return GT_ERR_UNSUPPORTED;
  }
  return run_fit(plan, X, A, B, C, G, obj_trace, dev_status, ws, stream, plan->opt.iters);
}

gt_status gt_plan_set_tuning(gt_plan* plan, int32_t bstep, int32_t tpass, int32_t split) {
  if (!plan || bstep < 0 || bstep > 2 || tpass < 0 || tpass > 1 || split < 0 || split > 2)
    return GT_ERR_ARG;
  // the prefetching and the older B-step kernels and the vector-ALU T pass are FP32-only: on a
  // 16-bit plan they would run the contraction on the FP32 X
  if (plan->opt.ttm_prec != GT_TTM_FP32 && (bstep != 0 || tpass != 0)) return GT_ERR_UNSUPPORTED;
  plan->tune_bstep = bstep;
  plan->tune_tpass = tpass;
  plan->tune_split = split;
  return GT_OK;
}

gt_status gt_plan_autotune(gt_plan* plan, const void* X, void* A, void* B, void* C, void* G,
                           void* ws, size_t ws_bytes, void* stream, gt_tune_result* out) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if (!X || !A || !B || !C || !G) return GT_ERR_ARG;
  if (plan->opt.dtype != GT_C64) return GT_ERR_UNSUPPORTED;
  if (plan->opt.ttm_prec != GT_TTM_FP32) {
    for (const auto& d : plan->desc)
      if (d.nt % 4 != 0) return GT_ERR_UNSUPPORTED;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    set_error_detail("gt_plan_autotune", hipErrorOutOfMemory);
    return GT_ERR_HIP;
  }
  // probe fits of up to 8 sweeps, so that the sweep loop (where the choices differ) outweighs
  // the initialisation
  const int iters = std::min(plan->opt.iters, 8);
  // time of a configuration: the faster of two probe fits after one untimed run, or < 0 on error
  auto probe = [&]() -> float {
    if (run_fit(plan, X, A, B, C, G, nullptr, nullptr, ws, stream, iters) != GT_OK) return -1.f;
    float best_ms = -1.f;
    for (int rep = 0; rep < 2; ++rep) {
      if (hipEventRecord(e0, s) != hipSuccess) return -1.f;
      if (run_fit(plan, X, A, B, C, G, nullptr, nullptr, ws, stream, iters) != GT_OK) return -1.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.f;
      float ms = -1.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.f;
      if (best_ms < 0.f || ms < best_ms) best_ms = ms;
    }
    return best_ms;
  };
  const LaunchCtx L0 = make_ctx(plan, ws, stream);
  const bool fused = fused_fit_ok(L0) && (L0.ttm_prec == GT_TTM_FP32 || fused_lowp_ok(L0));
  float best = probe();
  gt_status rc = best < 0.f ? GT_ERR_HIP : GT_OK;
  // coordinate search: each choice in turn over its values, the others held
  struct Knob {
    int* field;
    int nvals;
  };
  std::vector<Knob> knobs;
  if (fused) {
    knobs.push_back({&plan->tune_bstep, L0.ttm_prec == GT_TTM_FP32 ? 3 : 1});
    knobs.push_back({&plan->tune_tpass, L0.ttm_prec == GT_TTM_FP32 ? 2 : 1});
    if (!plan->parts.empty()) knobs.push_back({&plan->tune_split, 3});
  }
  for (const Knob& k : knobs) {
    if (rc != GT_OK) break;
    const int keep = *k.field;
    int best_v = keep;
    for (int v = 0; v < k.nvals; ++v) {
      if (v == keep) continue;
      *k.field = v;
      const float ms = probe();
      if (ms < 0.f) {
        rc = GT_ERR_HIP;
        break;
      }
      // a choice replaces the current one only when it is faster by more than 2 %, so that
      // run-to-run noise does not move the plan off its defaults
      if (ms < 0.98f * best) {
        best = ms;
        best_v = v;
      }
    }
    *k.field = best_v;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (out) *out = gt_tune_result{plan->tune_bstep, plan->tune_tpass, plan->tune_split, best};
  return rc;
}

gt_status gt_tucker_reconstruct(const gt_plan* plan, const void* A, const void* B, const void* C,
                                const void* G, void* Ht, void* Xhat, void* ws, size_t ws_bytes,
                                void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if (!C || !G || (Xhat && (!A || !B))) return GT_ERR_ARG;
  if (plan->opt.dtype != GT_C64) return GT_ERR_UNSUPPORTED;
  if (!Ht && !Xhat) return GT_OK;
  LaunchCtx L = make_ctx(plan, ws, stream);
  return launch_reconstruct(L, plan->totals.sc, (const float2*)A, (const float2*)B,
                            (const float2*)C, (const float2*)G, (float2*)Ht, (float2*)Xhat);
}

static gt_status check_snr(const float* sigma2, int32_t n_snr) {
  if (!sigma2 || n_snr < 1 || n_snr > kMaxSnr) return GT_ERR_ARG;
  for (int k = 0; k < n_snr; ++k)
    if (!(sigma2[k] > 0.f) || sigma2[k] > 3e38f) return GT_ERR_ARG;
  return GT_OK;
}

gt_status gt_sinr_eval(const gt_plan* plan, const void* C, const void* G, const float* sigma2,
                       int32_t n_snr, void* sinr, int32_t* dev_status, void* ws, size_t ws_bytes,
                       void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if ((st = check_snr(sigma2, n_snr)) != GT_OK) return st;
  if (!C || !G || !sinr) return GT_ERR_ARG;
  LaunchCtx L = make_ctx(plan, ws, stream);
  if (plan->opt.dtype == GT_C128)
    return launch_sinr_c128(L, plan->totals.sc, false, nullptr, (const double2*)C, (const double2*)G,
                            sigma2, n_snr, (double*)sinr, plan->ns_max, dev_status);
  return launch_sinr(L, plan->totals.sc, false, nullptr, (const float2*)C, (const float2*)G, sigma2,
                     n_snr, (float*)sinr, plan->ns_max, dev_status);
}

gt_status gt_sinr_eval_system(const gt_plan* plan, const void* C, const void* G, const float* sigma2,
                              int32_t n_snr, int32_t mode, void* sinr, int32_t* dev_status, void* ws,
                              size_t ws_bytes, void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if ((st = check_snr(sigma2, n_snr)) != GT_OK) return st;
  if (!C || !G || !sinr) return GT_ERR_ARG;
  if (mode < GT_INTERF_NONE || mode > GT_INTERF_ALL || !plan->system) return GT_ERR_ARG;
  if (plan->opt.dtype != GT_C64 || !plan->sys_uniform) return GT_ERR_UNSUPPORTED;
  LaunchCtx L = make_ctx(plan, ws, stream);
  const int32_t* toff = reinterpret_cast<const int32_t*>(L.ws + plan->lay.sys_terms_off[mode]);
  const int32_t* terms = reinterpret_cast<const int32_t*>(L.ws + plan->lay.sys_terms[mode]);
  return launch_sinr_system(L, plan->totals.sc, toff, terms, (const float2*)C, (const float2*)G,
                            sigma2, n_snr, (float*)sinr, plan->ns_max, dev_status);
}

gt_status gt_combine_compressed(const gt_plan* plan, const void* C, const void* G, const void* U,
                                int32_t n_pts, void* Ht, void* ws, size_t ws_bytes, void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if (!C || !G || !U || !Ht || n_pts < 1 || n_pts > kMaxCombinePts) return GT_ERR_ARG;
  if (plan->opt.dtype != GT_C64) return GT_ERR_UNSUPPORTED;
  LaunchCtx L = make_ctx(plan, ws, stream);
  return launch_combine_core(L, n_pts, (const float2*)C, (const float2*)G, (const float2*)U,
                             (float2*)Ht);
}

gt_status gt_combine_full(const gt_plan* plan, const void* X, const void* U, int32_t n_pts, void* H,
                          void* ws, size_t ws_bytes, void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if (!X || !U || !H || n_pts < 1 || n_pts > kMaxCombinePts) return GT_ERR_ARG;
  if (plan->opt.dtype != GT_C64) return GT_ERR_UNSUPPORTED;
  LaunchCtx L = make_ctx(plan, ws, stream);
  return launch_combine_full(L, n_pts, (const float2*)X, (const float2*)U, (float2*)H);
}

gt_status gt_sinr_eval_full(const gt_plan* plan, const void* X, const float* sigma2, int32_t n_snr,
                            void* sinr, int32_t* dev_status, void* ws, size_t ws_bytes,
                            void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if ((st = check_snr(sigma2, n_snr)) != GT_OK) return st;
  if (!X || !sinr) return GT_ERR_ARG;
  LaunchCtx L = make_ctx(plan, ws, stream);
  if (plan->opt.dtype == GT_C128)
    return launch_sinr_c128(L, plan->totals.sc, true, (const double2*)X, nullptr, nullptr, sigma2,
                            n_snr, (double*)sinr, plan->ns_max, dev_status);
  return launch_sinr(L, plan->totals.sc, true, (const float2*)X, nullptr, nullptr, sigma2, n_snr,
                     (float*)sinr, plan->ns_max, dev_status);
}

gt_status gt_sinr_eval_backward(const gt_plan* plan, const void* C, const void* G,
                                const float* sigma2, int32_t n_snr, const void* grad_sinr,
                                void* grad_C, void* grad_G, int32_t* dev_status, void* ws,
                                size_t ws_bytes, void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if ((st = check_snr(sigma2, n_snr)) != GT_OK) return st;
  if (!C || !G || !grad_sinr || !grad_C || !grad_G) return GT_ERR_ARG;
  LaunchCtx L = make_ctx(plan, ws, stream);
  if (plan->opt.dtype == GT_C128)
    return launch_sinr_bwd_c128(L, plan->totals.sc, (const double2*)C, (const double2*)G, sigma2,
                                n_snr, (const double*)grad_sinr, (double2*)grad_C, (double2*)grad_G,
                                plan->ns_max, dev_status);
  return launch_sinr_bwd(L, plan->totals.sc, (const float2*)C, (const float2*)G, sigma2, n_snr,
                         (const float*)grad_sinr, (float2*)grad_C, (float2*)grad_G, plan->ns_max,
                         dev_status);
}

// ---------------------------------------------------------------------------------------
// The SINR adjoint in the library's static scratch, for callers that cannot allocate.  Each GPU
// the library runs on holds its own copy of `scratch` (from the first call on that GPU until
// the process ends); its device address is taken once per device with hipGetSymbolAddress and
// only that address is passed to copies and kernels.

static constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];
static constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's scratch, looked up on the first call on that device.
static gt_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error_detail("hipGetDevice", e);
    return GT_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxScratchDevices) return GT_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error_detail("hipGetSymbolAddress(scratch)", e != hipSuccess ? e : hipErrorInvalidSymbol);
      return GT_ERR_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GT_OK;
}

gt_status gt_sinr_eval_backward_static(const gt_plan* plan, const void* C, const void* G,
                                       const float* sigma2, int32_t n_snr, const void* grad_sinr,
                                       void* grad_C, void* grad_G, int32_t* dev_status,
                                       void* stream) {
  if (!plan) return GT_ERR_ARG;
  gt_status st = check_snr(sigma2, n_snr);
  if (st != GT_OK) return st;
  if (!C || !G || !grad_sinr || !grad_C || !grad_G) return GT_ERR_ARG;
  if ((size_t)plan->slay.total > kStaticScratchBytes) return GT_ERR_WORKSPACE;
  void* ptr = nullptr;
  if ((st = static_scratch(&ptr)) != GT_OK) return st;
  // the plan's tables (with dl/dHt offsets in this layout) into the scratch, ordered on the
  // stream before the kernels; dl/dHt needs no clearing (every entry read is written first)
  hipError_t e = hipMemcpyAsync(ptr, plan->sblob.data(), plan->sblob.size(), hipMemcpyHostToDevice,
                                reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    set_error_detail("gt_sinr_eval_backward_static", e);
    return GT_ERR_HIP;
  }
  LaunchCtx L = make_ctx_at(plan, plan->slay, ptr, stream);
  if (plan->opt.dtype == GT_C128)
    return launch_sinr_bwd_c128(L, plan->totals.sc, (const double2*)C, (const double2*)G, sigma2,
                                n_snr, (const double*)grad_sinr, (double2*)grad_C, (double2*)grad_G,
                                plan->ns_max, dev_status);
  return launch_sinr_bwd(L, plan->totals.sc, (const float2*)C, (const float2*)G, sigma2, n_snr,
                         (const float*)grad_sinr, (float2*)grad_C, (float2*)grad_G, plan->ns_max,
                         dev_status);
}

gt_status gt_tucker_reconstruct_backward(const gt_plan* plan, const void* A, const void* B,
                                         const void* C, const void* G, const void* grad_Ht,
                                         const void* grad_Xhat, void* grad_A, void* grad_B,
                                         void* grad_C, void* grad_G, void* ws, size_t ws_bytes,
                                         void* stream) {
  gt_status st = check_ws(plan, ws, ws_bytes);
  if (st != GT_OK) return st;
  if (!A || !B || !C || !G || !grad_A || !grad_B || !grad_C || !grad_G) return GT_ERR_ARG;
  if (plan->opt.dtype != GT_C64) return GT_ERR_UNSUPPORTED;
  LaunchCtx L = make_ctx(plan, ws, stream);
  return launch_reconstruct_bwd(L, plan->totals.sc, (const float2*)A, (const float2*)B,
                                (const float2*)C, (const float2*)G, (const float2*)grad_Ht,
                                (const float2*)grad_Xhat, (float2*)grad_A, (float2*)grad_B,
                                (float2*)grad_C, (float2*)grad_G);
}

gt_status gt_tucker_fit_backward(const gt_plan* plan) {
  (void)plan;
  return GT_ERR_UNSUPPORTED;
}

gt_status gt_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return GT_OK;
}

gt_status gt_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_clear_locked();
  return GT_OK;
}

gt_status gt_profile_query(const char* name, double* total_ms, int64_t* launches) {
  if (!name || !total_ms || !launches) return GT_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double tot = 0.0;
  int64_t cnt = 0;
  std::string pat(name);
  const bool prefix = !pat.empty() && pat.back() == '*';
  if (prefix) pat.pop_back();
  for (auto& r : g_prof) {
    // base name: the kernel's identifier without the parentheses and template arguments
    // that the launch macros record
    std::string base = r.name;
    if (!base.empty() && base[0] == '(') base.erase(0, 1);
    const size_t lt = base.find_first_of("<)");
    if (lt != std::string::npos) base.resize(lt);
    if (prefix ? base.compare(0, pat.size(), pat) != 0 : base != pat) continue;
    if (hipEventSynchronize(r.stop) != hipSuccess) return GT_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return GT_ERR_HIP;
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return GT_OK;
}

}  // extern "C"
