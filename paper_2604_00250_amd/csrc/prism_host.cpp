// Host side of libprism: argument validation, problem planning (mask
// compaction, neighbour tables, work items, reduction tiles), workspace
// sizing and kernel dispatch.  Implements the C ABI declared in prism.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/prism.h"
#include "prism_internal.h"

using namespace prism;

#ifndef PRISM_SOURCE_HASH
#define PRISM_SOURCE_HASH "unknown"
#endif

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PRISM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Bucket {
  int K, mode, learn_d, maxN;
  int item_begin, item_count;
  int xsplit;  // cross-wave buffer rows the launch needs
  int vpl;     // voxels per lane of the launch (1 for the persistent launch)
  int stream;  // 0: the caller's stream; s > 0: the problem's side stream s - 1
  int cls;     // persistent launch: register class of its items (persistent_class)
  int grid;    // persistent launch: blocks
};

constexpr int kSideStreams = 3;  // with the caller's: the four hardware queues a process gets

}  // namespace

struct prism_problem {
  int device = 0;
  ModelDev model{};
  prism_launch launch{};
  std::vector<prism_bucket_launch> bucket_launch;  // per-bucket overrides of `launch`
  std::vector<prism_group_desc> desc;       // mask pointers are not kept
  std::vector<GroupDev> groups;
  std::vector<ItemDev> items;
  std::vector<Bucket> buckets;
  std::vector<TileDev> tiles;
  std::vector<int32_t> tri_groups;
  std::vector<int32_t> acq_off;
  int max_field_chunks = 0;
  int spatial_c = -1;  // C of every group with the Eq. 7 prior (-1: none yet, 0: they differ)
  int max_item_nv = 0;  // voxels of the plan's largest work item
  int persistent_grid = 0;
  int64_t n_vox = 0, n_micro = 0, n_cal = 0, n_y = 0;
  size_t ws_rec = 0, ws_part = 0, ws_float = 0;  // element counts
  // device tables
  GroupDev* d_groups = nullptr;
  ItemDev* d_items = nullptr;
  TileDev* d_tiles = nullptr;
  float* d_bval = nullptr;
  float* d_bvec = nullptr;
  int32_t* d_coords = nullptr;
  int32_t* d_nbr = nullptr;
  float* d_ninv = nullptr;
  int32_t* d_grid = nullptr;
  int32_t* d_tri = nullptr;
  std::vector<int32_t> coords_host;         // packed voxel coordinates of every group
  // slab stitch table (prism_stitch_plan)
  bool st_planned = false;
  int64_t st_n_out = 0;
  int32_t* d_st_g = nullptr;
  int32_t* d_st_v = nullptr;
  float* d_st_w = nullptr;
  // optional timing of the fused kernel
  bool prof = false;
  std::vector<hipEvent_t> ev;
  mutable int ev_used = 0;
  // concurrent variant launches (prism_launch.concurrent): side streams and the
  // fork / join events, created by plan() when first needed
  std::vector<hipStream_t> side;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  int n_side_used = 0;               // side streams the current plan uses
  mutable std::mutex enqueue_mu;     // one call's fork / launches / join at a time

  void free_stitch() {
    (void)hipFree(d_st_g);
    (void)hipFree(d_st_v);
    (void)hipFree(d_st_w);
    d_st_g = nullptr;
    d_st_v = nullptr;
    d_st_w = nullptr;
    st_n_out = 0;
    st_planned = false;
  }
  void free_plan() {
    (void)hipFree(d_items);
    (void)hipFree(d_tiles);
    d_items = nullptr;
    d_tiles = nullptr;
  }
  ~prism_problem() {
    free_plan();
    (void)hipFree(d_groups);
    (void)hipFree(d_bval);
    (void)hipFree(d_bvec);
    (void)hipFree(d_coords);
    (void)hipFree(d_nbr);
    (void)hipFree(d_ninv);
    (void)hipFree(d_grid);
    (void)hipFree(d_tri);
    free_stitch();
    for (auto e : ev) (void)hipEventDestroy(e);
    for (auto e : ev_join) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (auto st : side) (void)hipStreamDestroy(st);
  }
};

namespace {

int n_bias_of(int bias) { return bias == PRISM_BIAS_POLY2 ? 10 : bias == PRISM_BIAS_TRILINEAR8 ? 512 : 0; }

// Measurement split of one item: with n_split = 0 the item's size picks it
// (few voxels -> more waves share each voxel row, each over a part of N).
int item_split(const prism_launch& L, int nv) {
  if (L.n_split > 0) return L.n_split;
  const int lane_vox = 64 * L.vox_per_lane;
  if (nv <= lane_vox) return 4;
  if (nv <= 2 * lane_vox) return 2;
  return 1;
}

int xsplit_of(int wn) { return (4 / wn) * (wn - 1); }  // cross-wave buffer rows

// The launch shape of group g: the problem's shape with the overrides of the
// group's bucket (N, K, mode, learned D), if any.  The persistent launch runs
// one voxel per lane.
prism_launch group_launch(const prism_problem* h, const GroupDev& g) {
  prism_launch L = h->launch;
  for (const prism_bucket_launch& b : h->bucket_launch)
    if (b.n_meas == g.N && b.K == g.K && b.mode == g.mode && b.learn_diffusivity == g.learn_d) {
      L.vox_per_lane = b.vox_per_lane;
      L.n_split = b.n_split;
      L.item_vox = b.item_vox;
    }
  if (L.persistent) L.vox_per_lane = 1;
  return L;
}

// Voxels per work item of a group under its launch shape.
int group_item_vox(const prism_problem* h, const prism_launch& L) {
  const int vpl = L.vox_per_lane;
  const int base_chunk = 64 * vpl * 4;  // voxels per block chunk with n_split = 1
  if (L.item_vox > 0) return L.item_vox;
  if (L.n_split > 0) {
    // one block chunk per item: the finest cut balances the compute units
    // best (brain-shaped volume, K = 3: 256-voxel items run the fused pass
    // 2.4% faster than 512-voxel ones)
    return 64 * vpl * (4 / L.n_split);
  }
  // split chosen per item: about six blocks per compute unit over the whole
  // problem, whole chunks
  const int64_t target = 256 * 6;
  int64_t per = (h->n_vox + target - 1) / target;
  per = ((per + base_chunk - 1) / base_chunk) * base_chunk;
  return (int)std::max<int64_t>(base_chunk, std::min<int64_t>(per, 8 * base_chunk));
}

// Staggered first round (prism_launch.stagger).  All blocks of a launch of equal
// items start together and run in step, so every block of a compute unit
// reaches its epilogue (parameter, moment and Eq. 7 traffic) at the same moment.
// The dispatcher deals blocks to the 8 XCDs in turn and, within an XCD, to its
// compute units in turn, so the first CUs/8 items of each XCD's run of items
// (xcd_item) are the first block of each of its compute units: cutting them to
// 64 voxels over four waves (about a quarter of a block's time) and 128 voxels
// over two (about half) leaves one block per compute unit out of phase with
// the others from then on.  Measured on the brain-shaped volume (743k voxels,
// N = 288, K = 3, MSE) on four boxes: the fused kernel 2.7-4% faster; shortening
// more items, or spreading them over more positions, gained less or lost.
// Returns the cut (voxels, n_split per item, in item order) or an empty vector
// where the scheme does not apply.
std::vector<std::pair<int, int>> staggered_cut(const prism_problem* h, const prism_launch& Lg,
                                               const GroupDev& g) {
  std::vector<std::pair<int, int>> cut;
  if (!Lg.stagger || Lg.persistent || h->groups.size() != 1 || Lg.vox_per_lane != 1 || Lg.n_split != 1 ||
      Lg.item_vox != 0)
    return cut;
  constexpr int kXcd = 8;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus < kXcd)
    return cut;
  const int waves = pass_waves_per_simd(g.K, g.mode, g.learn_d, 1);
  // the four-way split's cross-wave buffer must not cost the variant a block per CU
  constexpr size_t kLdsPerCu = 160 * 1024;
  if (pass_lds_per_block(g.N, 3, g.K, g.learn_d, 1) * (size_t)waves > kLdsPerCu) return cut;
  const int per_xcd = cus / kXcd, nq = per_xcd / 2, nh = per_xcd - nq;
  const int64_t head = (int64_t)kXcd * (nq * 64 + nh * 128);
  const int64_t full = (g.V - head) / 256, part = (g.V - head) % 256;
  if (g.V <= head || full < 2LL * cus * waves) return cut;  // fewer than two rounds of blocks
  const int n = (int)(kXcd * (nq + nh) + full + (part ? 1 : 0));
  const int q = n / kXcd, r = n % kXcd;
  int64_t v0 = 0;
  for (int x = 0; x < kXcd; ++x) {
    const int len = q + (x < r ? 1 : 0);
    for (int j = 0; j < len && v0 < g.V; ++j) {
      int nv = 256, ns = 1;
      if (j < nq) {
        nv = 64;
        ns = 4;
      } else if (j < nq + nh) {
        nv = 128;
        ns = 2;
      }
      nv = (int)std::min<int64_t>(nv, g.V - v0);
      cut.emplace_back(nv, ns);
      v0 += nv;
    }
  }
  if (v0 != g.V || (int)cut.size() != n) cut.clear();  // not reached; the plain cut then
  return cut;
}

// Work items, launch buckets and reduction tiles for the current launch shape.
int plan(prism_problem* h) {
  const prism_launch& L = h->launch;
  std::vector<ItemDev> items;
  std::vector<int> item_vpl;
  bool keep_order = false;  // a staggered cut is launched in its own order
  std::vector<std::vector<int>> per_group(h->groups.size());
  for (size_t gi = 0; gi < h->groups.size(); ++gi) {
    GroupDev& g = h->groups[gi];
    const prism_launch Lg = group_launch(h, g);
    const int item_vox = group_item_vox(h, Lg);
    if (Lg.n_split > 0 && item_vox % (64 * Lg.vox_per_lane * (4 / Lg.n_split)) != 0)
      return fail(PRISM_E_INVALID, "group %d: item_vox %d is not a multiple of the block chunk %d", (int)gi,
                  item_vox, 64 * Lg.vox_per_lane * (4 / Lg.n_split));
    int rec = 0;
    const std::vector<std::pair<int, int>> cut = staggered_cut(h, Lg, g);
    keep_order = keep_order || !cut.empty();
    for (int v0 = 0, i = 0; v0 < g.V; ++i) {
      ItemDev it{};
      it.group = (int)gi;
      it.v0 = v0;
      it.nv = cut.empty() ? std::min(item_vox, g.V - v0) : cut[i].first;
      it.rec = rec++;
      it.n_split = cut.empty() ? item_split(Lg, it.nv) : cut[i].second;
      it.kind = ((g.K - 1) * 2 + g.mode) * 2 + g.learn_d;
      per_group[gi].push_back((int)items.size());
      items.push_back(it);
      item_vpl.push_back(Lg.vox_per_lane);
      v0 += it.nv;
    }
    g.item_count = rec;
  }
  auto cost = [&](const ItemDev& a) { return (int64_t)a.nv * h->groups[a.group].N * (h->groups[a.group].K + 2); };
  std::vector<Bucket> buckets;
  std::vector<ItemDev> ordered;
  ordered.reserve(items.size());
  if (L.persistent) {
    // one launch per register class; items largest first (LPT) within each
    for (int cls = 0; cls < 2; ++cls) {
      Bucket b{0, 0, 0, 0, (int)ordered.size(), 0, 0, 1, 0, cls, 0};
      for (const ItemDev& it : items)
        if (persistent_class(h->groups[it.group].K) == cls) ordered.push_back(it);
      std::stable_sort(ordered.begin() + b.item_begin, ordered.end(),
                       [&](const ItemDev& a, const ItemDev& c) { return cost(a) > cost(c); });
      b.item_count = (int)ordered.size() - b.item_begin;
      for (int i = b.item_begin; i < (int)ordered.size(); ++i) {
        b.maxN = std::max(b.maxN, h->groups[ordered[i].group].N);
        b.xsplit = std::max(b.xsplit, xsplit_of(ordered[i].n_split));
      }
      if (b.item_count > 0) buckets.push_back(b);
    }
  } else {
    // one launch per kernel variant (K, mode, learned D, voxels per lane); items
    // inside a launch largest first (LPT)
    std::vector<bool> done(items.size(), false);
    for (size_t i0 = 0; i0 < items.size(); ++i0) {
      if (done[i0]) continue;
      const GroupDev& g0 = h->groups[items[i0].group];
      Bucket b{g0.K, g0.mode, g0.learn_d, 0, (int)ordered.size(), 0, 0, item_vpl[i0]};
      std::vector<ItemDev> bi;
      for (size_t i = i0; i < items.size(); ++i) {
        const GroupDev& g = h->groups[items[i].group];
        if (done[i] || g.K != b.K || g.mode != b.mode || g.learn_d != b.learn_d || item_vpl[i] != b.vpl) continue;
        done[i] = true;
        b.maxN = std::max(b.maxN, g.N);
        bi.push_back(items[i]);
      }
      if (!keep_order)
        std::stable_sort(bi.begin(), bi.end(), [&](const ItemDev& a, const ItemDev& c) { return cost(a) > cost(c); });
      for (const ItemDev& it : bi) b.xsplit = std::max(b.xsplit, xsplit_of(it.n_split));
      ordered.insert(ordered.end(), bi.begin(), bi.end());
      b.item_count = (int)bi.size();
      if (b.item_count > 0) buckets.push_back(b);
    }
  }
  // concurrent variant launches: each launch to the stream with the least work so
  // far, largest launch first (the caller's stream takes the first)
  int n_side = 0;
  if (L.concurrent && buckets.size() > 1) {
    n_side = std::min<int>(kSideStreams, (int)buckets.size() - 1);
    std::vector<int64_t> work(buckets.size(), 0);
    for (size_t b = 0; b < buckets.size(); ++b)
      for (int i = buckets[b].item_begin; i < buckets[b].item_begin + buckets[b].item_count; ++i)
        work[b] += cost(ordered[i]);
    std::vector<size_t> order(buckets.size());
    for (size_t b = 0; b < order.size(); ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) { return work[a] > work[c]; });
    std::vector<int64_t> load(n_side + 1, 0);
    for (size_t b : order) {
      const int st = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      buckets[b].stream = st;
      load[st] += work[b];
    }
  }
  // records and first-stage reduction tiles
  std::vector<TileDev> tiles;
  int64_t rec_off = 0;
  int max_fc = 0;
  for (size_t gi = 0; gi < h->groups.size(); ++gi) {
    GroupDev& g = h->groups[gi];
    g.rec_off = rec_off;
    rec_off += (int64_t)g.item_count * g.rec_stride;
    const int nrr = (g.item_count + 63) / 64;
    const int nfc = (g.rec_stride + 63) / 64;
    max_fc = std::max(max_fc, nfc);
    g.tile_begin = (int)tiles.size();
    g.tile_count = nrr * nfc;
    for (int fc = 0; fc < nfc; ++fc)
      for (int rr = 0; rr < nrr; ++rr) {
        TileDev t;
        t.group = (int)gi;
        t.r0 = rr * 64;
        t.nr = std::min(64, g.item_count - rr * 64);
        t.f0 = fc * 64;
        t.nf = std::min(64, g.rec_stride - fc * 64);
        t.out = (int)tiles.size() * 64;
        tiles.push_back(t);
      }
  }
  // the side streams and events (kept across plans; default priority)
  while ((int)h->side.size() < n_side) {
    hipStream_t st = nullptr;
    hipEvent_t ej = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      return fail(PRISM_E_ALLOC, "stream creation failed");
    h->side.push_back(st);
    if (hipEventCreateWithFlags(&ej, hipEventDisableTiming) != hipSuccess)
      return fail(PRISM_E_ALLOC, "event creation failed");
    h->ev_join.push_back(ej);
  }
  if (n_side > 0 && !h->ev_fork && hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess)
    return fail(PRISM_E_ALLOC, "event creation failed");
  h->n_side_used = n_side;
  h->free_plan();
  h->max_item_nv = 0;
  for (const ItemDev& it : ordered) h->max_item_nv = std::max(h->max_item_nv, it.nv);
  h->items = ordered;
  h->buckets = buckets;
  h->tiles = tiles;
  h->max_field_chunks = max_fc;
  h->ws_rec = (size_t)rec_off;
  h->ws_part = tiles.size() * 64;
  h->persistent_grid = 0;
  if (L.persistent && !h->buckets.empty()) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus <= 0)
      cus = 256;
    // max_blocks caps the launches' blocks together, shared out by work
    int64_t total = 0;
    std::vector<int64_t> work(h->buckets.size(), 0);
    for (size_t bi = 0; bi < h->buckets.size(); ++bi) {
      const Bucket& b = h->buckets[bi];
      for (int i = b.item_begin; i < b.item_begin + b.item_count; ++i) work[bi] += cost(ordered[i]);
      total += work[bi];
    }
    int left = L.max_blocks;
    for (size_t bi = 0; bi < h->buckets.size(); ++bi) {
      Bucket& b = h->buckets[bi];
      const int bpc = persistent_blocks_per_cu(b.cls, b.maxN, b.xsplit);
      int grid = std::min(b.item_count, cus * bpc);
      if (L.max_blocks > 0) {
        const int rest = (int)(h->buckets.size() - bi - 1);
        const int share = bi + 1 == h->buckets.size()
                              ? left
                              : (int)std::max<int64_t>(1, (int64_t)L.max_blocks * work[bi] / std::max<int64_t>(total, 1));
        grid = std::min(grid, std::max(1, std::min(share, left - rest)));
        left -= grid;
      }
      b.grid = std::max(1, grid);
      h->persistent_grid += b.grid;
    }
  }
  hipError_t e = upload(&h->d_items, h->items);
  if (e == hipSuccess) e = upload(&h->d_tiles, h->tiles);
  if (e == hipSuccess) {
    (void)hipFree(h->d_groups);
    h->d_groups = nullptr;
    e = upload(&h->d_groups, h->groups);
  }
  if (e != hipSuccess) return fail(PRISM_E_ALLOC, "device upload failed: %s", hipGetErrorString(e));
  return PRISM_OK;
}

int check_shape(int vpl, int n_split, int item_vox, const char* what) {
  if (vpl != 1 && vpl != 2) return fail(PRISM_E_INVALID, "%s: vox_per_lane must be 1 or 2 (got %d)", what, vpl);
  if (n_split != 0 && n_split != 1 && n_split != 2 && n_split != 4)
    return fail(PRISM_E_INVALID, "%s: n_split must be 0 (per item), 1, 2 or 4 (got %d)", what, n_split);
  if (item_vox < 0) return fail(PRISM_E_INVALID, "%s: item_vox must be >= 0", what);
  return PRISM_OK;
}

int check_launch(const prism_launch* L) {
  int rc = check_shape(L->vox_per_lane, L->n_split, L->item_vox, "launch");
  if (rc != PRISM_OK) return rc;
  if (L->persistent != 0 && L->persistent != 1)
    return fail(PRISM_E_INVALID, "persistent must be 0 or 1");
  if (L->max_blocks < 0) return fail(PRISM_E_INVALID, "max_blocks must be >= 0");
  if (L->stagger != 0 && L->stagger != 1) return fail(PRISM_E_INVALID, "stagger must be 0 or 1");
  if (L->concurrent != 0 && L->concurrent != 1) return fail(PRISM_E_INVALID, "concurrent must be 0 or 1");
  return PRISM_OK;
}

// The distinct (N, K, mode, learned D) buckets of a problem's groups, in order of first appearance.
std::vector<prism_bucket_launch> bucket_signatures(const prism_problem* h) {
  std::vector<prism_bucket_launch> out;
  for (const GroupDev& g : h->groups) {
    bool seen = false;
    for (const prism_bucket_launch& b : out)
      seen = seen || (b.n_meas == g.N && b.K == g.K && b.mode == g.mode && b.learn_diffusivity == g.learn_d);
    if (seen) continue;
    prism_bucket_launch b{};
    b.n_meas = g.N;
    b.K = g.K;
    b.mode = g.mode;
    b.learn_diffusivity = g.learn_d;
    const prism_launch L = group_launch(h, g);
    b.vox_per_lane = L.vox_per_lane;
    b.n_split = L.n_split;
    b.item_vox = L.item_vox;
    out.push_back(b);
  }
  return out;
}

}  // namespace

extern "C" {

int32_t prism_abi_version(void) { return PRISM_ABI_VERSION; }

const char* prism_last_error(void) { return g_last_error.c_str(); }

void prism_model_defaults(prism_model* m) {
  if (!m) return;
  m->d_csf = 3.0f;
  m->d_gm = 0.9f;
  m->d_res = 0.2f;
  m->d_par = 1.7f;
  m->d_perp = 0.4f;
  m->lam_sp = 0.01f;
  m->huber_delta = 0.05f;
  m->lam_rep = 0.01f;
  m->lam_sparse = 0.02f;
  m->tau_sparse = 0.15f;
  m->lam_alpha = 0.01f;
  m->lam_beta = 0.01f;
  m->lam_bias = 0.01f;
  m->lam_orphan = 0.01f;
  m->s0_orphan = 0.1f;
  m->lam_cont = 0.005f;
  m->lam_order = 0.01f;
  m->lam_tv = 0.01f;
}

int32_t prism_problem_create(prism_problem** out, const prism_group_desc* groups, int32_t n_groups,
                             const prism_acq* acqs, int32_t n_acq, const prism_model* model) {
  if (!out) return fail(PRISM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!groups || n_groups <= 0) return fail(PRISM_E_INVALID, "need at least one group");
  if (!acqs || n_acq <= 0) return fail(PRISM_E_INVALID, "need at least one acquisition");
  if (!model) return fail(PRISM_E_INVALID, "model is NULL");
  const float mv[] = {model->d_csf, model->d_gm, model->d_res, model->d_par, model->d_perp,
                      model->lam_sp, model->huber_delta, model->lam_rep, model->lam_sparse,
                      model->tau_sparse, model->lam_alpha, model->lam_beta, model->lam_bias,
                      model->lam_orphan, model->s0_orphan, model->lam_cont, model->lam_order,
                      model->lam_tv};
  for (float x : mv)
    if (!std::isfinite(x) || x < 0.0f) return fail(PRISM_E_INVALID, "model constants must be finite and >= 0");
  if (!(model->s0_orphan > 0.0f)) return fail(PRISM_E_INVALID, "s0_orphan must be > 0");
  if (!(model->d_par > 0.0f)) return fail(PRISM_E_INVALID, "d_par must be > 0");
  // acquisitions
  std::vector<int32_t> acq_off(n_acq);
  std::vector<float> bval, bvec;
  for (int a = 0; a < n_acq; ++a) {
    const prism_acq& q = acqs[a];
    if (q.n_meas < 1 || q.n_meas > PRISM_MAX_MEAS)
      return fail(PRISM_E_INVALID, "acquisition %d: n_meas %d outside 1..%d", a, q.n_meas, PRISM_MAX_MEAS);
    if (!q.bval || !q.bvec) return fail(PRISM_E_INVALID, "acquisition %d: NULL bval or bvec", a);
    acq_off[a] = (int32_t)bval.size();
    for (int n = 0; n < q.n_meas; ++n) {
      const float b = q.bval[n];
      const float gx = q.bvec[3 * n], gy = q.bvec[3 * n + 1], gz = q.bvec[3 * n + 2];
      if (!std::isfinite(b) || b < 0.0f)
        return fail(PRISM_E_INVALID, "acquisition %d: b-value %d is negative or not finite", a, n);
      if (!std::isfinite(gx) || !std::isfinite(gy) || !std::isfinite(gz))
        return fail(PRISM_E_INVALID, "acquisition %d: direction %d not finite", a, n);
      const float nrm = std::sqrt(gx * gx + gy * gy + gz * gz);
      if (b > 0.0f && std::fabs(nrm - 1.0f) > 1e-3f)
        return fail(PRISM_E_INVALID, "acquisition %d: direction %d is not a unit vector (|g| = %g)", a, n, nrm);
      bval.push_back(b);
      bvec.push_back(gx);
      bvec.push_back(gy);
      bvec.push_back(gz);
    }
  }
  prism_problem* h = new (std::nothrow) prism_problem();
  if (!h) return fail(PRISM_E_ALLOC, "host allocation failed");
  (void)hipGetDevice(&h->device);
  // set-up of this device's static workspace (prism_loss_grad_noalloc); a
  // failure is reported by that entry point, not here
  (void)static_scratch_setup(h->device);
  h->model = ModelDev{model->d_csf, model->d_gm, model->d_res, model->d_par, model->d_perp,
                      model->lam_sp, model->huber_delta, model->lam_rep, model->lam_sparse,
                      model->tau_sparse, model->lam_alpha, model->lam_beta, model->lam_bias,
                      model->lam_orphan, model->s0_orphan, model->lam_cont, model->lam_order,
                      model->lam_tv};
  std::vector<int32_t> coords, nbr, grid;
  std::vector<float> ninv;
  int64_t micro = 0, cal = 0, y = 0, vox = 0, wfl = 0;
  for (int gi = 0; gi < n_groups; ++gi) {
    const prism_group_desc& d = groups[gi];
    auto bad = [&](const char* what) {
      delete h;
      return fail(PRISM_E_INVALID, "group %d: %s", gi, what);
    };
    if (d.nx < 1 || d.ny < 1 || d.nz < 1 || d.nx > PRISM_MAX_EDGE || d.ny > PRISM_MAX_EDGE || d.nz > PRISM_MAX_EDGE)
      return bad("box edges must be in 1..1023");
    if (d.K < 1 || d.K > PRISM_MAX_K) return bad("K must be in 1..6");
    if (d.mode != PRISM_MSE && d.mode != PRISM_RICIAN) return bad("unknown data mode");
    if (d.bias != PRISM_BIAS_NONE && d.bias != PRISM_BIAS_POLY2 && d.bias != PRISM_BIAS_TRILINEAR8)
      return bad("unknown bias basis");
    if (d.acq < 0 || d.acq >= n_acq) return bad("acquisition index out of range");
    if (d.neighbourhood != 0 && d.neighbourhood != 6 && d.neighbourhood != 26)
      return bad("neighbourhood must be 0, 6 or 26");
    if (d.learn_diffusivity != 0 && d.learn_diffusivity != 1) return bad("learn_diffusivity must be 0 or 1");
    if (d.priors & ~0xFFu) return bad("unknown prior bits");
    const int64_t box = (int64_t)d.nx * d.ny * d.nz;
    if (box > (int64_t)1 << 31) return bad("box too large");
    // compaction in raster order
    std::vector<int32_t> idx;
    // the bias TV needs the face neighbours even without an Eq. 7 neighbourhood
    const int ntab = d.neighbourhood != 0 ? d.neighbourhood
                     : ((d.priors & PRISM_PRIOR_TV) && d.bias != PRISM_BIAS_NONE ? 6 : 0);
    const bool need_idx = ntab != 0 || d.bias == PRISM_BIAS_TRILINEAR8;
    if (need_idx) idx.assign((size_t)box, -1);
    int32_t V = 0;
    const size_t cbase = coords.size();
    for (int i = 0; i < d.nx; ++i)
      for (int j = 0; j < d.ny; ++j)
        for (int k = 0; k < d.nz; ++k) {
          const int64_t r = ((int64_t)i * d.ny + j) * d.nz + k;
          if (d.mask && !d.mask[r]) continue;
          if (need_idx) idx[(size_t)r] = V;
          coords.push_back(i | (j << 10) | (k << 20));
          ++V;
        }
    GroupDev g{};
    g.micro_off = micro;
    g.cal_off = cal;
    g.y_off = y;
    g.vox_off = (int64_t)cbase;
    g.V = V;
    g.N = acqs[d.acq].n_meas;
    g.K = d.K;
    g.C = d.K + 3;
    g.P = 4 * d.K + 5 + (d.learn_diffusivity ? 2 : 0);
    g.mode = d.mode;
    g.bias = d.bias;
    g.n_bias = n_bias_of(d.bias);
    g.learn_d = d.learn_diffusivity;
    g.nbh = d.neighbourhood;
    g.priors = (int32_t)d.priors;
    g.nx = d.nx;
    g.ny = d.ny;
    g.nz = d.nz;
    {
      const int32_t n3[3] = {d.nx, d.ny, d.nz};
      for (int a = 0; a < 3; ++a) {
        g.bsc[a] = n3[a] > 1 ? 2.0f / (float)(n3[a] - 1) : 0.0f;
        g.boff[a] = n3[a] > 1 ? -1.0f : 0.0f;
      }
    }
    g.acq_off = acq_off[d.acq];
    g.nb0 = 0;
    while (g.nb0 < g.N && bval[(size_t)g.acq_off + g.nb0] == 0.0f) ++g.nb0;
    g.rec_stride = kRecHead + 2 * g.N;
    g.invM = V > 0 ? 1.0f / (float)V : 0.0f;
    {
      const ModelDev& m = h->model;
      g.sdata = g.mode == PRISM_MSE ? 2.0f * g.invM : 1.0f;
      g.sc_sp = m.lam_sp * g.invM;
      g.sc_rep = m.lam_rep * g.invM;
      g.sc_spa = m.lam_sparse * g.invM;
      g.sc_orph = m.lam_orphan * g.invM;
      g.sc_ord = m.lam_order * g.invM;
      g.sc_tv = m.lam_tv * g.invM;
      g.sc_cont2 = -2.0f * m.lam_cont * g.invM;
      g.inv_s0o = 1.0f / m.s0_orphan;
      g.sc_orph_s0 = g.sc_orph / m.s0_orphan;
      const int32_t n3[3] = {d.nx, d.ny, d.nz};
      for (int a = 0; a < 3; ++a) g.tri_sc[a] = n3[a] > 1 ? 7.0f / (float)(n3[a] - 1) : 0.0f;
    }
    g.ntab = ntab;
    g.nbr_off = (int64_t)nbr.size();
    g.ninv_off = (int64_t)ninv.size();
    if (ntab != 0) {
      // face neighbours first (-x, +x, -y, +y, -z, +z), then the other 20 of 26
      std::vector<int> off = {-1, 0, 0, 1, 0, 0, 0, -1, 0, 0, 1, 0, 0, 0, -1, 0, 0, 1};
      if (ntab == 26)
        for (int a = -1; a <= 1; ++a)
          for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
              const int m = std::abs(a) + std::abs(b) + std::abs(c);
              if (m < 2) continue;
              off.push_back(a);
              off.push_back(b);
              off.push_back(c);
            }
      const int nq = (int)off.size() / 3;
      const size_t nb0 = nbr.size();
      nbr.resize(nb0 + (size_t)nq * V, -1);
      for (int32_t v = 0; v < V; ++v) {
        const int32_t pc = coords[cbase + v];
        const int i = pc & 1023, j = (pc >> 10) & 1023, k = (pc >> 20) & 1023;
        for (int q = 0; q < nq; ++q) {
          const int a = i + off[3 * q], b = j + off[3 * q + 1], c = k + off[3 * q + 2];
          if (a < 0 || b < 0 || c < 0 || a >= d.nx || b >= d.ny || c >= d.nz) continue;
          nbr[nb0 + (size_t)q * V + v] = idx[((size_t)a * d.ny + b) * d.nz + c];
        }
      }
      // 1/|N(x)| over the Eq. 7 neighbourhood
      ninv.resize(ninv.size() + (size_t)V, 0.0f);
      for (int32_t v = 0; v < V && d.neighbourhood != 0; ++v) {
        int cnt = 0;
        for (int q = 0; q < d.neighbourhood; ++q) cnt += nbr[nb0 + (size_t)q * V + v] >= 0;
        ninv[g.ninv_off + v] = cnt > 0 ? 1.0f / (float)cnt : 0.0f;
      }
    }
    g.grid_off = (int64_t)grid.size();
    if (d.bias == PRISM_BIAS_TRILINEAR8) {
      grid.insert(grid.end(), idx.begin(), idx.end());
      h->tri_groups.push_back(gi);
    }
    wfl = (wfl + 3) & ~(int64_t)3;  // 16-byte aligned buffers
    g.w_off = wfl;  // [V][C] residual weights, then [V][C] fractions
    if ((d.priors & PRISM_PRIOR_SPATIAL) && d.neighbourhood) {
      wfl += 2 * (int64_t)g.C * V;
      wfl = (wfl + 3) & ~(int64_t)3;
      h->spatial_c = h->spatial_c < 0 ? g.C : (h->spatial_c == g.C ? g.C : 0);
    }
    g.glb_off = wfl;
    if (d.bias == PRISM_BIAS_TRILINEAR8) wfl += V;
    wfl = (wfl + 3) & ~(int64_t)3;  // 16-byte aligned acquisition table
    g.acqtab_off = wfl;
    wfl += (int64_t)kAcqStride * g.N;
    micro += (int64_t)g.P * V;
    cal += g.n_bias + 2 * g.N + 1;
    y += (int64_t)g.N * V;
    vox += V;
    h->groups.push_back(g);
    prism_group_desc dc = d;
    dc.mask = nullptr;
    h->desc.push_back(dc);
  }
  h->n_vox = vox;
  h->n_micro = micro;
  h->n_cal = cal;
  h->n_y = y;
  h->ws_float = (size_t)wfl;
  h->acq_off = acq_off;
  h->coords_host = coords;
  // default launch shape: one voxel per lane (three waves per SIMD for the
  // common variants); split measurements across waves for small problems
  h->launch.vox_per_lane = 1;
  h->launch.n_split = vox < 65536 ? 4 : (vox < 262144 ? 2 : 1);
  if (n_groups > 64) h->launch.n_split = 0;  // many groups: split per item size
  h->launch.item_vox = 0;
  h->launch.persistent = 0;
  h->launch.max_blocks = 0;
  h->launch.stagger = 1;
  h->launch.concurrent = 1;
  hipError_t e = upload(&h->d_bval, bval);
  if (e == hipSuccess) e = upload(&h->d_bvec, bvec);
  if (e == hipSuccess) e = upload(&h->d_coords, coords);
  if (e == hipSuccess) e = upload(&h->d_nbr, nbr);
  if (e == hipSuccess) e = upload(&h->d_ninv, ninv);
  if (e == hipSuccess) e = upload(&h->d_grid, grid);
  if (e == hipSuccess) e = upload(&h->d_tri, h->tri_groups);
  if (e != hipSuccess) {
    delete h;
    return fail(PRISM_E_ALLOC, "device allocation failed: %s", hipGetErrorString(e));
  }
  int rc = plan(h);
  if (rc != PRISM_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return PRISM_OK;
}

int32_t prism_problem_destroy(prism_problem* h) {
  if (!h) return fail(PRISM_E_INVALID, "handle is NULL");
  delete h;
  return PRISM_OK;
}

int32_t prism_problem_info(const prism_problem* h, prism_problem_info_t* info) {
  if (!h || !info) return fail(PRISM_E_INVALID, "NULL argument");
  info->n_vox = h->n_vox;
  info->n_micro = h->n_micro;
  info->n_cal = h->n_cal;
  info->n_y = h->n_y;
  info->n_groups = (int32_t)h->groups.size();
  info->n_buckets = (int32_t)h->buckets.size();
  return PRISM_OK;
}

int32_t prism_group_info(const prism_problem* h, int32_t group, prism_group_info_t* info) {
  if (!h || !info) return fail(PRISM_E_INVALID, "NULL argument");
  if (group < 0 || group >= (int32_t)h->groups.size()) return fail(PRISM_E_INVALID, "group %d out of range", group);
  const GroupDev& g = h->groups[group];
  info->n_vox = g.V;
  info->n_meas = g.N;
  info->K = g.K;
  info->n_params_vox = g.P;
  info->n_bias = g.n_bias;
  info->n_cal = g.n_bias + 2 * g.N + 1;
  info->pad = 0;
  info->micro_offset = g.micro_off;
  info->cal_offset = g.cal_off;
  info->y_offset = g.y_off;
  return PRISM_OK;
}

int32_t prism_problem_tune_buckets(prism_problem* h, const prism_launch* launch,
                                   const prism_bucket_launch* buckets, int32_t n_buckets) {
  if (!h || !launch) return fail(PRISM_E_INVALID, "NULL argument");
  if (n_buckets < 0 || (n_buckets > 0 && !buckets)) return fail(PRISM_E_INVALID, "bad bucket array");
  int rc = check_launch(launch);
  if (rc != PRISM_OK) return rc;
  std::vector<prism_bucket_launch> bl(buckets, buckets + n_buckets);
  for (int i = 0; i < n_buckets; ++i) {
    const prism_bucket_launch& b = bl[i];
    char what[96];
    snprintf(what, sizeof(what), "bucket %d (N=%d, K=%d, mode %d, learned D %d)", i, b.n_meas, b.K, b.mode,
             b.learn_diffusivity);
    rc = check_shape(b.vox_per_lane, b.n_split, b.item_vox, what);
    if (rc != PRISM_OK) return rc;
    bool found = false;
    for (const GroupDev& g : h->groups)
      found = found || (b.n_meas == g.N && b.K == g.K && b.mode == g.mode && b.learn_diffusivity == g.learn_d);
    if (!found) return fail(PRISM_E_INVALID, "%s: no group of the problem is in this bucket", what);
    for (int j = 0; j < i; ++j)
      if (bl[j].n_meas == b.n_meas && bl[j].K == b.K && bl[j].mode == b.mode &&
          bl[j].learn_diffusivity == b.learn_diffusivity)
        return fail(PRISM_E_INVALID, "%s is given twice", what);
  }
  const prism_launch old = h->launch;
  const std::vector<prism_bucket_launch> old_b = h->bucket_launch;
  h->launch = *launch;
  h->bucket_launch = bl;
  rc = plan(h);
  if (rc != PRISM_OK) {
    const std::string msg = g_last_error;
    h->launch = old;
    h->bucket_launch = old_b;
    plan(h);
    g_last_error = msg;
  }
  return rc;
}

int32_t prism_problem_tune(prism_problem* h, const prism_launch* launch) {
  return prism_problem_tune_buckets(h, launch, nullptr, 0);
}

int32_t prism_problem_launch(const prism_problem* h, prism_launch* launch) {
  if (!h || !launch) return fail(PRISM_E_INVALID, "NULL argument");
  *launch = h->launch;
  return PRISM_OK;
}

int32_t prism_problem_buckets(const prism_problem* h, prism_bucket_launch* out, int32_t cap, int32_t* n) {
  if (!h || !n) return fail(PRISM_E_INVALID, "NULL argument");
  if (cap < 0 || (cap > 0 && !out)) return fail(PRISM_E_INVALID, "bad output array");
  const std::vector<prism_bucket_launch> b = bucket_signatures(h);
  *n = (int32_t)b.size();
  for (int i = 0; i < (int)b.size() && i < cap; ++i) out[i] = b[i];
  return PRISM_OK;
}

int32_t prism_problem_plan_info(const prism_problem* h, int32_t* n_items, int32_t* n_launches,
                                int32_t* persistent_blocks) {
  if (!h || !n_items || !n_launches || !persistent_blocks) return fail(PRISM_E_INVALID, "NULL argument");
  *n_items = (int32_t)h->items.size();
  *n_launches = (int32_t)h->buckets.size();
  *persistent_blocks = h->persistent_grid;
  return PRISM_OK;
}

const char* prism_build_id(void) { return PRISM_SOURCE_HASH; }

int32_t prism_workspace_bytes(const prism_problem* h, size_t* bytes) {
  if (!h || !bytes) return fail(PRISM_E_INVALID, "NULL argument");
  *bytes = align256(h->ws_rec * sizeof(double)) + align256(h->ws_part * sizeof(double)) +
           align256(h->ws_float * sizeof(float)) + align256(h->groups.size() * 3 * sizeof(double)) +
           256;  // + the persistent launch's item counter
  return PRISM_OK;
}

static PassArgs pass_args(const prism_problem* h, const float* y, const float* tm, const float* tc,
                          float* gm, double* rec, float* wsp, uint32_t* status) {
  PassArgs a{};
  a.groups = h->d_groups;
  a.items = h->d_items;
  a.bval = h->d_bval;
  a.bvec = h->d_bvec;
  a.coords = h->d_coords;
  a.nbr = h->d_nbr;
  a.ninv = h->d_ninv;
  a.y = y;
  a.th_micro = tm;
  a.th_cal = tc;
  a.g_micro = gm;
  a.rec = rec;
  a.wsp = wsp;
  a.status = status;
  a.model = h->model;
  a.n_split = h->launch.n_split;
  return a;
}

int32_t prism_synthesize(const prism_problem* h, const float* theta_micro, const float* theta_cal,
                         float* yhat, void* stream) {
  if (!h) return fail(PRISM_E_INVALID, "handle is NULL");
  if ((h->n_micro && !theta_micro) || !theta_cal || (h->n_y && !yhat))
    return fail(PRISM_E_INVALID, "NULL device pointer");
  hipStream_t s = (hipStream_t)stream;
  PassArgs a = pass_args(h, nullptr, theta_micro, theta_cal, nullptr, nullptr, nullptr, nullptr);
  a.synth_only = 1;
  a.yhat = yhat;
  // one synthesis launch per item of the plan's variant groups (the synthesis
  // kernel has no persistent form: it runs item by item per variant)
  for (size_t i = 0; i < h->items.size();) {
    const GroupDev& g0 = h->groups[h->items[i].group];
    size_t j = i;
    int maxN = 0;
    while (j < h->items.size()) {
      const GroupDev& g = h->groups[h->items[j].group];
      if (g.K != g0.K || g.learn_d != g0.learn_d) break;
      maxN = std::max(maxN, g.N);
      ++j;
    }
    a.item_base = (int)i;
    a.n_items = (int)(j - i);
    hipError_t e = launch_pass_maxn(a, g0.K, g0.mode, g0.learn_d, 1, maxN, s);
    if (e != hipSuccess) return hip_fail(e, "synthesis launch");
    i = j;
  }
  return PRISM_OK;
}

namespace {

// Workspace carve-up and the pass: Eq. 7 weights, fused pass, reductions, the
// trilinear bias adjoint.  `adam` (optional) turns on the fused update of the
// per-voxel parameters in the pass epilogue; with `cal_adam` also set, the
// calibration vector is updated where its gradient is written (k_reduce2,
// k_bias_tri) and the step counter advances in the call's first kernel.
struct CalAdam {
  float* th;
  float* m;
  float* v;
  int32_t* step;
  float lr, b1, b2, eps;
  int update;  // 0: theta_cal held fixed (the counter still advances)
};

// loss-history ring of a fused iteration (see prism_iteration_adam)
struct History {
  double* ring;
  const int32_t* step;
  int32_t len;
  int32_t adv;  // 1 when step[0] has already advanced when the loss rows are written
};

int run_pass(const prism_problem* h, const float* y, const float* theta_micro, const float* theta_cal,
             double* loss, float* grad_micro, float* grad_cal, void* workspace, uint32_t* status,
             hipStream_t s, const PassArgs* adam, const CalAdam* cal_adam = nullptr,
             const History* hist = nullptr) {
  char* ws = (char*)workspace;
  const size_t o_part = align256(h->ws_rec * sizeof(double));
  const size_t o_float = o_part + align256(h->ws_part * sizeof(double));
  const size_t o_calsq = o_float + align256(h->ws_float * sizeof(float));
  const size_t o_counter = o_calsq + align256(h->groups.size() * 3 * sizeof(double));
  double* rec = (double*)ws;
  double* part = (double*)(ws + o_part);
  float* wsp = (float*)(ws + o_float);
  double* calsq = (double*)(ws + o_calsq);
  int32_t* counter = (int32_t*)(ws + o_counter);
  const bool have_items = !h->items.empty();
  PassArgs a = pass_args(h, y, theta_micro, theta_cal, grad_micro, rec, wsp, status);
  a.n_groups = (int)h->groups.size();
  // the calibration prior's sums of squares come from the call's first kernel
  // (before any parameter changes) whenever there is one
  a.calsq = have_items ? calsq : nullptr;
  if (adam) {
    a.adam = 1;
    a.th_upd = adam->th_upd;
    a.m_micro = adam->m_micro;
    a.v_micro = adam->v_micro;
    a.step = adam->step;
    a.lr = adam->lr;
    a.b1 = adam->b1;
    a.b2 = adam->b2;
    a.eps = adam->eps;
    if (cal_adam) {
      a.step_advance = cal_adam->step;
      a.step_ready = 1;
    }
  }
  hipError_t e = launch_stage(a, (int)h->groups.size(), s);
  if (e != hipSuccess) return hip_fail(e, "acquisition staging launch");
  if (!h->items.empty()) {
    a.item_base = 0;
    a.n_items = (int)h->items.size();
    e = launch_spatial(a, (int)h->items.size(), std::max(h->spatial_c, 0), h->max_item_nv, s);
    a.step_advance = nullptr;  // advanced once, by the first kernel
    if (e != hipSuccess) return hip_fail(e, "spatial-prior launch");
  }
  // concurrent variant launches fork from the caller's stream and join it again
  const int n_side = h->n_side_used;
  std::unique_lock<std::mutex> lock(h->enqueue_mu, std::defer_lock);
  if (n_side > 0) {
    lock.lock();
    e = hipEventRecord(h->ev_fork, s);
    for (int i = 0; e == hipSuccess && i < n_side; ++i) e = hipStreamWaitEvent(h->side[i], h->ev_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "stream fork");
  }
  for (const Bucket& b : h->buckets) {
    a.item_base = b.item_begin;
    a.n_items = b.item_count;
    a.n_split = b.xsplit;
    hipStream_t bs = b.stream > 0 ? h->side[b.stream - 1] : s;
    // per-launch timing only for launches on the caller's stream
    const bool timed = h->prof && bs == s && h->ev_used + 2 <= (int)h->ev.size();
    if (timed) (void)hipEventRecord(h->ev[h->ev_used], s);
    if (h->launch.persistent)
      e = launch_pass_persistent(a, b.cls, b.maxN, b.grid, counter + 32 * b.cls, bs);
    else
      e = launch_pass_maxn(a, b.K, b.mode, b.learn_d, b.vpl, b.maxN, bs);
    if (e != hipSuccess) return hip_fail(e, "fused-pass launch");
    if (timed) {
      (void)hipEventRecord(h->ev[h->ev_used + 1], s);
      h->ev_used += 2;
    }
  }
  if (n_side > 0) {
    for (int i = 0; e == hipSuccess && i < n_side; ++i) {
      e = hipEventRecord(h->ev_join[i], h->side[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, h->ev_join[i], 0);
    }
    if (e != hipSuccess) return hip_fail(e, "stream join");
    lock.unlock();
  }
  ReduceArgs r{};
  r.groups = h->d_groups;
  r.tiles = h->d_tiles;
  r.rec = rec;
  r.part = part;
  r.th_cal = theta_cal;
  r.g_cal = grad_cal;
  r.loss = loss;
  r.wsp = wsp;
  r.grid = h->d_grid;
  r.coords = h->d_coords;
  r.status = status;
  r.model = h->model;
  r.n_tiles = (int)h->tiles.size();
  r.n_groups = (int)h->groups.size();
  r.calsq = a.calsq;
  if (cal_adam && cal_adam->update) {
    r.cal_adam = 1;
    r.th_cal_upd = cal_adam->th;
    r.m_cal = cal_adam->m;
    r.v_cal = cal_adam->v;
    r.step = cal_adam->step;
    r.lr = cal_adam->lr;
    r.b1 = cal_adam->b1;
    r.b2 = cal_adam->b2;
    r.eps = cal_adam->eps;
  }
  if (hist && hist->ring) {
    r.hist = hist->ring;
    r.hist_step = hist->step;
    r.hist_len = hist->len;
    r.hist_adv = hist->adv;
  }
  e = launch_reduce(r, h->max_field_chunks, s);
  if (e != hipSuccess) return hip_fail(e, "reduction launch");
  e = launch_bias_trilinear(r, h->d_tri, (int)h->tri_groups.size(), s);
  if (e != hipSuccess) return hip_fail(e, "trilinear-bias launch");
  return PRISM_OK;
}

int check_pass_args(const prism_problem* h, const float* y, const float* theta_micro, const float* theta_cal,
                    const double* loss, const float* grad_micro, const float* grad_cal, const void* workspace,
                    size_t workspace_bytes, const uint32_t* status) {
  if (!h) return fail(PRISM_E_INVALID, "handle is NULL");
  if ((h->n_y && !y) || (h->n_micro && (!theta_micro || !grad_micro)) || !theta_cal || !grad_cal ||
      !loss || !status)
    return fail(PRISM_E_INVALID, "NULL device pointer");
  size_t need = 0;
  prism_workspace_bytes(h, &need);
  if (need > 0 && !workspace) return fail(PRISM_E_INVALID, "workspace is NULL");
  if (workspace_bytes < need)
    return fail(PRISM_E_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  return PRISM_OK;
}

}  // namespace

int32_t prism_loss_grad(const prism_problem* h, const float* y, const float* theta_micro,
                        const float* theta_cal, double* loss, float* grad_micro, float* grad_cal,
                        void* workspace, size_t workspace_bytes, uint32_t* status, void* stream) {
  int rc = check_pass_args(h, y, theta_micro, theta_cal, loss, grad_micro, grad_cal, workspace,
                           workspace_bytes, status);
  if (rc != PRISM_OK) return rc;
  return run_pass(h, y, theta_micro, theta_cal, loss, grad_micro, grad_cal, workspace, status,
                  (hipStream_t)stream, nullptr);
}

static_assert(PRISM_NOALLOC_WORKSPACE_BYTES == kStaticScratchBytes, "static workspace size");

int32_t prism_loss_grad_noalloc(const prism_problem* h, const float* y, const float* theta_micro,
                                const float* theta_cal, double* loss, float* grad_micro,
                                float* grad_cal, uint32_t* status, void* stream) {
  if (!h) return fail(PRISM_E_INVALID, "handle is NULL");
  size_t need = 0;
  prism_workspace_bytes(h, &need);
  if (need > kStaticScratchBytes)
    return fail(PRISM_E_WORKSPACE,
                "the problem needs %zu bytes of workspace; the static workspace of "
                "prism_loss_grad_noalloc holds %zu (use prism_loss_grad with a caller workspace)",
                need, kStaticScratchBytes);
  hipError_t e = hipSuccess;
  void* ws = static_scratch(h->device, &e);
  if (!ws) return hip_fail(e, "static workspace of the problem's device");
  int rc = check_pass_args(h, y, theta_micro, theta_cal, loss, grad_micro, grad_cal, ws,
                           kStaticScratchBytes, status);
  if (rc != PRISM_OK) return rc;
  return run_pass(h, y, theta_micro, theta_cal, loss, grad_micro, grad_cal, ws, status,
                  (hipStream_t)stream, nullptr);
}

int32_t prism_iteration_adam(const prism_problem* h, const float* y, float* theta_micro,
                             float* theta_cal, float* m_micro, float* v_micro, float* m_cal,
                             float* v_cal, int32_t* step, float lr, float beta1, float beta2,
                             float eps, int32_t update_cal, double* loss, double* loss_history,
                             int32_t history_len, float* grad_micro, float* grad_cal, void* workspace,
                             size_t workspace_bytes, uint32_t* status, void* stream) {
  int rc = check_pass_args(h, y, theta_micro, theta_cal, loss, grad_micro, grad_cal, workspace,
                           workspace_bytes, status);
  if (rc != PRISM_OK) return rc;
  if (loss_history && history_len < 1) return fail(PRISM_E_INVALID, "history_len must be >= 1");
  if (!step || (h->n_micro && (!m_micro || !v_micro)) || (update_cal && (!m_cal || !v_cal)))
    return fail(PRISM_E_INVALID, "NULL device pointer");
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
    return fail(PRISM_E_INVALID, "Adam hyper-parameters out of range");
  hipStream_t s = (hipStream_t)stream;
  bool fuse = true;  // the continuity prior reads neighbours' parameters during the pass
  for (const GroupDev& g : h->groups)
    if ((g.priors & PRISM_PRIOR_CONTINUITY) && g.nbh > 0) fuse = false;
  if (fuse && !h->items.empty()) {
    // one call: the step counter advances in the first kernel, the per-voxel
    // parameters are updated in the fused pass, the calibration vector where
    // its gradient is written
    PassArgs ad{};
    ad.th_upd = theta_micro;
    ad.m_micro = m_micro;
    ad.v_micro = v_micro;
    ad.step = step;
    ad.lr = lr;
    ad.b1 = beta1;
    ad.b2 = beta2;
    ad.eps = eps;
    CalAdam ca{theta_cal, m_cal, v_cal, step, lr, beta1, beta2, eps, update_cal ? 1 : 0};
    const History hi{loss_history, step, history_len, 1};  // the first kernel advanced step[0]
    return run_pass(h, y, theta_micro, theta_cal, loss, grad_micro, grad_cal, workspace, status, s, &ad, &ca,
                    &hi);
  }
  if (fuse) {
    PassArgs ad{};
    ad.th_upd = theta_micro;
    ad.m_micro = m_micro;
    ad.v_micro = v_micro;
    ad.step = step;
    ad.lr = lr;
    ad.b1 = beta1;
    ad.b2 = beta2;
    ad.eps = eps;
    const History hi{loss_history, step, history_len, 0};  // advanced by the Adam launch below
    rc = run_pass(h, y, theta_micro, theta_cal, loss, grad_micro, grad_cal, workspace, status, s, &ad, nullptr,
                  &hi);
    if (rc != PRISM_OK) return rc;
  } else {
    const History hi{loss_history, step, history_len, 0};
    rc = run_pass(h, y, theta_micro, theta_cal, loss, grad_micro, grad_cal, workspace, status, s, nullptr,
                  nullptr, &hi);
    if (rc != PRISM_OK) return rc;
    hipError_t e = launch_adam(theta_micro, grad_micro, m_micro, v_micro, h->n_micro, lr, beta1, beta2, eps,
                               step, s, false);
    if (e != hipSuccess) return hip_fail(e, "Adam launch");
  }
  hipError_t e = launch_adam(theta_cal, grad_cal, m_cal, v_cal, update_cal ? h->n_cal : 0, lr, beta1, beta2,
                             eps, step, s, true);
  if (e != hipSuccess) return hip_fail(e, "Adam launch");
  return PRISM_OK;
}

int32_t prism_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                        float beta1, float beta2, float eps, int32_t* step, void* stream) {
  if (n < 0) return fail(PRISM_E_INVALID, "n must be >= 0");
  if (!step || (n > 0 && (!p || !g || !m || !v))) return fail(PRISM_E_INVALID, "NULL device pointer");
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
    return fail(PRISM_E_INVALID, "Adam hyper-parameters out of range");
  hipError_t e = launch_adam(p, g, m, v, n, lr, beta1, beta2, eps, step, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "Adam launch");
  return PRISM_OK;
}

int32_t prism_rprop_step(float* p, const float* g, float* prev, float* step, int64_t n,
                         float eta_minus, float eta_plus, float step_min, float step_max,
                         void* stream) {
  if (n < 0) return fail(PRISM_E_INVALID, "n must be >= 0");
  if (n > 0 && (!p || !g || !prev || !step)) return fail(PRISM_E_INVALID, "NULL device pointer");
  if (!(eta_minus > 0.0f && eta_minus < 1.0f) || !(eta_plus > 1.0f) || !(step_min >= 0.0f) ||
      !(step_max >= step_min))
    return fail(PRISM_E_INVALID, "Rprop hyper-parameters out of range");
  hipError_t e = launch_rprop(p, g, prev, step, n, eta_minus, eta_plus, step_min, step_max,
                              (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "Rprop launch");
  return PRISM_OK;
}

int32_t prism_rician_terms(const float* z, float* log_i0e, float* one_minus_ratio, float* q, int64_t n,
                           void* stream) {
  if (n < 0) return fail(PRISM_E_INVALID, "n must be >= 0");
  if (n > 0 && (!z || !log_i0e || !one_minus_ratio || !q)) return fail(PRISM_E_INVALID, "NULL device pointer");
  hipError_t e = launch_rician_terms(z, log_i0e, one_minus_ratio, q, n, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "special-function launch");
  return PRISM_OK;
}

int32_t prism_stitch_plan(prism_problem* h, int32_t nx, int32_t ny, int32_t nz, const int32_t* z0,
                          int64_t* n_out) {
  if (!h || !z0 || !n_out) return fail(PRISM_E_INVALID, "NULL argument");
  const int G = (int)h->groups.size();
  if (nx < 1 || ny < 1 || nz < 1 || nx > PRISM_MAX_EDGE || ny > PRISM_MAX_EDGE || nz > PRISM_MAX_EDGE)
    return fail(PRISM_E_INVALID, "volume edges must be in 1..1023");
  const GroupDev& g0 = h->groups[0];
  for (int g = 0; g < G; ++g) {
    const GroupDev& gd = h->groups[g];
    if (gd.nx != nx || gd.ny != ny) return fail(PRISM_E_INVALID, "slab %d: box %dx%d differs from the volume's %dx%d", g, gd.nx, gd.ny, nx, ny);
    if (gd.K != g0.K || gd.learn_d != g0.learn_d) return fail(PRISM_E_INVALID, "slab %d: K or learn_diffusivity differs", g);
    if (z0[g] < 0 || z0[g] + gd.nz > nz) return fail(PRISM_E_INVALID, "slab %d: slices %d..%d outside the volume", g, z0[g], z0[g] + gd.nz - 1);
    if (g > 0 && z0[g] <= z0[g - 1]) return fail(PRISM_E_INVALID, "slab starts must increase strictly");
    if (g > 1 && z0[g] < z0[g - 2] + h->groups[g - 2].nz) return fail(PRISM_E_INVALID, "slab %d: a slice lies in more than two slabs", g);
  }
  // blend weights per slab and slice: linear ramps over the overlaps
  std::vector<std::vector<float>> w(G);
  for (int g = 0; g < G; ++g) {
    const int a = z0[g], t = h->groups[g].nz;
    const int o_lo = g > 0 ? std::max(0, z0[g - 1] + h->groups[g - 1].nz - a) : 0;
    const int o_hi = g + 1 < G ? std::max(0, a + t - z0[g + 1]) : 0;
    w[g].assign((size_t)t, 1.0f);
    for (int k = 0; k < t; ++k) {
      double x = 1.0;
      if (o_lo) x = std::min(x, (k + 1.0) / (o_lo + 1.0));
      if (o_hi) x = std::min(x, (double)(t - k) / (o_hi + 1.0));
      w[g][(size_t)k] = (float)x;
    }
  }
  // up to two sources per raster position of the volume
  const size_t R = (size_t)nx * ny * nz;
  std::vector<int32_t> ag(R, -1), av(R, -1), bg(R, -1), bv(R, -1);
  for (int g = 0; g < G; ++g) {
    const GroupDev& gd = h->groups[g];
    for (int32_t v = 0; v < gd.V; ++v) {
      const int32_t pc = h->coords_host[(size_t)gd.vox_off + v];
      const size_t r = ((size_t)(pc & 1023) * ny + ((pc >> 10) & 1023)) * nz + z0[g] + ((pc >> 20) & 1023);
      if (ag[r] < 0) {
        ag[r] = g;
        av[r] = v;
      } else {
        bg[r] = g;
        bv[r] = v;
      }
    }
  }
  int64_t n = 0;
  for (size_t r = 0; r < R; ++r) n += ag[r] >= 0;
  std::vector<int32_t> sg((size_t)2 * n), sv((size_t)2 * n);
  std::vector<float> sw((size_t)2 * n);
  int64_t o = 0;
  for (size_t r = 0; r < R; ++r) {
    if (ag[r] < 0) continue;
    const int zk = (int)(r % nz);
    const float wa = w[ag[r]][(size_t)(zk - z0[ag[r]])];
    const float wb = bg[r] >= 0 ? w[bg[r]][(size_t)(zk - z0[bg[r]])] : 0.0f;
    sg[o] = ag[r];
    sv[o] = av[r];
    sg[n + o] = bg[r];
    sv[n + o] = bv[r];
    sw[o] = bg[r] >= 0 ? wa / (wa + wb) : 1.0f;
    sw[n + o] = bg[r] >= 0 ? wb / (wa + wb) : 0.0f;
    ++o;
  }
  h->free_stitch();
  hipError_t e = upload(&h->d_st_g, sg);
  if (e == hipSuccess) e = upload(&h->d_st_v, sv);
  if (e == hipSuccess) e = upload(&h->d_st_w, sw);
  if (e != hipSuccess) {
    h->free_stitch();
    return fail(PRISM_E_ALLOC, "device allocation failed: %s", hipGetErrorString(e));
  }
  h->st_n_out = n;
  h->st_planned = true;
  *n_out = n;
  return PRISM_OK;
}

int32_t prism_stitch_maps(const prism_problem* h, const float* theta_micro, float* maps, void* stream) {
  if (!h) return fail(PRISM_E_INVALID, "handle is NULL");
  if (!h->st_planned) return fail(PRISM_E_INVALID, "no stitch plan (call prism_stitch_plan first)");
  if (h->st_n_out == 0) return PRISM_OK;
  if (!theta_micro || !maps) return fail(PRISM_E_INVALID, "NULL device pointer");
  StitchArgs a{};
  a.groups = h->d_groups;
  a.src_g = h->d_st_g;
  a.src_v = h->d_st_v;
  a.src_w = h->d_st_w;
  a.th_micro = theta_micro;
  a.maps = maps;
  a.n_out = h->st_n_out;
  hipError_t e = launch_stitch(a, h->groups[0].K, h->groups[0].learn_d, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stitch launch");
  return PRISM_OK;
}

int32_t prism_profile_enable(prism_problem* h, int32_t enable, int32_t max_launches) {
  if (!h) return fail(PRISM_E_INVALID, "handle is NULL");
  for (auto e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
  h->ev_used = 0;
  h->prof = enable != 0;
  if (!h->prof) return PRISM_OK;
  if (max_launches < 1) return fail(PRISM_E_INVALID, "max_launches must be >= 1");
  h->ev.resize((size_t)max_launches * 2);
  for (auto& e : h->ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return hip_fail(r, "hipEventCreate");
  }
  return PRISM_OK;
}

int32_t prism_profile_read(prism_problem* h, double* total_ms, int32_t* launches) {
  if (!h || !total_ms || !launches) return fail(PRISM_E_INVALID, "NULL argument");
  double tot = 0.0;
  const int n = h->ev_used / 2;
  if (n > 0) {
    hipError_t r = hipEventSynchronize(h->ev[h->ev_used - 1]);
    if (r != hipSuccess) return hip_fail(r, "hipEventSynchronize");
  }
  for (int i = 0; i < n; ++i) {
    float ms = 0.0f;
    hipError_t r = hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]);
    if (r != hipSuccess) return hip_fail(r, "hipEventElapsedTime");
    tot += ms;
  }
  *total_ms = tot;
  *launches = n;
  h->ev_used = 0;
  return PRISM_OK;
}

}  // extern "C"
