// Host side of multi-stream batches (declarations and contract in
// include/chaosvid.h): one tick of many video streams as one keystream
// launch per generator variant and one persistent rounds launch per channel
// count, with every table the tick needs sent to the device in one copy.
//
// A tick is planned on the host:
//  - chains: every band generator of every item (Sec. 3, Eq. 5), with its
//    output placed in one keystream workspace shared by the tick; chains are
//    sorted by length so that a wavefront holds chains of similar length;
//  - jobs: one per (item, frame), assigned to groups of G workgroups longest
//    first, each to the group with the least work so far;
//  - shift tables of Eq. (1), one per frame.
// The tables are written into a pinned staging buffer (two, used in turn so
// that the host can plan tick t+1 while tick t runs) and copied to the device
// with one copy.  When the tick's structure repeats, the whole sequence --
// copy, keystream launches, rounds launches, error-flag read-back -- is
// replayed from a HIP graph captured the first time.
//
// Keystream prefetch (shape.prefetch): the keystream of a frame depends only
// on its key's generator state (Algorithm 2), so once a tick's keystream is
// generated (or adopted), the next tick's -- the same keys and frame counts,
// one tick on -- is generated on a private stream into the other of two
// keystream buffers while this tick's rounds run (on compute units that the
// rounds launches leave free for it when ticks are queued back to back).  It advances a shadow copy of the keys'
// generator states, made on the tick's stream right after the tick's
// keystream, so the prefetch never touches a key; a next tick that matches
// takes the keystream and copies the shadow states into the keys on its own
// stream, in the same launch that starts the following prefetch's shadow.
// A run of equal ticks thus costs max(keystream, rounds) per tick instead of
// their sum.  A tick that does not match generates its own keystream into
// the buffer the prefetch does not write, and the prefetched work is dropped.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include "runtime.h"

using namespace cv::rt;

namespace {

constexpr uint32_t kSpinLimit = 1u << 21;  // about two seconds of polling per barrier
// Frame jobs are launched in classes: by channel count (3, 4) and by whether
// the row-run kernel takes runs of 12 pixels per lane (W a multiple of 12)
// or of 4 -- class (C == 4) * 2 + (W % 12 != 0) -- except that a tick with
// jobs of both widths for one channel count launches them together, in
// class 4 + (C == 4), on the kernel that picks the run length per job (one
// launch instead of two: groups freed by one kind take jobs of the other).
constexpr int kClasses = 6;
int job_class(const cv::Geom& g) { return (g.C == 4 ? 2 : 0) + (g.W % 12 != 0 ? 1 : 0); }
uint32_t class_C(int c) { return c >= 4 ? (c == 5 ? 4u : 3u) : (c >= 2 ? 4u : 3u); }
uint32_t class_KQ(int c) { return c >= 4 ? 0u : (c & 1) ? 4u : 12u; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Everything that the launches of a tick take as arguments; two ticks with
// equal signatures enqueue the same work on different table contents.
struct Signature {
  size_t blob_bytes = 0;
  uint8_t* d_blob = nullptr;
  uint8_t* d_ks = nullptr;
  uint8_t* d_scratch = nullptr;
  uint32_t* d_counters = nullptr;
  uint32_t n_chains[cv::kPrbgVariants] = {};
  size_t chain_off[cv::kPrbgVariants] = {};
  uint32_t groups[kClasses] = {};  // per job class
  uint32_t n_slots[kClasses] = {};
  uint32_t G = 0, threads = 0, tile_cap = 0;
  bool rows[kClasses] = {};
  size_t lds[kClasses] = {};
  size_t job_off[kClasses] = {}, gj_off[kClasses] = {}, go_off[kClasses] = {}, sl_off[kClasses] = {};
  uint64_t scratch_stride = 0;
  bool operator==(const Signature& o) const {
    bool eq = blob_bytes == o.blob_bytes && d_blob == o.d_blob && d_ks == o.d_ks &&
              d_scratch == o.d_scratch && d_counters == o.d_counters && G == o.G &&
              threads == o.threads && tile_cap == o.tile_cap && scratch_stride == o.scratch_stride;
    for (int v = 0; v < cv::kPrbgVariants; v++) eq = eq && n_chains[v] == o.n_chains[v] && chain_off[v] == o.chain_off[v];
    for (int c = 0; c < kClasses; c++)
      eq = eq && groups[c] == o.groups[c] && n_slots[c] == o.n_slots[c] && rows[c] == o.rows[c] &&
           lds[c] == o.lds[c] && job_off[c] == o.job_off[c] && gj_off[c] == o.gj_off[c] &&
           go_off[c] == o.go_off[c] && sl_off[c] == o.sl_off[c];
    return eq;
  }
};

// One pinned staging buffer with the graph that copies from it.
struct Slot {
  uint8_t* h_blob = nullptr;
  size_t cap = 0;
  hipEvent_t copied = nullptr;  // the tick that read h_blob has copied it
  bool pending = false;
  hipGraphExec_t exec = nullptr;
  Signature sig;
  bool has_sig = false;
};

struct Span {
  hipEvent_t a, b;
  int kind;  // 0 = keystream, 1 = rounds
  uint64_t work;
};

// The keystream prefetch of one batch.  Generator states advance in one of
// two shadow buffers, used in turn by successive prefetches; keystream goes
// to the keystream buffer the tick does not use.
struct Prefetch {
  struct Entry {
    const cv_key* k;
    uint64_t serial, epoch, frame_index;  // the key as the next tick must find it
    uint32_t n_frames;
    uint64_t ks_off;     // its keystream in the prefetch's keystream buffer
    uint64_t state_off;  // its generator states in the prefetch's shadow buffer (doubles)
  };
  SideStreams side;                    // private streams (default priority)
  hipEvent_t ks_ready = nullptr;       // tick's stream: keystream generated or adopted, states copied
  hipEvent_t done[2] = {};             // per shadow buffer: the last prefetch using it is complete
  bool used[2] = {};
  hipEvent_t copied = nullptr;         // the chain-table copy has read h_table
  bool copy_pending = false;
  uint8_t* h_table = nullptr;          // pinned chain tables
  size_t h_cap = 0;
  uint8_t* d_table = nullptr;
  size_t d_cap = 0;
  uint8_t* d_shadow[2] = {};
  size_t shadow_cap[2] = {};
  std::vector<Entry> entries;
  bool valid = false;  // entries describe the last prefetch launched
  int target = -1;     // keystream buffer of the last prefetch launched (-1: none yet)
  int shadow = -1;     // its shadow buffer
};

// The next prefetch, planned before the tick that launches it.
struct NextPrefetch {
  std::vector<Prefetch::Entry> entries;
  std::vector<cv::PlcmChain> chains[cv::kPrbgVariants];
  std::vector<cv::StateCopy> gather;  // generator states into the shadow buffer
  int target = 0, shadow = 0;
  uint64_t steps = 0;
  uint32_t workgroups = 0;
};

}  // namespace

struct cv_batch {
  int device = 0;
  cv_batch_shape shape{1024, 8, 0, 1, 0, 1};
  size_t lds_max = 0;
  hipStream_t cap = nullptr;  // private stream that graphs are captured on
  std::array<Slot, 2> slot;
  uint32_t turn = 0;
  uint8_t* d_blob = nullptr;
  size_t blob_cap = 0;
  uint32_t reserve_cus = 0;  // compute units per XCD the rounds launches leave to others
  uint8_t* d_ks[2] = {};  // keystream buffers: a tick's and a prefetch's
  size_t ks_cap[2] = {};
  Prefetch pf;
  uint8_t* d_scratch = nullptr;
  size_t scratch_cap = 0;
  uint32_t* d_counters = nullptr;
  size_t counters_cap = 0;  // groups
  uint32_t* d_err = nullptr;
  uint32_t* h_err = nullptr;  // pinned copy of d_err, written at the end of every tick
  bool failed = false;        // a tick timed out: d_err stays set
  hipEvent_t done = nullptr;  // end of the last tick
  hipStream_t last_stream = nullptr;
  bool ran = false;
  cv_batch_info info{};
  bool profiling = false;
  std::vector<Span> spans;
  std::vector<hipEvent_t> event_pool;
  cv_profile prof{};
};

namespace {

// ------------------------------------------------------------ the plan ---
struct Plan {
  std::vector<cv::PlcmChain> chains[cv::kPrbgVariants];  // by generator variant
  std::vector<cv::BatchJob> jobs[kClasses];  // by job class; ks and gm hold offsets until fill_blob
  std::vector<uint32_t> group_jobs[kClasses], group_off[kClasses];
  std::vector<uint32_t> gm;              // shift tables of every frame job
  std::vector<cv::StateCopy> copies;     // generator-state copies of the tick's hooks
  uint32_t reserve_cus = 0;              // compute units per XCD the rounds leave free
  uint64_t scratch_stride = 0;
  uint32_t groups[kClasses] = {};
  uint32_t wide[kClasses] = {};           // groups larger than the shape's G
  std::vector<uint32_t> slots[kClasses];  // per workgroup of the launch (cv::batch_slot)
  bool rows[kClasses] = {};  // the row-run kernel (else the pixel-word one)
  size_t lds[kClasses] = {};
  uint64_t steps = 0, frame_rounds = 0;
};

cv_status check_items(const cv_batch* b, const cv_batch_item* items, size_t n_items) {
  if (n_items && !items) return fail(CV_E_INVAL, "items is NULL");
  struct Range {
    uintptr_t lo, hi;
    bool out;
  };
  std::vector<Range> ranges;
  std::vector<const cv_key*> keys;
  for (size_t i = 0; i < n_items; i++) {
    const cv_batch_item& it = items[i];
    if (!it.key) return fail(CV_E_INVAL, "item key is NULL");
    if (it.n_frames == 0) continue;
    if (it.key->device != b->device) return fail(CV_E_INVAL, "item key lives on another device");
    if (it.decrypt != 0 && it.decrypt != 1) return fail(CV_E_INVAL, "item decrypt must be 0 or 1");
    cv_status s = check_frames_args(it.key, it.in, it.out, it.s_c, it.n_frames);
    if (s != CV_OK) return s;
    // one keystream launch covers the item's frames: a chain's steps must fit 31 bits
    for (const cv::PlcmChain& c : it.key->h_chains)
      if ((c.nbytes + 5) / 6 * (uint64_t)it.n_frames >= (1ull << 31))
        return fail(CV_E_INVAL, "too many frames of one stream in one tick");
    const uint64_t bytes = (uint64_t)it.n_frames * it.key->F;
    ranges.push_back({(uintptr_t)it.in, (uintptr_t)it.in + bytes, false});
    ranges.push_back({(uintptr_t)it.out, (uintptr_t)it.out + bytes, true});
    keys.push_back(it.key);
  }
  std::sort(keys.begin(), keys.end());
  if (std::adjacent_find(keys.begin(), keys.end()) != keys.end())
    return fail(CV_E_INVAL, "a key appears in more than one item of the tick");
  // an output may overlap nothing; inputs may overlap each other
  std::sort(ranges.begin(), ranges.end(), [](const Range& x, const Range& y) { return x.lo < y.lo; });
  uintptr_t end_all = 0, end_out = 0;
  for (const Range& r : ranges) {
    if ((r.out && r.lo < end_all) || (!r.out && r.lo < end_out))
      return fail(CV_E_INVAL, "an output buffer overlaps another buffer of the tick");
    end_all = std::max(end_all, r.hi);
    if (r.out) end_out = std::max(end_out, r.hi);
  }
  return CV_OK;
}

// A job as the planner sees it: work of one band-round (r rounds of at most
// max_band_rows rows of W pixels) and its band count.
struct JobLoad {
  uint64_t unit;
  uint32_t n, job;
  // on the critical path of a group of G: r rounds of ceil(n/G) bands
  uint64_t cost(uint32_t G) const { return unit * ((n + G - 1) / G); }
};

// One group of a launch: its XCD, its first slot there and its size.
struct GroupDesc {
  uint32_t xcd, first, G;
};

// Groups of the XCDs' `slots` workgroups each: `nb` groups of size B spread
// over the XCDs (at most slots/B on one), every other slot in groups of G0;
// listed XCD by XCD in turn, so that consecutive groups sit on different XCDs.
std::vector<GroupDesc> partition(uint32_t slots, uint32_t G0, uint32_t nb, uint32_t B) {
  std::vector<GroupDesc> per[8];
  for (uint32_t x = 0; x < 8; x++) {
    uint32_t s = 0;
    for (uint32_t q = x; q < nb && s + B <= slots; q += 8, s += B) per[x].push_back({x, s, B});
    for (; s + G0 <= slots; s += G0) per[x].push_back({x, s, G0});
  }
  std::vector<GroupDesc> out;
  for (size_t k = 0;; k++) {
    const size_t before = out.size();
    for (uint32_t x = 0; x < 8; x++)
      if (k < per[x].size()) out.push_back(per[x][k]);
    if (out.size() == before) break;
  }
  return out;
}

// Longest job first onto the group where it would finish first; returns the
// largest group load and each job's group in `where`.
uint64_t place(const std::vector<JobLoad>& order, const std::vector<GroupDesc>& groups,
               std::vector<uint32_t>* where) {
  std::vector<uint64_t> load(groups.size(), 0);
  uint64_t span = 0;
  if (where) where->assign(order.size(), 0);
  for (size_t j = 0; j < order.size(); j++) {
    size_t best = 0;
    uint64_t best_end = ~0ull;
    for (size_t q = 0; q < groups.size(); q++) {
      const uint64_t end = load[q] + order[j].cost(groups[q].G);
      if (end < best_end) {
        best_end = end;
        best = q;
      }
    }
    load[best] = best_end;
    span = std::max(span, best_end);
    if (where) (*where)[j] = (uint32_t)best;
  }
  return span;
}

// Longest chains first, so that a wavefront holds chains of similar length.
void sort_chains(std::vector<cv::PlcmChain> (&chains)[cv::kPrbgVariants]) {
  for (auto& cs : chains)
    std::stable_sort(cs.begin(), cs.end(), [](const cv::PlcmChain& x, const cv::PlcmChain& y) {
      return x.nbytes * x.frames > y.nbytes * y.frames;
    });
}

// Tables of one tick: the chains of `cj` and the frame jobs of `fj`.
cv_status plan_tick(const cv_batch* b, const std::vector<ChainJob>& cj,
                    const std::vector<FrameJob>& fj, Plan& P) {
  const uint32_t G = b->shape.group_wgs, threads = b->shape.threads;
  for (const ChainJob& c : cj) {
    const int v = prbg_variant(c.k);
    for (const cv::PlcmChain& c0 : c.k->h_chains) {
      cv::PlcmChain ch = c0;
      ch.out_off = c.ks_off + c0.out_off;
      ch.frame_stride = c.frame_stride ? c.frame_stride : c0.frame_stride;
      ch.frames = c.frames;
      P.chains[v].push_back(ch);
    }
    P.steps += prbg_steps(c.k, c.frames);
  }
  sort_chains(P.chains);
  uint64_t gm = 0, pwf_max = 0;
  for (const FrameJob& f : fj) {
    gm += f.k->g.H;
    pwf_max = std::max<uint64_t>(pwf_max, (uint64_t)f.k->g.H * f.k->g.W * 4);
  }
  P.scratch_stride = align_up(pwf_max, 256);
  P.gm.resize(gm);
  gm = 0;
  std::vector<JobLoad> order[kClasses];  // per class
  // both widths of one channel count in this tick: one launch for them
  bool kind[kClasses] = {};
  for (const FrameJob& f : fj) kind[job_class(f.k->g)] = true;
  const bool merge[2] = {kind[0] && kind[1], kind[2] && kind[3]};
  auto class_of = [&](const Geom& g) {
    const int c = job_class(g);
    return merge[c / 2] ? 4 + c / 2 : c;
  };
  // the row-run kernel takes a class's jobs when it takes every one
  bool rows_ok[kClasses];
  for (bool& x : rows_ok) x = threads == 1024;
  size_t lds_pw[kClasses] = {}, lds_rows[kClasses] = {};
  for (const FrameJob& f : fj) {
    const Geom& g = f.k->g;
    shift_table(g.H, g.W, f.s_c, P.gm.data() + gm);
    const int ci = class_of(g);
    // the LDS tiling: the largest tiles that fit, capped by the shape
    const uint32_t cap = b->shape.tile_rows_max ? b->shape.tile_rows_max : 0xFFFFFFFFu;
    const uint32_t tile = std::min(pw_tile_rows(g, threads, b->lds_max), cap);
    if (tile == 0) return fail(CV_E_INVAL, "frame too wide for the batch's workgroup size");
    lds_pw[ci] = std::max(lds_pw[ci], cv::round_pw_lds_bytes(g, tile));
    const uint32_t te = std::min(cv::rounds_skew_tile_rows(g, b->lds_max), cap);
    const uint32_t td = std::min(cv::batch_unskew_tile_rows(g, b->lds_max), cap);
    rows_ok[ci] = rows_ok[ci] && te > 0 && td > 0;
    if (rows_ok[ci])
      lds_rows[ci] = std::max(lds_rows[ci], cv::batch_rows_lds_bytes(g, f.decrypt != 0, f.decrypt ? td : te));
    cv::BatchJob J{};
    J.in = f.in;
    J.out = f.out;
    J.in_last = f.in_last;
    // offsets of the keystream (from the tick's base) and of the shift table (from the
    // table area), turned into device addresses by fill_blob
    J.ks = (const uint8_t*)(uintptr_t)f.ks_off;
    J.gm = (const uint32_t*)(uintptr_t)(gm * 4);
    J.g = g;
    J.decrypt = f.decrypt;
    J.tile_rows = tile;
    J.tile_enc = te;
    J.tile_dec = td;
    order[ci].push_back({(uint64_t)g.r * f.k->max_band_rows * g.W, g.n, (uint32_t)P.jobs[ci].size()});
    P.jobs[ci].push_back(J);
    P.frame_rounds += g.r;
    gm += g.H;
  }
  // per job class: the groups (sizes chosen for the tick's jobs) and the
  // jobs on them, longest first onto the group where each finishes first
  for (int ci = 0; ci < kClasses; ci++) {
    if (P.jobs[ci].empty()) continue;
    P.rows[ci] = rows_ok[ci];
    P.lds[ci] = rows_ok[ci] ? lds_rows[ci] : lds_pw[ci];
    const uint32_t slots = cv::batch_resident_slots(class_C(ci), class_KQ(ci), P.rows[ci], threads,
                                                    P.lds[ci], b->device, P.reserve_cus, G);
    if (slots < G) return fail(CV_E_INVAL, "batch launch shape does not fit on the device");
    std::vector<JobLoad>& ord = order[ci];
    std::stable_sort(ord.begin(), ord.end(),
                     [G](const JobLoad& x, const JobLoad& y) { return x.cost(G) > y.cost(G); });
    std::vector<GroupDesc> groups = partition(slots, G, 0, G);
    if (b->shape.max_groups) {
      // fixed shape: groups of G only, at most max_groups of them
      groups.resize(std::min<size_t>(groups.size(), b->shape.max_groups));
    } else {
      // larger groups for jobs with more bands than G, when that shortens the tick
      uint32_t wide = 0;
      for (const JobLoad& o : ord) wide += o.n > G;
      uint64_t best = place(ord, groups, nullptr);
      for (uint32_t B = 2 * G; B <= slots && wide; B += G) {
        for (uint32_t nb = 1; nb <= std::min(wide, 8 * (slots / B)); nb++) {
          std::vector<GroupDesc> cand = partition(slots, G, nb, B);
          const uint64_t span = place(ord, cand, nullptr);
          if (span < best) {
            best = span;
            groups = std::move(cand);
          }
        }
      }
    }
    std::vector<uint32_t> where;
    place(ord, groups, &where);
    // groups that received jobs, renumbered in order
    std::vector<std::vector<uint32_t>> per(groups.size());
    for (size_t q = 0; q < ord.size(); q++) per[where[q]].push_back(ord[q].job);
    std::vector<uint32_t> id(groups.size(), cv::kIdleSlot);
    uint32_t used = 0;
    P.group_off[ci].push_back(0);
    for (size_t q = 0; q < groups.size(); q++) {
      if (per[q].empty()) continue;
      id[q] = used++;
      P.wide[ci] += groups[q].G > G;
      P.group_jobs[ci].insert(P.group_jobs[ci].end(), per[q].begin(), per[q].end());
      P.group_off[ci].push_back((uint32_t)P.group_jobs[ci].size());
    }
    P.groups[ci] = used;
    P.slots[ci].assign(8 * slots, cv::kIdleSlot);
    for (size_t q = 0; q < groups.size(); q++) {
      if (id[q] == cv::kIdleSlot) continue;
      for (uint32_t w = 0; w < groups[q].G; w++)
        P.slots[ci][8 * (groups[q].first + w) + groups[q].xcd] = cv::batch_slot(id[q], w, groups[q].G);
    }
  }
  return CV_OK;
}

// --------------------------------------------------------- workspace ---
cv_status grow(uint8_t** p, size_t* cap, size_t want, const char* what) {
  if (want <= *cap) return CV_OK;
  CV_HIP(hipDeviceSynchronize());  // the old buffer may still be in use
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  const size_t sz = align_up(want + want / 4, 1 << 20);
  if (hipMalloc(p, sz) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(CV_E_NOMEM, std::string(what) + " allocation failed");
  }
  *cap = sz;
  return CV_OK;
}

void drop_graphs(cv_batch* b) {
  for (Slot& s : b->slot) {
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    s.exec = nullptr;
    s.has_sig = false;
  }
}

// Layout of the blob: chains (3 variants), jobs, group tables, shift tables.
struct Layout {
  size_t chain_off[cv::kPrbgVariants], job_off[kClasses], gj_off[kClasses], go_off[kClasses],
      sl_off[kClasses], gm_off, copies_off, bytes;
};

Layout layout(const Plan& P) {
  Layout L{};
  size_t o = 0;
  for (int v = 0; v < cv::kPrbgVariants; v++) {
    L.chain_off[v] = o;
    o = align_up(o + P.chains[v].size() * sizeof(cv::PlcmChain), 16);
  }
  for (int c = 0; c < kClasses; c++) {
    L.job_off[c] = o;
    o = align_up(o + P.jobs[c].size() * sizeof(cv::BatchJob), 16);
    L.gj_off[c] = o;
    o = align_up(o + P.group_jobs[c].size() * 4, 16);
    L.go_off[c] = o;
    o = align_up(o + P.group_off[c].size() * 4, 16);
    L.sl_off[c] = o;
    o = align_up(o + P.slots[c].size() * 4, 16);
  }
  L.gm_off = o;
  o = align_up(o + P.gm.size() * 4, 16);
  L.copies_off = o;
  L.bytes = align_up(o + P.copies.size() * sizeof(cv::StateCopy), 256);
  return L;
}

cv_status ensure_pinned(Slot& s, size_t bytes) {
  if (bytes <= s.cap) return CV_OK;
  if (s.pending) {
    CV_HIP(hipEventSynchronize(s.copied));
    s.pending = false;
  }
  if (s.h_blob) (void)hipHostFree(s.h_blob);
  s.h_blob = nullptr;
  s.cap = 0;
  const size_t sz = align_up(bytes + bytes / 4, 1 << 16);
  if (hipHostMalloc(&s.h_blob, sz) != hipSuccess) {
    (void)hipGetLastError();
    s.h_blob = nullptr;
    return fail(CV_E_NOMEM, "pinned staging allocation failed");
  }
  s.cap = sz;
  if (s.exec) (void)hipGraphExecDestroy(s.exec);  // it copies from the old buffer
  s.exec = nullptr;
  s.has_sig = false;
  return CV_OK;
}

// Write the tables into the slot's staging buffer with device addresses.
void fill_blob(const cv_batch* b, const Plan& P, const Layout& L, uint8_t* h,
               const uint8_t* ks_base) {
  for (int v = 0; v < cv::kPrbgVariants; v++)
    if (!P.chains[v].empty())
      memcpy(h + L.chain_off[v], P.chains[v].data(), P.chains[v].size() * sizeof(cv::PlcmChain));
  const uint8_t* d_gm = b->d_blob + L.gm_off;
  for (int c = 0; c < kClasses; c++) {
    cv::BatchJob* J = (cv::BatchJob*)(h + L.job_off[c]);
    for (size_t q = 0; q < P.jobs[c].size(); q++) {
      J[q] = P.jobs[c][q];
      J[q].ks = (const uint8_t*)((uintptr_t)ks_base + (uintptr_t)P.jobs[c][q].ks);
      J[q].gm = (const uint32_t*)(d_gm + (uintptr_t)P.jobs[c][q].gm);
    }
    if (!P.group_jobs[c].empty())
      memcpy(h + L.gj_off[c], P.group_jobs[c].data(), P.group_jobs[c].size() * 4);
    if (!P.group_off[c].empty())
      memcpy(h + L.go_off[c], P.group_off[c].data(), P.group_off[c].size() * 4);
    if (!P.slots[c].empty()) memcpy(h + L.sl_off[c], P.slots[c].data(), P.slots[c].size() * 4);
  }
  if (!P.gm.empty()) memcpy(h + L.gm_off, P.gm.data(), P.gm.size() * 4);
  if (!P.copies.empty()) memcpy(h + L.copies_off, P.copies.data(), P.copies.size() * sizeof(cv::StateCopy));
}

Signature signature(const cv_batch* b, const Plan& P, const Layout& L, uint8_t* ks_base) {
  Signature s;
  s.blob_bytes = L.bytes;
  s.d_blob = b->d_blob;
  s.d_ks = ks_base;
  s.d_scratch = b->d_scratch;
  s.d_counters = b->d_counters;
  for (int v = 0; v < cv::kPrbgVariants; v++) {
    s.n_chains[v] = (uint32_t)P.chains[v].size();
    s.chain_off[v] = L.chain_off[v];
  }
  for (int c = 0; c < kClasses; c++) {
    s.groups[c] = P.groups[c];
    s.n_slots[c] = (uint32_t)P.slots[c].size();
    s.sl_off[c] = L.sl_off[c];
    s.rows[c] = P.rows[c];
    s.lds[c] = P.lds[c];
    s.job_off[c] = L.job_off[c];
    s.gj_off[c] = L.gj_off[c];
    s.go_off[c] = L.go_off[c];
  }
  s.G = b->shape.group_wgs;
  s.threads = b->shape.threads;
  s.tile_cap = b->shape.tile_rows_max;
  s.scratch_stride = P.scratch_stride;
  return s;
}

hipEvent_t pooled(cv_batch* b) {
  if (!b->event_pool.empty()) {
    hipEvent_t e = b->event_pool.back();
    b->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

cv_status drain(cv_batch* b) {
  for (Span& sp : b->spans) {
    CV_HIP(hipEventSynchronize(sp.b));
    float ms = 0.f;
    CV_HIP(hipEventElapsedTime(&ms, sp.a, sp.b));
    if (sp.kind == 0) {
      b->prof.prbg_ms += ms;
      b->prof.prbg_launches++;
      b->prof.prbg_steps += sp.work;
    } else {
      b->prof.round_ms += ms;
      b->prof.round_launches++;
      b->prof.round_frames += sp.work;
    }
    b->event_pool.push_back(sp.a);
    b->event_pool.push_back(sp.b);
  }
  b->spans.clear();
  return CV_OK;
}

// Enqueue the tick (copy, launches, flag read-back) on stream st.  With
// `timed`, every launch is bracketed by events (not allowed while capturing).
cv_status enqueue_tick(cv_batch* b, const Plan& P, const Layout& L, const Slot& s, hipStream_t st,
                       bool timed, uint8_t* ks_base, const TickHooks* hooks = nullptr) {
  CV_HIP(hipMemcpyAsync(b->d_blob, s.h_blob, L.bytes, hipMemcpyHostToDevice, st));
  bool has_chains = false;
  for (const auto& cs : P.chains) has_chains = has_chains || !cs.empty();
  bool has_jobs = false;
  for (const auto& js : P.jobs) has_jobs = has_jobs || !js.empty();
  hipEvent_t ta = nullptr;
  if (timed && has_chains && (ta = pooled(b))) CV_HIP(hipEventRecord(ta, st));
  for (int v = 0; v < cv::kPrbgVariants; v++)
    if (!P.chains[v].empty())
      CV_HIP(cv::launch_prbg_plcm((const cv::PlcmChain*)(b->d_blob + L.chain_off[v]),
                                  (uint32_t)P.chains[v].size(), ks_base, 0, v, st));
  if (ta) {
    hipEvent_t tb = pooled(b);
    if (tb) {
      CV_HIP(hipEventRecord(tb, st));
      b->spans.push_back({ta, tb, 0, P.steps});
    }
  }
  if (hooks) {
    for (hipEvent_t e : hooks->waits) CV_HIP(hipStreamWaitEvent(st, e, 0));
    CV_HIP(cv::launch_copy_states((const cv::StateCopy*)(b->d_blob + L.copies_off),
                                  (uint32_t)P.copies.size(), st));
    if (hooks->ks_ready) CV_HIP(hipEventRecord(hooks->ks_ready, st));
  }
  ta = nullptr;
  if (timed && has_jobs && (ta = pooled(b))) CV_HIP(hipEventRecord(ta, st));
  for (int c = 0; c < kClasses; c++) {
    if (P.jobs[c].empty()) continue;
    cv::BatchArgs a{};
    a.jobs = (const cv::BatchJob*)(b->d_blob + L.job_off[c]);
    a.group_jobs = (const uint32_t*)(b->d_blob + L.gj_off[c]);
    a.group_off = (const uint32_t*)(b->d_blob + L.go_off[c]);
    a.slots = (const uint32_t*)(b->d_blob + L.sl_off[c]);
    a.n_slots = (uint32_t)P.slots[c].size();
    a.scratch = b->d_scratch;
    a.scratch_stride = P.scratch_stride;
    a.counters = b->d_counters;
    a.err = b->d_err;
    a.groups = P.groups[c];
    a.spin_limit = kSpinLimit;
    CV_HIP(cv::launch_batch_rounds(a, class_C(c), class_KQ(c), P.rows[c], b->shape.threads, P.lds[c], st));
  }
  if (ta) {
    hipEvent_t tb = pooled(b);
    if (tb) {
      CV_HIP(hipEventRecord(tb, st));
      b->spans.push_back({ta, tb, 1, P.frame_rounds});
    }
  }
  CV_HIP(hipMemcpyAsync(b->h_err, b->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  return CV_OK;
}

// A tick that timed out at a group barrier (or found a group spread over
// XCDs) set the flag; the copy at the end of every tick brings it back.
cv_status check_flag(cv_batch* b, bool wait) {
  if (b->failed) return fail(CV_E_HIP, "an earlier tick of this batch timed out at a group barrier");
  if (!b->ran) return CV_OK;
  if (wait) {
    CV_HIP(hipEventSynchronize(b->done));
  } else if (hipEventQuery(b->done) != hipSuccess) {
    (void)hipGetLastError();
    return CV_OK;
  }
  if (*b->h_err) {
    b->failed = true;
    return fail(CV_E_HIP,
                "a batch tick timed out at a group barrier or found a group spread over XCDs; "
                "its output is invalid");
  }
  return CV_OK;
}

cv_status prepare(cv_batch* b, const std::vector<ChainJob>& cj, const std::vector<FrameJob>& fj,
                  Plan& P, Layout& L, const TickHooks* hooks = nullptr) {
  if (hooks) P.copies = hooks->copies;
  P.reserve_cus = std::max(b->reserve_cus, hooks ? hooks->reserve_cus : 0u);
  cv_status s = plan_tick(b, cj, fj, P);
  if (s != CV_OK) return s;
  L = layout(P);
  const uint32_t gmax = *std::max_element(P.groups, P.groups + kClasses);
  if ((s = grow(&b->d_blob, &b->blob_cap, L.bytes, "batch table")) != CV_OK) return s;
  if ((s = grow(&b->d_scratch, &b->scratch_cap, std::max<uint64_t>(2 * P.scratch_stride * gmax, 256),
                "batch scratch")) != CV_OK)
    return s;
  size_t cbytes = b->counters_cap * 128;
  if ((s = grow((uint8_t**)&b->d_counters, &cbytes, 128ull * std::max<uint32_t>(gmax, 8),
                "batch counters")) != CV_OK)
    return s;
  b->counters_cap = cbytes / 128;
  return CV_OK;
}

// Order this call's stream after the batch's previous tick.
cv_status order_after_last(cv_batch* b, hipStream_t st) {
  if (b->ran && st != b->last_stream) CV_HIP(hipStreamWaitEvent(st, b->done, 0));
  return CV_OK;
}

// Staging slot for the next tick, free for the host to write.
cv_status next_slot(cv_batch* b, size_t bytes, Slot** out) {
  Slot& sl = b->slot[b->turn];
  b->turn ^= 1;
  cv_status s = ensure_pinned(sl, bytes);
  if (s != CV_OK) return s;
  if (sl.pending) {  // the tick before last may still be copying from this buffer
    CV_HIP(hipEventSynchronize(sl.copied));
    sl.pending = false;
  }
  *out = &sl;
  return CV_OK;
}

// Capture the tick into the slot's graph (when its signature changed) and launch it.
cv_status launch_graph(cv_batch* b, const Plan& P, const Layout& L, Slot& sl, uint8_t* ks_base,
                       hipStream_t st) {
  const Signature sig = signature(b, P, L, ks_base);
  if (!(sl.has_sig && sl.sig == sig)) {
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    sl.exec = nullptr;
    sl.has_sig = false;
    CV_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    cv_status s = enqueue_tick(b, P, L, sl, b->cap, false, ks_base);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &graph);
    if (s != CV_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&sl.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      sl.exec = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    sl.sig = sig;
    sl.has_sig = true;
    b->info.graph_captures++;
  } else {
    b->info.graph_replays++;
  }
  CV_HIP(hipGraphLaunch(sl.exec, st));
  return CV_OK;
}

// Items outside the pixel-word conditions run on their key's own path.
// (2DLASM keys too: the batched keystream launch runs PLCM generators only.)
bool item_eligible(const cv_batch* b, const cv_batch_item& it) {
  return it.key->map == CV_MAP_PLCM &&
         pw_eligible(it.key, it.in, it.out, b->shape.threads, b->lds_max);
}

// Chains and frame jobs of the items that take the batched kernels, with
// their keystream laid out item after item from offset 0; the others are
// listed in `fallback`.
void collect(const cv_batch* b, const cv_batch_item* items, size_t n_items,
             std::vector<ChainJob>& cj, std::vector<FrameJob>& fj, std::vector<size_t>& fallback,
             std::vector<size_t>& eligible, uint64_t& ks) {
  ks = 0;
  for (size_t i = 0; i < n_items; i++) {
    const cv_batch_item& it = items[i];
    if (it.n_frames == 0) continue;
    if (!item_eligible(b, it)) {
      fallback.push_back(i);
      continue;
    }
    eligible.push_back(i);
    const cv_key* k = it.key;
    const uint64_t rF = (uint64_t)k->g.r * k->F;
    cj.push_back({k, ks, 0, it.n_frames});
    for (uint32_t t = 0; t < it.n_frames; t++)
      fj.push_back({k, it.in + (uint64_t)t * k->F, it.out + (uint64_t)t * k->F,
                    it.in + (uint64_t)it.n_frames * k->F - 4, ks + t * rF, it.s_c[t],
                    (uint32_t)it.decrypt});
    ks += it.n_frames * rF;
  }
}

// Grow keystream buffer `i`; a prefetch that wrote the old buffer is lost.
cv_status grow_ks(cv_batch* b, int i, uint64_t bytes) {
  const uint8_t* old = b->d_ks[i];
  cv_status s = grow(&b->d_ks[i], &b->ks_cap[i], std::max<uint64_t>(bytes, 16), "batch keystream");
  if (b->d_ks[i] != old && b->pf.target == i) b->pf.valid = false;
  return s;
}

cv_status ensure_prefetch(cv_batch* b) {
  Prefetch& pf = b->pf;
  hipError_t e = hipSuccess;
  for (hipEvent_t* ev : {&pf.ks_ready, &pf.done[0], &pf.done[1], &pf.copied})
    if (e == hipSuccess && !*ev) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "prefetch events");
  return CV_OK;
}

// Does the tick take the prefetched keystream?  Every batched item's key
// must be one the prefetch covered, unchanged since (same key object, state
// not set from outside, same frame index), with the frame count predicted,
// and no key covered may be missing.  `prev` receives each item's entry.
bool prefetch_matches(const cv_batch* b, const cv_batch_item* items,
                      const std::vector<size_t>& eligible, std::vector<const Prefetch::Entry*>* prev) {
  const Prefetch& pf = b->pf;
  if (!pf.valid || pf.entries.size() != eligible.size()) return false;
  std::map<const cv_key*, const Prefetch::Entry*> by_key;
  for (const Prefetch::Entry& e : pf.entries) by_key[e.k] = &e;
  prev->clear();
  for (size_t i : eligible) {
    const cv_batch_item& it = items[i];
    const auto f = by_key.find(it.key);
    if (f == by_key.end()) return false;
    const Prefetch::Entry& e = *f->second;
    if (e.serial != it.key->serial || e.epoch != it.key->state_epoch ||
        e.frame_index != it.key->frame_index || e.n_frames != it.n_frames)
      return false;
    prev->push_back(&e);
  }
  return true;
}

// Plan the prefetch that follows this tick: the same items one tick on, into
// keystream buffer `target`.  Its generator states start as copies made on
// the tick's stream after the tick's keystream: from the keys, or on a tick
// that takes a prefetch (`prev`), from that prefetch's shadow states, which
// the same launch copies into the keys.  False when its memory cannot be had.
bool plan_prefetch(cv_batch* b, const cv_batch_item* items, const std::vector<size_t>& eligible,
                   const std::vector<const Prefetch::Entry*>* prev, int target, NextPrefetch& np) {
  Prefetch& pf = b->pf;
  np.target = target;
  np.shadow = pf.shadow == 0 ? 1 : 0;
  uint64_t ks = 0, states = 0;
  for (size_t i : eligible) {
    const cv_batch_item& it = items[i];
    const cv_key* k = it.key;
    np.entries.push_back({k, k->serial, k->state_epoch, k->frame_index + it.n_frames, it.n_frames, ks,
                          states});
    ks += it.n_frames * (uint64_t)k->g.r * k->F;
    states += 2ull * k->g.n;
  }
  if (grow_ks(b, target, ks) != CV_OK ||
      grow(&pf.d_shadow[np.shadow], &pf.shadow_cap[np.shadow], std::max<uint64_t>(states * 8, 256),
           "prefetch states") != CV_OK)
    return false;
  double* sh = (double*)pf.d_shadow[np.shadow];
  const double* from = prev ? (const double*)pf.d_shadow[pf.shadow] : nullptr;
  for (size_t j = 0; j < np.entries.size(); j++) {
    const Prefetch::Entry& e = np.entries[j];
    const cv_key* k = e.k;
    const uint64_t nd = 2ull * k->g.n;
    np.gather.push_back({prev ? from + (*prev)[j]->state_off : k->d_state, sh + e.state_off, nd});
    const int v = prbg_variant(k);
    for (const cv::PlcmChain& c0 : k->h_chains) {
      cv::PlcmChain ch = c0;
      ch.state = sh + e.state_off + (c0.state - k->d_state);
      ch.out_off = e.ks_off + c0.out_off;
      ch.frames = e.n_frames;
      np.chains[v].push_back(ch);
    }
    np.steps += prbg_steps(k, e.n_frames);
  }
  sort_chains(np.chains);
  for (int v = 0; v < cv::kPrbgVariants; v++)
    np.workgroups += cv::prbg_plcm_workgroups((uint32_t)np.chains[v].size(), v);
  return true;
}

// Launch the planned prefetch on the private stream beside the tick's
// stream st: its chain tables go up (after the previous prefetch, which read
// the same device table: the same stream, or its completion event), then its
// keystream launches wait for the tick's stream to have its keystream and
// the shadow states (pf.ks_ready).
cv_status launch_prefetch(cv_batch* b, NextPrefetch& np, hipStream_t st) {
  Prefetch& pf = b->pf;
  const hipStream_t prev = pf.side.last;
  hipStream_t ps = nullptr;
  cv_status ss = side_stream(pf.side, b->device, st, &ps);
  if (ss != CV_OK) return ss;
  if (prev && prev != ps && pf.shadow >= 0 && pf.used[pf.shadow])
    CV_HIP(hipStreamWaitEvent(ps, pf.done[pf.shadow], 0));
  size_t chain_off[cv::kPrbgVariants], bytes = 0;
  for (int v = 0; v < cv::kPrbgVariants; v++) {
    chain_off[v] = bytes;
    bytes += align_up(np.chains[v].size() * sizeof(cv::PlcmChain), 256);
  }
  if (pf.copy_pending) {  // the previous prefetch may still be copying from h_table
    CV_HIP(hipEventSynchronize(pf.copied));
    pf.copy_pending = false;
  }
  if (pf.h_cap < bytes) {
    if (pf.h_table) (void)hipHostFree(pf.h_table);
    pf.h_table = nullptr;
    pf.h_cap = 0;
    if (hipHostMalloc(&pf.h_table, bytes) != hipSuccess) {
      (void)hipGetLastError();
      pf.h_table = nullptr;
      return CV_OK;  // no prefetch this time
    }
    pf.h_cap = bytes;
  }
  if (grow(&pf.d_table, &pf.d_cap, bytes, "prefetch tables") != CV_OK) return CV_OK;
  for (int v = 0; v < cv::kPrbgVariants; v++)
    if (!np.chains[v].empty())
      memcpy(pf.h_table + chain_off[v], np.chains[v].data(), np.chains[v].size() * sizeof(cv::PlcmChain));
  CV_HIP(hipMemcpyAsync(pf.d_table, pf.h_table, bytes, hipMemcpyHostToDevice, ps));
  CV_HIP(hipEventRecord(pf.copied, ps));
  pf.copy_pending = true;
  CV_HIP(hipStreamWaitEvent(ps, pf.ks_ready, 0));
  hipEvent_t ta = b->profiling ? pooled(b) : nullptr;
  if (ta) CV_HIP(hipEventRecord(ta, ps));
  for (int v = 0; v < cv::kPrbgVariants; v++)
    if (!np.chains[v].empty())
      CV_HIP(cv::launch_prbg_plcm((const cv::PlcmChain*)(pf.d_table + chain_off[v]),
                                  (uint32_t)np.chains[v].size(), b->d_ks[np.target], 0, v, ps));
  if (ta) {
    hipEvent_t tb = pooled(b);
    if (tb) {
      CV_HIP(hipEventRecord(tb, ps));
      b->spans.push_back({ta, tb, 0, np.steps});
    } else {
      b->event_pool.push_back(ta);
    }
  }
  CV_HIP(hipEventRecord(pf.done[np.shadow], ps));
  pf.used[np.shadow] = true;
  pf.entries = std::move(np.entries);
  pf.target = np.target;
  pf.shadow = np.shadow;
  pf.valid = true;
  return CV_OK;
}

cv_status run_tick(cv_batch* b, const cv_batch_item* items, size_t n_items, hipStream_t st) {
  std::vector<ChainJob> cj;
  std::vector<FrameJob> fj;
  std::vector<size_t> fallback, eligible;
  uint64_t ks = 0;
  collect(b, items, n_items, cj, fj, fallback, eligible, ks);
  Prefetch& pf = b->pf;
  std::vector<const Prefetch::Entry*> prev;
  const bool hit = prefetch_matches(b, items, eligible, &prev);
  if (pf.valid) (hit ? b->info.prefetch_hits : b->info.prefetch_misses)++;
  // keystream buffer: the prefetched one, else one that no prefetch writes
  const int buf = hit ? pf.target : (pf.target == 0 ? 1 : 0);
  cv_status s = hit ? CV_OK : grow_ks(b, buf, ks);
  if (s != CV_OK) return s;
  bool ahead = b->shape.prefetch && !eligible.empty();
  if (ahead && (s = ensure_prefetch(b)) != CV_OK) return s;
  NextPrefetch np;
  ahead = ahead && plan_prefetch(b, items, eligible, hit ? &prev : nullptr, 1 - buf, np);
  if ((s = order_after_last(b, st)) != CV_OK) return s;
  for (size_t i : eligible)  // after the keys' own calls on other streams
    if ((s = key_order_wait(items[i].key, st)) != CV_OK) return s;
  for (size_t i : fallback) {
    const cv_batch_item& it = items[i];
    if ((s = crypt_frames(it.key, it.decrypt != 0, it.in, it.out, it.s_c, it.n_frames, st)) != CV_OK)
      return s;
  }
  b->info.last_fallback_items = (uint32_t)fallback.size();
  TickHooks hooks;
  if (hit) {
    // the prefetched keystream, laid out item by item in the prefetch's
    // order; its generator states become the keys' states
    const double* sh = (const double*)pf.d_shadow[pf.shadow];
    size_t q = 0;
    for (size_t j = 0; j < eligible.size(); j++) {
      const cv_batch_item& it = items[eligible[j]];
      const uint64_t rF = (uint64_t)it.key->g.r * it.key->F;
      for (uint32_t t = 0; t < it.n_frames; t++) fj[q++].ks_off = prev[j]->ks_off + t * rF;
      hooks.copies.push_back({sh + prev[j]->state_off, it.key->d_state, 2ull * it.key->g.n});
    }
    hooks.waits.push_back(pf.done[pf.shadow]);
    cj.clear();
  }
  if (ahead) {
    // the next prefetch's shadow buffer is free once the last prefetch that used it is done
    if (pf.used[np.shadow]) hooks.waits.push_back(pf.done[np.shadow]);
    hooks.copies.insert(hooks.copies.end(), np.gather.begin(), np.gather.end());
    hooks.ks_ready = pf.ks_ready;
    // while earlier ticks are still running (ticks queued back to back), the
    // prefetch is on the critical path: the rounds leave it compute units;
    // after an idle device (ticks that arrive in real time) the rounds take
    // them all and the prefetch catches up in the idle time after them
    bool busy = false;
    if (b->ran) {
      busy = hipEventQuery(b->done) == hipErrorNotReady;
      (void)hipGetLastError();
    }
    if (busy) hooks.reserve_cus = (np.workgroups + 7) / 8;
  }
  pf.valid = false;
  const bool hooked = hit || ahead;
  if ((s = batch_enqueue(b, cj, fj, b->d_ks[buf], st, hooked ? &hooks : nullptr)) != CV_OK) return s;
  for (size_t i : eligible) items[i].key->frame_index += items[i].n_frames;
  return ahead ? launch_prefetch(b, np, st) : CV_OK;
}

}  // namespace

namespace cv {
namespace rt {

cv_status batch_enqueue(cv_batch* b, const std::vector<ChainJob>& cj, const std::vector<FrameJob>& fj,
                        uint8_t* ks_base, hipStream_t st, const TickHooks* hooks) {
  Plan P;
  Layout L;
  cv_status s = prepare(b, cj, fj, P, L, hooks);
  if (s != CV_OK) return s;
  b->info.last_jobs = 0;
  b->info.last_groups = 0;
  b->info.last_wide_groups = 0;
  for (int c = 0; c < kClasses; c++) {
    b->info.last_jobs += (uint32_t)P.jobs[c].size();
    b->info.last_groups += P.groups[c];
    b->info.last_wide_groups += P.wide[c];
  }
  b->info.last_chains = 0;
  for (const auto& cs : P.chains) b->info.last_chains += (uint32_t)cs.size();
  if (cj.empty() && fj.empty()) return CV_OK;
  Slot* sp = nullptr;
  if ((s = next_slot(b, L.bytes, &sp)) != CV_OK) return s;
  fill_blob(b, P, L, sp->h_blob, ks_base);
  if (b->profiling || !b->shape.use_graph || hooks)
    s = enqueue_tick(b, P, L, *sp, st, b->profiling, ks_base, hooks);
  else
    s = launch_graph(b, P, L, *sp, ks_base, st);
  if (s != CV_OK) return s;
  CV_HIP(hipEventRecord(sp->copied, st));
  sp->pending = true;
  return CV_OK;
}

bool batch_flag_set(const cv_batch* b) { return b->failed || *b->h_err != 0; }

void batch_set_reserve(cv_batch* b, uint32_t cus_per_xcd) { b->reserve_cus = cus_per_xcd; }

}  // namespace rt
}  // namespace cv

namespace {

void release(cv_batch* b) {
  drop_graphs(b);
  for (Slot& s : b->slot) {
    if (s.h_blob) (void)hipHostFree(s.h_blob);
    if (s.copied) (void)hipEventDestroy(s.copied);
  }
  for (Span& sp : b->spans) {
    b->event_pool.push_back(sp.a);
    b->event_pool.push_back(sp.b);
  }
  for (hipEvent_t e : b->event_pool) (void)hipEventDestroy(e);
  if (b->d_blob) (void)hipFree(b->d_blob);
  for (uint8_t* p : b->d_ks)
    if (p) (void)hipFree(p);
  Prefetch& pf = b->pf;
  if (pf.h_table) (void)hipHostFree(pf.h_table);
  if (pf.d_table) (void)hipFree(pf.d_table);
  for (uint8_t* p : pf.d_shadow)
    if (p) (void)hipFree(p);
  for (hipEvent_t e : {pf.ks_ready, pf.done[0], pf.done[1], pf.copied})
    if (e) (void)hipEventDestroy(e);
  side_streams_free(pf.side);
  if (b->d_scratch) (void)hipFree(b->d_scratch);
  if (b->d_counters) (void)hipFree(b->d_counters);
  if (b->d_err) (void)hipFree(b->d_err);
  if (b->h_err) (void)hipHostFree(b->h_err);
  if (b->done) (void)hipEventDestroy(b->done);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

cv_status check_shape(const cv_batch_shape& s) {
  if (s.threads < 256 || s.threads > 1024 || s.threads % 64)
    return fail(CV_E_INVAL, "threads must be a multiple of 64 in 256..1024");
  if (s.group_wgs < 1 || s.group_wgs > 64) return fail(CV_E_INVAL, "group_wgs must be in 1..64");
  if (s.use_graph > 1) return fail(CV_E_INVAL, "use_graph must be 0 or 1");
  if (s.prefetch > 1) return fail(CV_E_INVAL, "prefetch must be 0 or 1");
  return CV_OK;
}

}  // namespace

namespace {

// Shape class of a tick for the autotuner cache: the sorted multiset of its
// batched items' (H, W, C, n, r, direction, frames), and the device's LDS.
std::string tune_key(const cv_batch* b, const cv_batch_item* items, size_t n_items) {
  std::vector<std::string> parts;
  for (size_t i = 0; i < n_items; i++) {
    const cv_batch_item& it = items[i];
    if (it.n_frames == 0 || !item_eligible(b, it)) continue;
    const Geom& g = it.key->g;
    char buf[96];
    snprintf(buf, sizeof buf, "%ux%ux%u/n%u/r%u/%c%u", g.H, g.W, g.C, g.n, g.r,
             it.decrypt ? 'd' : 'e', it.n_frames);
    parts.push_back(buf);
  }
  std::sort(parts.begin(), parts.end());
  std::string k = "batch|lds" + std::to_string(b->lds_max);
  for (size_t i = 0; i < parts.size();) {
    size_t j = i;
    while (j < parts.size() && parts[j] == parts[i]) j++;
    k += "|" + std::to_string(j - i) + "*" + parts[i];
    i = j;
  }
  return k;
}

}  // namespace

extern "C" {

cv_status cv_batch_create(int device, cv_batch** out) {
  if (!out) return fail(CV_E_INVAL, "NULL argument");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(CV_E_INVAL, "no such HIP device");
  DeviceGuard dg(device);
  cv_batch* b = new cv_batch();
  b->device = device;
  b->lds_max = lds_limit(device);
  hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  for (Slot& s : b->slot)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.copied, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&b->d_err, sizeof(uint32_t));
  if (e == hipSuccess) e = hipHostMalloc(&b->h_err, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(b->d_err, 0, sizeof(uint32_t));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release(b);
    return fail(e == hipErrorOutOfMemory ? CV_E_NOMEM : CV_E_HIP, "cv_batch_create failed");
  }
  *b->h_err = 0;
  *out = b;
  return CV_OK;
}

void cv_batch_free(cv_batch* b) {
  if (!b) return;
  DeviceGuard dg(b->device);
  (void)hipDeviceSynchronize();
  release(b);
}

cv_status cv_batch_get_shape(const cv_batch* b, cv_batch_shape* shape) {
  if (!b || !shape) return fail(CV_E_INVAL, "NULL argument");
  *shape = b->shape;
  return CV_OK;
}

cv_status cv_batch_set_shape(cv_batch* b, const cv_batch_shape* shape) {
  if (!b || !shape) return fail(CV_E_INVAL, "NULL argument");
  cv_status s = check_shape(*shape);
  if (s != CV_OK) return s;
  b->shape = *shape;
  return CV_OK;
}

cv_status cv_batch_run(cv_batch* b, const cv_batch_item* items, size_t n_items, void* stream) {
  if (!b) return fail(CV_E_INVAL, "batch is NULL");
  cv_status s = check_items(b, items, n_items);
  if (s != CV_OK) return s;
  for (size_t i = 0; i < n_items; i++)
    if (items[i].n_frames && (s = check_async_errors(items[i].key, false)) != CV_OK) return s;
  if ((s = check_flag(b, false)) != CV_OK) return s;
  DeviceGuard dg(b->device);
  hipStream_t st = (hipStream_t)stream;
  if ((s = run_tick(b, items, n_items, st)) != CV_OK) return s;
  CV_HIP(hipEventRecord(b->done, st));
  b->last_stream = st;
  b->ran = true;
  b->info.ticks++;
  return CV_OK;
}

cv_status cv_batch_sync(cv_batch* b) {
  if (!b) return fail(CV_E_INVAL, "batch is NULL");
  DeviceGuard dg(b->device);
  return check_flag(b, true);
}

cv_status cv_batch_get_info(const cv_batch* b, cv_batch_info* info) {
  if (!b || !info) return fail(CV_E_INVAL, "NULL argument");
  *info = b->info;
  return CV_OK;
}

cv_status cv_batch_autotune(cv_batch* b, const cv_batch_item* items, size_t n_items, void* stream,
                            cv_batch_shape* best) {
  if (!b) return fail(CV_E_INVAL, "batch is NULL");
  cv_status s = check_items(b, items, n_items);
  if (s != CV_OK) return s;
  if ((s = check_flag(b, false)) != CV_OK) return s;
  DeviceGuard dg(b->device);
  hipStream_t st = (hipStream_t)stream;
  const cv_batch_shape keep = b->shape;
  // the tick's shape class: its batched frame jobs' geometries and directions
  const std::string key = tune_key(b, items, n_items);
  std::map<std::string, int64_t> cached;
  if (tune_lookup(key, &cached) && cached.count("threads") && cached.count("group_wgs") &&
      cached.count("max_groups") && cached.count("tile_rows_max")) {
    cv_batch_shape c = keep;
    c.threads = (uint32_t)cached["threads"];
    c.group_wgs = (uint32_t)cached["group_wgs"];
    c.max_groups = (uint32_t)cached["max_groups"];
    c.tile_rows_max = (uint32_t)cached["tile_rows_max"];
    if (check_shape(c) == CV_OK) {
      b->shape = c;
      b->info.tune_cache_hits++;
      if (best) *best = c;
      return CV_OK;
    }
  }
  if ((s = order_after_last(b, st)) != CV_OK) return s;
  const bool prof = b->profiling;
  b->profiling = true;  // time each rounds launch
  cv_batch_shape win = keep;
  double win_ms = -1.0;
  const int kb = b->pf.target == 0 ? 1 : 0;  // a keystream buffer no prefetch writes
  // candidates: the kernel (512 threads: pixel-word, 1024: row-run), G, the
  // groups in flight (0 = all resident, else half the resident groups) and
  // the LDS tiling (0 = the largest tiles, else half their rows)
  const uint32_t threads_c[] = {512, 1024}, G_c[] = {4, 8, 16, 32};
  for (uint32_t th : threads_c) {
    for (uint32_t G : G_c) {
      for (int half_groups = 0; half_groups < 2 && s == CV_OK; half_groups++) {
        for (int half_tiles = 0; half_tiles < 2 && s == CV_OK; half_tiles++) {
          b->shape = keep;
          b->shape.threads = th;
          b->shape.group_wgs = G;
          b->shape.max_groups = 0;
          b->shape.tile_rows_max = 0;
          std::vector<ChainJob> cj;
          std::vector<FrameJob> fj;
          std::vector<size_t> fallback, eligible;
          uint64_t ks = 0;
          collect(b, items, n_items, cj, fj, fallback, eligible, ks);
          if (fj.empty()) break;
          if (half_tiles) {
            // half the rows of the largest tile of any job
            uint32_t rows = 0;
            for (const FrameJob& f : fj) {
              const Geom& g = f.k->g;
              rows = std::max(rows, std::max(pw_tile_rows(g, th, b->lds_max),
                                             std::max(cv::rounds_skew_tile_rows(g, b->lds_max),
                                                      cv::batch_unskew_tile_rows(g, b->lds_max))));
            }
            if (rows < 2) continue;
            b->shape.tile_rows_max = rows / 2;
          }
          if ((s = grow_ks(b, kb, ks)) != CV_OK) break;
          Plan P;
          Layout L;
          if ((s = prepare(b, {}, fj, P, L)) != CV_OK) {
            // a shape this tick cannot use (too wide for the workgroup) is skipped
            if (s == CV_E_INVAL) {
              s = CV_OK;
              continue;
            }
            break;
          }
          if (half_groups) {
            const uint32_t gmax = *std::max_element(P.groups, P.groups + kClasses);
            if (gmax < 16) continue;
            b->shape.max_groups = gmax / 2 / 8 * 8;
            Plan P2;
            if ((s = prepare(b, {}, fj, P2, L)) != CV_OK) break;
            P = std::move(P2);
          }
          Slot* sp = nullptr;
          if ((s = next_slot(b, L.bytes, &sp)) != CV_OK) break;
          Slot& sl = *sp;
          fill_blob(b, P, L, sl.h_blob, b->d_ks[kb]);
          if ((s = drain(b)) != CV_OK) break;
          b->prof = cv_profile{};
          for (int rep = 0; rep < 4 && s == CV_OK; rep++) s = enqueue_tick(b, P, L, sl, st, true, b->d_ks[kb]);
          if (s != CV_OK) break;
          CV_HIP(hipEventRecord(sl.copied, st));
          sl.pending = true;
          // the first launch warms up; the rest are timed
          if (!b->spans.empty()) {
            Span first = b->spans.front();
            b->spans.erase(b->spans.begin());
            if ((s = drain(b)) != CV_OK) break;
            b->event_pool.push_back(first.a);
            b->event_pool.push_back(first.b);
          }
          b->info.tune_shapes_timed++;
          const double ms = b->prof.round_ms / std::max<uint64_t>(1, b->prof.round_launches);
          if (win_ms < 0 || ms < win_ms) {
            win_ms = ms;
            win = b->shape;
          }
        }
      }
      if (s != CV_OK) break;
    }
    if (s != CV_OK) break;
  }
  CV_HIP(hipEventRecord(b->done, st));
  b->last_stream = st;
  b->ran = true;
  cv_status s2 = drain(b);
  b->profiling = prof;
  b->prof = cv_profile{};
  b->shape = s == CV_OK ? win : keep;
  if (s != CV_OK) return s;
  if (s2 != CV_OK) return s2;
  if ((s = check_flag(b, true)) != CV_OK) return s;
  if (win_ms >= 0)
    (void)tune_store(key, {{"threads", b->shape.threads}, {"group_wgs", b->shape.group_wgs},
                           {"max_groups", b->shape.max_groups},
                           {"tile_rows_max", b->shape.tile_rows_max}});
  if (best) *best = b->shape;
  return CV_OK;
}

cv_status cv_batch_set_profiling(cv_batch* b, int on) {
  if (!b) return fail(CV_E_INVAL, "batch is NULL");
  DeviceGuard dg(b->device);
  cv_status s = drain(b);
  if (s != CV_OK) return s;
  b->profiling = on != 0;
  b->prof = cv_profile{};
  return CV_OK;
}

cv_status cv_batch_get_profile(cv_batch* b, cv_profile* prof) {
  if (!b || !prof) return fail(CV_E_INVAL, "NULL argument");
  if (!b->profiling) return fail(CV_E_STATE, "profiling is off");
  DeviceGuard dg(b->device);
  cv_status s = drain(b);
  if (s != CV_OK) return s;
  *prof = b->prof;
  return CV_OK;
}

}  // extern "C"
