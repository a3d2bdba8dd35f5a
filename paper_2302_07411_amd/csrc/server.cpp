// Serving loop of libchaosvid (declarations and contract in
// include/chaosvid.h): many live streams on one device, driven by one
// worker thread.
//
// Per stream, the worker keeps a ring of `ring_frames` keystream frames in
// a device arena.  The keystream of frame f depends only on the key's
// generator state (Algorithm 2), so it is produced before the frame
// arrives: the worker keeps one keystream launch in flight on its own HIP
// stream, covering every stream with a free ring slot, and gives streams
// with short generator chains several frames per launch so that no chain
// waits long for the longest one.  Frames submitted by the caller queue per
// stream; whenever fewer than two rounds ticks are in flight, the worker
// takes every queued frame whose keystream is ready, from every stream, into
// one tick of the batched rounds kernel on a second HIP stream (continuous
// batching).  A frame's ring slot is reused once its tick has completed.
//
// Locking: one mutex guards the stream table and every counter; HIP calls
// are made by the worker with the mutex released, on job lists it copied
// out under the mutex.  Callers' threads never make HIP calls except in
// cv_stream_open (key setup) and cv_stream_close / cv_server_free.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace cv::rt;
using Clock = std::chrono::steady_clock;

namespace {

constexpr uint32_t kLatencyLog = 4096;   // per-stream latencies kept for polling
constexpr uint32_t kMaxStreams = 4096;
constexpr uint32_t kMaxTicksInFlight = 2;
constexpr uint32_t kThreads = 1024;      // rounds workgroup size

// First-fit sub-allocator of the keystream arena (offsets, 256-byte units).
class Arena {
 public:
  void reset(size_t cap) {
    cap_ = cap;
    free_.clear();
    if (cap) free_[0] = cap;
    used_ = 0;
  }
  // Offset of a block of `n` bytes, or SIZE_MAX if none is free.
  size_t alloc(size_t n) {
    n = (n + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, left = it->second - n;
      free_.erase(it);
      if (left) free_[off + n] = left;
      used_ += n;
      return off;
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) / 256 * 256;
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t cap() const { return cap_; }

 private:
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
};

// Device memory for keystream rings: chunks from hipMalloc, each split by
// its own Arena.  Rings are handed out as device addresses.
class Pool {
 public:
  ~Pool() {
    for (Chunk& c : chunks_) (void)hipFree(c.mem);
  }
  // Device memory of `bytes` (a multiple of 256), or null.
  static uint8_t* allocate(size_t bytes) {
    uint8_t* mem = nullptr;
    if (bytes == 0 || hipMalloc(&mem, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return mem;
  }
  // Take `mem` (from allocate) as a new chunk.
  void add(uint8_t* mem, size_t bytes) {
    chunks_.push_back({mem, Arena()});
    chunks_.back().sub.reset(bytes);
  }
  uint8_t* alloc(size_t n) {
    for (Chunk& c : chunks_) {
      const size_t off = c.sub.alloc(n);
      if (off != SIZE_MAX) return c.mem + off;
    }
    return nullptr;
  }
  void release(uint8_t* p, size_t n) {
    for (Chunk& c : chunks_)
      if (p >= c.mem && p < c.mem + c.sub.cap()) {
        c.sub.release((size_t)(p - c.mem), n);
        return;
      }
  }
  size_t used() const {
    size_t u = 0;
    for (const Chunk& c : chunks_) u += c.sub.used();
    return u;
  }
  size_t cap() const {
    size_t t = 0;
    for (const Chunk& c : chunks_) t += c.sub.cap();
    return t;
  }

 private:
  struct Chunk {
    uint8_t* mem;
    Arena sub;
  };
  std::vector<Chunk> chunks_;
};

struct Pending {
  uint64_t ticket;
  const uint8_t* in;
  uint8_t* out;
  uint32_t s_c;
  Clock::time_point t_submit;
};

struct Part {
  cv_stream* st;
  uint64_t ticket;
  Clock::time_point t_submit;
};

struct Tick {
  hipEvent_t ev = nullptr;
  Clock::time_point t_launch;
  bool batched = false;
  std::vector<Part> parts;
};

}  // namespace

struct cv_stream {
  cv_server* srv = nullptr;
  cv_key* key = nullptr;
  bool decrypt = false;
  uint32_t D = 0;             // ring depth (frames)
  uint32_t Q = 0;             // queue depth (frames in flight)
  uint64_t rF = 0;            // keystream bytes per frame
  uint64_t steps_per_frame = 0;  // longest chain's steps per frame
  uint8_t* ring = nullptr;    // keystream ring: D frames of rF bytes
  size_t ring_bytes = 0;
  bool pw = false;            // geometry takes the batched kernels
  // counters (server mutex)
  uint64_t submitted = 0;     // tickets issued
  uint64_t ks_issued = 0;     // keystream frames launched
  uint64_t ks_ready = 0;      // keystream frames generated
  uint64_t dispatched = 0;    // frames handed to rounds ticks
  uint64_t completed = 0;     // frames done
  std::deque<Pending> queue;  // submitted, not yet dispatched
  std::vector<double> lat;    // latency (ms) of ticket t at t % kLatencyLog
  bool closing = false;
  bool in_ks_launch = false;
  uint64_t starved_mark = 0;  // tickets below this were counted as starved
};

struct cv_server {
  int device = 0;
  size_t lds_max = 0;
  uint32_t ring_frames = 3, queue_frames = 8;
  uint32_t split = 0;      // quarters of every XCD's CUs for the keystream (0: shared CUs)
  Pool pool;                 // keystream rings
  bool grow = false;         // budget 0: the pool grows while the device has free memory
  cv_batch* rb = nullptr;  // rounds ticks
  cv_batch* kb = nullptr;  // keystream launches
  hipStream_t s_rounds = nullptr, s_ks = nullptr;
  hipEvent_t ks_ev = nullptr;
  std::vector<hipEvent_t> ev_pool;
  std::mutex mu;
  std::condition_variable work_cv, done_cv;
  std::thread worker;
  bool stop = false;
  cv_status err = CV_OK;
  std::string err_msg;
  std::vector<cv_stream*> streams;
  std::vector<std::pair<cv_stream*, uint32_t>> ks_launch;  // in flight
  bool ks_busy = false;
  // 2DLASM streams' keystream: one launch over all their chains, from a
  // chain table staged in pinned memory, with the launch's own word for a
  // sine that could not be rounded
  cv::LasmChain* d_lasm = nullptr;
  cv::LasmChain* h_lasm = nullptr;
  size_t lasm_cap = 0;  // chains
  uint32_t* d_lasm_err = nullptr;
  uint32_t* h_lasm_err = nullptr;
  Clock::time_point ks_launch_t;
  std::deque<Tick> ticks;
  cv_server_stats stats{};
};

namespace {

// Set the server's sticky error (mutex held).
void set_error(cv_server* S, cv_status s, const std::string& msg) {
  if (S->err == CV_OK) {
    S->err = s;
    S->err_msg = msg;
  }
  S->done_cv.notify_all();
}

hipEvent_t take_event(cv_server* S) {
  if (!S->ev_pool.empty()) {
    hipEvent_t e = S->ev_pool.back();
    S->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess ? e : nullptr;
}

// A 2DLASM stream's share of a keystream launch (its own generator launch).
struct LasmJob {
  cv_key* k;
  uint64_t ks_off;
  uint32_t frames;
};

// Frames of keystream to generate for each stream in the next launch (mutex held).
void plan_keystream(cv_server* S, std::vector<ChainJob>& cj, std::vector<LasmJob>& lj) {
  uint64_t longest = 0;
  for (cv_stream* st : S->streams)
    if (!st->closing && st->ks_issued - st->completed < st->D)
      longest = std::max(longest, st->steps_per_frame);
  for (cv_stream* st : S->streams) {
    if (st->closing) continue;
    const uint64_t free = st->D - (st->ks_issued - st->completed);
    if (free == 0) continue;
    const uint64_t contiguous = st->D - st->ks_issued % st->D;  // no wrap within a launch
    const uint64_t share = std::max<uint64_t>(1, longest / std::max<uint64_t>(1, st->steps_per_frame));
    const uint32_t k = (uint32_t)std::min({free, contiguous, share});
    // keystream addresses are absolute (the launches get a null base)
    const uint64_t off = (uint64_t)(uintptr_t)st->ring + (st->ks_issued % st->D) * st->rF;
    if (st->key->map == CV_MAP_PLCM)
      cj.push_back({st->key, off, 0, k});
    else
      lj.push_back({st->key, off, k});
    S->ks_launch.push_back({st, k});
    st->ks_issued += k;
    st->in_ks_launch = true;
  }
}

// One keystream launch over the chains of every 2DLASM stream in `lj` on
// the keystream stream (mutex not held; the previous keystream launch, which
// read the same tables, is complete).  Chains are sorted by length so that
// the chains of a workgroup end together.
cv_status launch_lasm_keystream(cv_server* S, const std::vector<LasmJob>& lj) {
  std::vector<cv::LasmChain> ch;
  for (const LasmJob& l : lj)
    for (const cv::LasmChain& c : l.k->h_lchains) {
      cv::LasmChain x = c;
      x.out_off = l.ks_off + c.out_off;  // absolute: the launch gets a null base
      x.frames = l.frames;
      ch.push_back(x);
    }
  std::stable_sort(ch.begin(), ch.end(), [](const cv::LasmChain& a, const cv::LasmChain& b) {
    return a.nbytes * a.frames > b.nbytes * b.frames;
  });
  if (!S->d_lasm_err) {
    if (hipMalloc(&S->d_lasm_err, sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc(&S->h_lasm_err, sizeof(uint32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(CV_E_NOMEM, "2DLASM error word allocation failed");
    }
    *S->h_lasm_err = 0;
    CV_HIP(hipMemcpyAsync(S->d_lasm_err, S->h_lasm_err, sizeof(uint32_t), hipMemcpyHostToDevice,
                          S->s_ks));
  }
  if (ch.size() > S->lasm_cap) {
    if (S->d_lasm) (void)hipFree(S->d_lasm);
    if (S->h_lasm) (void)hipHostFree(S->h_lasm);
    S->d_lasm = nullptr;
    S->h_lasm = nullptr;
    S->lasm_cap = 0;
    const size_t cap = ch.size() + ch.size() / 2;
    if (hipMalloc(&S->d_lasm, cap * sizeof(cv::LasmChain)) != hipSuccess ||
        hipHostMalloc(&S->h_lasm, cap * sizeof(cv::LasmChain)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(CV_E_NOMEM, "2DLASM chain table allocation failed");
    }
    S->lasm_cap = cap;
  }
  memcpy(S->h_lasm, ch.data(), ch.size() * sizeof(cv::LasmChain));
  CV_HIP(hipMemcpyAsync(S->d_lasm, S->h_lasm, ch.size() * sizeof(cv::LasmChain),
                        hipMemcpyHostToDevice, S->s_ks));
  CV_HIP(cv::launch_prbg_lasm(S->d_lasm, (uint32_t)ch.size(), nullptr, 0, 0, S->d_lasm_err,
                              S->s_ks));
  CV_HIP(hipMemcpyAsync(S->h_lasm_err, S->d_lasm_err, sizeof(uint32_t), hipMemcpyDeviceToHost,
                        S->s_ks));
  return CV_OK;
}

// Queued frames with keystream ready, from every stream (mutex held).
void plan_rounds(cv_server* S, std::vector<FrameJob>& fj, std::vector<Pending>& solo,
                 std::vector<cv_stream*>& solo_st, Tick& t) {
  for (cv_stream* st : S->streams) {
    for (const Pending& p : st->queue) {
      if (p.ticket < st->ks_ready || p.ticket < st->starved_mark) continue;
      st->starved_mark = p.ticket + 1;  // counted once
      S->stats.starved_frames++;
    }
    while (!st->queue.empty() && st->queue.front().ticket < st->ks_ready) {
      const Pending p = st->queue.front();
      st->queue.pop_front();
      const cv_key* k = st->key;
      const uint64_t ks_off = (uint64_t)(uintptr_t)st->ring + (p.ticket % st->D) * st->rF;
      if (st->pw && pw_eligible(k, p.in, p.out, kThreads, S->lds_max)) {
        fj.push_back({k, p.in, p.out, p.in + k->F - 4, ks_off, p.s_c, (uint32_t)st->decrypt});
      } else {
        solo.push_back(p);
        solo_st.push_back(st);
      }
      t.parts.push_back({st, p.ticket, p.t_submit});
      st->dispatched++;
    }
  }
}

// Rounds of frames outside the batched kernels' conditions, on their key's path.
cv_status run_solo(cv_server* S, const std::vector<Pending>& solo,
                   const std::vector<cv_stream*>& solo_st) {
  for (size_t i = 0; i < solo.size(); i++) {
    cv_stream* st = solo_st[i];
    const Pending& p = solo[i];
    cv_status s = ensure_workspace(st->key, 1);
    if (s == CV_OK) s = upload_shift_tables(st->key, &p.s_c, 1, S->s_rounds);
    if (s == CV_OK)
      s = run_rounds(st->key, st->decrypt, p.in, p.out, st->ring + (p.ticket % st->D) * st->rF, 1,
                     S->s_rounds);
    if (s != CV_OK) return s;
  }
  return CV_OK;
}

// Budget 0: admission by the device's free memory now.  A new chunk of at
// least 4 GiB (or the ring) is allocated while the free memory, less a
// reserve of a sixteenth of the total for other allocations, holds it.
// Called without the server mutex; returns the chunk (null if none) and its size.
uint8_t* new_chunk(size_t ring_bytes, size_t* bytes) {
  size_t free_b = 0, total = 0;
  if (hipMemGetInfo(&free_b, &total) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  const size_t reserve = total / 16, need = (ring_bytes + 255) / 256 * 256;
  if (free_b < reserve + need) return nullptr;
  *bytes = std::min(free_b - reserve, std::max<size_t>(need, 4ull << 30)) / 256 * 256;
  return Pool::allocate(*bytes);
}

// Release a stream's ring (mutex held) and then, with the mutex released,
// its key.
// The server's two HIP streams.  With `quarters` = q in 1..3, the keystream
// stream may use q quarters of the compute units of every XCD (mask bits i
// with (i/8) % 4 < q: 8q CUs per XCD whether consecutive mask bits walk the
// CUs of one XCD or alternate between XCDs) and the rounds stream the rest,
// so that neither kernel slows the other's wavefronts; the rounds launch is
// then sized for the CUs it has.  q = 0: both streams use every CU.
hipError_t make_streams(cv_server* S, uint32_t quarters) {
  if (S->s_rounds) (void)hipStreamDestroy(S->s_rounds);
  if (S->s_ks) (void)hipStreamDestroy(S->s_ks);
  S->s_rounds = S->s_ks = nullptr;
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device);
  if (e != hipSuccess) return e;
  cv_batch_shape shape{kThreads, 8, 0, 0, 0};
  S->split = cus >= 64 && cus % 32 == 0 ? std::min<uint32_t>(quarters, 3) : 0;
  if (S->split) {
    std::vector<uint32_t> ks((cus + 31) / 32, 0), rd((cus + 31) / 32, 0);
    for (int i = 0; i < cus; i++) ((uint32_t)(i / 8) % 4 < S->split ? ks : rd)[i / 32] |= 1u << (i % 32);
    e = hipExtStreamCreateWithCUMask(&S->s_ks, (uint32_t)ks.size(), ks.data());
    if (e == hipSuccess) e = hipExtStreamCreateWithCUMask(&S->s_rounds, (uint32_t)rd.size(), rd.data());
    if (e != hipSuccess) {  // masks not supported here: share the CUs
      (void)hipGetLastError();
      if (S->s_ks) (void)hipStreamDestroy(S->s_ks);
      if (S->s_rounds) (void)hipStreamDestroy(S->s_rounds);
      S->s_ks = S->s_rounds = nullptr;
      S->split = 0;
    }
  }
  if (!S->split) {
    e = hipStreamCreateWithFlags(&S->s_ks, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s_rounds, hipStreamNonBlocking);
  }
  (void)cv_batch_set_shape(S->rb, &shape);
  (void)cv_batch_set_shape(S->kb, &shape);
  // with the split, the rounds launches are sized for the CUs their stream may use
  batch_set_reserve(S->rb, S->split * (uint32_t)cus / 32);
  return e;
}

void free_stream(cv_server* S, cv_stream* st, std::unique_lock<std::mutex>* lk) {
  S->pool.release(st->ring, st->ring_bytes);
  if (lk) lk->unlock();
  cv_key_free(st->key);
  delete st;
  if (lk) lk->lock();
}

void worker_main(cv_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progressed = false;
    // keystream launch done: its frames become usable
    if (S->ks_busy && hipEventQuery(S->ks_ev) == hipSuccess) {
      for (auto& [st, k] : S->ks_launch) {
        st->ks_ready += k;
        st->in_ks_launch = false;
      }
      if (S->h_lasm_err && *S->h_lasm_err)
        set_error(S, CV_E_HIP, "a 2DLASM sine could not be rounded with certainty");
      S->ks_launch.clear();
      S->ks_busy = false;
      S->stats.keystream_ms +=
          std::chrono::duration<double, std::milli>(Clock::now() - S->ks_launch_t).count();
      progressed = true;
    }
    // rounds ticks done, in order
    while (!S->ticks.empty() && hipEventQuery(S->ticks.front().ev) == hipSuccess) {
      Tick& t = S->ticks.front();
      if (t.batched && batch_flag_set(S->rb))
        set_error(S, CV_E_HIP, "a rounds tick timed out at a group barrier; its frames are invalid");
      const Clock::time_point now = Clock::now();
      for (const Part& p : t.parts) {
        p.st->lat[p.ticket % kLatencyLog] =
            std::chrono::duration<double, std::milli>(now - p.t_submit).count();
        p.st->completed++;
      }
      S->stats.frames_done += t.parts.size();
      S->stats.rounds_ms += std::chrono::duration<double, std::milli>(now - t.t_launch).count();
      S->ev_pool.push_back(t.ev);
      S->ticks.pop_front();
      progressed = true;
      S->done_cv.notify_all();
    }
    (void)hipGetLastError();  // a query of an unfinished event leaves hipErrorNotReady behind
    // streams being closed: free once nothing of theirs is in flight
    for (size_t i = 0; i < S->streams.size();) {
      cv_stream* st = S->streams[i];
      if (st->closing && st->completed == st->submitted && !st->in_ks_launch) {
        S->streams.erase(S->streams.begin() + i);
        free_stream(S, st, &lk);
        S->done_cv.notify_all();
        progressed = true;
        continue;
      }
      i++;
    }
    if (S->err == CV_OK && S->ticks.size() < kMaxTicksInFlight) {
      std::vector<FrameJob> fj;
      std::vector<Pending> solo;
      std::vector<cv_stream*> solo_st;
      Tick t;
      plan_rounds(S, fj, solo, solo_st, t);
      if (!t.parts.empty()) {
        t.ev = take_event(S);
        t.t_launch = Clock::now();
        t.batched = !fj.empty();
        lk.unlock();
        cv_status s = run_solo(S, solo, solo_st);
        if (s == CV_OK && !fj.empty()) s = batch_enqueue(S->rb, {}, fj, nullptr, S->s_rounds);
        std::string msg = s != CV_OK ? cv_last_error() : "";
        hipError_t e = t.ev ? hipEventRecord(t.ev, S->s_rounds) : hipErrorOutOfMemory;
        lk.lock();
        if (s != CV_OK) set_error(S, s, msg);
        else if (e != hipSuccess) set_error(S, CV_E_HIP, "event record failed");
        else {
          S->ticks.push_back(std::move(t));
          S->stats.rounds_ticks++;
        }
        progressed = true;
      }
    }
    if (S->err == CV_OK && !S->ks_busy && !S->stop) {
      std::vector<ChainJob> cj;
      std::vector<LasmJob> lj;
      plan_keystream(S, cj, lj);
      if (!cj.empty() || !lj.empty()) {
        uint64_t frames = 0;
        for (auto& c : cj) frames += c.frames;
        for (auto& l : lj) frames += l.frames;
        S->ks_launch_t = Clock::now();
        lk.unlock();
        cv_status s = cj.empty() ? CV_OK : batch_enqueue(S->kb, cj, {}, nullptr, S->s_ks);
        if (s == CV_OK && !lj.empty()) s = launch_lasm_keystream(S, lj);
        std::string msg = s != CV_OK ? cv_last_error() : "";
        hipError_t e = hipEventRecord(S->ks_ev, S->s_ks);
        lk.lock();
        if (s != CV_OK) set_error(S, s, msg);
        else if (e != hipSuccess) set_error(S, CV_E_HIP, "event record failed");
        S->ks_busy = true;
        S->stats.keystream_launches++;
        S->stats.keystream_frames += frames;
        progressed = true;
      }
    }
    if (S->err != CV_OK) {
      // nothing more will complete: release waiters
      S->done_cv.notify_all();
    }
    const bool idle = S->ticks.empty() && !S->ks_busy;
    if (S->stop && idle) break;
    if (S->stop && S->err != CV_OK) {
      lk.unlock();
      (void)hipDeviceSynchronize();
      lk.lock();
      break;
    }
    if (!progressed) {
      if (idle && !S->stop)
        S->work_cv.wait_for(lk, std::chrono::milliseconds(2));
      else
        S->work_cv.wait_for(lk, std::chrono::microseconds(50));
    }
  }
}

cv_status server_error(const cv_server* S) {
  return S->err == CV_OK ? CV_OK : fail(S->err, "server stopped: " + S->err_msg);
}

void destroy(cv_server* S) {
  if (S->worker.joinable()) {
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->stop = true;
    }
    S->work_cv.notify_all();
    S->worker.join();
  }
  DeviceGuard dg(S->device);
  (void)hipDeviceSynchronize();
  for (cv_stream* st : S->streams) free_stream(S, st, nullptr);
  S->streams.clear();
  for (Tick& t : S->ticks) S->ev_pool.push_back(t.ev);
  for (hipEvent_t e : S->ev_pool)
    if (e) (void)hipEventDestroy(e);
  if (S->ks_ev) (void)hipEventDestroy(S->ks_ev);
  cv_batch_free(S->rb);
  cv_batch_free(S->kb);
  if (S->s_rounds) (void)hipStreamDestroy(S->s_rounds);
  if (S->s_ks) (void)hipStreamDestroy(S->s_ks);
  if (S->d_lasm) (void)hipFree(S->d_lasm);
  if (S->h_lasm) (void)hipHostFree(S->h_lasm);
  if (S->d_lasm_err) (void)hipFree(S->d_lasm_err);
  if (S->h_lasm_err) (void)hipHostFree(S->h_lasm_err);
  delete S;
}

}  // namespace

extern "C" {

cv_status cv_server_create(int device, size_t hbm_budget, cv_server** out) {
  if (!out) return fail(CV_E_INVAL, "NULL argument");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(CV_E_INVAL, "no such HIP device");
  DeviceGuard dg(device);
  const bool grow = hbm_budget == 0;
  hbm_budget = hbm_budget / 256 * 256;
  if (!grow && hbm_budget == 0) return fail(CV_E_INVAL, "hbm_budget below 256 bytes");
  cv_server* S = new cv_server();
  S->grow = grow;
  S->device = device;
  S->lds_max = lds_limit(device);
  cv_status s = cv_batch_create(device, &S->rb);
  if (s == CV_OK) s = cv_batch_create(device, &S->kb);
  if (s != CV_OK) {
    destroy(S);
    return s;
  }
  // ticks change shape every time: launch kernel by kernel, groups of 8
  hipError_t e = make_streams(S, 1);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ks_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    destroy(S);
    return hip_fail(e, "cv_server_create");
  }
  if (!grow) {
    uint8_t* mem = Pool::allocate(hbm_budget);
    if (!mem) {
      destroy(S);
      return fail(CV_E_NOMEM, "keystream arena allocation failed");
    }
    S->pool.add(mem, hbm_budget);
  }
  S->stats.hbm_budget = S->pool.cap();
  S->worker = std::thread(worker_main, S);
  *out = S;
  return CV_OK;
}

cv_status cv_server_tune(cv_server* S, uint32_t ring_frames, uint32_t queue_frames,
                         int split_cus) {
  if (!S) return fail(CV_E_INVAL, "server is NULL");
  if (ring_frames < 1 || ring_frames > 64 || queue_frames < 1 || queue_frames > 64)
    return fail(CV_E_INVAL, "ring_frames and queue_frames must be in 1..64");
  if (split_cus < 0 || split_cus > 3) return fail(CV_E_INVAL, "split_cus must be in 0..3");
  std::lock_guard<std::mutex> g(S->mu);
  if ((uint32_t)split_cus != S->split) {
    if (!S->streams.empty() || S->ks_busy || !S->ticks.empty())
      return fail(CV_E_STATE, "the compute-unit split can change only with no stream open");
    DeviceGuard dg(S->device);
    (void)hipStreamSynchronize(S->s_ks);
    (void)hipStreamSynchronize(S->s_rounds);
    hipError_t e = make_streams(S, (uint32_t)split_cus);
    if (e != hipSuccess) {
      set_error(S, CV_E_HIP, "stream creation failed");
      return hip_fail(e, "cv_server_tune");
    }
  }
  S->ring_frames = ring_frames;
  S->queue_frames = queue_frames;
  return CV_OK;
}

void cv_server_free(cv_server* S) {
  if (!S) return;
  (void)cv_server_drain(S);
  destroy(S);
}

cv_status cv_server_drain(cv_server* S) {
  if (!S) return fail(CV_E_INVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  S->done_cv.wait(lk, [&] {
    if (S->err != CV_OK) return true;
    for (cv_stream* st : S->streams)
      if (st->completed != st->submitted) return false;
    return true;
  });
  return server_error(S);
}

cv_status cv_server_get_stats(cv_server* S, cv_server_stats* stats) {
  if (!S || !stats) return fail(CV_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  *stats = S->stats;
  stats->open_streams = (uint32_t)S->streams.size();
  stats->split_cus = S->split;
  stats->hbm_used = S->pool.used();
  return CV_OK;
}

cv_status cv_stream_open(cv_server* S, const cv_geom* geom, cv_map map, const double* p_m,
                         size_t n_doubles, int decrypt, cv_stream** out) {
  if (!S || !out) return fail(CV_E_INVAL, "NULL argument");
  *out = nullptr;
  if (decrypt != 0 && decrypt != 1) return fail(CV_E_INVAL, "decrypt must be 0 or 1");
  cv_key* k = nullptr;
  cv_status s = cv_keysetup(geom, map, p_m, n_doubles, S->device, &k);
  if (s != CV_OK) return s;
  cv_stream* st = new cv_stream();
  st->srv = S;
  st->key = k;
  st->decrypt = decrypt != 0;
  st->rF = (uint64_t)k->g.r * k->F;
  for (const cv::PlcmChain& c : k->h_chains)
    st->steps_per_frame = std::max<uint64_t>(st->steps_per_frame, (c.nbytes + 5) / 6);
  st->pw = (k->g.C == 3 || k->g.C == 4) && k->g.W % 16 == 0;
  st->lat.assign(kLatencyLog, -1.0);
  {
    std::unique_lock<std::mutex> lk(S->mu);
    if ((s = server_error(S)) == CV_OK) {
      st->D = S->ring_frames;
      st->Q = S->queue_frames;
      st->ring_bytes = st->D * st->rF;
      if (S->streams.size() >= kMaxStreams) {
        s = fail(CV_E_AGAIN, "too many open streams");
      } else {
        st->ring = S->pool.alloc(st->ring_bytes);
        if (!st->ring && S->grow) {
          lk.unlock();  // allocate without holding up the worker
          size_t bytes = 0;
          uint8_t* mem = new_chunk(st->ring_bytes, &bytes);
          lk.lock();
          if (mem) {
            S->pool.add(mem, bytes);
            S->stats.hbm_budget = S->pool.cap();
          }
          st->ring = S->pool.alloc(st->ring_bytes);
        }
        if (!st->ring) {
          s = fail(CV_E_AGAIN, S->grow ? "the device's free memory (less a reserve of 1/16 of it) "
                                         "cannot hold this stream's keystream ring now"
                                       : "the server's device-memory budget cannot hold this "
                                         "stream's keystream ring now");
        } else if (S->streams.size() >= kMaxStreams) {  // others opened while unlocked
          S->pool.release(st->ring, st->ring_bytes);
          st->ring = nullptr;
          s = fail(CV_E_AGAIN, "too many open streams");
        } else {
          S->streams.push_back(st);
        }
      }
    }
  }
  if (s != CV_OK) {
    cv_key_free(k);
    delete st;
    return s;
  }
  S->work_cv.notify_all();
  *out = st;
  return CV_OK;
}

cv_status cv_stream_submit(cv_stream* st, const uint8_t* frame, uint8_t* out, uint32_t s_c,
                           uint64_t* ticket) {
  if (!st || !frame || !out || !ticket) return fail(CV_E_INVAL, "NULL argument");
  if (s_c == 0) return fail(CV_E_INVAL, "confusion seed s_c must be >= 1");
  if (ranges_overlap(frame, st->key->F, out, st->key->F)) return fail(CV_E_INVAL, "frame and out overlap");
  cv_server* S = st->srv;
  {
    std::lock_guard<std::mutex> g(S->mu);
    cv_status s = server_error(S);
    if (s != CV_OK) return s;
    if (st->closing) return fail(CV_E_STATE, "stream is closing");
    if (st->submitted - st->completed >= st->Q) return fail(CV_E_AGAIN, "stream queue is full");
    *ticket = st->submitted;
    st->queue.push_back({st->submitted, frame, out, s_c, Clock::now()});
    st->submitted++;
  }
  S->work_cv.notify_all();
  return CV_OK;
}

cv_status cv_stream_poll(cv_stream* st, uint64_t ticket, int* done, double* latency_ms) {
  if (!st || !done) return fail(CV_E_INVAL, "NULL argument");
  cv_server* S = st->srv;
  std::lock_guard<std::mutex> g(S->mu);
  if (ticket >= st->submitted) return fail(CV_E_INVAL, "ticket not issued");
  *done = ticket < st->completed;
  if (latency_ms)
    *latency_ms = (*done && ticket + kLatencyLog >= st->completed) ? st->lat[ticket % kLatencyLog]
                                                                   : -1.0;
  if (!*done) return server_error(S);
  return CV_OK;
}

cv_status cv_stream_close(cv_stream* st) {
  if (!st) return fail(CV_E_INVAL, "stream is NULL");
  cv_server* S = st->srv;
  std::unique_lock<std::mutex> lk(S->mu);
  st->closing = true;
  S->work_cv.notify_all();
  // the worker frees the stream once its frames and keystream launch are done
  S->done_cv.wait(lk, [&] {
    return S->err != CV_OK ||
           std::find(S->streams.begin(), S->streams.end(), st) == S->streams.end();
  });
  if (S->err != CV_OK) return server_error(S);  // freed with the server
  return CV_OK;
}

}  // extern "C"
