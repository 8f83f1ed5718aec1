// Continuous-batching request server over a prepared polar_batch (C ABI in
// include/polar.h, polar_server_*).
//
// Requests (1..n frames of one code) are admitted first come, first served
// as soon as the device memory they need is free.  LLRs and results in host
// memory go through the server's own device pools: each frame-length class
// (one per distinct N among the batch's codes) owns a ring of fixed-size
// LLR slots in one device LLR pool and a ring of bits slots in one device
// bits pool, so such a request holds one contiguous slot range of each ring
// it needs: one host-to-device copy per request in, one copy out.  LLRs and
// results already in device memory are read and written in place; they use
// no slot, and count instead against a byte budget of caller memory that
// admitted, unfinished requests may reference.
//
// polar_server_poll() does all the work on the caller's thread: it retires
// finished steps (their results are already in pinned host memory), admits
// waiting requests, and launches a new step over every admitted frame not
// yet launched, as long as a stream is free (at most kMaxStepsPerClass steps
// of one frame length in flight).  A step is the new requests'
// LLR copies, the frame descriptors, one persistent batch decode, the result
// copies and an event, all on one of the server's streams; a step overlaps
// the one before it on the device, and requests that arrive while a step
// runs join the next one.
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <new>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

// Ring of n slots: allocation at the head, release in any order, the tail
// advancing over released ranges.  Ranges never wrap (an end gap too small
// for a request is skipped and counted as used until the tail passes it).
struct Ring {
  int n = 0, head = 0, tail = 0, used = 0;
  std::vector<int> len;  // at a range start: its length; negated once released
  std::vector<int> gap;  // at a skipped end gap start: its length

  void init(int slots) {
    n = slots;
    head = tail = used = 0;
    len.assign(slots, 0);
    gap.assign(slots, 0);
  }
  // whether alloc(k) would succeed (same rules, nothing changed)
  bool fits(int k) const {
    if (k <= 0 || k > n || used + k > n) return false;
    if (used == 0) return true;
    if (head >= tail) return n - head >= k || tail >= k;
    return tail - head >= k;
  }
  int take(int k) {
    const int s = head;
    len[s] = k;
    head += k;
    if (head == n) head = 0;
    used += k;
    return s;
  }
  int alloc(int k) {
    if (k <= 0 || k > n || used + k > n) return -1;
    if (used == 0) head = tail = 0;
    if (head >= tail) {
      if (n - head >= k) return take(k);
      if (tail >= k) {  // skip the end gap, continue at the front
        const int g = n - head;
        gap[head] = g;
        used += g;
        head = 0;
        return take(k);
      }
      return -1;
    }
    return tail - head >= k ? take(k) : -1;
  }
  void release(int s) {
    len[s] = -len[s];
    while (used > 0) {
      if (gap[tail] > 0) {
        used -= gap[tail];
        gap[tail] = 0;
        tail = 0;
      } else if (len[tail] < 0) {
        const int k = -len[tail];
        len[tail] = 0;
        used -= k;
        tail += k;
        if (tail == n) tail = 0;
      } else {
        break;
      }
    }
  }
};

struct SizeClass {
  int n = 0;                // frame length
  int llr_bytes = 0;        // bytes of one LLR slot
  int bits_bytes = 0;       // bytes of one bits slot (largest ceil(K/8) of the class)
  size_t llr_base = 0;      // byte offset of slot 0 in the LLR pool
  size_t bits_base = 0;     // byte offset of slot 0 in the bits pool
  Ring llr_ring;            // LLR slots of requests with host LLRs
  Ring bits_ring;           // bits slots of requests with host results
};

struct Request {
  int code = 0, cls = 0, nframes = 0;
  int llr_slot = -1;        // first slot of its range in the class's LLR ring (host LLRs)
  int bits_slot = -1;       // first slot of its range in the class's bits ring (host results)
  const uint8_t* dev_llr = nullptr;  // LLRs already in device memory (else staged)
  uint8_t* bits = nullptr;  // caller's output: host memory, or device memory if dev_bits
  bool dev_bits = false;
  size_t dev_bytes = 0;     // caller device memory it references (budgeted)
  size_t stage_off = 0;     // its LLR copy in the pinned staging ring
  size_t stage_len = 0;     // bytes taken there, including a skipped end gap
  size_t stage_end = 0;     // end of its bytes in the ring
  int64_t stage_seq = -1;   // its staging segment (allocation order)
};

// A staging allocation; segments are released in any order, the tail
// advancing over released ones.
struct StageSeg {
  size_t end = 0, len = 0;
  bool done = false;
};

struct Step {
  hipEvent_t done = nullptr;
  int stream = 0;
  int cls = 0;  // its length class
  std::vector<int64_t> reqs;
};

// Steps of one length class in flight at once.  With more, the long class
// (N = 32768, most of the device time) takes every stream at high load and
// the others queue behind it: at 90% of the batch capacity the served p99
// was 0.9-1.7 ms with no cap and 0.57 ms with 2 (one MI355X, 3 streams).
constexpr int kMaxStepsPerClass = 2;

}  // namespace

struct polar_server {
  const polar_batch* batch = nullptr;
  int device = 0;       // the batch's device: every launch goes there
  bool failed = false;  // a HIP call failed: requests in flight are lost
  int elem = 1;
  std::vector<int> code_n, code_rb, code_cls;
  std::vector<SizeClass> cls;
  std::vector<int> cls_steps;  // steps in flight per length class
  size_t dev_budget = 0;  // caller device bytes admitted requests may reference
  size_t dev_used = 0;
  uint8_t* d_llr = nullptr;
  uint8_t* d_bits = nullptr;
  uint8_t* h_bits = nullptr;  // pinned mirror of the bits pool
  uint8_t* h_stage = nullptr;  // pinned staging ring for request LLRs
  size_t stage_size = 0, stage_head = 0, stage_tail = 0, stage_used = 0;
  std::deque<StageSeg> stage_segs;  // live staging allocations, oldest first
  int64_t stage_base = 0;           // sequence number of stage_segs.front()
  uint64_t* d_desc = nullptr;  // one descriptor region per stream
  uint64_t* h_desc = nullptr;
  int desc_cap = 0;            // frames one step can carry
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<bool> busy;
  std::deque<int64_t> waiting;   // submitted, not yet admitted
  std::deque<int64_t> admitted;  // admitted, not yet launched
  std::deque<Step> inflight;
  std::unordered_map<int64_t, Request> reqs;
  int64_t next_id = 1;
  std::vector<uint64_t> sort_tmp;  // scratch of group_by_code
};

namespace {

// Device work is only valid on the batch's device, and after a failed HIP
// call the server's steps are in an unknown state.
polar_status usable(const polar_server* s) {
  if (s->failed) return POLAR_EDEVICE;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != s->device) return POLAR_ESTATE;
  return POLAR_OK;
}

void free_server(polar_server* s) {
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  if (s->d_llr) (void)hipFree(s->d_llr);
  if (s->d_bits) (void)hipFree(s->d_bits);
  if (s->d_desc) (void)hipFree(s->d_desc);
  if (s->h_bits) (void)hipHostFree(s->h_bits);
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  if (s->h_desc) (void)hipHostFree(s->h_desc);
  delete s;
}

// Staging allocation at the head of the ring (release: stage_release).
bool stage_alloc(polar_server* s, size_t bytes, size_t* off, size_t* taken) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes > s->stage_size || s->stage_used + bytes > s->stage_size) return false;
  if (s->stage_used == 0) s->stage_head = s->stage_tail = 0;
  if (s->stage_head >= s->stage_tail) {
    if (s->stage_size - s->stage_head >= bytes) {
      *off = s->stage_head;
      *taken = bytes;
    } else if (s->stage_tail >= bytes) {
      *off = 0;
      *taken = bytes + (s->stage_size - s->stage_head);  // the skipped end gap goes with it
    } else {
      return false;
    }
  } else if (s->stage_tail - s->stage_head >= bytes) {
    *off = s->stage_head;
    *taken = bytes;
  } else {
    return false;
  }
  s->stage_head = *off + bytes;
  if (s->stage_head == s->stage_size) s->stage_head = 0;
  s->stage_used += *taken;
  return true;
}

void stage_release(polar_server* s, const Request& r) {
  s->stage_segs[(size_t)(r.stage_seq - s->stage_base)].done = true;
  while (!s->stage_segs.empty() && s->stage_segs.front().done) {
    const StageSeg& g = s->stage_segs.front();
    s->stage_used -= g.len;
    s->stage_tail = g.end == s->stage_size ? 0 : g.end;
    s->stage_segs.pop_front();
    ++s->stage_base;
  }
  if (s->stage_used == 0) s->stage_head = s->stage_tail = 0;
}

// Moves waiting requests to admitted while the memory they need is free
// (FIFO): LLR slots for host LLRs, bits slots for host results, budget
// bytes for caller device memory.
void admit(polar_server* s) {
  while (!s->waiting.empty()) {
    Request& r = s->reqs[s->waiting.front()];
    SizeClass& c = s->cls[r.cls];
    if (!r.dev_llr && !c.llr_ring.fits(r.nframes)) break;
    if (!r.dev_bits && !c.bits_ring.fits(r.nframes)) break;
    if (s->dev_used + r.dev_bytes > s->dev_budget) break;
    if (!r.dev_llr) r.llr_slot = c.llr_ring.alloc(r.nframes);
    if (!r.dev_bits) r.bits_slot = c.bits_ring.alloc(r.nframes);
    s->dev_used += r.dev_bytes;
    s->admitted.push_back(s->waiting.front());
    s->waiting.pop_front();
  }
}

// One step over the admitted requests of length class ci (oldest first) on
// stream st.
// Stable counting sort of nd descriptors (pairs of words, code index in the
// low byte of the first) by code, so that neighbouring waves of the step
// run the same decoder.
void group_by_code(uint64_t* d, int nd, int ncodes, std::vector<uint64_t>& tmp) {
  int count[257] = {0};
  for (int j = 0; j < nd; ++j) ++count[(d[2 * j] & 255u) + 1];
  int used = 0;
  for (int c = 1; c <= ncodes; ++c) used += count[c] ? 1 : 0;
  if (used < 2) return;
  for (int c = 0; c < ncodes; ++c) count[c + 1] += count[c];
  tmp.resize(2 * (size_t)nd);
  for (int j = 0; j < nd; ++j) {
    const int k = count[d[2 * j] & 255u]++;
    tmp[2 * (size_t)k] = d[2 * j];
    tmp[2 * (size_t)k + 1] = d[2 * j + 1];
  }
  std::copy(tmp.begin(), tmp.end(), d);
}

polar_status launch_class(polar_server* s, int ci, int st) {
  hipStream_t stream = s->streams[st];
  uint64_t* hd = s->h_desc + 2 * (size_t)s->desc_cap * st;
  uint64_t* dd = s->d_desc + 2 * (size_t)s->desc_cap * st;
  Step step;
  step.stream = st;
  step.cls = ci;
  int nd = 0;
  std::deque<int64_t> rest;
  bool full = false;
  while (!s->admitted.empty()) {
    const int64_t id = s->admitted.front();
    s->admitted.pop_front();
    Request& r = s->reqs[id];
    if (r.cls != ci || full || nd + r.nframes > s->desc_cap) {
      if (r.cls == ci) full = true;  // keep the class in order
      rest.push_back(id);
      continue;
    }
    const SizeClass& c = s->cls[r.cls];
    const size_t llr_off = c.llr_base + (size_t)(r.llr_slot < 0 ? 0 : r.llr_slot) * c.llr_bytes;
    const size_t bits_off = c.bits_base + (size_t)(r.bits_slot < 0 ? 0 : r.bits_slot) * c.bits_bytes;
    // LLR element offset from the pool base: the request's slot for staged
    // requests; for requests already in device memory, the signed distance
    // to the caller's buffer (the kernel's 64-bit address sum wraps to it)
    int64_t first;
    if (r.dev_llr) {
      first = (int64_t)((intptr_t)r.dev_llr - (intptr_t)s->d_llr) / s->elem;
    } else {
      first = (int64_t)(llr_off / (size_t)s->elem);
      if (hipMemcpyAsync(s->d_llr + llr_off, s->h_stage + r.stage_off, (size_t)r.nframes * c.llr_bytes,
                         hipMemcpyHostToDevice, stream) != hipSuccess)
        return POLAR_EDEVICE;
    }
    // output: the request's bits slots, or the caller's device buffer
    // (signed distance from the bits pool base)
    const int rb = s->code_rb[r.code];
    const int64_t out0 = r.dev_bits ? (int64_t)((intptr_t)r.bits - (intptr_t)s->d_bits) : (int64_t)bits_off;
    const int64_t ostep = r.dev_bits ? rb : c.bits_bytes;
    for (int j = 0; j < r.nframes; ++j) {
      hd[2 * nd] = (uint64_t)r.code | ((uint64_t)(out0 + (int64_t)j * ostep) << 8);
      hd[2 * nd + 1] = (uint64_t)(first + (int64_t)j * c.n);
      ++nd;
    }
    step.reqs.push_back(id);
  }
  s->admitted.swap(rest);
  if (nd == 0) return POLAR_OK;
  group_by_code(hd, nd, (int)s->code_n.size(), s->sort_tmp);
  if (hipMemcpyAsync(dd, hd, (size_t)nd * 16, hipMemcpyHostToDevice, stream) != hipSuccess) return POLAR_EDEVICE;
  if (polar_batch_decode_desc(s->batch, dd, nd, s->d_llr, s->d_bits, stream) != POLAR_OK) return POLAR_EDEVICE;
  // results to pinned host memory: one copy per slot range of each length
  // class touched by the step (ring ranges are contiguous unless they wrap)
  for (size_t ci = 0; ci < s->cls.size(); ++ci) {
    int lo = -1, hi = -1;
    bool wrapped = false;
    for (int64_t id : step.reqs) {
      const Request& r = s->reqs[id];
      if (r.cls != (int)ci || r.dev_bits) continue;
      if (lo >= 0 && r.bits_slot < lo) wrapped = true;
      if (lo < 0 || r.bits_slot < lo) lo = r.bits_slot;
      hi = std::max(hi, r.bits_slot + r.nframes);
    }
    if (lo < 0) continue;
    const SizeClass& c = s->cls[ci];
    if (wrapped) {  // copy each request's range
      for (int64_t id : step.reqs) {
        const Request& r = s->reqs[id];
        if (r.cls != (int)ci || r.dev_bits) continue;
        const size_t off = c.bits_base + (size_t)r.bits_slot * c.bits_bytes;
        if (hipMemcpyAsync(s->h_bits + off, s->d_bits + off, (size_t)r.nframes * c.bits_bytes,
                           hipMemcpyDeviceToHost, stream) != hipSuccess)
          return POLAR_EDEVICE;
      }
    } else {
      const size_t off = c.bits_base + (size_t)lo * c.bits_bytes;
      if (hipMemcpyAsync(s->h_bits + off, s->d_bits + off, (size_t)(hi - lo) * c.bits_bytes, hipMemcpyDeviceToHost,
                         stream) != hipSuccess)
        return POLAR_EDEVICE;
    }
  }
  step.done = s->events[st];
  if (hipEventRecord(step.done, stream) != hipSuccess) return POLAR_EDEVICE;
  s->busy[st] = true;
  ++s->cls_steps[ci];
  s->inflight.push_back(std::move(step));
  return POLAR_OK;
}

// Launches steps while streams are free: each over one length class, the
// class of the oldest admitted request first, so short codes do not wait
// for the decodes of long ones, skipping classes that already have
// kMaxStepsPerClass steps in flight.
polar_status launch(polar_server* s) {
  while (!s->admitted.empty()) {
    int st = -1;
    for (size_t i = 0; i < s->busy.size(); ++i)
      if (!s->busy[i]) {
        st = (int)i;
        break;
      }
    if (st < 0) return POLAR_OK;
    int ci = -1;
    for (int64_t id : s->admitted) {
      const int c = s->reqs[id].cls;
      if (s->cls_steps[c] < kMaxStepsPerClass) {
        ci = c;
        break;
      }
    }
    if (ci < 0) return POLAR_OK;
    const polar_status e = launch_class(s, ci, st);
    if (e != POLAR_OK) return e;
  }
  return POLAR_OK;
}

// Retires finished steps (in any order); appends their request ids (to
// done while cap allows, and to all when given).
polar_status retire(polar_server* s, int64_t* done, int cap, int* ndone, std::vector<int64_t>* all = nullptr) {
  for (auto si = s->inflight.begin(); si != s->inflight.end();) {
    Step& step = *si;
    const hipError_t q = hipEventQuery(step.done);
    if (q == hipErrorNotReady) {
      ++si;
      continue;
    }
    if (q != hipSuccess) return POLAR_EDEVICE;
    for (int64_t id : step.reqs) {
      auto it = s->reqs.find(id);
      Request& r = it->second;
      const SizeClass& c = s->cls[r.cls];
      const int rb = s->code_rb[r.code];
      if (!r.dev_bits) {
        const uint8_t* src = s->h_bits + c.bits_base + (size_t)r.bits_slot * c.bits_bytes;
        for (int j = 0; j < r.nframes; ++j) memcpy(r.bits + (size_t)j * rb, src + (size_t)j * c.bits_bytes, rb);
        s->cls[r.cls].bits_ring.release(r.bits_slot);
      }
      if (!r.dev_llr) {
        s->cls[r.cls].llr_ring.release(r.llr_slot);
        stage_release(s, r);
      }
      s->dev_used -= r.dev_bytes;
      if (*ndone < cap && done) done[*ndone] = id;
      if (all) all->push_back(id);
      ++*ndone;
      s->reqs.erase(it);
    }
    s->busy[step.stream] = false;
    --s->cls_steps[step.cls];
    si = s->inflight.erase(si);
  }
  return POLAR_OK;
}

}  // namespace

extern "C" {

polar_server* polar_server_create(const polar_batch* batch, const polar_code* const* codes, int ncodes,
                                  int slots_per_class, int streams, size_t staging_bytes, size_t device_bytes) {
  if (!batch || !codes || ncodes < 1 || ncodes != (int)batch->plans.size() || slots_per_class < 0 ||
      (slots_per_class == 0 && device_bytes == 0) || streams < 1 || streams > 8 || staging_bytes < 4096 ||
      !batch->prepared) {
    polar_set_status(!batch || (batch && !batch->prepared) ? (batch ? POLAR_ESTATE : POLAR_EINVAL) : POLAR_EINVAL);
    return nullptr;
  }
  polar_server* s = polar::alloc_fails() ? nullptr : new (std::nothrow) polar_server;
  if (!s) {
    polar_set_status(POLAR_ENOMEM);
    return nullptr;
  }
  polar_status st = POLAR_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != batch->device) st = POLAR_ESTATE;
  try {
    s->batch = batch;
    s->device = batch->device;
    s->elem = batch->llr_type == POLAR_LLR_F32 ? 4 : 1;
    for (int i = 0; i < ncodes && st == POLAR_OK; ++i) {
      if (!codes[i] || codes[i]->plan.n != batch->plans[i].n || codes[i]->plan.frozen != batch->plans[i].frozen) {
        st = POLAR_EINVAL;
        break;
      }
      s->code_n.push_back(codes[i]->plan.n);
      s->code_rb.push_back((codes[i]->plan.k + 7) / 8);
      int c = -1;
      for (size_t j = 0; j < s->cls.size(); ++j)
        if (s->cls[j].n == codes[i]->plan.n) c = (int)j;
      if (c < 0) {
        SizeClass sc;
        sc.n = codes[i]->plan.n;
        sc.llr_bytes = sc.n * s->elem;
        s->cls.push_back(sc);
        c = (int)s->cls.size() - 1;
      }
      s->code_cls.push_back(c);
      s->cls[c].bits_bytes = std::max(s->cls[c].bits_bytes, (codes[i]->plan.k + 7) / 8);
    }
    if (st == POLAR_OK) {
      // pools of at least 256 bytes: their bases anchor the descriptor offsets
      size_t llr_total = 256, bits_total = 256;
      size_t cap = 0;  // most frames of one class admitted at once
      for (SizeClass& c : s->cls) {
        c.bits_bytes = (c.bits_bytes + 15) & ~15;
        c.llr_base = llr_total;
        c.bits_base = bits_total;
        llr_total += (size_t)slots_per_class * c.llr_bytes;
        bits_total += (size_t)slots_per_class * c.bits_bytes;
        c.llr_ring.init(slots_per_class);
        c.bits_ring.init(slots_per_class);
        // frames with host LLRs or host results hold a slot of one ring
        // each; frames with both in device memory cost at least N LLR bytes
        cap = std::max(cap, 2 * (size_t)slots_per_class + device_bytes / (size_t)c.llr_bytes);
      }
      if (cap > ((size_t)1 << 24)) cap = (size_t)1 << 24;
      s->desc_cap = (int)cap;
      s->cls_steps.assign(s->cls.size(), 0);
      s->dev_budget = device_bytes;
      s->sort_tmp.reserve(2 * (size_t)s->desc_cap);  // steps never allocate for it
      s->stage_size = staging_bytes;
      if (polar::dev_malloc((void**)&s->d_llr, llr_total) != hipSuccess ||
          polar::dev_malloc((void**)&s->d_bits, bits_total) != hipSuccess ||
          polar::dev_malloc((void**)&s->d_desc, (size_t)streams * s->desc_cap * 16) != hipSuccess ||
          polar::pinned_malloc((void**)&s->h_bits, bits_total) != hipSuccess ||
          polar::pinned_malloc((void**)&s->h_stage, staging_bytes) != hipSuccess ||
          polar::pinned_malloc((void**)&s->h_desc, (size_t)streams * s->desc_cap * 16) != hipSuccess)
        st = POLAR_ENOMEM;
      for (int i = 0; i < streams && st == POLAR_OK; ++i) {
        hipStream_t hs = nullptr;
        hipEvent_t ev = nullptr;
        if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) {
          st = POLAR_EDEVICE;
          break;
        }
        s->streams.push_back(hs);
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
          st = POLAR_EDEVICE;
          break;
        }
        s->events.push_back(ev);
        s->busy.push_back(false);
      }
    }
  } catch (const std::bad_alloc&) {
    st = POLAR_ENOMEM;
  }
  if (st != POLAR_OK) {
    free_server(s);
    polar_set_status(st);
    return nullptr;
  }
  polar_set_status(POLAR_OK);
  return s;
}

polar_status polar_server_submit(polar_server* s, int code_index, int nframes, const void* llr, int where,
                                 uint8_t* bits, int64_t* id) {
  const int llr_on_device = where & POLAR_SERVER_LLR_DEVICE;
  if (!s || code_index < 0 || code_index >= (int)s->code_n.size() || nframes < 1 || !llr || !bits || !id)
    return polar_set_status(POLAR_EINVAL);
  if (s->failed) return polar_set_status(POLAR_EDEVICE);
  const SizeClass& c = s->cls[s->code_cls[code_index]];
  const bool bits_on_device = (where & POLAR_SERVER_BITS_DEVICE) != 0;
  if (llr_on_device && ((uintptr_t)llr % (uintptr_t)s->elem) != 0) return polar_set_status(POLAR_EINVAL);
  const size_t bytes = (size_t)nframes * c.llr_bytes;
  Request r;
  r.code = code_index;
  r.cls = s->code_cls[code_index];
  r.nframes = nframes;
  r.bits = bits;
  r.dev_bits = bits_on_device;
  r.dev_bytes = (llr_on_device ? bytes : 0) + (bits_on_device ? (size_t)nframes * s->code_rb[code_index] : 0);
  // requests that could never be admitted
  if ((!llr_on_device && nframes > c.llr_ring.n) || (!bits_on_device && nframes > c.bits_ring.n) ||
      r.dev_bytes > s->dev_budget || (size_t)nframes > (size_t)s->desc_cap)
    return polar_set_status(POLAR_EINVAL);
  if (llr_on_device) {
    r.dev_llr = (const uint8_t*)llr;
  } else {
    const size_t head0 = s->stage_head, tail0 = s->stage_tail, used0 = s->stage_used;
    if (!stage_alloc(s, bytes, &r.stage_off, &r.stage_len)) return polar_set_status(POLAR_EAGAIN);
    r.stage_end = r.stage_off + ((bytes + 255) & ~(size_t)255);
    try {
      StageSeg g;
      g.end = r.stage_end;
      g.len = r.stage_len;
      s->stage_segs.push_back(g);
    } catch (const std::bad_alloc&) {
      s->stage_head = head0;  // undo the allocation
      s->stage_tail = tail0;
      s->stage_used = used0;
      return polar_set_status(POLAR_ENOMEM);
    }
    r.stage_seq = s->stage_base + (int64_t)s->stage_segs.size() - 1;
    memcpy(s->h_stage + r.stage_off, llr, bytes);
  }
  try {
    const int64_t rid = s->next_id++;
    s->reqs.emplace(rid, r);
    s->waiting.push_back(rid);
    *id = rid;
  } catch (const std::bad_alloc&) {
    return polar_set_status(POLAR_ENOMEM);
  }
  return polar_set_status(POLAR_OK);
}

polar_status polar_server_poll(polar_server* s, int64_t* done_ids, int cap, int* ndone) {
  if (!s || cap < 0 || !ndone) return polar_set_status(POLAR_EINVAL);
  *ndone = 0;
  const polar_status u = usable(s);
  if (u != POLAR_OK) return polar_set_status(u);
  try {
    polar_status st = retire(s, done_ids, cap, ndone);
    if (st == POLAR_OK) {
      admit(s);
      st = launch(s);
    }
    if (st != POLAR_OK) {
      s->failed = true;
      return polar_set_status(st);
    }
  } catch (const std::bad_alloc&) {
    return polar_set_status(POLAR_ENOMEM);
  }
  return polar_set_status(POLAR_OK);
}

polar_status polar_server_run_trace(polar_server* s, int nreq, const double* arrival_s, const int32_t* code_index,
                                    const int32_t* nframes, const void* const* llr, uint8_t* const* bits,
                                    double* completion_s) {
  if (!s || nreq < 0 || (nreq > 0 && (!arrival_s || !code_index || !nframes || !llr || !bits || !completion_s)))
    return polar_set_status(POLAR_EINVAL);
  const polar_status u = usable(s);
  if (u != POLAR_OK) return polar_set_status(u);
  typedef std::chrono::steady_clock clk;
  const clk::time_point t0 = clk::now();
  auto since = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };
  try {
    std::unordered_map<int64_t, int> which;
    std::vector<int64_t> done;
    int next = 0, finished = 0;
    while (finished < nreq) {
      const double now = since();
      while (next < nreq && arrival_s[next] <= now) {
        int64_t id = 0;
        const polar_status st = polar_server_submit(s, code_index[next], nframes[next], llr[next],
                                                    POLAR_SERVER_LLR_DEVICE | POLAR_SERVER_BITS_DEVICE, bits[next], &id);
        if (st != POLAR_OK) return st;
        which[id] = next++;
      }
      done.clear();
      int nd = 0;
      polar_status st = retire(s, nullptr, 0, &nd, &done);
      if (st == POLAR_OK) {
        admit(s);
        st = launch(s);
      }
      if (st != POLAR_OK) {
        s->failed = true;
        return polar_set_status(st);
      }
      if (!done.empty()) {
        const double t = since();
        for (int64_t id : done) {
          auto it = which.find(id);
          if (it != which.end()) {
            completion_s[it->second] = t;
            which.erase(it);
            ++finished;
          }
        }
      }
    }
  } catch (const std::bad_alloc&) {
    return polar_set_status(POLAR_ENOMEM);
  }
  return polar_set_status(POLAR_OK);
}

polar_status polar_server_pending(const polar_server* s, int* waiting, int* admitted, int* inflight_steps) {
  if (!s) return polar_set_status(POLAR_EINVAL);
  if (waiting) *waiting = (int)s->waiting.size();
  if (admitted) *admitted = (int)s->admitted.size();
  if (inflight_steps) *inflight_steps = (int)s->inflight.size();
  return polar_set_status(POLAR_OK);
}

polar_status polar_server_device_bytes(const polar_server* s, size_t* in_use, size_t* budget) {
  if (!s) return polar_set_status(POLAR_EINVAL);
  if (in_use) *in_use = s->dev_used;
  if (budget) *budget = s->dev_budget;
  return polar_set_status(POLAR_OK);
}

void polar_server_destroy(polar_server* s) {
  if (!s) return;
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  free_server(s);
}

}  // extern "C"
