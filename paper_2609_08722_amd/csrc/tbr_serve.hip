// tbr_serve.hip -- continuous batching of replay requests (tbr_serve_* in
// include/tbr.h).
//
// A scheduler thread owns the device side. Registered programs are copied
// once into a caller-provided device arena and stay resident. Submitted
// requests wait in a FIFO; each scheduler tick
//   1. retires finished launches (their HIP event has completed), freeing
//      the requests' arena bytes and slots,
//   2. admits queued requests in order while a slot is free and the arena
//      can hold the request's HBM footprint: its prepared stroke records,
//      and the outputs it asked the server to hold (arena_outputs),
//   3. packs every admitted-but-not-launched request into ONE persistent
//      launch (k_serve) over a list of (request, 16x16 tile) work items.
//      A tick is a captured hipGraph built once per stream: one copy of
//      the tick's descriptors and work list from pinned staging, a fill
//      kernel that clears the work cursor, one stroke-preparation launch
//      for all the tick's requests (k_serve_prep) and k_serve. Each tick
//      only updates the copy size and the two launches' grids and
//      arguments, then launches the graph.
// Launches rotate over several streams, so requests admitted while others
// are still on the GPU run concurrently with them. Each tile runs the same
// per-pixel device functions as tbr_render, so results do not depend on the
// mix. A host-only "fake device" executor (no HIP calls) models completion
// time for scheduler tests on machines without a GPU.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "tbr.h"
#include "tbr_kernels.hpp"

using namespace tbr;

namespace tbr {
extern thread_local std::string g_err;  // shared with tbr_last_error()
}  // namespace tbr

namespace {

tbr_status sfail(tbr_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
tbr_status sfail(tbr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing free list.
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0;
};

struct Program {
  int n, k;
  size_t off = 0, bytes = 0;  // arena copy: cx|cy|angle|length|half_width|logits|palette
};

enum ReqState { kQueued, kAdmitted, kRunning, kDone, kFailed, kCancelled };

// Arena-held outputs of a request, in this order after its stroke records.
struct OutLayout {
  size_t rgb, label, owner, total;  // offsets from the outputs' start; total bytes
};

OutLayout out_layout(int width, int height, int32_t mask) {
  OutLayout L{};
  const size_t P = (size_t)width * height;
  size_t off = 0;
  L.rgb = off;
  if (mask & TBR_OUT_RGB) off = align_up(off + P * 3 * sizeof(float));
  L.label = off;
  if (mask & TBR_OUT_LABEL) off = align_up(off + P * sizeof(int32_t));
  L.owner = off;
  if (mask & TBR_OUT_OWNER) off = align_up(off + P * sizeof(int32_t));
  L.total = off;
  return L;
}

struct Request {
  tbr_request req;
  uint64_t ticket;
  int n = 0, k = 0;
  size_t rec_off = 0, rec_bytes = 0;  // the footprint: records, then arena outputs
  size_t out_bytes = 0;
  OutLayout out{};
  int tiles = 0;
  ReqState state = kQueued;
  double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
};

// Launch buffers of one tick, at `off` in the arena and mirrored in pinned
// host staging: [ServeDesc x max_slots | ServePrep x max_slots |
// uint2 items x max_tick_items], then (device only) the work cursor.
struct TickLayout {
  size_t desc, prep, items, cursor, staging, total;
};

TickLayout tick_layout(const tbr_serve_opts* o);

struct Tick {
  bool busy = false;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  size_t off = 0;                // arena offset of the device launch buffers
  char* h_stage = nullptr;       // pinned staging, TickLayout::staging bytes
  hipGraph_t graph = nullptr;    // copy -> fill cursor -> prep -> serve
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t n_copy = nullptr, n_fill = nullptr, n_prep = nullptr, n_serve = nullptr;
  std::vector<uint64_t> tickets;
  double fake_done = 0;  // fake executor: modelled completion time
  bool fake_fail = false;  // fake executor: this launch reports a device error
};

}  // namespace

struct tbr_server {
  tbr_serve_opts opts{};
  char* base = nullptr;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  uint64_t next_program = 1, next_ticket = 1;
  std::map<uint64_t, Program> programs;
  std::map<uint64_t, Request> requests;
  std::deque<uint64_t> queue;    // submitted, not admitted (FIFO)
  std::vector<uint64_t> ready;   // admitted, not launched
  std::vector<Tick> ticks;
  int admitted = 0;              // admitted or running
  size_t fixed = 0;              // arena bytes held for good: launch buffers, programs
  int64_t launch_count = 0;
  tbr_serve_stats stats{};
  std::string error;             // first device error (fatal for the server)
};

namespace {

size_t program_bytes(int n, int k) {
  return align_up(((size_t)5 * n + (size_t)n * k + (size_t)3 * k) * sizeof(float));
}
size_t record_bytes(int n) { return align_up((size_t)(n > 0 ? n : 1) * sizeof(StrokeRec)); }

int tiles_of(const tbr_request& r) {
  return ((r.width + 15) / 16) * ((r.height + 15) / 16);
}

TickLayout tick_layout(const tbr_serve_opts* o) {
  TickLayout L{};
  size_t off = 0;
  L.desc = off;
  off = align_up(off + (size_t)o->max_slots * sizeof(ServeDesc));
  L.prep = off;
  off = align_up(off + (size_t)o->max_slots * sizeof(ServePrep));
  L.items = off;
  off = align_up(off + (size_t)o->max_tick_items * sizeof(uint2));
  L.staging = off;
  L.cursor = off;
  off = align_up(off + sizeof(int));
  L.total = off;
  return L;
}

// Kernel node parameters of the tick graph.
hipKernelNodeParams prep_node(int blocks, void** args) {
  hipKernelNodeParams kp{};
  kp.func = reinterpret_cast<void*>(&k_serve_prep);
  kp.gridDim = dim3(std::max(blocks, 1));
  kp.blockDim = dim3(256);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  return kp;
}

hipKernelNodeParams serve_node(int n_items, void** args) {
  hipKernelNodeParams kp{};
  kp.func = reinterpret_cast<void*>(&k_serve);
  // persistent grid: at most 8 blocks per CU, never more blocks than items
  kp.gridDim = dim3(std::max(1, std::min(n_items, 256 * 8)));
  kp.blockDim = dim3(256);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  return kp;
}

// Build the tick's graph once (with placeholder sizes that every launch
// overwrites). Returns a HIP error code.
hipError_t build_tick_graph(tbr_server* s, Tick& tk);

// Called with the lock held.
void retire(tbr_server* s) {
  const double t = now_s();
  for (auto& tk : s->ticks) {
    if (!tk.busy) continue;
    bool failed = false;
    if (s->opts.fake_device) {
      if (t < tk.fake_done) continue;
      failed = tk.fake_fail;
      if (failed && s->error.empty()) s->error = "device error (fake executor)";
    } else {
      hipError_t e = hipEventQuery(tk.done);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) {
        failed = true;
        if (s->error.empty()) s->error = hipGetErrorString(e);
      }
    }
    for (uint64_t id : tk.tickets) {
      auto it = s->requests.find(id);
      if (it == s->requests.end()) continue;
      Request& r = it->second;
      r.state = failed ? kFailed : kDone;
      r.t_done = t;
      // the records are free once the launch is over; arena outputs stay
      // until tbr_serve_release (or, for a failed request, its poll)
      s->arena.release(r.rec_off, r.rec_bytes);
      --s->admitted;
      if (!failed) {
        ++s->stats.completed;
        s->stats.pixel_strokes += (int64_t)r.req.width * r.req.height * r.n;
      }
    }
    tk.tickets.clear();
    tk.busy = false;
  }
}

void admit(tbr_server* s) {
  const double t = now_s();
  while (!s->queue.empty() && s->admitted < s->opts.max_slots) {
    uint64_t id = s->queue.front();
    Request& r = s->requests[id];
    size_t off;
    if (!s->arena.alloc(r.rec_bytes + r.out_bytes, &off)) break;  // wait for memory (FIFO)
    r.rec_off = off;
    r.state = kAdmitted;
    r.t_admit = t;
    s->queue.pop_front();
    s->ready.push_back(id);
    ++s->admitted;
  }
}

tbr_status launch(tbr_server* s) {
  if (s->ready.empty()) return TBR_OK;
  Tick* tk = nullptr;
  for (auto& c : s->ticks)
    if (!c.busy) {
      tk = &c;
      break;
    }
  if (!tk) return TBR_OK;
  // pack ready requests (in admission order) while the work list has room
  std::vector<uint64_t> take;
  int n_items = 0;
  size_t used = 0;
  // A request of at least solo_tiles tiles runs in a launch of its own:
  // requests of one launch retire together, so a large request packed with
  // small ones would hold them back, or be held back by them.
  const int solo = s->opts.solo_tiles;
  for (uint64_t id : s->ready) {
    Request& r = s->requests[id];
    if (take.size() >= (size_t)s->opts.max_slots) break;
    if (n_items + r.tiles > s->opts.max_tick_items) break;
    const bool big = solo > 0 && r.tiles >= solo;
    if (big && !take.empty()) break;
    take.push_back(id);
    n_items += r.tiles;
    ++used;
    if (big) break;
  }
  if (take.empty()) return TBR_OK;
  s->ready.erase(s->ready.begin(), s->ready.begin() + used);
  const double t = now_s();
  tk->busy = true;
  tk->tickets = take;
  ++s->stats.launches;
  ++s->launch_count;
  if (s->opts.fake_device) {
    tk->fake_fail = s->opts.fake_fail_launch > 0 && s->launch_count == s->opts.fake_fail_launch;
    double cost = 0;
    for (uint64_t id : take) {
      Request& r = s->requests[id];
      r.state = kRunning;
      r.t_start = t;
      cost += (double)r.req.width * r.req.height * r.n * s->opts.fake_ns_per_pixel_stroke * 1e-9;
    }
    tk->fake_done = t + cost;
    return TBR_OK;
  }
  const TickLayout TL = tick_layout(&s->opts);
  ServeDesc* h_desc = reinterpret_cast<ServeDesc*>(tk->h_stage + TL.desc);
  ServePrep* h_prep = reinterpret_cast<ServePrep*>(tk->h_stage + TL.prep);
  uint2* h_items = reinterpret_cast<uint2*>(tk->h_stage + TL.items);
  char* dbase = s->base + tk->off;
  int item = 0, blocks = 0;
  for (size_t j = 0; j < take.size(); ++j) {
    Request& r = s->requests[take[j]];
    const Program& pg = s->programs[r.req.program_id];
    float* pbase = reinterpret_cast<float*>(s->base + pg.off);
    const int n = pg.n, k = pg.k;
    KProgram kp{n, k, pbase, pbase + n, pbase + 2 * n, pbase + 3 * n, pbase + 4 * n,
                pbase + 5 * n, pbase + 5 * n + (size_t)n * k};
    // default 0.7 pixel, rounded once from double as tbr_render callers do
    float tau_min = r.req.tau_min > 0.f ? r.req.tau_min : (float)(0.7 / (double)r.req.width);
    KOpts ko{r.req.tau, tau_min, r.req.tau_c, r.req.eps_floor};
    StrokeRec* recs = reinterpret_cast<StrokeRec*>(s->base + r.rec_off);
    ServePrep q{};
    q.prog = kp;
    q.opts = ko;
    q.out = recs;
    q.block0 = blocks;
    h_prep[j] = q;
    blocks += (n + 255) / 256;
    ServeDesc d{};
    d.recs = recs;
    d.palette = kp.palette;
    char* outs = s->base + r.rec_off + r.rec_bytes;
    const int32_t m = r.req.arena_outputs;
    d.rgb = (m & TBR_OUT_RGB) ? reinterpret_cast<float*>(outs + r.out.rgb) : r.req.rgb;
    d.label = (m & TBR_OUT_LABEL) ? reinterpret_cast<int32_t*>(outs + r.out.label) : r.req.label;
    d.owner = (m & TBR_OUT_OWNER) ? reinterpret_cast<int32_t*>(outs + r.out.owner) : r.req.owner;
    d.n = n;
    d.width = r.req.width;
    d.height = r.req.height;
    d.tiles_x = (r.req.width + 15) / 16;
    d.soft = r.req.mode == TBR_SOFT ? 1 : 0;
    h_desc[j] = d;
    for (int q2 = 0; q2 < r.tiles; ++q2) h_items[item++] = make_uint2((unsigned)j, (unsigned)q2);
    r.state = kRunning;
    r.t_start = t;
  }
  // update the tick graph: copy size, prep grid, serve grid and arguments
  const ServePrep* d_prep = reinterpret_cast<const ServePrep*>(dbase + TL.prep);
  const ServeDesc* d_desc = reinterpret_cast<const ServeDesc*>(dbase + TL.desc);
  const uint2* d_items = reinterpret_cast<const uint2*>(dbase + TL.items);
  int* d_cursor = reinterpret_cast<int*>(dbase + TL.cursor);
  int n_req = (int)take.size();
  void* prep_args[2] = {&d_prep, &n_req};
  void* serve_args[4] = {&d_desc, &d_items, &n_items, &d_cursor};
  hipKernelNodeParams pp = prep_node(blocks, prep_args);
  hipKernelNodeParams sp = serve_node(n_items, serve_args);
  const size_t bytes = TL.items + (size_t)n_items * sizeof(uint2);
  hipError_t e = hipGraphExecMemcpyNodeSetParams1D(tk->exec, tk->n_copy, dbase, tk->h_stage,
                                                  bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(tk->exec, tk->n_prep, &pp);
  if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(tk->exec, tk->n_serve, &sp);
  if (e == hipSuccess) e = hipGraphLaunch(tk->exec, tk->stream);
  if (e == hipSuccess) e = hipEventRecord(tk->done, tk->stream);
  if (e != hipSuccess) return sfail(TBR_E_DEVICE, "serve launch: %s", hipGetErrorString(e));
  return TBR_OK;
}

hipError_t build_tick_graph(tbr_server* s, Tick& tk) {
  const TickLayout TL = tick_layout(&s->opts);
  char* dbase = s->base + tk.off;
  const ServePrep* d_prep = reinterpret_cast<const ServePrep*>(dbase + TL.prep);
  const ServeDesc* d_desc = reinterpret_cast<const ServeDesc*>(dbase + TL.desc);
  const uint2* d_items = reinterpret_cast<const uint2*>(dbase + TL.items);
  int* d_cursor = reinterpret_cast<int*>(dbase + TL.cursor);
  int one = 1, zero = 0, n_req = 1, n_items = 0;
  hipError_t e = hipGraphCreate(&tk.graph, 0);
  if (e != hipSuccess) return e;
  e = hipGraphAddMemcpyNode1D(&tk.n_copy, tk.graph, nullptr, 0, dbase, tk.h_stage, TL.staging,
                              hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  // the cursor is cleared by a fill kernel, not a memset node
  void* fill_args[3] = {&d_cursor, &one, &zero};
  hipKernelNodeParams fp{};
  fp.func = reinterpret_cast<void*>(&k_fill_i32);
  fp.gridDim = dim3(1);
  fp.blockDim = dim3(64);
  fp.kernelParams = fill_args;
  e = hipGraphAddKernelNode(&tk.n_fill, tk.graph, &tk.n_copy, 1, &fp);
  if (e != hipSuccess) return e;
  void* prep_args[2] = {&d_prep, &n_req};
  hipKernelNodeParams pp = prep_node(1, prep_args);
  e = hipGraphAddKernelNode(&tk.n_prep, tk.graph, &tk.n_fill, 1, &pp);
  if (e != hipSuccess) return e;
  void* serve_args[4] = {&d_desc, &d_items, &n_items, &d_cursor};
  hipKernelNodeParams sp = serve_node(n_items, serve_args);
  e = hipGraphAddKernelNode(&tk.n_serve, tk.graph, &tk.n_prep, 1, &sp);
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&tk.exec, tk.graph, nullptr, nullptr, 0);
}

void worker_loop(tbr_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    retire(s);
    admit(s);
    if (s->error.empty()) {
      tbr_status st = launch(s);
      if (st != TBR_OK && s->error.empty()) s->error = g_err;
    }
    bool busy = false;
    for (auto& tk : s->ticks) busy |= tk.busy;
    // sleep briefly while launches run; wake at once on submit / stop
    s->cv.wait_for(lk, std::chrono::microseconds(busy ? 50 : 2000));
  }
}

tbr_status check_serve_opts(const tbr_serve_opts* o) {
  if (!o) return sfail(TBR_E_INVALID, "opts is NULL");
  if (o->max_slots < 1 || o->max_queue < 1 || o->max_tick_items < 1)
    return sfail(TBR_E_INVALID, "max_slots, max_queue and max_tick_items must be >= 1");
  if (o->streams < 1 || o->streams > 4) return sfail(TBR_E_INVALID, "streams must be 1..4");
  if (!o->fake_device && (!o->arena || o->arena_bytes == 0))
    return sfail(TBR_E_INVALID, "arena is NULL or empty");
  if (o->fake_device && !(o->fake_ns_per_pixel_stroke >= 0.f))
    return sfail(TBR_E_INVALID, "fake_ns_per_pixel_stroke must be >= 0");
  return TBR_OK;
}

}  // namespace

extern "C" {

size_t tbr_serve_tick_bytes(const tbr_serve_opts* opts) {
  if (!opts || opts->max_slots < 1 || opts->max_tick_items < 1) return 0;
  return tick_layout(opts).total;
}

size_t tbr_serve_program_bytes(int32_t n_strokes, int32_t n_palette) {
  if (n_strokes < 0 || n_palette < 1) return 0;
  return program_bytes(n_strokes, n_palette);
}

size_t tbr_serve_request_bytes(int32_t n_strokes) {
  if (n_strokes < 0) return 0;
  return record_bytes(n_strokes);
}

size_t tbr_serve_output_bytes(int32_t width, int32_t height, int32_t arena_outputs) {
  if (width < 1 || height < 1 || (arena_outputs & ~TBR_OUT_ALL)) return 0;
  return out_layout(width, height, arena_outputs).total;
}

tbr_status tbr_serve_create(const tbr_serve_opts* opts, tbr_server** out) {
  tbr_status st;
  if ((st = check_serve_opts(opts))) return st;
  if (!out) return sfail(TBR_E_INVALID, "out is NULL");
  tbr_server* s = new tbr_server();
  s->opts = *opts;
  s->base = static_cast<char*>(opts->arena);
  s->arena.init(opts->arena_bytes);
  s->ticks.resize(opts->streams);
  const TickLayout TL = tick_layout(opts);
  for (auto& tk : s->ticks) {
    size_t off;
    if (!s->arena.alloc(TL.total, &off)) {
      tbr_serve_destroy(s);
      return sfail(TBR_E_NOMEM, "arena too small for %d launch buffers", opts->streams);
    }
    tk.off = off;
    s->fixed += align_up(TL.total);
    if (!opts->fake_device) {
      hipError_t e = hipStreamCreateWithFlags(&tk.stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&tk.done, hipEventDisableTiming);
      if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&tk.h_stage), TL.staging,
                          hipHostMallocDefault);
      if (e == hipSuccess) e = build_tick_graph(s, tk);
      if (e != hipSuccess) {
        tbr_serve_destroy(s);
        return sfail(TBR_E_DEVICE, "serve create: %s", hipGetErrorString(e));
      }
    }
  }
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return TBR_OK;
}

tbr_status tbr_serve_register_program(tbr_server* s, const tbr_program* p, uint64_t* program_id) {
  if (!s || !p || !program_id) return sfail(TBR_E_INVALID, "null argument");
  if (p->n_strokes < 0 || p->n_palette < 1 || p->n_palette > 64)
    return sfail(TBR_E_INVALID, "n_strokes %d / n_palette %d out of range", p->n_strokes,
                 p->n_palette);
  if (!s->opts.fake_device &&
      (!p->palette || (p->n_strokes > 0 && (!p->cx || !p->cy || !p->angle || !p->length ||
                                             !p->half_width || !p->logits))))
    return sfail(TBR_E_INVALID, "a program array is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  Program pg;
  pg.n = p->n_strokes;
  pg.k = p->n_palette;
  pg.bytes = program_bytes(pg.n, pg.k);
  if (!s->arena.alloc(pg.bytes, &pg.off))
    return sfail(TBR_E_NOMEM, "arena cannot hold a %d-stroke program", pg.n);
  if (!s->opts.fake_device) {
    const int n = pg.n, k = pg.k;
    float* dst = reinterpret_cast<float*>(s->base + pg.off);
    const float* srcs[7] = {p->cx, p->cy, p->angle, p->length, p->half_width, p->logits, p->palette};
    size_t cnt[7] = {(size_t)n, (size_t)n, (size_t)n, (size_t)n, (size_t)n, (size_t)n * k,
                     (size_t)3 * k};
    hipError_t e = hipSuccess;
    for (int f = 0; f < 7 && e == hipSuccess; ++f) {
      if (cnt[f]) e = hipMemcpy(dst, srcs[f], cnt[f] * sizeof(float), hipMemcpyDeviceToDevice);
      dst += cnt[f];
    }
    if (e != hipSuccess) {
      s->arena.release(pg.off, pg.bytes);
      return sfail(TBR_E_DEVICE, "register copy: %s", hipGetErrorString(e));
    }
  }
  *program_id = s->next_program++;
  s->programs[*program_id] = pg;
  s->fixed += align_up(pg.bytes);
  return TBR_OK;
}

tbr_status tbr_serve_submit(tbr_server* s, const tbr_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return sfail(TBR_E_INVALID, "null argument");
  if (req->mode != TBR_SOFT && req->mode != TBR_HARD)
    return sfail(TBR_E_INVALID, "mode must be TBR_SOFT or TBR_HARD");
  if (req->width < 1 || req->width > 16384 || req->height < 1 || req->height > 16384)
    return sfail(TBR_E_INVALID, "canvas %dx%d outside 1..16384", req->width, req->height);
  if (!(req->tau >= 0.f) || !(req->tau_c >= 0.f) || !(req->eps_floor > 0.f))
    return sfail(TBR_E_INVALID, "tau, tau_c must be >= 0 and eps_floor > 0");
  const int32_t m = req->arena_outputs;
  if (m & ~TBR_OUT_ALL) return sfail(TBR_E_INVALID, "arena_outputs %d is not a TBR_OUT_* mask", m);
  if (req->mode == TBR_SOFT && (m & (TBR_OUT_LABEL | TBR_OUT_OWNER)))
    return sfail(TBR_E_INVALID, "a soft request has only an rgb output");
  if (((m & TBR_OUT_RGB) && req->rgb) || ((m & TBR_OUT_LABEL) && req->label) ||
      ((m & TBR_OUT_OWNER) && req->owner))
    return sfail(TBR_E_INVALID, "an output held in the arena must have a NULL pointer");
  if (!s->opts.fake_device) {
    const bool rgb = req->rgb || (m & TBR_OUT_RGB);
    if (req->mode == TBR_SOFT && !rgb) return sfail(TBR_E_INVALID, "soft request without rgb");
    if (req->mode == TBR_HARD && !rgb && !req->label && !req->owner && !(m & TBR_OUT_LABEL) &&
        !(m & TBR_OUT_OWNER))
      return sfail(TBR_E_INVALID, "hard request without any output");
  }
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->error.empty()) return sfail(TBR_E_DEVICE, "server failed: %s", s->error.c_str());
  auto pit = s->programs.find(req->program_id);
  if (pit == s->programs.end()) return sfail(TBR_E_NOTFOUND, "unknown program id");
  Request r;
  r.req = *req;
  r.n = pit->second.n;
  r.k = pit->second.k;
  r.rec_bytes = record_bytes(r.n);
  r.out = out_layout(req->width, req->height, m);
  r.out_bytes = r.out.total;
  r.tiles = tiles_of(*req);
  if (r.tiles > s->opts.max_tick_items)
    return sfail(TBR_E_NOMEM, "request has %d tiles > max_tick_items %d", r.tiles,
                 s->opts.max_tick_items);
  if (r.rec_bytes + r.out_bytes > s->arena.size() - s->fixed)
    return sfail(TBR_E_NOMEM, "request footprint %zu bytes exceeds the arena's %zu free of "
                 "launch buffers and programs", r.rec_bytes + r.out_bytes,
                 s->arena.size() - s->fixed);
  if ((int)s->queue.size() >= s->opts.max_queue) return sfail(TBR_E_CAPACITY, "queue full");
  r.ticket = s->next_ticket++;
  r.t_submit = now_s();
  s->requests[r.ticket] = r;
  s->queue.push_back(r.ticket);
  ++s->stats.submitted;
  *ticket = r.ticket;
  lk.unlock();
  s->cv.notify_one();
  return TBR_OK;
}

tbr_status tbr_serve_poll(tbr_server* s, uint64_t ticket, tbr_result* out) {
  if (!s || !out) return sfail(TBR_E_INVALID, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return sfail(TBR_E_NOTFOUND, "unknown ticket");
  const Request& r = it->second;
  out->t_submit = r.t_submit;
  out->t_admit = r.t_admit;
  out->t_start = r.t_start;
  out->t_done = r.t_done;
  out->pixel_strokes = (int64_t)r.req.width * r.req.height * r.n;
  out->rgb = r.req.rgb;
  out->label = r.req.label;
  out->owner = r.req.owner;
  if (r.state == kDone) {
    out->status = TBR_OK;
    if (r.out_bytes == 0) {
      s->requests.erase(it);
      return TBR_OK;
    }
    // outputs held in the arena: their addresses, until tbr_serve_release
    const int32_t m = r.req.arena_outputs;
    char* outs = s->opts.fake_device ? nullptr : s->base + r.rec_off + r.rec_bytes;
    if (outs) {
      if (m & TBR_OUT_RGB) out->rgb = reinterpret_cast<float*>(outs + r.out.rgb);
      if (m & TBR_OUT_LABEL) out->label = reinterpret_cast<int32_t*>(outs + r.out.label);
      if (m & TBR_OUT_OWNER) out->owner = reinterpret_cast<int32_t*>(outs + r.out.owner);
    }
    return TBR_OK;
  }
  if (r.state == kFailed) {
    out->status = TBR_E_DEVICE;
    if (r.out_bytes) s->arena.release(r.rec_off + r.rec_bytes, r.out_bytes);
    s->requests.erase(it);
    return sfail(TBR_E_DEVICE, "request failed on the device: %s", s->error.c_str());
  }
  if (r.state == kCancelled) {
    out->status = TBR_E_CANCELLED;
    s->requests.erase(it);
    return TBR_E_CANCELLED;
  }
  if (!s->error.empty()) {
    out->status = TBR_E_DEVICE;
    return sfail(TBR_E_DEVICE, "server failed: %s", s->error.c_str());
  }
  out->status = TBR_PENDING;
  return TBR_PENDING;
}

tbr_status tbr_serve_release(tbr_server* s, uint64_t ticket) {
  if (!s) return sfail(TBR_E_INVALID, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return sfail(TBR_E_NOTFOUND, "unknown ticket");
  Request& r = it->second;
  if (r.state != kDone) {
    if (r.state == kFailed || r.state == kCancelled)
      return sfail(TBR_E_INVALID, "the ticket ended without outputs: poll it");
    return TBR_PENDING;
  }
  if (r.out_bytes) s->arena.release(r.rec_off + r.rec_bytes, r.out_bytes);
  s->requests.erase(it);
  lk.unlock();
  s->cv.notify_one();  // the freed bytes may admit a waiting request
  return TBR_OK;
}

tbr_status tbr_serve_cancel(tbr_server* s, uint64_t ticket) {
  if (!s) return sfail(TBR_E_INVALID, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return sfail(TBR_E_NOTFOUND, "unknown ticket");
  if (it->second.state != kQueued) return TBR_PENDING;  // already admitted: runs to completion
  auto q = std::find(s->queue.begin(), s->queue.end(), ticket);
  if (q != s->queue.end()) s->queue.erase(q);
  it->second.state = kCancelled;
  ++s->stats.cancelled;
  return TBR_OK;
}

tbr_status tbr_serve_get_stats(tbr_server* s, tbr_serve_stats* out) {
  if (!s || !out) return sfail(TBR_E_INVALID, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  *out = s->stats;
  out->queued = (int64_t)s->queue.size();
  out->in_flight = s->admitted;
  out->arena_used = s->arena.used();
  out->arena_bytes = s->arena.size();
  return TBR_OK;
}

void tbr_serve_destroy(tbr_server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& tk : s->ticks) {
    if (tk.stream) (void)hipStreamSynchronize(tk.stream);
    if (tk.exec) (void)hipGraphExecDestroy(tk.exec);
    if (tk.graph) (void)hipGraphDestroy(tk.graph);
    if (tk.done) (void)hipEventDestroy(tk.done);
    if (tk.stream) (void)hipStreamDestroy(tk.stream);
    if (tk.h_stage) (void)hipHostFree(tk.h_stage);
  }
  delete s;
}

double tbr_serve_now(void) { return now_s(); }

}  // extern "C"
