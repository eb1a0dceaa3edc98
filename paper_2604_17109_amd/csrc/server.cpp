// Request server with continuous batching for real-valued Ising requests (the
// MIMO detection service of Suppl. "PIMI FPGA implementation for MIMO
// detection", host-side task scheduling; here on one GPU).
//
// Device-resident slot table: per N class (N rounded up to 32) a fixed array
// of slots split into chunks of `max_batch` slots.  A request is admitted into
// the open chunk of its class when a chunk and the device-memory budget allow;
// its binary64 couplings are copied into the chunk's pinned staging area and
// quantised and packed into MFMA fragments on the device at launch.
// pim_server_flush launches every due chunk on one of several streams (one
// whose last launch has finished, if any): upload, the FP8/BF16 sweep over the chunk's
// requests (32-trial waves), the binary64 re-rank and selection, and the
// readback of the selected states into pinned memory, all asynchronous.  New
// arrivals keep being admitted into fresh chunks and launched on other
// streams while earlier chunks run, so their work overlaps on the device.
// pim_server_poll collects finished chunks without blocking and frees them.
//
// Every request's noise comes from counter stream = its request id, so its
// result does not depend on the chunk, slot or launch it lands in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace pim {
namespace {

// Seconds on the host's monotonic clock (CLOCK_MONOTONIC on Linux).
double mono_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Chunk {
  int cls = 0;
  int count = 0;                 // requests admitted into this chunk
  bool launched = false;
  std::chrono::steady_clock::time_point first;  // admission of its first request
  hipEvent_t done = nullptr;
  std::vector<uint32_t> ids;
  std::vector<int32_t> ns;
  std::vector<double> t_admit;   // per request: admission time (host monotonic clock, s)
  double t_launch = 0.0;         // when pim_server_flush issued the chunk
  // pinned host staging (inputs) and results, each one contiguous block
  // (h_in / d_in, h_out / d_out) of sections; the result block is read back
  // by one copy.  Both host blocks are mapped into the device's address space
  // (dh_in / dh_out) and copied by kernels on the chunk's stream.
  uint8_t* h_in = nullptr;
  uint8_t* d_in = nullptr;
  uint8_t* h_out = nullptr;
  uint8_t* d_out = nullptr;
  uint8_t* dh_in = nullptr;
  uint8_t* dh_out = nullptr;
  size_t in_bytes = 0, out_bytes = 0;
  uint8_t* h_frag = nullptr;
  float* h_hf = nullptr;
  float* h_scale = nullptr;
  double* h_j64 = nullptr;
  double* h_h64 = nullptr;
  uint32_t* h_sid = nullptr;
  MimoSlot* h_slots = nullptr;   // MIMO requests: per slot dimensions and H / y offset
  double* h_hy = nullptr;        // MIMO requests: H then y of each request, packed
  size_t hy_used = 0;            // doubles of h_hy in use
  size_t max_work = 0, max_hy = 0;  // largest mapping workspace / H + y among its MIMO requests
  double* h_xm = nullptr;        // results: x_m per slot
  int8_t* h_spins = nullptr;
  double* h_e = nullptr;
  int32_t* h_sel = nullptr;
  // device
  uint8_t* d_frag = nullptr;
  float* d_hf = nullptr;
  float* d_scale = nullptr;
  double* d_j64 = nullptr;
  double* d_h64 = nullptr;
  uint32_t* d_sid = nullptr;
  MimoSlot* d_slots = nullptr;
  double* d_hy = nullptr;
  double* d_xm = nullptr;
  const double** d_j64p = nullptr;
  const double** d_h64p = nullptr;
  int8_t* d_final = nullptr;
  int8_t* d_best = nullptr;
  int32_t* d_stats = nullptr;
  double* d_rerank = nullptr;
  int8_t* d_sel_spins = nullptr;
  double* d_sel_e = nullptr;
  int32_t* d_sel_i = nullptr;
};

struct Klass {
  int nt = 0, npad = 0;
  size_t frag = 0;
  std::vector<Chunk*> chunks;
  int open = -1;                 // chunk accepting requests, or -1
};

// Persistent host workers for the per-request parts of pim_server_submit
// (validation and staging copies of large binary64 couplings).  run() hands
// out item indices through an atomic counter; the calling thread works too
// and returns when every item is done.
class Pool {
 public:
  explicit Pool(int workers) {
    for (int i = 0; i < workers; ++i) threads_.emplace_back([this] { loop(); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> g(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }
  // f(i) for i in [0, count) on the workers and the calling thread; returns
  // when every call has returned.  f must not throw.
  void run(int count, const std::function<void(int)>& f) {
    if (count <= 0) return;
    {
      std::lock_guard<std::mutex> g(m_);
      fn_ = &f;
      total_ = count;
      next_.store(0);
      active_ = (int)threads_.size();
      ++gen_;
    }
    cv_.notify_all();
    for (int i; (i = next_.fetch_add(1)) < count;) f(i);
    std::unique_lock<std::mutex> g(m_);
    done_cv_.wait(g, [this] { return active_ == 0; });
    fn_ = nullptr;
  }

 private:
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int)>* f;
      int total;
      {
        std::unique_lock<std::mutex> g(m_);
        cv_.wait(g, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        f = fn_;
        total = total_;
      }
      for (int i; (i = next_.fetch_add(1)) < total;) (*f)(i);
      std::lock_guard<std::mutex> g(m_);
      if (--active_ == 0) done_cv_.notify_one();
    }
  }
  std::vector<std::thread> threads_;
  std::mutex m_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* fn_ = nullptr;
  int total_ = 0, active_ = 0;
  std::atomic<int> next_{0};
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// Checks a request (J finite, symmetric with a zero diagonal; h finite) while
// staging it: J (n x n) into j64 (np x np, zero-padded) and h into h64 (np,
// zero-padded).  J is walked in kTile x kTile tiles, each compared with and
// copied together with its transpose, so both stay in cache and J is read
// once.  This call handles the tile rows that start in [i0, i1): their tiles
// on and right of the diagonal (and the transposes, which land in other rows
// but in columns below i1, so no element is written by two calls), and the
// diagonal, padding columns and h of rows i0 .. i1 - 1; the call whose range
// ends at n also clears the padding rows.  Returns false (staging then
// incomplete) if the request is invalid in that part.
constexpr int kTile = 16;

bool validate_and_stage_rows(const double* J, const double* h, int n, size_t np, double* j64, double* h64, int i0,
                             int i1) {
  for (int i = i0; i < i1; ++i) {
    if (J[(size_t)i * n + i] != 0.0 || (h && !std::isfinite(h[i]))) return false;
    h64[i] = h ? h[i] : 0.0;
  }
  for (int ib = i0; ib < i1; ib += kTile)
    for (int jb = ib; jb < n; jb += kTile) {
      const int ie = std::min(ib + kTile, n), je = std::min(jb + kTile, n);
      for (int i = ib; i < ie; ++i)
        for (int j = std::max(jb, i + 1); j < je; ++j) {
          const double a = J[(size_t)i * n + j];
          if (!std::isfinite(a) || a != J[(size_t)j * n + i]) return false;
          j64[(size_t)i * np + j] = a;
          j64[(size_t)j * np + i] = a;
        }
    }
  for (int i = i0; i < i1; ++i) {
    j64[(size_t)i * np + i] = 0.0;
    std::fill(j64 + (size_t)i * np + n, j64 + (size_t)(i + 1) * np, 0.0);
  }
  if (i1 == n) {
    std::fill(h64 + n, h64 + np, 0.0);
    std::fill(j64 + (size_t)n * np, j64 + np * np, 0.0);
  }
  return true;
}

// Submissions whose couplings total fewer elements than kParallelElems run on
// the calling thread alone (waking the workers would cost more than it
// saves), with one exception: a submission of fewer than kFewRequests
// requests that still holds kSplitElems elements splits its requests of at
// least kSplitN spins into strips of kTile rows, so that one large request is
// staged by several threads.  Large submissions keep whole requests as work
// items, which keeps each request's reads in one thread's cache.
constexpr size_t kParallelElems = (size_t)1 << 17;
constexpr size_t kSplitElems = (size_t)1 << 15;
constexpr int kFewRequests = 8;
constexpr int kSplitN = 96;

}  // namespace
}  // namespace pim

struct pim_server {
  pim_server_config cfg{};
  bool mimo = false;                 // requests are MIMO problems (H, y), mapped on the device
  pim::Rule rule;
  std::vector<double> beta, eta;
  std::vector<pim::Klass> classes;   // index nt - 1
  float* d_thtab = nullptr;
  int32_t* d_zero = nullptr;         // class ids (all 0) for max_batch instances
  int32_t* d_cancel = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> stream_idle;  // recorded after the last launch on each stream
  int next_stream = 0;
  std::deque<pim::Chunk*> inflight;  // launch order
  size_t bytes = 0;                  // device bytes held by slots
  std::unique_ptr<pim::Pool> pool;   // submit workers
};

using namespace pim;

namespace {

struct Layout;
Layout layout(const pim_server* s, const Klass& k);

void free_chunk(Chunk* c) {
  if (c->done) (void)hipEventDestroy(c->done);
  for (void* p : {(void*)c->h_in, (void*)c->h_out})
    if (p) (void)hipHostFree(p);
  for (void* p : {(void*)c->d_in, (void*)c->d_out, (void*)c->d_j64p, (void*)c->d_h64p, (void*)c->d_final,
                  (void*)c->d_best, (void*)c->d_stats, (void*)c->d_rerank})
    dev_free(p, nullptr);
  delete c;
}

template <typename T>
bool host_alloc(T** p, size_t count, unsigned flags = hipHostMallocDefault) {
  return hipHostMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T), flags) == hipSuccess;
}
template <typename T>
bool dev_alloc_n(T** p, size_t count) {
  *p = (T*)dev_alloc(std::max<size_t>(count, 1) * sizeof(T), nullptr);
  return *p != nullptr;
}

// Offsets (each 256-B aligned) of the input block and of the result block
// (spins | energies | (trial, step, tracked) | x_m of MIMO requests).  Couplings
// staged on the host: frag | hf | scale | j64 | h64 | sid, all uploaded from the
// host copy.  MIMO requests: sid | slots | hy first (the part uploaded from the
// host, host_in_bytes), then the device-only frag | hf | scale | j64 | h64.
struct Layout {
  size_t frag, hf, scale, j64, h64, pmax, sid, slots, hy, in_bytes, host_in_bytes;
  size_t spins, e, sel, xm, out_bytes;
};
size_t al(size_t x) { return (x + 255) & ~size_t(255); }
// Doubles of H (Nr x Nt complex) and y (Nr complex) a MIMO request of class
// npad can bring: Nr <= npad / 2 and Nt <= npad / 2.
size_t hy_slot_doubles(size_t np) { return np * np / 2 + np; }
// x_m values returned per MIMO request: 2 Nt <= min(npad, PIM_MAX_N_LDS / 2).
size_t xm_stride(size_t np) { return std::min<size_t>(np, PIM_MAX_N_LDS / 2); }
Layout layout(const pim_server* s, const Klass& k) {
  const size_t B = s->cfg.max_batch, np = k.npad;
  Layout L{};
  if (s->mimo) {
    L.sid = 0;
    L.slots = al(B * 4);
    L.hy = al(L.slots + B * sizeof(MimoSlot));
    L.host_in_bytes = al(L.hy + B * hy_slot_doubles(np) * 8);
    L.frag = L.host_in_bytes;
  } else {
    L.frag = 0;
  }
  L.hf = al(L.frag + B * k.frag);
  L.scale = al(L.hf + B * np * 4);
  L.j64 = al(L.scale + B * 4);
  L.h64 = al(L.j64 + B * np * np * 8);
  L.pmax = al(L.h64 + B * np * 8);
  if (s->mimo) {
    L.in_bytes = al(L.pmax + B * kPackSlices * 8);
  } else {
    L.sid = al(L.pmax + B * kPackSlices * 8);
    L.in_bytes = al(L.sid + B * 4);
    L.host_in_bytes = L.in_bytes;
  }
  L.spins = 0;
  L.e = al(B * np);
  L.sel = al(L.e + B * 8);
  L.xm = al(L.sel + 3 * B * 4);
  L.out_bytes = s->mimo ? al(L.xm + B * xm_stride(np) * 8) : L.xm;
  return L;
}

Chunk* new_chunk(pim_server* s, int cls) {
  const Klass& k = s->classes[cls];
  const size_t B = s->cfg.max_batch, R = s->cfg.trials, np = k.npad;
  const Layout L = layout(s, k);
  auto* c = new Chunk();
  c->cls = cls;
  c->in_bytes = L.in_bytes;
  c->out_bytes = L.out_bytes;
  bool ok = hipEventCreateWithFlags(&c->done, hipEventDisableTiming) == hipSuccess;
  // coherent (not cached by the device) and device-mapped, so copy kernels
  // can read the staged requests and write the results directly
  const unsigned hflags = hipHostMallocMapped | hipHostMallocCoherent;
  ok = ok && host_alloc(&c->h_in, L.host_in_bytes, hflags) && host_alloc(&c->h_out, L.out_bytes, hflags) &&
       dev_alloc_n(&c->d_in, L.in_bytes) && dev_alloc_n(&c->d_out, L.out_bytes);
  if (ok)
    ok = hipHostGetDevicePointer((void**)&c->dh_in, c->h_in, 0) == hipSuccess &&
         hipHostGetDevicePointer((void**)&c->dh_out, c->h_out, 0) == hipSuccess && c->dh_in && c->dh_out;
  ok = ok && dev_alloc_n(&c->d_j64p, B) && dev_alloc_n(&c->d_h64p, B) && dev_alloc_n(&c->d_final, B * R * np) &&
       dev_alloc_n(&c->d_best, B * R * np) && dev_alloc_n(&c->d_stats, 5 * B * R) &&
       dev_alloc_n(&c->d_rerank, B * R);
  if (ok) {
    if (s->mimo) {
      c->h_slots = reinterpret_cast<MimoSlot*>(c->h_in + L.slots);
      c->h_hy = reinterpret_cast<double*>(c->h_in + L.hy);
      c->d_slots = reinterpret_cast<MimoSlot*>(c->d_in + L.slots);
      c->d_hy = reinterpret_cast<double*>(c->d_in + L.hy);
      c->h_xm = reinterpret_cast<double*>(c->h_out + L.xm);
      c->d_xm = reinterpret_cast<double*>(c->d_out + L.xm);
    } else {
      c->h_frag = c->h_in + L.frag;
      c->h_hf = reinterpret_cast<float*>(c->h_in + L.hf);
      c->h_scale = reinterpret_cast<float*>(c->h_in + L.scale);
      c->h_j64 = reinterpret_cast<double*>(c->h_in + L.j64);
      c->h_h64 = reinterpret_cast<double*>(c->h_in + L.h64);
    }
    c->h_sid = reinterpret_cast<uint32_t*>(c->h_in + L.sid);
    c->d_frag = c->d_in + L.frag;
    c->d_hf = reinterpret_cast<float*>(c->d_in + L.hf);
    c->d_scale = reinterpret_cast<float*>(c->d_in + L.scale);
    c->d_j64 = reinterpret_cast<double*>(c->d_in + L.j64);
    c->d_h64 = reinterpret_cast<double*>(c->d_in + L.h64);
    c->d_sid = reinterpret_cast<uint32_t*>(c->d_in + L.sid);
    c->h_spins = reinterpret_cast<int8_t*>(c->h_out + L.spins);
    c->h_e = reinterpret_cast<double*>(c->h_out + L.e);
    c->h_sel = reinterpret_cast<int32_t*>(c->h_out + L.sel);
    c->d_sel_spins = reinterpret_cast<int8_t*>(c->d_out + L.spins);
    c->d_sel_e = reinterpret_cast<double*>(c->d_out + L.e);
    c->d_sel_i = reinterpret_cast<int32_t*>(c->d_out + L.sel);
    // per-request pointer tables of the re-rank, fixed for the chunk's lifetime
    std::vector<const double*> jp(B), hp(B);
    for (size_t i = 0; i < B; ++i) {
      jp[i] = c->d_j64 + i * np * np;
      hp[i] = c->d_h64 + i * np;
    }
    ok = hipMemcpy((void*)c->d_j64p, jp.data(), B * sizeof(void*), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy((void*)c->d_h64p, hp.data(), B * sizeof(void*), hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) {
    free_chunk(c);
    return nullptr;
  }
  return c;
}

// A chunk of class cls with room (not launched, not full), or nullptr when
// none can be had.  Full chunks stay staged until the next flush.
Chunk* chunk_for(pim_server* s, int cls) {
  Klass& k = s->classes[cls];
  if (k.open >= 0 && !k.chunks[k.open]->launched && k.chunks[k.open]->count < s->cfg.max_batch)
    return k.chunks[k.open];
  k.open = -1;
  for (size_t i = 0; i < k.chunks.size(); ++i)
    if (!k.chunks[i]->launched && k.chunks[i]->count < s->cfg.max_batch) {
      k.open = (int)i;
      return k.chunks[i];
    }
  if ((int)k.chunks.size() >= s->cfg.slots_per_class / s->cfg.max_batch) return nullptr;
  const Layout L = layout(s, k);
  const size_t B = s->cfg.max_batch, R = s->cfg.trials;
  const size_t need = L.in_bytes + L.out_bytes + B * (2 * sizeof(void*) + R * (2 * (size_t)k.npad + 5 * 4 + 8));
  if (s->cfg.hbm_budget && s->bytes + need > s->cfg.hbm_budget) return nullptr;
  Chunk* c = new_chunk(s, cls);
  if (!c) return nullptr;
  s->bytes += need;
  k.chunks.push_back(c);
  k.open = (int)k.chunks.size() - 1;
  return c;
}

hipError_t launch_chunk(pim_server* s, Chunk* c, hipStream_t st) {
  const Klass& k = s->classes[c->cls];
  const size_t B = c->count, R = s->cfg.trials, np = k.npad;
  // the used part of each input section (the result block is small and read
  // back whole)
  hipError_t e = hipSuccess;
  if (s->mimo) {
    // ids, slot records and the packed (H, y) are one contiguous prefix of
    // the block: one upload (a copy kernel reading the mapped host block, so
    // the chunk never waits on a copy engine), then the Ising instances are
    // built on the device
    const Layout L = layout(s, k);
    e = launch_copy_bytes(c->d_in, c->dh_in, L.hy + c->hy_used * 8, st);
    if (e != hipSuccess) return e;
    MimoMapArgs ma{};
    ma.slots = c->d_slots;
    ma.hy = c->d_hy;
    ma.j64 = c->d_j64;
    ma.h64 = c->d_h64;
    ma.xm = c->d_xm;
    ma.npad = (int)np;
    ma.xm_stride = (int)xm_stride(np);
    ma.count = (int)B;
    e = launch_mimo_map(ma, c->max_work, c->max_hy, st);
  } else {
    // the used part of each staged section, by copy kernels (see above)
    const size_t off_j = (uint8_t*)c->h_j64 - c->h_in, off_h = (uint8_t*)c->h_h64 - c->h_in,
                 off_s = (uint8_t*)c->h_sid - c->h_in;
    e = launch_copy_bytes(c->d_j64, c->dh_in + off_j, B * np * np * 8, st);
    if (e == hipSuccess) e = launch_copy_bytes(c->d_h64, c->dh_in + off_h, B * np * 8, st);
    if (e == hipSuccess) e = launch_copy_bytes(c->d_sid, c->dh_in + off_s, B * 4, st);
  }
  if (e != hipSuccess) return e;
  RealPackArgs pa{};
  pa.j64 = c->d_j64;
  pa.h64 = c->d_h64;
  pa.frag = c->d_frag;
  pa.hf = c->d_hf;
  pa.scale = c->d_scale;
  pa.pmax = reinterpret_cast<double*>(c->d_in + layout(s, k).pmax);
  pa.frag_bytes = k.frag;
  pa.npad = (int)np;
  pa.count = (int)B;
  e = launch_pack_real(pa, s->cfg.prec, st);
  if (e != hipSuccess) return e;
  SweepRealArgs a{};
  a.jfrag = c->d_frag;
  a.scale = c->d_scale;
  a.h = c->d_hf;
  a.thtab = s->d_thtab;
  a.inst_class = s->d_zero;
  a.inst_stream = c->d_sid;
  a.target = nullptr;
  a.init = nullptr;
  a.final_s = c->d_final;
  a.best_s = c->d_best;
  a.e_best = reinterpret_cast<float*>(c->d_stats);
  a.t_best = c->d_stats + B * R;
  a.first_hit = c->d_stats + 2 * B * R;
  a.e_final = reinterpret_cast<float*>(c->d_stats + 3 * B * R);
  a.steps_done = c->d_stats + 4 * B * R;
  a.cancel = s->d_cancel;
  a.n = (int)np;
  a.npad = (int)np;
  a.R = (int)R;
  a.T = s->cfg.steps;
  a.start_step = 0;
  a.k0 = (uint32_t)s->cfg.seed;
  a.k1 = (uint32_t)(s->cfg.seed >> 32);
  e = launch_sweep_real(a, (int)B, k.nt, s->cfg.prec, true, st);
  if (e != hipSuccess) return e;
  RerankArgs ra{};
  ra.j64 = c->d_j64p;
  ra.h64 = c->d_h64p;
  ra.best_s = c->d_best;
  ra.t_best = a.t_best;
  ra.e_best = c->d_stats;
  ra.energy = c->d_rerank;
  ra.out_spins = c->d_sel_spins;
  ra.out_energy = c->d_sel_e;
  ra.out_trial = c->d_sel_i;
  ra.out_step = c->d_sel_i + B;
  ra.out_tracked = c->d_sel_i + 2 * B;
  ra.n = (int)np;  // couplings and fields are zero-padded to npad
  ra.npad = (int)np;
  ra.R = (int)R;
  ra.count = (int)B;
  e = launch_rerank_select(ra, st);
  if (e == hipSuccess) e = launch_copy_bytes(c->dh_out, c->d_out, c->out_bytes, st);
  if (e == hipSuccess) e = hipEventRecord(c->done, st);
  return e;
}

}  // namespace

namespace {

pim_status server_create(const pim_server_config* cfg, bool mimo, pim_server** out) {
  try {
    if (!cfg || !out) return fail(PIM_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (cfg->max_n < 1 || cfg->max_n > PIM_MAX_N_LDS)
      return fail(PIM_ERR_INVALID, "max_n = %d outside [1, %d]", cfg->max_n, PIM_MAX_N_LDS);
    if (cfg->trials < 1 || cfg->steps < 1) return fail(PIM_ERR_INVALID, "trials and steps must be >= 1");
    if (!cfg->beta || !cfg->eta) return fail(PIM_ERR_INVALID, "beta and eta must be non-NULL");
    if (cfg->prec != PIM_PREC_FP8 && cfg->prec != PIM_PREC_BF16) return fail(PIM_ERR_INVALID, "unknown precision");
    if (cfg->streams < 1 || cfg->streams > 16) return fail(PIM_ERR_INVALID, "streams must be in [1, 16]");
    if (cfg->max_batch < 1 || cfg->max_batch > 65535) return fail(PIM_ERR_INVALID, "max_batch outside [1, 65535]");
    if (cfg->slots_per_class < cfg->max_batch)
      return fail(PIM_ERR_INVALID, "slots_per_class must be >= max_batch");
    for (int t = 0; t < cfg->steps; ++t)
      if (!(std::isfinite(cfg->beta[t]) && cfg->beta[t] >= 0 && std::isfinite(cfg->eta[t]) && cfg->eta[t] >= 0))
        return fail(PIM_ERR_INVALID, "beta[%d] / eta[%d] must be finite and >= 0", t, t);
    pim_params p{};
    p.n = cfg->max_n;
    p.j_scale = cfg->j_scale;
    p.xi = cfg->xi;
    p.levels = cfg->levels;
    p.noise = cfg->noise;
    p.noise_bits = 8;
    p.noise_table = cfg->noise_table;
    float tab[kTabEntries];
    pim_status st = pim_compile_table_real(&p, 1.0, 0.0, tab);  // validates the rule parameters
    if (st != PIM_OK) return st;
    auto* s = new pim_server();
    s->cfg = *cfg;
    s->mimo = mimo;
    s->beta.assign(cfg->beta, cfg->beta + cfg->steps);
    s->eta.assign(cfg->eta, cfg->eta + cfg->steps);
    s->cfg.beta = s->beta.data();
    s->cfg.eta = s->eta.data();
    s->cfg.noise_table = nullptr;
    // the rule, compiled once for every step: one table class for all requests
    {
      Rule r;
      r.real = true;
      r.n = cfg->max_n;
      r.c = cfg->j_scale;
      r.xi = cfg->xi;
      r.levels = cfg->levels;
      r.noise = cfg->noise;
      if (cfg->noise_table) r.ztab.assign(cfg->noise_table, cfg->noise_table + kNoiseVals);
      else (void)builtin_noise_table(cfg->noise, r.ztab);
      s->rule = r;
    }
    std::vector<float> tabs((size_t)cfg->steps * kTabEntries);
    for (int t = 0; t < cfg->steps; ++t) {
      float th[kMaxLevels];
      int32_t um[2 * kMaxLevels];
      compile_step_real(s->rule, s->beta[t], s->eta[t], th, um);
      theta_by_noise_real(th, um, s->rule.levels, tabs.data() + (size_t)t * kTabEntries);
    }
    bool ok = dev_alloc_n(&s->d_thtab, tabs.size()) && dev_alloc_n(&s->d_zero, cfg->max_batch) &&
              dev_alloc_n(&s->d_cancel, 1);
    if (ok) {
      std::vector<int32_t> z(cfg->max_batch, 0);
      ok = hipMemcpy(s->d_thtab, tabs.data(), tabs.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(s->d_zero, z.data(), z.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(s->d_cancel, z.data(), 4, hipMemcpyHostToDevice) == hipSuccess;
    }
    for (int i = 0; ok && i < cfg->streams; ++i) {
      hipStream_t q = nullptr;
      hipEvent_t ev = nullptr;
      ok = hipStreamCreateWithFlags(&q, hipStreamNonBlocking) == hipSuccess;
      if (ok) s->streams.push_back(q);
      ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
      if (ok) s->stream_idle.push_back(ev);
    }
    s->classes.resize((PIM_MAX_N_LDS + 31) / 32);
    for (size_t c = 0; c < s->classes.size(); ++c) {
      s->classes[c].nt = (int)c + 1;
      s->classes[c].npad = 32 * ((int)c + 1);
      s->classes[c].frag = real_frag_bytes(cfg->prec, (int)c + 1);
    }
    // chunks allocated up front for every class up to max_n (pinned and
    // device allocations are slow; doing them here keeps them off the
    // request path)
    for (size_t c = 0; ok && c < s->classes.size(); ++c) {
      if (s->classes[c].npad - 31 > cfg->max_n) break;
      const int want = std::min(cfg->prealloc_chunks, cfg->slots_per_class / cfg->max_batch);
      for (int i = 0; ok && i < want; ++i) {
        Chunk* ch = chunk_for(s, (int)c);
        ok = ch != nullptr;
        if (ok) s->classes[c].open = -1;
        if (ok && i + 1 < want) ch->launched = true;  // keep chunk_for from handing it out again
      }
      for (Chunk* ch : s->classes[c].chunks) ch->launched = false;
    }
    if (!ok) {
      pim_server_destroy(s);
      return fail(PIM_ERR_NOMEM, "server set-up failed");
    }
    // submit workers: up to 15 besides the caller (a GPU's share of host
    // cores), none on a single-core host
    const int hw = (int)std::thread::hardware_concurrency();
    const int workers = std::min(hw, 16) - 1;
    if (workers > 0) s->pool.reset(new Pool(workers));
    *out = s;
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_server_create");
  }
}

}  // namespace

extern "C" {

pim_status pim_server_create(const pim_server_config* cfg, pim_server** out) {
  return server_create(cfg, false, out);
}

pim_status pim_server_create_mimo(const pim_server_config* cfg, pim_server** out) {
  return server_create(cfg, true, out);
}

pim_status pim_server_submit_mimo(pim_server* s, int32_t count, const uint32_t* ids, const int32_t* dims,
                                  const double* esn0, const double* const* H, const double* const* y,
                                  int32_t* admitted) {
  try {
    if (!s || !ids || !dims || !esn0 || !H || !y || !admitted) return fail(PIM_ERR_INVALID, "NULL argument");
    *admitted = 0;
    if (!s->mimo) return fail(PIM_ERR_STATE, "this server takes (J, h) requests (pim_server_submit)");
    for (int r = 0; r < count; ++r) {
      const int nr = dims[4 * r], nt = dims[4 * r + 1], qam = dims[4 * r + 2], map = dims[4 * r + 3];
      const bool known = (qam == 4 || qam == 16) && (map == PIM_MIMO_ML || map == PIM_MIMO_DI);
      const int n = (map == PIM_MIMO_ML && qam == 4) ? 2 * nt : 4 * nt;
      const int np = 32 * ((n + 31) / 32);
      if (!known || nt < 1 || nt > PIM_MAX_N_LDS / 4 || n > s->cfg.max_n || nr < 1 || 2 * nr > np ||
          ids[r] >= (1u << 24) || !H[r] || !y[r] || (map == PIM_MIMO_DI && !(std::isfinite(esn0[r]) && esn0[r] > 0.0)))
        return fail(PIM_ERR_INVALID, "request %d (id %u): need qam 4 or 16, a known mapping, 1 <= nt <= %d, "
                    "N <= max_n, 1 <= 2 nr <= N rounded up to 32, id < 2^24, esn0 > 0 finite (DI)",
                    r, ids[r], PIM_MAX_N_LDS / 4);
      const size_t nh = 2 * (size_t)nr * nt, ny = 2 * (size_t)nr;
      for (size_t i = 0; i < nh; ++i)
        if (!std::isfinite(H[r][i])) return fail(PIM_ERR_INVALID, "request %d (id %u): H is not finite", r, ids[r]);
      for (size_t i = 0; i < ny; ++i)
        if (!std::isfinite(y[r][i])) return fail(PIM_ERR_INVALID, "request %d (id %u): y is not finite", r, ids[r]);
      Chunk* c = chunk_for(s, np / 32 - 1);
      if (!c) return PIM_OK;  // no slot: the caller polls and submits the rest later
      const size_t sl = c->count;
      if (c->count == 0) {
        c->first = std::chrono::steady_clock::now();
        c->hy_used = 0;
        c->max_work = c->max_hy = 0;
      }
      std::memcpy(c->h_hy + c->hy_used, H[r], nh * 8);
      std::memcpy(c->h_hy + c->hy_used + nh, y[r], ny * 8);
      c->h_slots[sl] = MimoSlot{nr, nt, qam, map, esn0[r], (int64_t)c->hy_used};
      c->hy_used += nh + ny;
      c->max_work = std::max(c->max_work, mimo_map_work_doubles(nr, nt));
      c->max_hy = std::max(c->max_hy, nh + ny);
      c->h_sid[sl] = ids[r];
      c->ids.push_back(ids[r]);
      c->ns.push_back(n);
      c->t_admit.push_back(mono_now());
      ++c->count;
      ++*admitted;
    }
    return PIM_OK;
  } catch (const std::bad_alloc&) {
    return fail(PIM_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_server_submit_mimo");
  }
}

pim_status pim_server_submit(pim_server* s, int32_t count, const uint32_t* ids, const int32_t* ns,
                             const double* const* J, const double* const* h, int32_t* admitted) {
  try {
    if (!s || !ids || !ns || !J || !admitted) return fail(PIM_ERR_INVALID, "NULL argument");
    *admitted = 0;
    if (s->mimo) return fail(PIM_ERR_STATE, "this server takes MIMO requests (pim_server_submit_mimo)");
    if (count <= 0) return PIM_OK;
    // (1) argument checks, in order up to the first failure
    int f = 0;
    size_t elems = 0;
    for (; f < count; ++f) {
      const int n = ns[f];
      if (n < 1 || n > s->cfg.max_n || ids[f] >= (1u << 24) || !J[f]) break;
      elems += (size_t)n * n;
    }
    const bool few = f < kFewRequests;
    const bool par = s->pool && (elems >= kParallelElems || (few && elems >= kSplitElems));
    auto run = [&](int items, const std::function<void(int)>& fn) {
      if (par) {
        s->pool->run(items, fn);
      } else {
        for (int i = 0; i < items; ++i) fn(i);
      }
    };
    // (2) slots in order until none is free (allocation may happen here)
    std::vector<std::pair<Chunk*, size_t>> place;
    place.reserve(f);
    int took = 0;
    for (; took < f; ++took) {
      const int n = ns[took];
      const int cls = (n + 31) / 32 - 1;
      Chunk* c = chunk_for(s, cls);
      if (!c) break;  // no slot: the caller polls and submits the rest later
      const size_t sl = c->count;
      if (c->count == 0) c->first = std::chrono::steady_clock::now();
      c->h_sid[sl] = ids[took];
      c->ids.push_back(ids[took]);
      c->ns.push_back(n);
      c->t_admit.push_back(0.0);
      ++c->count;
      place.emplace_back(c, sl);
    }
    // (3) content checks and staging copies of the binary64 couplings in one
    //     pass per request (quantisation and packing happen on the device at
    //     launch)
    //     work items: whole requests, or strips of kTile rows of the large
    //     ones when the pool is in use; a failed item clears its request's flag
    struct Item {
      int r, i0, i1;
    };
    std::vector<Item> items;
    items.reserve(took);
    for (int r = 0; r < took; ++r) {
      const int n = ns[r];
      if (par && few && n >= kSplitN)
        for (int i0 = 0; i0 < n; i0 += kTile) items.push_back({r, i0, std::min(i0 + kTile, n)});
      else
        items.push_back({r, 0, n});
    }
    std::unique_ptr<std::atomic<uint8_t>[]> ok(new std::atomic<uint8_t>[took]);
    for (int r = 0; r < took; ++r) ok[r].store(1, std::memory_order_relaxed);
    run((int)items.size(), [&](int k) {
      const Item& it = items[k];
      Chunk* c = place[it.r].first;
      const size_t sl = place[it.r].second, np = s->classes[c->cls].npad;
      if (!validate_and_stage_rows(J[it.r], h ? h[it.r] : nullptr, ns[it.r], np, c->h_j64 + sl * np * np,
                                   c->h_h64 + sl * np, it.i0, it.i1))
        ok[it.r].store(0, std::memory_order_relaxed);
    });
    int g = 0;
    while (g < took && ok[g].load(std::memory_order_relaxed)) ++g;
    if (g < took) {
      // an invalid request: it and the ones after it give their slots back
      // (the last ones taken in each chunk, so in reverse order)
      for (int r = took - 1; r >= g; --r) {
        Chunk* c = place[r].first;
        --c->count;
        c->ids.pop_back();
        c->ns.pop_back();
        c->t_admit.pop_back();
      }
      *admitted = g;
      return fail(PIM_ERR_INVALID, "request %d (id %u): J must be finite and symmetric with a zero diagonal, "
                  "h finite", g, ids[g]);
    }
    // requests before an invalid one are admitted (and counted) as usual
    const double t_adm = mono_now();
    for (int r = 0; r < took; ++r) place[r].first->t_admit[place[r].second] = t_adm;
    *admitted = took;
    if (took == f && f < count)
      return fail(PIM_ERR_INVALID, "request %d (id %u): n outside [1, max_n], id >= 2^24 or J NULL", f, ids[f]);
    return PIM_OK;
  } catch (const std::bad_alloc&) {
    return fail(PIM_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_server_submit");
  }
}

pim_status pim_server_flush(pim_server* s, int32_t* launched) {
  try {
    if (!s) return fail(PIM_ERR_INVALID, "server is NULL");
    int total = 0;
    const auto now = std::chrono::steady_clock::now();
    const double wait = s->cfg.max_wait_us;
    for (Klass& k : s->classes) {
      // a class with a chunk still in flight (launched, not yet collected)
      bool busy = false;
      for (const Chunk* c : k.chunks) busy = busy || c->launched;
      for (size_t ci = 0; ci < k.chunks.size(); ++ci) {
      Chunk* c = k.chunks[ci];
      if (c->launched || c->count == 0) continue;
      // a partly filled chunk waits for company up to max_wait_us, but only
      // while an earlier chunk of its class is in flight: an idle class
      // launches at once
      const double age = std::chrono::duration<double, std::micro>(now - c->first).count();
      if (c->count < s->cfg.max_batch && wait > 0.0 && busy && age < wait) continue;
      if (k.open == (int)ci) k.open = -1;
      // an idle stream if there is one, so a small chunk does not queue
      // behind a long one; otherwise the next stream in turn
      const int ns = (int)s->streams.size();
      int si = s->next_stream;
      for (int i = 0; i < ns; ++i) {
        const int cand = (s->next_stream + i) % ns;
        if (hipEventQuery(s->stream_idle[cand]) == hipSuccess) {
          si = cand;
          break;
        }
      }
      s->next_stream = (si + 1) % ns;
      hipStream_t st = s->streams[si];
      c->t_launch = mono_now();
      hipError_t e = launch_chunk(s, c, st);
      if (e == hipSuccess) e = hipEventRecord(s->stream_idle[si], st);
      if (e != hipSuccess) return fail(PIM_ERR_DEVICE, "server launch failed: %s", hipGetErrorString(e));
      c->launched = true;
      busy = true;
      s->inflight.push_back(c);
      total += c->count;
      }
    }
    if (launched) *launched = total;
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_server_flush");
  }
}

pim_status pim_server_poll(pim_server* s, int32_t max, uint32_t* ids, int8_t* states, double* energies,
                           int32_t* done) {
  return pim_server_poll_mimo(s, max, ids, states, energies, nullptr, nullptr, done);
}

pim_status pim_server_poll_times(pim_server* s, int32_t max, uint32_t* ids, int8_t* states, double* energies,
                                 double* times, int32_t* done) {
  return pim_server_poll_mimo(s, max, ids, states, energies, nullptr, times, done);
}

pim_status pim_server_poll_mimo(pim_server* s, int32_t max, uint32_t* ids, int8_t* states, double* energies,
                                double* xm, double* times, int32_t* done) {
  try {
    if (!s || !ids || !done) return fail(PIM_ERR_INVALID, "NULL argument");
    *done = 0;
    const double t_seen = times ? mono_now() : 0.0;
    // finished chunks in any order (streams complete independently)
    for (auto it = s->inflight.begin(); it != s->inflight.end();) {
      Chunk* c = *it;
      if (*done + c->count > max) break;
      const hipError_t q = hipEventQuery(c->done);
      if (q == hipErrorNotReady) {
        ++it;
        continue;
      }
      if (q != hipSuccess) return fail(PIM_ERR_DEVICE, "server work failed: %s", hipGetErrorString(q));
      const size_t np = s->classes[c->cls].npad;
      for (int r = 0; r < c->count; ++r) {
        const int o = *done + r;
        ids[o] = c->ids[r];
        if (states) {
          std::memset(states + (size_t)o * PIM_MAX_N_LDS, 0, PIM_MAX_N_LDS);
          std::memcpy(states + (size_t)o * PIM_MAX_N_LDS, c->h_spins + (size_t)r * np, c->ns[r]);
        }
        if (energies) energies[o] = c->h_e[r];
        if (xm) {
          double* row = xm + (size_t)o * (PIM_MAX_N_LDS / 2);
          std::fill(row, row + PIM_MAX_N_LDS / 2, 0.0);
          if (s->mimo) std::memcpy(row, c->h_xm + (size_t)r * xm_stride(np), 2 * c->h_slots[r].nt * sizeof(double));
        }
        if (times) {
          times[3 * (size_t)o] = c->t_admit[r];
          times[3 * (size_t)o + 1] = c->t_launch;
          times[3 * (size_t)o + 2] = t_seen;
        }
      }
      *done += c->count;
      c->count = 0;
      c->launched = false;
      c->ids.clear();
      c->ns.clear();
      c->t_admit.clear();
      c->hy_used = 0;
      c->max_work = c->max_hy = 0;
      it = s->inflight.erase(it);
    }
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_server_poll");
  }
}

pim_status pim_server_pending(pim_server* s, int32_t* staged, int32_t* in_flight) {
  if (!s) return fail(PIM_ERR_INVALID, "server is NULL");
  int a = 0, b = 0;
  for (const Klass& k : s->classes)
    for (const Chunk* c : k.chunks)
      if (!c->launched) a += c->count;
  for (const Chunk* c : s->inflight) b += c->count;
  if (staged) *staged = a;
  if (in_flight) *in_flight = b;
  return PIM_OK;
}

void pim_server_destroy(pim_server* s) {
  if (!s) return;
  for (hipStream_t q : s->streams) (void)hipStreamSynchronize(q);
  for (Klass& k : s->classes)
    for (Chunk* c : k.chunks) free_chunk(c);
  for (hipEvent_t ev : s->stream_idle) (void)hipEventDestroy(ev);
  for (hipStream_t q : s->streams) (void)hipStreamDestroy(q);
  dev_free(s->d_thtab, nullptr);
  dev_free(s->d_zero, nullptr);
  dev_free(s->d_cancel, nullptr);
  delete s;
}

}  // extern "C"
