// C ABI of the PIMI sweep library: validation, handles, allocation, schedule
// upload, launches and result readout.  Every entry point catches everything
// and reports a pim_status; no exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace pim {
namespace {

thread_local std::string g_last_error;

struct AllocHooks {
  pim_alloc_fn alloc = nullptr;
  pim_free_fn free_fn = nullptr;
  void* user = nullptr;
};
AllocHooks g_alloc;

}  // namespace

pim_status fail(pim_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

void* dev_alloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 16;
  if (g_alloc.alloc) return g_alloc.alloc(bytes, (void*)s, g_alloc.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  if (g_alloc.free_fn) {
    g_alloc.free_fn(p, (void*)s, g_alloc.user);
    return;
  }
  (void)hipFree(p);
}

}  // namespace pim

using namespace pim;

namespace {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return fail(PIM_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

template <typename T>
pim_status alloc_dev(T** p, size_t count, hipStream_t s) {
  *p = (T*)dev_alloc(count * sizeof(T), s);
  if (!*p) return fail(PIM_ERR_NOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
  return PIM_OK;
}

// Several device buffers carved out of one allocation (256-byte aligned
// sub-buffers): one allocator call instead of one per buffer, which matters
// when the allocator is a callback into the caller's runtime.
class Carver {
 public:
  template <typename T>
  void add(T** p, size_t count) {
    const size_t off = total_;
    total_ += (std::max<size_t>(count * sizeof(T), 1) + 255) & ~(size_t)255;
    set_.push_back([p, off](uint8_t* base) { *p = reinterpret_cast<T*>(base + off); });
  }
  pim_status commit(uint8_t** arena, hipStream_t s) {
    *arena = static_cast<uint8_t*>(dev_alloc(total_, s));
    if (!*arena) return fail(PIM_ERR_NOMEM, "device allocation of %zu bytes failed", total_);
    for (auto& f : set_) f(*arena);
    return PIM_OK;
  }
  // the offset the next add() will get
  size_t mark() const { return total_; }

 private:
  std::vector<std::function<void(uint8_t*)>> set_;
  size_t total_ = 0;
};

// Cancel flags of all batches live in pinned, device-mapped slabs of 1024
// flags that stay allocated for the life of the process: a pinned allocation
// per batch would cost tens of microseconds at every batch creation.
class CancelFlags {
 public:
  bool acquire(int32_t** h, int32_t** d) {
    std::lock_guard<std::mutex> g(m_);
    if (free_.empty()) {
      int32_t* hs = nullptr;
      int32_t* ds = nullptr;
      if (hipHostMalloc((void**)&hs, kSlab * sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess)
        return false;
      if (hipHostGetDevicePointer((void**)&ds, hs, 0) != hipSuccess) {
        (void)hipHostFree(hs);
        return false;
      }
      for (int i = kSlab - 1; i >= 0; --i) free_.push_back({hs + i, ds + i});
    }
    *h = free_.back().first;
    *d = free_.back().second;
    free_.pop_back();
    __atomic_store_n(*h, 0, __ATOMIC_SEQ_CST);
    return true;
  }
  void release(int32_t* h, int32_t* d) {
    std::lock_guard<std::mutex> g(m_);
    free_.push_back({h, d});
  }

 private:
  static constexpr int kSlab = 1024;
  std::mutex m_;
  std::vector<std::pair<int32_t*, int32_t*>> free_;
};
CancelFlags g_cancel_flags;

// Pinned staging of the step tables, shared by every batch: held (locked)
// from compilation until the upload has completed, grown on demand and kept
// for the life of the process.
struct TableStaging {
  std::mutex m;
  void* p = nullptr;
  size_t bytes = 0;
};
TableStaging g_tab_staging;

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

pim_status validate_params(const pim_params* p, Rule& r) {
  if (!p) return fail(PIM_ERR_INVALID, "params is NULL");
  if (p->n < 1 || p->n > PIM_MAX_N) return fail(PIM_ERR_INVALID, "n = %d outside [1, %d]", p->n, PIM_MAX_N);
  if (!std::isfinite(p->j_scale) || !(p->j_scale > 0.0))
    return fail(PIM_ERR_INVALID, "j_scale must be finite and > 0");
  if (!finite_nonneg(p->xi)) return fail(PIM_ERR_INVALID, "xi must be finite and >= 0");
  if (p->levels < 2 || p->levels > kMaxLevels)
    return fail(PIM_ERR_INVALID, "levels = %d outside [2, %d]", p->levels, kMaxLevels);
  if (p->noise != PIM_NOISE_GAUSS && p->noise != PIM_NOISE_UNIFORM)
    return fail(PIM_ERR_INVALID, "unknown noise law %d", p->noise);
  if (p->noise_bits != kNoiseBits)
    return fail(PIM_ERR_UNSUPPORTED, "noise_bits = %d (only %d is implemented)", p->noise_bits, kNoiseBits);
  if (p->rng_stream >= (1u << 24)) return fail(PIM_ERR_INVALID, "rng_stream must be < 2^24");
  r.n = p->n;
  r.c = p->j_scale;
  r.xi = p->xi;
  r.levels = p->levels;
  r.noise = p->noise;
  r.stream = p->rng_stream;
  if (p->noise_table) {
    r.ztab.assign(p->noise_table, p->noise_table + kNoiseVals);
    for (int u = 0; u < kNoiseVals; ++u) {
      if (!std::isfinite(r.ztab[u])) return fail(PIM_ERR_INVALID, "noise_table[%d] is not finite", u);
      if (u && r.ztab[u] < r.ztab[u - 1]) return fail(PIM_ERR_INVALID, "noise_table is not non-decreasing at %d", u);
    }
  } else if (!builtin_noise_table(p->noise, r.ztab)) {
    return fail(PIM_ERR_INVALID, "no built-in table for noise law %d", p->noise);
  }
  return PIM_OK;
}

pim_status validate_couplings(const int8_t* J, const int32_t* h, int n) {
  if (!J) return fail(PIM_ERR_INVALID, "J is NULL");
  for (int i = 0; i < n; ++i) {
    if (J[(size_t)i * n + i] != 0) return fail(PIM_ERR_INVALID, "J[%d][%d] != 0 (diagonal must be zero)", i, i);
    int64_t bound = h ? std::llabs((long long)h[i]) : 0;
    for (int j = 0; j < n; ++j) {
      const int8_t v = J[(size_t)i * n + j];
      if (v != J[(size_t)j * n + i]) return fail(PIM_ERR_INVALID, "J is not symmetric at (%d, %d)", i, j);
      if (v == -128) return fail(PIM_ERR_INVALID, "J[%d][%d] = -128 (use [-127, 127])", i, j);
      bound += std::abs((int)v);
    }
    if (bound > kFieldLimit)
      return fail(PIM_ERR_INVALID, "row %d: sum_j |J_ij| + |h_i| = %lld exceeds %d", i, (long long)bound, kFieldLimit);
  }
  return PIM_OK;
}

pim_status check_spins(const int8_t* s, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (s[i] != 1 && s[i] != -1) return fail(PIM_ERR_INVALID, "spin value %d at %zu is not +-1", (int)s[i], i);
  return PIM_OK;
}

hipError_t wait_last_run(pim_batch* b);

void free_batch_buffers(pim_batch* b) {
  for (pim_batch* part : b->parts) {
    (void)wait_last_run(part);
    free_batch_buffers(part);
    delete part;
  }
  b->parts.clear();
  for (hipStream_t f : b->fork) (void)hipStreamDestroy(f);
  for (hipEvent_t j : b->join) (void)hipEventDestroy(j);
  b->fork.clear();
  b->join.clear();
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  hipStream_t s = b->stream;
  dev_free(b->d_arena, s);  // the fixed-size buffers, carved at creation
  dev_free(b->d_multi, s);
  dev_free(b->d_j8pad, s);
  dev_free(b->d_trace, s);
  dev_free(b->d_thtab, s);
  dev_free(b->d_steptab, s);
  if (b->h_cancel) g_cancel_flags.release(b->h_cancel, b->d_cancel);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
}

int32_t* stat_ptr(pim_batch* b, int which) { return b->d_stats + (size_t)which * b->count * b->R; }

// Re-evaluates every trial's best state in binary64 and selects each
// instance's lowest-energy trial on the device, then reads the selection back
// in one go (once per run).
pim_status ensure_selection(pim_batch* b) {
  if (b->reranked) return PIM_OK;
  RerankArgs ra{};
  ra.j8 = b->d_jptrs;
  ra.h = b->has_h ? b->d_hptrs : nullptr;
  ra.j64 = b->real ? b->d_j64ptrs : nullptr;
  ra.h64 = (b->real && b->has_h) ? b->d_h64ptrs : nullptr;
  ra.best_s = b->d_best;
  ra.t_best = stat_ptr(b, 1);
  ra.e_best = stat_ptr(b, 0);
  ra.energy = b->d_rerank;
  ra.out_spins = b->d_sel_spins;
  ra.out_energy = b->d_sel_e;
  ra.out_trial = b->d_sel_i;
  ra.out_step = b->d_sel_i + b->count;
  ra.out_tracked = b->d_sel_i + 2 * b->count;
  ra.n = b->n;
  ra.npad = b->npad;
  ra.R = b->R;
  ra.count = b->count;
  HIP_TRY(launch_rerank_select(ra, b->stream));
  b->h_sel_spins.resize((size_t)b->count * b->npad);
  b->h_sel_e.resize(b->count);
  b->h_sel_i.resize((size_t)3 * b->count);
  // the three outputs are adjacent in the arena: one readback of the span
  const uint8_t* lo = reinterpret_cast<const uint8_t*>(b->d_sel_spins);
  const uint8_t* hi = reinterpret_cast<const uint8_t*>(b->d_sel_i + 3 * b->count);
  std::vector<uint8_t> span(hi - lo);
  HIP_TRY(hipMemcpyAsync(span.data(), lo, span.size(), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  std::memcpy(b->h_sel_spins.data(), span.data(), b->h_sel_spins.size());
  std::memcpy(b->h_sel_e.data(), span.data() + (reinterpret_cast<const uint8_t*>(b->d_sel_e) - lo),
              b->count * sizeof(double));
  std::memcpy(b->h_sel_i.data(), span.data() + (reinterpret_cast<const uint8_t*>(b->d_sel_i) - lo),
              3 * b->count * sizeof(int32_t));
  b->reranked = true;
  return PIM_OK;
}

pim_status check_batch_ready(pim_batch* b, int32_t inst) {
  if (!b) return fail(PIM_ERR_INVALID, "batch is NULL");
  if (b->sticky_error) return fail(PIM_ERR_DEVICE, "batch is in an error state after a failed device call");
  if (!b->ran) return fail(PIM_ERR_STATE, "no run has been issued on this batch");
  if (inst < 0 || inst >= b->count) return fail(PIM_ERR_INVALID, "instance index %d outside [0, %d)", inst, b->count);
  return PIM_OK;
}

// steps_done < T on any trial of the batch means the run was cancelled.
pim_status cancelled_any(pim_batch* b) {
  std::vector<int32_t> done((size_t)b->count * b->R);
  HIP_TRY(hipMemcpyAsync(done.data(), stat_ptr(b, 4), done.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                         b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (size_t c = 0; c < done.size(); ++c)
    if (done[c] < b->last_T) return fail(PIM_ERR_CANCELLED, "run was cancelled after %d of %d steps", done[c], b->last_T);
  return PIM_OK;
}

// steps_done < T on any trial of the instance means the run was cancelled.
pim_status cancelled_status(pim_batch* b, int32_t inst) {
  std::vector<int32_t> done(b->R);
  HIP_TRY(hipMemcpyAsync(done.data(), stat_ptr(b, 4) + (size_t)inst * b->R, b->R * sizeof(int32_t),
                         hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int a = 0; a < b->R; ++a)
    if (done[a] < b->last_T) return fail(PIM_ERR_CANCELLED, "run was cancelled after %d of %d steps", done[a], b->last_T);
  return PIM_OK;
}

// A batch of instances of uneven N: one simple part per distinct N, each with
// its own buffers; the composite maps instance indices to (part, local index).
pim_status create_composite(pim_instance* const* insts, int32_t count, int32_t trials, const int8_t* init_spins,
                            hipStream_t s, pim_batch** out) {
  std::vector<int> ns;
  for (int k = 0; k < count; ++k) ns.push_back(insts[k]->rule.n);
  std::vector<int> distinct(ns);
  std::sort(distinct.begin(), distinct.end());
  distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
  std::vector<size_t> init_off(count + 1, 0);
  for (int k = 0; k < count; ++k) init_off[k + 1] = init_off[k] + (size_t)trials * ns[k];
  if (init_spins) {
    pim_status st = check_spins(init_spins, init_off[count]);
    if (st != PIM_OK) return st;
  }
  auto* b = new pim_batch();
  b->count = count;
  b->R = trials;
  b->n = 0;
  b->real = insts[0]->rule.real;
  b->prec = insts[0]->prec;
  b->stream = s;
  b->insts.assign(insts, insts + count);
  b->part_of.assign(count, -1);
  b->local_of.assign(count, -1);
  auto bail = [&](pim_status st) {
    free_batch_buffers(b);
    delete b;
    return st;
  };
  for (size_t p = 0; p < distinct.size(); ++p) {
    std::vector<pim_instance*> sub;
    std::vector<int8_t> sub_init;
    for (int k = 0; k < count; ++k)
      if (ns[k] == distinct[p]) {
        b->part_of[k] = (int)p;
        b->local_of[k] = (int)sub.size();
        sub.push_back(insts[k]);
        if (init_spins) sub_init.insert(sub_init.end(), init_spins + init_off[k], init_spins + init_off[k + 1]);
      }
    pim_batch* part = nullptr;
    pim_status st = pim_batch_create(sub.data(), (int32_t)sub.size(), trials, init_spins ? sub_init.data() : nullptr,
                                     (void*)s, &part);
    if (st != PIM_OK) return bail(st);
    b->parts.push_back(part);
    b->has_h |= part->has_h;
    hipStream_t f = nullptr;
    hipEvent_t j = nullptr;
    if (hipStreamCreateWithFlags(&f, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess)
      return bail(fail(PIM_ERR_DEVICE, "stream / event creation failed"));
    b->fork.push_back(f);
    b->join.push_back(j);
  }
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess)
    return bail(fail(PIM_ERR_DEVICE, "stream / event creation failed"));
  *out = b;
  return PIM_OK;
}

// Waits on the host for the batch's last run: ev1 is recorded after every
// launch of a run, and every later call on the batch synchronises before it
// returns, so nothing of the batch is in flight after it.  Waiting on the
// event rather than on the run's stream keeps working when the caller has
// destroyed that stream since.
hipError_t wait_last_run(pim_batch* b) {
  if (!b->ran || !b->ev1) return hipSuccess;
  return hipEventSynchronize(b->ev1);
}

// Every run of a batch reuses its buffers.  A call on another stream than the
// batch's previous one first waits for the previous run, since the two
// streams are not otherwise ordered.
hipError_t settle_stream(pim_batch* b, hipStream_t s) {
  if (b->stream == s) return hipSuccess;
  hipError_t e = wait_last_run(b);
  if (e == hipSuccess) b->stream = s;
  return e;
}

struct RunCtx {
  int T = 0, L = 0;
  bool real = false, mfma = false, seq = false;
  bool f4 = false;  // the streamed kernel on e2m1 operands
  std::vector<int32_t> tgt;
  std::vector<float> tgtf;
};

// Validates the schedule, compiles and uploads the step tables of a simple
// (single-N) batch on stream s and fills ctx for run_launch.
pim_status run_prepare(pim_batch* b, const pim_schedule* sc, hipStream_t s, RunCtx& ctx) {
  {
    if (!b) return fail(PIM_ERR_INVALID, "batch is NULL");
    if (b->sticky_error) return fail(PIM_ERR_DEVICE, "batch is in an error state after a failed device call");
    if (!sc) return fail(PIM_ERR_INVALID, "schedule is NULL");
    if (sc->steps < 1) return fail(PIM_ERR_INVALID, "steps must be >= 1");
    if (!sc->beta || !sc->eta) return fail(PIM_ERR_INVALID, "beta and eta must be non-NULL");
    if (sc->start_step < 0 || (int64_t)sc->start_step + sc->steps >= (int64_t)1 << 31)
      return fail(PIM_ERR_INVALID, "start_step + steps must lie in [0, 2^31)");
    if (sc->kernel != PIM_KERNEL_MFMA_I8 && sc->kernel != PIM_KERNEL_PLAIN_F32 && sc->kernel != PIM_KERNEL_SEQ_I8 &&
        sc->kernel != PIM_KERNEL_MFMA_F4)
      return fail(PIM_ERR_INVALID, "unknown kernel %d", sc->kernel);
    if (sc->kernel == PIM_KERNEL_MFMA_F4 && b->real)
      return fail(PIM_ERR_UNSUPPORTED, "e2m1 operands take integer instances");
    if (sc->kernel == PIM_KERNEL_SEQ_I8 && b->real)
      return fail(PIM_ERR_UNSUPPORTED, "the sequential kernel takes integer instances");
    // recording runs take the int8 kernel (also when e2m1 operands were asked for)
    if (sc->record_states && ((sc->kernel != PIM_KERNEL_MFMA_I8 && sc->kernel != PIM_KERNEL_MFMA_F4) || b->real))
      return fail(PIM_ERR_UNSUPPORTED, "state recording is implemented for the int8 MFMA kernel");
    if (b->n > PIM_MAX_N_LDS &&
        ((sc->kernel != PIM_KERNEL_MFMA_I8 && sc->kernel != PIM_KERNEL_MFMA_F4) || sc->record_states))
      return fail(PIM_ERR_UNSUPPORTED, "N = %d > %d runs only the matrix-core kernels, without state recording",
                  b->n, PIM_MAX_N_LDS);
    if (sc->use_target && !sc->target) return fail(PIM_ERR_INVALID, "use_target set without target energies");
    const int T = sc->steps;
    for (int t = 0; t < T; ++t)
      if (!finite_nonneg(sc->beta[t]) || !finite_nonneg(sc->eta[t]))
        return fail(PIM_ERR_INVALID, "beta[%d] / eta[%d] must be finite and >= 0", t, t);
    for (int k = 0; sc->use_target && k < b->count; ++k)
      if (std::isnan(sc->target[k])) return fail(PIM_ERR_INVALID, "target[%d] is NaN", k);
    // targets: integer batches compare E <= floor(target), real ones in binary32
    std::vector<int32_t> tgt(b->count, INT32_MIN);
    std::vector<float> tgtf(b->count, -INFINITY);
    if (sc->use_target)
      for (int k = 0; k < b->count; ++k) {
        const double f = std::floor(sc->target[k]);
        tgt[k] = f >= (double)INT32_MAX ? INT32_MAX : (f <= (double)INT32_MIN + 1 ? INT32_MIN + 1 : (int32_t)f);
        // largest binary32 value <= target, so E <= tgtf <=> E <= target for binary32 E
        float tf = (float)sc->target[k];
        if ((double)tf > sc->target[k]) tf = std::nextafter(tf, -INFINITY);
        tgtf[k] = tf;
      }
    if (hipError_t e0 = settle_stream(b, s); e0 != hipSuccess) {
      b->sticky_error = true;
      return fail(PIM_ERR_DEVICE, "waiting for the previous stream failed: %s", hipGetErrorString(e0));
    }
    const int L = b->insts[0]->rule.levels;
    const int ncls = (int)b->class_rep.size();
    const bool real = b->real;
    // ---- compile ----
    std::vector<int32_t> steptab;
    const bool seq = sc->kernel == PIM_KERNEL_SEQ_I8;
    // the matrix-core and sequential kernels all read the (u, s) tables
    const bool mfma = sc->kernel == PIM_KERNEL_MFMA_I8 || sc->kernel == PIM_KERNEL_MFMA_F4 || seq;
    const size_t entry = real ? 4 : 2;  // bytes per table entry
    const size_t thtab_need = mfma ? (size_t)ncls * T * kTabEntries * entry : 0;
    // the tables on the device already hold this schedule: nothing to compile
    // or upload (they depend only on beta, eta and the batch's fixed rules)
    const bool tab_cached = mfma && b->tab_valid && b->d_thtab && b->thtab_bytes >= thtab_need &&
                            b->tab_beta.size() == (size_t)T &&
                            std::memcmp(b->tab_beta.data(), sc->beta, (size_t)T * sizeof(double)) == 0 &&
                            std::memcmp(b->tab_eta.data(), sc->eta, (size_t)T * sizeof(double)) == 0;
    std::unique_lock<std::mutex> staging_lock(g_tab_staging.m, std::defer_lock);
    if (mfma && !tab_cached) {
      b->tab_valid = false;
      const size_t need = thtab_need;
      staging_lock.lock();  // held until the upload below has completed
      if (need > g_tab_staging.bytes) {
        if (g_tab_staging.p) (void)hipHostFree(g_tab_staging.p);
        g_tab_staging.p = nullptr;
        g_tab_staging.bytes = 0;
        if (hipHostMalloc(&g_tab_staging.p, need, hipHostMallocDefault) != hipSuccess)
          return fail(PIM_ERR_NOMEM, "pinned staging allocation of %zu bytes failed", need);
        g_tab_staging.bytes = need;
      }
      void* out = g_tab_staging.p;
      parallel_for(T * ncls, [&](int lo, int hi) {
        int32_t th[kMaxLevels], um[2 * kMaxLevels];
        float thf[kMaxLevels];
        for (int i = lo; i < hi; ++i) {
          const int c = i / T, t = i % T;
          const Rule& r = b->insts[b->class_rep[c]]->rule;
          const size_t off = ((size_t)c * T + t) * kTabEntries;
          if (real) {
            compile_step_real(r, sc->beta[t], sc->eta[t], thf, um);
            theta_by_noise_real(thf, um, r.levels, static_cast<float*>(out) + off);
          } else {
            compile_step(r, sc->beta[t], sc->eta[t], th, um);
            theta_by_noise(th, um, r.levels, static_cast<int16_t*>(out) + off);
          }
        }
      });
    } else {
      for (int k = 0; k < b->count; ++k)
        if (b->insts[k]->rule.levels != L)
          return fail(PIM_ERR_UNSUPPORTED, "the plain kernel needs one LUT size per batch");
      const int w = (L - 1) + 2 * L;
      steptab.resize((size_t)ncls * T * w);
      for (int c = 0; c < ncls; ++c) {
        const Rule& r = b->insts[b->class_rep[c]]->rule;
        for (int t = 0; t < T; ++t) {
          int32_t* row = &steptab[((size_t)c * T + t) * w];
          if (real) {
            float thf[kMaxLevels];
            compile_step_real(r, sc->beta[t], sc->eta[t], thf, row + (L - 1));
            std::memcpy(row, thf, (L - 1) * sizeof(float));  // float bits in the int32 row
          } else {
            compile_step(r, sc->beta[t], sc->eta[t], row, row + (L - 1));
          }
        }
      }
    }
    // ---- upload ----
    if (mfma && thtab_need > b->thtab_bytes) {
      dev_free(b->d_thtab, s);
      b->d_thtab = nullptr;
      b->thtab_bytes = 0;
      b->d_thtab = dev_alloc(thtab_need, s);
      if (!b->d_thtab) return fail(PIM_ERR_NOMEM, "device allocation of %zu bytes failed", thtab_need);
      b->thtab_bytes = thtab_need;
    }
    if (!mfma && steptab.size() * 4 > b->steptab_bytes) {
      dev_free(b->d_steptab, s);
      b->d_steptab = nullptr;
      b->steptab_bytes = 0;
      pim_status st = alloc_dev(&b->d_steptab, steptab.size(), s);
      if (st != PIM_OK) return st;
      b->steptab_bytes = steptab.size() * 4;
    }
    auto device_fail = [&](hipError_t e, const char* what) {
      b->sticky_error = true;
      return fail(PIM_ERR_DEVICE, "%s failed: %s", what, hipGetErrorString(e));
    };
    hipError_t e = hipSuccess;
    b->recorded = false;
    if (sc->record_states) {
      const size_t need = (size_t)b->count * b->R * ((size_t)T + 1) * b->npad;
      if (need / ((size_t)T + 1) != (size_t)b->count * b->R * b->npad)
        return fail(PIM_ERR_INVALID, "recorded trajectory size overflows");
      if (need > b->trace_bytes) {
        dev_free(b->d_trace, s);
        b->d_trace = nullptr;
        b->trace_bytes = 0;
        pim_status st = alloc_dev(&b->d_trace, need, s);
        if (st != PIM_OK) return st;
        b->trace_bytes = need;
      }
    }
    if (seq && !b->d_j8pad) {
      // row-major int8 J with rows padded to npad, for the sequential kernel
      const size_t per = (size_t)b->npad * b->npad;
      pim_status st = alloc_dev(&b->d_j8pad, per * b->count, s);
      if (st != PIM_OK) return st;
      e = hipMemsetAsync(b->d_j8pad, 0, per * b->count, s);
      for (int k = 0; k < b->count && e == hipSuccess; ++k)
        e = hipMemcpy2DAsync(b->d_j8pad + per * k, b->npad, b->insts[k]->d_j8, b->n, b->n, b->n,
                             hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return device_fail(e, "sequential coupling layout");
    }
    if (mfma && !tab_cached) e = hipMemcpyAsync(b->d_thtab, g_tab_staging.p, thtab_need, hipMemcpyHostToDevice, s);
    else if (!mfma) e = hipMemcpyAsync(b->d_steptab, steptab.data(), steptab.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->d_target, real ? (const void*)tgtf.data() : (const void*)tgt.data(), b->count * 4,
                         hipMemcpyHostToDevice, s);
    // the host tables must stay alive until the copies are done
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);  // copies already queued still read the host tables
      return device_fail(e, "schedule upload");
    }
    if (mfma && !tab_cached) {
      b->tab_beta.assign(sc->beta, sc->beta + T);
      b->tab_eta.assign(sc->eta, sc->eta + T);
      b->tab_valid = true;
    }
    __atomic_store_n(b->h_cancel, 0, __ATOMIC_SEQ_CST);
    ctx.T = T;
    ctx.L = L;
    ctx.real = real;
    ctx.mfma = mfma;
    ctx.seq = seq;
    ctx.f4 = sc->kernel == PIM_KERNEL_MFMA_F4 && b->d_jfrag4 && !sc->record_states;
    ctx.tgt = std::move(tgt);
    ctx.tgtf = std::move(tgtf);
    return PIM_OK;
  }
}

// Arguments of the integer matrix-core sweep of a simple batch.
SweepArgs int_sweep_args(pim_batch* b, const pim_schedule* sc, uint64_t seed, int T) {
  SweepArgs a{};
  a.jfrag = b->d_jfrag;
  a.trace = sc->record_states ? b->d_trace : nullptr;
  a.h = b->has_h ? b->d_h : nullptr;
  a.thtab = static_cast<const int16_t*>(b->d_thtab);
  a.inst_class = b->d_class;
  a.inst_stream = b->d_stream_ids;
  a.target = sc->use_target ? b->d_target : nullptr;
  a.init = b->d_init;
  a.final_s = b->d_final;
  a.best_s = b->d_best;
  a.e_best = stat_ptr(b, 0);
  a.t_best = stat_ptr(b, 1);
  a.first_hit = stat_ptr(b, 2);
  a.e_final = stat_ptr(b, 3);
  a.steps_done = stat_ptr(b, 4);
  a.cancel = b->d_cancel;
  a.n = b->n;
  a.npad = b->npad;
  a.R = b->R;
  a.T = T;
  a.start_step = sc->start_step;
  a.k0 = (uint32_t)seed;
  a.k1 = (uint32_t)(seed >> 32);
  a.waves = b->waves;
  a.count = b->count;
  return a;
}

// Launches the prepared run of a simple batch on stream s (asynchronous).
hipError_t run_launch(pim_batch* b, const pim_schedule* sc, uint64_t seed, const RunCtx& ctx, hipStream_t s) {
  {
    const int T = ctx.T, L = ctx.L;
    const bool real = ctx.real, mfma = ctx.mfma, seq = ctx.seq;
    const std::vector<int32_t>& tgt = ctx.tgt;
    const std::vector<float>& tgtf = ctx.tgtf;
    hipError_t e = hipSuccess;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (seq) {
      SeqArgs a{};
      a.j8pad = b->d_j8pad;
      a.h = b->has_h ? b->d_h : nullptr;
      a.thtab = static_cast<const int16_t*>(b->d_thtab);
      a.inst_class = b->d_class;
      a.inst_stream = b->d_stream_ids;
      a.target = sc->use_target ? b->d_target : nullptr;
      a.init = b->d_init;
      a.final_s = b->d_final;
      a.best_s = b->d_best;
      a.e_best = stat_ptr(b, 0);
      a.t_best = stat_ptr(b, 1);
      a.first_hit = stat_ptr(b, 2);
      a.e_final = stat_ptr(b, 3);
      a.steps_done = stat_ptr(b, 4);
      a.cancel = b->d_cancel;
      a.n = b->n;
      a.npad = b->npad;
      a.R = b->R;
      a.T = T;
      a.start_step = sc->start_step;
      a.k0 = k0;
      a.k1 = k1;
      e = launch_sweep_seq(a, b->count, b->nt, b->has_h, s);
    } else if (mfma && !real) {
      SweepArgs a = int_sweep_args(b, sc, seed, T);
      if (ctx.f4) {
        a.jfrag = reinterpret_cast<const int8_t*>(b->d_jfrag4);
        e = b->nt * 32 > PIM_MAX_N_LDS ? launch_sweep_big4(a, b->count, b->nt, b->has_h, s)
                                       : launch_sweep_mfma4(a, b->count, b->nt, b->has_h, s);
      } else {
        e = b->nt * 32 > PIM_MAX_N_LDS ? launch_sweep_big(a, b->count, b->nt, b->has_h, s)
                                       : launch_sweep_mfma(a, b->count, b->nt, b->has_h, s);
      }
    } else if (mfma) {
      SweepRealArgs a{};
      a.jfrag = reinterpret_cast<const uint8_t*>(b->d_jfrag);
      a.scale = b->d_scale;
      a.h = b->has_h ? reinterpret_cast<const float*>(b->d_h) : nullptr;
      a.thtab = static_cast<const float*>(b->d_thtab);
      a.inst_class = b->d_class;
      a.inst_stream = b->d_stream_ids;
      a.target = sc->use_target ? reinterpret_cast<const float*>(b->d_target) : nullptr;
      a.init = b->d_init;
      a.final_s = b->d_final;
      a.best_s = b->d_best;
      a.e_best = reinterpret_cast<float*>(stat_ptr(b, 0));
      a.t_best = stat_ptr(b, 1);
      a.first_hit = stat_ptr(b, 2);
      a.e_final = reinterpret_cast<float*>(stat_ptr(b, 3));
      a.steps_done = stat_ptr(b, 4);
      a.cancel = b->d_cancel;
      a.n = b->n;
      a.npad = b->npad;
      a.R = b->R;
      a.T = T;
      a.start_step = sc->start_step;
      a.k0 = k0;
      a.k1 = k1;
      e = launch_sweep_real(a, b->count, b->nt, b->prec, b->has_h, s);
    } else {
      const int w = (L - 1) + 2 * L;
      for (int k = 0; k < b->count && e == hipSuccess; ++k) {
        const size_t cell0 = (size_t)k * b->R;
        PlainArgs a{};
        a.jf32 = b->insts[k]->d_jf32;
        a.h = (!real && b->insts[k]->has_h) ? b->insts[k]->d_h : nullptr;
        a.hf = (real && b->insts[k]->has_h) ? b->insts[k]->d_hf : nullptr;
        a.steptab = b->d_steptab + (size_t)b->inst_class[k] * T * w;
        a.init = b->d_init ? b->d_init + cell0 * b->npad : nullptr;
        a.final_s = b->d_final + cell0 * b->npad;
        a.best_s = b->d_best + cell0 * b->npad;
        a.e_best = stat_ptr(b, 0) + cell0;
        a.t_best = stat_ptr(b, 1) + cell0;
        a.first_hit = stat_ptr(b, 2) + cell0;
        a.e_final = stat_ptr(b, 3) + cell0;
        a.steps_done = stat_ptr(b, 4) + cell0;
        a.cancel = b->d_cancel;
        a.n = b->n;
        a.npad = b->npad;
        a.jstride = b->insts[k]->jstride;
        a.R = b->R;
        a.T = T;
        a.start_step = sc->start_step;
        a.levels = L;
        a.use_target = sc->use_target ? 1 : 0;
        if (real) std::memcpy(&a.target, &tgtf[k], 4);
        else a.target = tgt[k];
        a.stream = b->insts[k]->rule.stream;
        a.k0 = k0;
        a.k1 = k1;
        e = launch_sweep_plain(a, real, s);
      }
    }
    return e;
  }
}

// Compute units of the current device (cached per device).
int device_cus() {
  static std::mutex m;
  static std::vector<int> cus;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1 << 30;
  std::lock_guard<std::mutex> lock(m);
  if ((int)cus.size() <= dev) cus.resize(dev + 1, 0);
  if (cus[dev] == 0 && hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1 << 30;
  return cus[dev];
}

// Parts mp of composite b that run the streamed kernel, all on e2m1 operands
// (f4) or all on int8, as one launch: each
// instance's trial blocks stay on one XCD (workgroups 8k + x run on XCD x),
// instances go to the least-loaded XCD longest first, and each XCD takes its
// workgroups longest first, so short ones fill in behind long ones instead of
// the parts' launches sharing the CUs among themselves.  The part arguments
// and the work list are uploaded when they differ from the last upload (after
// the batch's previous run, which may still read them).
pim_status stage_multi(pim_batch* b, const std::vector<pim_schedule>& psc, uint64_t seed, int T,
                       const std::vector<size_t>& mp, bool f4, hipStream_t s, const MultiPart** d_parts,
                       const int4** d_work, int* nwork, int* nitems, int* nt_max, bool* has_h) {
  constexpr int kX = 8;
  std::vector<MultiPart> parts(mp.size());
  struct Item {
    int part, inst, bpi;
    double cost;
  };
  std::vector<Item> items;
  *nt_max = 0;
  *has_h = false;
  for (size_t i : mp) *has_h |= b->parts[i]->has_h;
  for (size_t i = 0; i < mp.size(); ++i) {
    pim_batch* pb = b->parts[mp[i]];
    std::memset(&parts[i], 0, sizeof(MultiPart));
    parts[i].a = int_sweep_args(pb, &psc[mp[i]], seed, T);
    if (f4) parts[i].a.jfrag = reinterpret_cast<const int8_t*>(pb->d_jfrag4);  // else the int8 fragments
    parts[i].a.h = *has_h ? pb->d_h : nullptr;  // zeros for instances without fields
    parts[i].a.target = pb->d_target;     // the launch drops it when targets are off
    parts[i].a.k0 = parts[i].a.k1 = 0;    // per run: kernel arguments
    parts[i].a.T = parts[i].a.start_step = 0;
    parts[i].nt = pb->nt;
    *nt_max = std::max(*nt_max, pb->nt);
    const int bpi = (pb->R + 127) / 128;
    const double c = f4 ? big4_step_cost(pb->nt) : big_step_cost(pb->nt);
    for (int k = 0; k < pb->count; ++k) items.push_back({(int)i, k, bpi, c});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
  std::vector<std::vector<int4>> lists(kX);
  std::vector<double> load(kX, 0.0);
  for (const Item& it : items) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += it.bpi * it.cost;
    for (int t = 0; t < it.bpi; ++t) lists[x].push_back(int4{it.part, it.inst, t, 0});
  }
  size_t depth = 0;
  for (const auto& l : lists) depth = std::max(depth, l.size());
  std::vector<int4> work(depth * kX, int4{-1, 0, 0, 0});
  size_t items_total = 0;
  for (int x = 0; x < kX; ++x) {
    items_total += lists[x].size();
    for (size_t k = 0; k < lists[x].size(); ++k) work[k * kX + x] = lists[x][k];
  }
  *nitems = (int)items_total;
  const size_t pbytes = (parts.size() * sizeof(MultiPart) + 255) & ~(size_t)255;
  const size_t bytes = pbytes + work.size() * sizeof(int4);
  std::vector<uint8_t> host(bytes, 0);
  std::memcpy(host.data(), parts.data(), parts.size() * sizeof(MultiPart));
  std::memcpy(host.data() + pbytes, work.data(), work.size() * sizeof(int4));
  auto device_fail = [&](hipError_t e, const char* what) {
    b->sticky_error = true;
    return fail(PIM_ERR_DEVICE, "%s failed: %s", what, hipGetErrorString(e));
  };
  if (host != b->h_multi) {
    hipError_t e = wait_last_run(b);
    if (e != hipSuccess) return device_fail(e, "waiting for the previous run");
    if (bytes > b->multi_cap) {
      dev_free(b->d_multi, s);
      b->d_multi = static_cast<uint8_t*>(dev_alloc(bytes, s));
      b->multi_cap = b->d_multi ? bytes : 0;
      if (!b->d_multi) return fail(PIM_ERR_NOMEM, "device allocation of %zu bytes failed", bytes);
    }
    e = hipMemcpyAsync(b->d_multi, host.data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host copy goes out of scope
    if (e != hipSuccess) {
      b->h_multi.clear();
      return device_fail(e, "work list upload");
    }
    b->h_multi.swap(host);
  }
  *d_parts = reinterpret_cast<const MultiPart*>(b->d_multi);
  *d_work = reinterpret_cast<const int4*>(b->d_multi + pbytes);
  *nwork = (int)work.size();
  return PIM_OK;
}

// Run-state bookkeeping after a successful launch.
void run_mark(pim_batch* b, const pim_schedule* sc) {
  b->ran = true;
  b->recorded = sc->record_states != 0;
  b->reranked = false;
  b->cancelled_checked = -1;
  b->last_T = sc->steps;
  b->last_start = sc->start_step;
}

}  // namespace

extern "C" {

int32_t pim_abi_version(void) { return PIM_ABI_VERSION; }

const char* pim_last_error(void) { return g_last_error.c_str(); }

pim_status pim_set_allocator(pim_alloc_fn alloc, pim_free_fn free_fn, void* user) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(PIM_ERR_INVALID, "alloc and free must both be set or both be NULL");
  g_alloc.alloc = alloc;
  g_alloc.free_fn = free_fn;
  g_alloc.user = user;
  return PIM_OK;
}

pim_status pim_compile_step(const pim_params* params, double beta, double eta, int32_t* theta,
                            int32_t* u_min) {
  try {
    Rule r;
    pim_status st = validate_params(params, r);
    if (st != PIM_OK) return st;
    if (!finite_nonneg(beta) || !finite_nonneg(eta)) return fail(PIM_ERR_INVALID, "beta and eta must be finite and >= 0");
    if (!theta || !u_min) return fail(PIM_ERR_INVALID, "output pointer is NULL");
    compile_step(r, beta, eta, theta, u_min);
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_compile_step");
  }
}

pim_status pim_compile_table(const pim_params* params, double beta, double eta, int16_t* table) {
  try {
    Rule r;
    pim_status st = validate_params(params, r);
    if (st != PIM_OK) return st;
    if (!finite_nonneg(beta) || !finite_nonneg(eta)) return fail(PIM_ERR_INVALID, "beta and eta must be finite and >= 0");
    if (!table) return fail(PIM_ERR_INVALID, "output pointer is NULL");
    int32_t th[kMaxLevels], um[2 * kMaxLevels];
    compile_step(r, beta, eta, th, um);
    theta_by_noise(th, um, r.levels, table);
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_compile_table");
  }
}

pim_status pim_compile_table_real(const pim_params* params, double beta, double eta, float* table) {
  try {
    Rule r;
    pim_status st = validate_params(params, r);
    if (st != PIM_OK) return st;
    if (!finite_nonneg(beta) || !finite_nonneg(eta)) return fail(PIM_ERR_INVALID, "beta and eta must be finite and >= 0");
    if (!table) return fail(PIM_ERR_INVALID, "output pointer is NULL");
    float th[kMaxLevels];
    int32_t um[2 * kMaxLevels];
    compile_step_real(r, beta, eta, th, um);
    theta_by_noise_real(th, um, r.levels, table);
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_compile_table_real");
  }
}

pim_status pim_quantize(const double* J, int32_t n, int32_t prec, double* J_out, double* scale_out) {
  if (!J || !J_out) return fail(PIM_ERR_INVALID, "NULL argument");
  if (n < 1 || n > PIM_MAX_N_LDS) return fail(PIM_ERR_INVALID, "n = %d outside [1, %d]", n, PIM_MAX_N_LDS);
  if (prec != PIM_PREC_FP8 && prec != PIM_PREC_BF16) return fail(PIM_ERR_INVALID, "unknown precision %d", prec);
  const size_t nn = (size_t)n * n;
  for (size_t i = 0; i < nn; ++i)
    if (!std::isfinite(J[i])) return fail(PIM_ERR_INVALID, "J is not finite");
  const float scale = real_scale(J, nn, prec);
  for (size_t i = 0; i < nn; ++i) J_out[i] = (double)scale * quantized_value(J[i], prec, scale);
  if (scale_out) *scale_out = scale;
  return PIM_OK;
}

pim_status pim_create_real(const double* J, const double* h, const pim_params* params, int32_t prec, void* stream,
                           pim_instance** out) {
  try {
    if (!out) return fail(PIM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    Rule r;
    pim_status st = validate_params(params, r);
    if (st != PIM_OK) return st;
    if (prec != PIM_PREC_FP8 && prec != PIM_PREC_BF16) return fail(PIM_ERR_INVALID, "unknown precision %d", prec);
    if (!J) return fail(PIM_ERR_INVALID, "J is NULL");
    const int n = r.n;
    if (n > PIM_MAX_N_LDS)
      return fail(PIM_ERR_UNSUPPORTED, "real-valued instances need N <= %d (N = %d)", PIM_MAX_N_LDS, n);
    for (int i = 0; i < n; ++i) {
      if (J[(size_t)i * n + i] != 0.0) return fail(PIM_ERR_INVALID, "J[%d][%d] != 0 (diagonal must be zero)", i, i);
      if (h && !std::isfinite(h[i])) return fail(PIM_ERR_INVALID, "h[%d] is not finite", i);
      for (int j = 0; j < n; ++j) {
        const double v = J[(size_t)i * n + j];
        if (!std::isfinite(v)) return fail(PIM_ERR_INVALID, "J[%d][%d] is not finite", i, j);
        if (v != J[(size_t)j * n + i]) return fail(PIM_ERR_INVALID, "J is not symmetric at (%d, %d)", i, j);
      }
    }
    r.real = true;
    hipStream_t s = (hipStream_t)stream;
    auto* inst = new pim_instance();
    inst->rule = std::move(r);
    inst->prec = prec;
    inst->nt = (n + 31) / 32;
    inst->npad = inst->nt * 32;
    inst->jstride = (n + 3) & ~3;
    inst->has_h = false;
    if (h)
      for (int i = 0; i < n; ++i) inst->has_h |= (h[i] != 0.0);
    inst->scale = real_scale(J, (size_t)n * n, prec);
    inst->frag_bytes = real_frag_bytes(prec, inst->nt);
    // device arena: fragments, FP32 J, fl32(h), binary64 h (built on the
    // host in one block of the same layout and uploaded by one copy), then
    // the binary64 J (copied straight from the caller's array)
    Carver cv;
    const size_t o_frag = cv.mark();
    cv.add(&inst->d_jfrag, inst->frag_bytes);
    const size_t o_jf = cv.mark();
    cv.add(&inst->d_jf32, (size_t)inst->npad * inst->jstride);
    const size_t o_hf = cv.mark();
    cv.add(&inst->d_hf, (size_t)inst->npad);
    const size_t o_h64 = cv.mark();
    cv.add(&inst->d_h64, (size_t)n);
    const size_t staged = cv.mark();
    cv.add(&inst->d_j64, (size_t)n * n);
    std::vector<uint8_t> host(staged, 0);
    pack_real_fragments(J, n, inst->nt, prec, inst->scale, host.data() + o_frag);
    float* jf = reinterpret_cast<float*>(host.data() + o_jf);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) jf[(size_t)i * inst->jstride + j] = (float)J[(size_t)i * n + j];
    float* hf = reinterpret_cast<float*>(host.data() + o_hf);
    double* h64 = reinterpret_cast<double*>(host.data() + o_h64);
    if (h)
      for (int i = 0; i < n; ++i) {
        hf[i] = (float)h[i];
        h64[i] = h[i];
      }
    st = cv.commit(&inst->d_arena, s);
    if (st != PIM_OK) {
      pim_destroy(inst);
      return st;
    }
    hipError_t e = hipMemcpyAsync(inst->d_arena, host.data(), staged, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(inst->d_j64, J, (size_t)n * n * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);  // copies already queued still read the host buffers
      pim_destroy(inst);
      return fail(PIM_ERR_DEVICE, "copying the instance to the device failed: %s", hipGetErrorString(e));
    }
    *out = inst;
    return PIM_OK;
  } catch (const std::bad_alloc&) {
    return fail(PIM_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_create_real");
  }
}

pim_status pim_create(const int8_t* J, const int32_t* h, const pim_params* params, void* stream,
                      pim_instance** out) {
  try {
    if (!out) return fail(PIM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    Rule r;
    pim_status st = validate_params(params, r);
    if (st != PIM_OK) return st;
    st = validate_couplings(J, h, r.n);
    if (st != PIM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    auto* inst = new pim_instance();
    inst->rule = std::move(r);
    const int n = inst->rule.n;
    inst->nt = n <= PIM_MAX_N_LDS ? (n + 31) / 32 : big_tiles(n);
    inst->npad = inst->nt * 32;
    inst->has_h = false;
    if (h)
      for (int i = 0; i < n; ++i) inst->has_h |= (h[i] != 0);
    inst->frag_bytes = (size_t)inst->nt * inst->nt * 1024;
    // e2m1 fragments as well when every coupling is e2m1-exact
    if (f4_couplings(J, (size_t)n * n)) inst->frag4_bytes = f4_frag_bytes(inst->nt);
    inst->jstride = (n + 3) & ~3;
    // device arena: fragments, FP32 J, h (built on the host in one block of
    // the same layout and uploaded by one copy), then the int8 J (copied
    // straight from the caller's array)
    Carver cv;
    const size_t o_frag = cv.mark();
    cv.add(&inst->d_jfrag, inst->frag_bytes);
    const size_t o_frag4 = cv.mark();
    if (inst->frag4_bytes) cv.add(&inst->d_jfrag4, inst->frag4_bytes);
    const size_t o_jf = cv.mark();
    cv.add(&inst->d_jf32, (size_t)inst->npad * inst->jstride);
    const size_t o_h = cv.mark();
    cv.add(&inst->d_h, (size_t)inst->npad);
    const size_t staged = cv.mark();
    cv.add(&inst->d_j8, (size_t)n * n);
    std::vector<uint8_t> host(staged, 0);
    pack_mfma_fragments(J, n, inst->nt, reinterpret_cast<int8_t*>(host.data() + o_frag));
    if (inst->frag4_bytes) pack_f4_fragments(J, n, inst->nt, host.data() + o_frag4);
    float* jf = reinterpret_cast<float*>(host.data() + o_jf);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) jf[(size_t)i * inst->jstride + j] = (float)J[(size_t)i * n + j];
    if (h) std::memcpy(host.data() + o_h, h, (size_t)n * sizeof(int32_t));
    st = cv.commit(&inst->d_arena, s);
    if (st != PIM_OK) {
      pim_destroy(inst);
      return st;
    }
    hipError_t e = hipMemcpyAsync(inst->d_arena, host.data(), staged, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(inst->d_j8, J, (size_t)n * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host staging buffers go out of scope
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);  // copies already queued still read the host buffers
      pim_destroy(inst);
      return fail(PIM_ERR_DEVICE, "copying the instance to the device failed: %s", hipGetErrorString(e));
    }
    *out = inst;
    return PIM_OK;
  } catch (const std::bad_alloc&) {
    return fail(PIM_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_create");
  }
}

void pim_destroy(pim_instance* inst) {
  if (!inst) return;
  dev_free(inst->d_arena, nullptr);  // every device buffer of the instance
  delete inst;
}

pim_status pim_batch_create(pim_instance* const* insts, int32_t count, int32_t trials,
                            const int8_t* init_spins, void* stream, pim_batch** out) {
  try {
    if (!out) return fail(PIM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!insts || count < 1) return fail(PIM_ERR_INVALID, "need at least one instance");
    if (trials < 1 || trials > (1 << 24)) return fail(PIM_ERR_INVALID, "trials = %d outside [1, 2^24]", trials);
    if (count > 65535) return fail(PIM_ERR_INVALID, "count = %d exceeds 65535", count);
    bool mixed = false;
    for (int k = 0; k < count; ++k) {
      if (!insts[k]) return fail(PIM_ERR_INVALID, "instance %d is NULL", k);
      if (insts[k]->rule.real != insts[0]->rule.real || insts[k]->prec != insts[0]->prec)
        return fail(PIM_ERR_UNSUPPORTED, "integer and real instances, or two precisions, in one batch");
      mixed |= insts[k]->rule.n != insts[0]->rule.n;
    }
    if (mixed) return create_composite(insts, count, trials, init_spins, (hipStream_t)stream, out);
    const int n = insts[0]->rule.n;
    if (init_spins) {
      pim_status st = check_spins(init_spins, (size_t)count * trials * n);
      if (st != PIM_OK) return st;
    }
    hipStream_t s = (hipStream_t)stream;
    auto* b = new pim_batch();
    b->insts.assign(insts, insts + count);
    b->count = count;
    b->R = trials;
    b->n = n;
    b->nt = insts[0]->nt;
    b->npad = insts[0]->npad;
    b->real = insts[0]->rule.real;
    b->prec = insts[0]->prec;
    b->frag_bytes = insts[0]->frag_bytes;
    b->frag4_bytes = insts[0]->frag4_bytes;
    for (int k = 0; k < count; ++k)
      if (!insts[k]->d_jfrag4) b->frag4_bytes = 0;  // e2m1 only when every instance has it
    b->stream = s;
    for (int k = 0; k < count; ++k) b->has_h |= insts[k]->has_h;
    // table classes: instances whose compiled tables coincide share one
    b->inst_class.resize(count);
    for (int k = 0; k < count; ++k) {
      int cls = -1;
      for (size_t c = 0; c < b->class_rep.size(); ++c)
        if (insts[b->class_rep[c]]->rule.same_table_class(insts[k]->rule)) { cls = (int)c; break; }
      if (cls < 0) {
        cls = (int)b->class_rep.size();
        b->class_rep.push_back(k);
      }
      b->inst_class[k] = cls;
    }
    const size_t frag = b->frag_bytes;
    const size_t cells = (size_t)count * trials;
    // the arena starts with the per-instance tables filled on the host (one
    // upload), then the device-only buffers; the three selection outputs are
    // last and adjacent (one readback)
    Carver cv;
    const size_t o_class = cv.mark();
    cv.add(&b->d_class, (size_t)count);
    const size_t o_sid = cv.mark();
    cv.add(&b->d_stream_ids, (size_t)count);
    const size_t o_jp = cv.mark();
    cv.add(&b->d_jptrs, (size_t)count);
    const size_t o_hp = cv.mark();
    cv.add(&b->d_hptrs, (size_t)count);
    const size_t o_jp64 = cv.mark();
    cv.add(&b->d_j64ptrs, (size_t)count);
    const size_t o_hp64 = cv.mark();
    cv.add(&b->d_h64ptrs, (size_t)count);
    const size_t o_scale = cv.mark();
    cv.add(&b->d_scale, (size_t)count);
    const size_t tables = cv.mark();
    cv.add(&b->d_jfrag, frag * count);
    if (b->frag4_bytes) cv.add(&b->d_jfrag4, b->frag4_bytes * count);
    cv.add(&b->d_h, (size_t)count * b->npad);
    cv.add(&b->d_final, cells * b->npad);
    cv.add(&b->d_best, cells * b->npad);
    cv.add(&b->d_stats, cells * 5);
    cv.add(&b->d_target, (size_t)count);
    cv.add(&b->d_rerank, cells);
    if (init_spins) cv.add(&b->d_init, cells * b->npad);
    cv.add(&b->d_sel_spins, (size_t)count * b->npad);
    cv.add(&b->d_sel_e, (size_t)count);
    cv.add(&b->d_sel_i, (size_t)3 * count);
    pim_status st = cv.commit(&b->d_arena, s);
    if (st != PIM_OK) {
      free_batch_buffers(b);
      delete b;
      return st;
    }
    hipError_t e = g_cancel_flags.acquire(&b->h_cancel, &b->d_cancel) ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipEventCreate(&b->ev0);
    if (e == hipSuccess) e = hipEventCreate(&b->ev1);
    std::vector<uint8_t> host(tables, 0);
    auto* sid = reinterpret_cast<uint32_t*>(host.data() + o_sid);
    auto* jp = reinterpret_cast<const int8_t**>(host.data() + o_jp);
    auto* hp = reinterpret_cast<const int32_t**>(host.data() + o_hp);
    auto* jp64 = reinterpret_cast<const double**>(host.data() + o_jp64);
    auto* hp64 = reinterpret_cast<const double**>(host.data() + o_hp64);
    auto* scales = reinterpret_cast<float*>(host.data() + o_scale);
    std::memcpy(host.data() + o_class, b->inst_class.data(), (size_t)count * sizeof(int32_t));
    for (int k = 0; k < count; ++k) {
      sid[k] = insts[k]->rule.stream;
      jp[k] = insts[k]->d_j8;
      hp[k] = insts[k]->d_h;
      jp64[k] = insts[k]->d_j64;
      hp64[k] = insts[k]->d_h64;
      scales[k] = insts[k]->scale;
    }
    for (int k = 0; k < count && e == hipSuccess; ++k) {
      e = hipMemcpyAsync(b->d_jfrag + frag * k, insts[k]->d_jfrag, frag, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess && b->frag4_bytes)
        e = hipMemcpyAsync(b->d_jfrag4 + b->frag4_bytes * k, insts[k]->d_jfrag4, b->frag4_bytes,
                           hipMemcpyDeviceToDevice, s);
      const void* hsrc = b->real ? (const void*)insts[k]->d_hf : (const void*)insts[k]->d_h;
      if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_h + (size_t)k * b->npad, hsrc, b->npad * 4, hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_arena, host.data(), tables, hipMemcpyHostToDevice, s);
    std::vector<int8_t> init_pad;
    if (e == hipSuccess && init_spins) {
      init_pad.assign(cells * b->npad, (int8_t)1);
      for (size_t c = 0; c < cells; ++c) std::memcpy(&init_pad[c * b->npad], init_spins + c * n, n);
      e = hipMemcpyAsync(b->d_init, init_pad.data(), init_pad.size(), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);  // copies already queued still read the host buffers
      free_batch_buffers(b);
      delete b;
      return fail(PIM_ERR_DEVICE, "batch setup failed: %s", hipGetErrorString(e));
    }
    *out = b;
    return PIM_OK;
  } catch (const std::bad_alloc&) {
    return fail(PIM_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_batch_create");
  }
}

void pim_batch_destroy(pim_batch* b) {
  if (!b) return;
  // the last run's work has finished before its buffers and its cancel flag
  // slot are released
  (void)wait_last_run(b);
  free_batch_buffers(b);
  delete b;
}

pim_status pim_cancel(pim_batch* b) {
  if (b && !b->parts.empty()) {
    for (pim_batch* part : b->parts) (void)pim_cancel(part);
    return PIM_OK;
  }
  if (!b || !b->h_cancel) return fail(PIM_ERR_INVALID, "batch is NULL");
  __atomic_store_n(b->h_cancel, 1, __ATOMIC_SEQ_CST);
  return PIM_OK;
}

pim_status pim_run(pim_batch* b, const pim_schedule* sc, uint64_t seed, void* stream) {
  try {
    if (!b) return fail(PIM_ERR_INVALID, "batch is NULL");
    if (b->sticky_error) return fail(PIM_ERR_DEVICE, "batch is in an error state after a failed device call");
    hipStream_t s = stream ? (hipStream_t)stream : b->stream;
    if (b->parts.empty()) {
      RunCtx ctx;
      pim_status st = run_prepare(b, sc, s, ctx);
      if (st != PIM_OK) return st;
      hipError_t e = hipEventRecord(b->ev0, s);
      if (e == hipSuccess) e = run_launch(b, sc, seed, ctx, s);
      if (e == hipSuccess) e = hipEventRecord(b->ev1, s);
      if (e != hipSuccess) {
        b->sticky_error = true;
        return fail(PIM_ERR_DEVICE, "sweep launch failed: %s", hipGetErrorString(e));
      }
      run_mark(b, sc);
      return PIM_OK;
    }
    // uneven N: prepare every part, then capture all launches as parallel
    // branches of one graph and launch it
    if (!sc) return fail(PIM_ERR_INVALID, "schedule is NULL");
    if (sc->use_target && !sc->target) return fail(PIM_ERR_INVALID, "use_target set without target energies");
    const size_t P = b->parts.size();
    std::vector<std::vector<double>> tg(P);
    std::vector<pim_schedule> psc(P, *sc);
    if (sc->use_target)
      for (int k = 0; k < b->count; ++k) tg[b->part_of[k]].push_back(sc->target[k]);
    if (hipError_t e0 = settle_stream(b, s); e0 != hipSuccess) {
      b->sticky_error = true;
      return fail(PIM_ERR_DEVICE, "waiting for the previous stream failed: %s", hipGetErrorString(e0));
    }
    std::vector<RunCtx> ctx(P);
    for (size_t p = 0; p < P; ++p) {
      if (sc->use_target) psc[p].target = tg[p].data();
      pim_status st = run_prepare(b->parts[p], &psc[p], s, ctx[p]);
      if (st != PIM_OK) return st;
    }
    // streamed parts (N > 256): one launch over a longest-first work list, on
    // e2m1 operands when at least two parts run on them, else on int8
    std::vector<char> in_multi(P, 0);
    std::vector<size_t> mp4, mp8;
    for (size_t p = 0; p < P; ++p)
      if (b->parts[p]->nt * 32 > PIM_MAX_N_LDS && ctx[p].mfma && !ctx[p].real && !ctx[p].seq)
        (ctx[p].f4 ? mp4 : mp8).push_back(p);
    const bool multi_f4 = mp4.size() >= 2;
    const std::vector<size_t>& mp = multi_f4 ? mp4 : mp8;
    const MultiPart* d_parts = nullptr;
    const int4* d_work = nullptr;
    int nwork = 0, nitems = 0, nt_max = 0;
    bool multi_h = false;
    if (mp.size() >= 2) {
      pim_status st =
          stage_multi(b, psc, seed, ctx[0].T, mp, multi_f4, s, &d_parts, &d_work, &nwork, &nitems, &nt_max, &multi_h);
      if (st != PIM_OK) return st;
      for (size_t p : mp) in_multi[p] = 1;
    }
    const MultiRun run{(uint32_t)seed, (uint32_t)(seed >> 32), ctx[0].T, sc->start_step, sc->use_target ? 1 : 0};
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    hipError_t e = hipEventRecord(b->fork_ev, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->fork_ev, 0);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t ce = hipEventRecord(b->fork_ev, b->cap);
      // the one launch of the streamed parts first: its longest workgroups take
      // the CUs before the small parts' launches are dispatched.  When it has
      // a workgroup for every CU its longest-first schedule leaves almost no
      // idle tail, and the other parts' workgroups, run beside it, only delay
      // its long ones: they then wait for it (measured at 128 SK-1 instances
      // of N = 100..1000, 10^4 steps: 382 against 396 ms)
      const bool chain = nwork > 0 && nitems >= device_cus();
      std::vector<size_t> order;
      if (nwork > 0) order.push_back(mp[0]);
      for (size_t p = 0; p < P; ++p)
        if (!in_multi[p]) order.push_back(p);
      for (size_t i = 0; i < order.size() && ce == hipSuccess; ++i) {
        const size_t p = order[i];
        const bool multi_head = nwork > 0 && p == mp[0];
        ce = hipStreamWaitEvent(b->fork[p], (chain && !multi_head) ? b->join[mp[0]] : b->fork_ev, 0);
        if (ce == hipSuccess)
          ce = !multi_head ? run_launch(b->parts[p], &psc[p], seed, ctx[p], b->fork[p])
               : multi_f4  ? launch_sweep_big4_multi(d_parts, d_work, nwork, nt_max, multi_h, run, b->fork[p])
                           : launch_sweep_big_multi(d_parts, d_work, nwork, nt_max, multi_h, run, b->fork[p]);
        if (ce == hipSuccess) ce = hipEventRecord(b->join[p], b->fork[p]);
        if (ce == hipSuccess) ce = hipStreamWaitEvent(b->cap, b->join[p], 0);
      }
      e = hipStreamEndCapture(b->cap, &b->graph);  // always end the capture
      if (ce != hipSuccess) e = ce;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipEventRecord(b->ev0, s);
    if (e == hipSuccess) e = hipGraphLaunch(b->gexec, s);
    if (e == hipSuccess) e = hipEventRecord(b->ev1, s);
    if (e != hipSuccess) {
      b->sticky_error = true;
      return fail(PIM_ERR_DEVICE, "graph launch failed: %s", hipGetErrorString(e));
    }
    for (size_t p = 0; p < P; ++p) run_mark(b->parts[p], &psc[p]);
    run_mark(b, sc);
    return PIM_OK;
  } catch (const std::bad_alloc&) {
    return fail(PIM_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_run");
  }
}

pim_status pim_tune(pim_batch* b, int32_t steps, void* stream, int32_t* waves_out) {
  try {
    if (!b) return fail(PIM_ERR_INVALID, "batch is NULL");
    if (steps < 1) return fail(PIM_ERR_INVALID, "steps must be >= 1");
    if (b->real) return fail(PIM_ERR_UNSUPPORTED, "tuning is implemented for the int8 MFMA kernel");
    std::vector<pim_batch*> targets = b->parts;
    if (targets.empty()) targets.push_back(b);
    std::vector<double> beta(steps, 1.0), eta(steps, 0.5);
    pim_schedule sc{};
    sc.steps = steps;
    sc.beta = beta.data();
    sc.eta = eta.data();
    sc.kernel = PIM_KERNEL_MFMA_I8;
    for (size_t p = 0; p < targets.size(); ++p) {
      pim_batch* t = targets[p];
      if (t->npad > PIM_MAX_N_LDS) {  // the streamed kernel has a fixed 4-wave workgroup
        if (waves_out) waves_out[p] = 4;
        continue;
      }
      const int cand[3] = {4, 2, 1};
      int best_w = 4;
      float best_ms = 0.0f;
      for (int w : cand) {
        t->waves = w;
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {  // first run warms up
          pim_status st = pim_run(t, &sc, 12345, stream);
          if (st == PIM_OK) st = pim_kernel_time(t, &ms);
          if (st != PIM_OK) return st;
        }
        if (w == cand[0] || ms < best_ms) {
          best_ms = ms;
          best_w = w;
        }
      }
      t->waves = best_w;
      if (waves_out) waves_out[p] = best_w;
    }
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_tune");
  }
}

pim_status pim_states(pim_batch* b, int32_t inst, int32_t trial, int8_t* states) {
  try {
    if (b && !b->parts.empty() && inst >= 0 && inst < b->count)
      return pim_states(b->parts[b->part_of[inst]], b->local_of[inst], trial, states);
    pim_status st = check_batch_ready(b, inst);
    if (st != PIM_OK) return st;
    if (!b->recorded) return fail(PIM_ERR_STATE, "the last run did not record its states");
    if (trial < 0 || trial >= b->R) return fail(PIM_ERR_INVALID, "trial %d outside [0, %d)", trial, b->R);
    if (!states) return fail(PIM_ERR_INVALID, "states is NULL");
    const size_t rows = (size_t)b->last_T + 1;
    const int8_t* src = b->d_trace + ((size_t)inst * b->R + trial) * rows * b->npad;
    HIP_TRY(hipMemcpy2DAsync(states, b->n, src, b->npad, b->n, rows, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_states");
  }
}

pim_status pim_flip_counts(pim_batch* b, int32_t inst, int64_t* num, int64_t* den) {
  try {
    if (b && !b->parts.empty() && inst >= 0 && inst < b->count)
      return pim_flip_counts(b->parts[b->part_of[inst]], b->local_of[inst], num, den);
    pim_status st = check_batch_ready(b, inst);
    if (st != PIM_OK) return st;
    if (!b->recorded) return fail(PIM_ERR_STATE, "the last run did not record its states");
    if (!num || !den) return fail(PIM_ERR_INVALID, "NULL argument");
    const int T = b->last_T;
    unsigned long long* d = nullptr;
    st = alloc_dev(&d, 2 * (size_t)T, b->stream);
    if (st != PIM_OK) return st;
    FlipRateArgs fa{};
    fa.trace = b->d_trace + (size_t)inst * b->R * ((size_t)T + 1) * b->npad;
    fa.j8 = b->insts[inst]->d_j8;
    fa.num = d;
    fa.den = d + T;
    fa.n = b->n;
    fa.npad = b->npad;
    fa.R = b->R;
    fa.T = T;
    hipError_t e = launch_flip_rate(fa, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(num, d, T * 8, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(den, d + T, T * 8, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    dev_free(d, b->stream);
    if (e != hipSuccess) return fail(PIM_ERR_DEVICE, "pim_flip_counts failed: %s", hipGetErrorString(e));
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_flip_counts");
  }
}

pim_status pim_kernel_time(pim_batch* b, float* ms) {
  if (!b || !ms) return fail(PIM_ERR_INVALID, "NULL argument");
  if (!b->ran) return fail(PIM_ERR_STATE, "no run has been issued on this batch");
  HIP_TRY(hipEventSynchronize(b->ev1));
  HIP_TRY(hipEventElapsedTime(ms, b->ev0, b->ev1));
  return PIM_OK;
}

pim_status pim_energy(const pim_instance* inst, const int8_t* spins, int32_t count, double* out, void* stream) {
  try {
    if (!inst || !spins || !out) return fail(PIM_ERR_INVALID, "NULL argument");
    if (count < 1) return fail(PIM_ERR_INVALID, "count must be >= 1");
    const int n = inst->rule.n;
    // device memory (the caller's device buffer) is read in place; anything
    // the runtime does not know as device memory is a host array
    bool on_device = false;
    {
      hipPointerAttribute_t attr{};
      if (hipPointerGetAttributes(&attr, spins) == hipSuccess)
        on_device = attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
      else
        (void)hipGetLastError();  // an unknown pointer is host memory, not an error
    }
    pim_status st = on_device ? PIM_OK : check_spins(spins, (size_t)count * n);
    if (st != PIM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    int8_t* d_s = nullptr;
    double* d_o = nullptr;
    if (!on_device) st = alloc_dev(&d_s, (size_t)count * n, s);
    if (st == PIM_OK) st = alloc_dev(&d_o, (size_t)count, s);
    if (st != PIM_OK) {
      dev_free(d_s, s);
      return st;
    }
    EnergyArgs ea{};
    ea.jf32 = inst->d_jf32;
    ea.h = (!inst->rule.real && inst->has_h) ? inst->d_h : nullptr;
    ea.jf64 = inst->rule.real ? inst->d_j64 : nullptr;
    ea.hf64 = (inst->rule.real && inst->has_h) ? inst->d_h64 : nullptr;
    ea.spins = on_device ? spins : d_s;
    ea.out = d_o;
    ea.n = n;
    ea.jstride = inst->jstride;
    ea.stride = n;
    ea.count = count;
    hipError_t e = on_device ? hipSuccess : hipMemcpyAsync(d_s, spins, (size_t)count * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_energy_f64(ea, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d_o, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    else (void)hipStreamSynchronize(s);  // a queued copy may still read the caller's spins
    dev_free(d_s, s);
    dev_free(d_o, s);
    if (e != hipSuccess) return fail(PIM_ERR_DEVICE, "pim_energy failed: %s", hipGetErrorString(e));
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_energy");
  }
}

pim_status pim_best(pim_batch* b, int32_t inst, int8_t* spins_out, double* e_out, int32_t* trial_out,
                    int32_t* step_out) {
  try {
    if (b && !b->parts.empty() && inst >= 0 && inst < b->count) {
      if (b->sticky_error) return fail(PIM_ERR_DEVICE, "batch is in an error state after a failed device call");
      return pim_best(b->parts[b->part_of[inst]], b->local_of[inst], spins_out, e_out, trial_out, step_out);
    }
    pim_status st = check_batch_ready(b, inst);
    if (st != PIM_OK) return st;
    st = ensure_selection(b);
    if (st != PIM_OK) {
      b->sticky_error = true;
      return st;
    }
    const double e = b->h_sel_e[inst];
    const int32_t trial = b->h_sel_i[inst];
    const int32_t step = b->h_sel_i[b->count + inst];
    const int32_t tracked = b->h_sel_i[2 * b->count + inst];
    if (!b->real && (double)tracked != e)
      return fail(PIM_ERR_DEVICE, "tracked energy %d disagrees with the binary64 re-evaluation %.17g", tracked, e);
    if (spins_out) std::memcpy(spins_out, &b->h_sel_spins[(size_t)inst * b->npad], b->n);
    if (e_out) *e_out = e;
    if (trial_out) *trial_out = trial;
    if (step_out) *step_out = step;
    if (b->cancelled_checked < 0) {
      st = cancelled_any(b);
      b->cancelled_checked = (st == PIM_OK) ? 0 : 1;
    }
    if (b->cancelled_checked == 1)
      return fail(PIM_ERR_CANCELLED, "run was cancelled; results are partial");
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_best");
  }
}

pim_status pim_trials(pim_batch* b, int32_t inst, double* best_e, int32_t* best_step, int32_t* first_hit,
                      double* final_e, int8_t* best_spins, int8_t* final_spins) {
  try {
    if (b && !b->parts.empty() && inst >= 0 && inst < b->count) {
      if (b->sticky_error) return fail(PIM_ERR_DEVICE, "batch is in an error state after a failed device call");
      return pim_trials(b->parts[b->part_of[inst]], b->local_of[inst], best_e, best_step, first_hit, final_e,
                        best_spins, final_spins);
    }
    pim_status st = check_batch_ready(b, inst);
    if (st != PIM_OK) return st;
    const int R = b->R;
    const size_t cell0 = (size_t)inst * R;
    std::vector<int32_t> tmp(R);
    auto fetch = [&](int which, std::vector<int32_t>& dst) -> pim_status {
      HIP_TRY(hipMemcpyAsync(dst.data(), stat_ptr(b, which) + cell0, R * 4, hipMemcpyDeviceToHost, b->stream));
      HIP_TRY(hipStreamSynchronize(b->stream));
      return PIM_OK;
    };
    auto energy_of = [&](int32_t v) -> double {
      if (!b->real) return (double)v;
      float f;
      std::memcpy(&f, &v, 4);
      return (double)f;
    };
    if (best_e) {
      if ((st = fetch(0, tmp)) != PIM_OK) return st;
      for (int a = 0; a < R; ++a) best_e[a] = energy_of(tmp[a]);
    }
    if (best_step) {
      if ((st = fetch(1, tmp)) != PIM_OK) return st;
      std::copy(tmp.begin(), tmp.end(), best_step);
    }
    if (first_hit) {
      if ((st = fetch(2, tmp)) != PIM_OK) return st;
      std::copy(tmp.begin(), tmp.end(), first_hit);
    }
    if (final_e) {
      if ((st = fetch(3, tmp)) != PIM_OK) return st;
      for (int a = 0; a < R; ++a) final_e[a] = energy_of(tmp[a]);
    }
    if (best_spins || final_spins) {
      std::vector<int8_t> sp((size_t)R * b->npad);
      for (int which = 0; which < 2; ++which) {
        int8_t* dst = which ? final_spins : best_spins;
        if (!dst) continue;
        const int8_t* src = (which ? b->d_final : b->d_best) + cell0 * b->npad;
        HIP_TRY(hipMemcpyAsync(sp.data(), src, sp.size(), hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
        for (int a = 0; a < R; ++a) std::memcpy(dst + (size_t)a * b->n, &sp[(size_t)a * b->npad], b->n);
      }
    }
    return cancelled_status(b, inst);
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_trials");
  }
}

}  // extern "C"
