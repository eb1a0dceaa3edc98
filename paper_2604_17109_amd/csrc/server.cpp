// Request server with continuous batching for real-valued Ising requests (the
// MIMO detection service of Suppl. "PIMI FPGA implementation for MIMO
// detection", host-side task scheduling; here on one GPU).
//
// Device-resident slot table: per N class (N rounded up to 32) a fixed array
// of slots split into chunks of `max_batch` slots.  A request is admitted into
// the open chunk of its class when a chunk and the device-memory budget allow;
// its couplings are quantised and packed on the host into the chunk's pinned
// staging area.  pim_server_flush launches every open chunk on the next of
// several streams: upload, the persistent FP8/BF16 sweep over the chunk's
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
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "internal.hpp"

namespace pim {
namespace {

struct Chunk {
  int cls = 0;
  int count = 0;                 // requests admitted into this chunk
  bool launched = false;
  hipEvent_t done = nullptr;
  std::vector<uint32_t> ids;
  std::vector<int32_t> ns;
  // pinned host staging (inputs) and results
  uint8_t* h_frag = nullptr;
  float* h_hf = nullptr;
  float* h_scale = nullptr;
  double* h_j64 = nullptr;
  double* h_h64 = nullptr;
  uint32_t* h_sid = nullptr;
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

}  // namespace
}  // namespace pim

struct pim_server {
  pim_server_config cfg{};
  pim::Rule rule;
  std::vector<double> beta, eta;
  std::vector<pim::Klass> classes;   // index nt - 1
  float* d_thtab = nullptr;
  int32_t* d_zero = nullptr;         // class ids (all 0) for max_batch instances
  int32_t* d_cancel = nullptr;
  std::vector<hipStream_t> streams;
  int next_stream = 0;
  std::deque<pim::Chunk*> inflight;  // launch order
  size_t bytes = 0;                  // device bytes held by slots
};

using namespace pim;

namespace {

size_t chunk_device_bytes(const pim_server* s, const Klass& k) {
  const size_t B = s->cfg.max_batch, R = s->cfg.trials, np = k.npad;
  return B * (k.frag + np * 4 + 4 + np * np * 8 + np * 8 + 4 + 2 * sizeof(void*)) +
         B * R * (2 * np + 5 * 4 + 8) + B * (np + 8 + 12);
}

void free_chunk(Chunk* c) {
  if (c->done) (void)hipEventDestroy(c->done);
  for (void* p : {(void*)c->h_frag, (void*)c->h_hf, (void*)c->h_scale, (void*)c->h_j64, (void*)c->h_h64,
                  (void*)c->h_sid, (void*)c->h_spins, (void*)c->h_e, (void*)c->h_sel})
    if (p) (void)hipHostFree(p);
  for (void* p : {(void*)c->d_frag, (void*)c->d_hf, (void*)c->d_scale, (void*)c->d_j64, (void*)c->d_h64,
                  (void*)c->d_sid, (void*)c->d_j64p, (void*)c->d_h64p, (void*)c->d_final, (void*)c->d_best,
                  (void*)c->d_stats, (void*)c->d_rerank, (void*)c->d_sel_spins, (void*)c->d_sel_e,
                  (void*)c->d_sel_i})
    dev_free(p, nullptr);
  delete c;
}

template <typename T>
bool host_alloc(T** p, size_t count) {
  return hipHostMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault) == hipSuccess;
}
template <typename T>
bool dev_alloc_n(T** p, size_t count) {
  *p = (T*)dev_alloc(std::max<size_t>(count, 1) * sizeof(T), nullptr);
  return *p != nullptr;
}

Chunk* new_chunk(pim_server* s, int cls) {
  const Klass& k = s->classes[cls];
  const size_t B = s->cfg.max_batch, R = s->cfg.trials, np = k.npad;
  auto* c = new Chunk();
  c->cls = cls;
  bool ok = hipEventCreateWithFlags(&c->done, hipEventDisableTiming) == hipSuccess;
  ok = ok && host_alloc(&c->h_frag, B * k.frag) && host_alloc(&c->h_hf, B * np) && host_alloc(&c->h_scale, B) &&
       host_alloc(&c->h_j64, B * np * np) && host_alloc(&c->h_h64, B * np) && host_alloc(&c->h_sid, B) &&
       host_alloc(&c->h_spins, B * np) && host_alloc(&c->h_e, B) && host_alloc(&c->h_sel, 3 * B);
  ok = ok && dev_alloc_n(&c->d_frag, B * k.frag) && dev_alloc_n(&c->d_hf, B * np) && dev_alloc_n(&c->d_scale, B) &&
       dev_alloc_n(&c->d_j64, B * np * np) && dev_alloc_n(&c->d_h64, B * np) && dev_alloc_n(&c->d_sid, B) &&
       dev_alloc_n(&c->d_j64p, B) && dev_alloc_n(&c->d_h64p, B) && dev_alloc_n(&c->d_final, B * R * np) &&
       dev_alloc_n(&c->d_best, B * R * np) && dev_alloc_n(&c->d_stats, 5 * B * R) &&
       dev_alloc_n(&c->d_rerank, B * R) && dev_alloc_n(&c->d_sel_spins, B * np) && dev_alloc_n(&c->d_sel_e, B) &&
       dev_alloc_n(&c->d_sel_i, 3 * B);
  if (ok) {  // per-request pointer tables of the re-rank, fixed for the chunk's lifetime
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
  const size_t need = chunk_device_bytes(s, k);
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
  hipError_t e = hipMemcpyAsync(c->d_frag, c->h_frag, B * k.frag, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_hf, c->h_hf, B * np * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_scale, c->h_scale, B * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_j64, c->h_j64, B * np * np * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_h64, c->h_h64, B * np * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_sid, c->h_sid, B * 4, hipMemcpyHostToDevice, st);
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
  if (e == hipSuccess) e = hipMemcpyAsync(c->h_spins, c->d_sel_spins, B * np, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->h_e, c->d_sel_e, B * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->h_sel, c->d_sel_i, 3 * B * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(c->done, st);
  return e;
}

}  // namespace

extern "C" {

pim_status pim_server_create(const pim_server_config* cfg, pim_server** out) {
  try {
    if (!cfg || !out) return fail(PIM_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (cfg->max_n < 1 || cfg->max_n > PIM_MAX_N_LDS)
      return fail(PIM_ERR_INVALID, "max_n = %d outside [1, %d]", cfg->max_n, PIM_MAX_N_LDS);
    if (cfg->trials < 1 || cfg->steps < 1) return fail(PIM_ERR_INVALID, "trials and steps must be >= 1");
    if (!cfg->beta || !cfg->eta) return fail(PIM_ERR_INVALID, "beta and eta must be non-NULL");
    if (cfg->prec != PIM_PREC_FP8 && cfg->prec != PIM_PREC_BF16) return fail(PIM_ERR_INVALID, "unknown precision");
    if (cfg->streams < 1 || cfg->streams > 8) return fail(PIM_ERR_INVALID, "streams must be in [1, 8]");
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
      ok = hipStreamCreateWithFlags(&q, hipStreamNonBlocking) == hipSuccess;
      if (ok) s->streams.push_back(q);
    }
    s->classes.resize((PIM_MAX_N_LDS + 31) / 32);
    for (size_t c = 0; c < s->classes.size(); ++c) {
      s->classes[c].nt = (int)c + 1;
      s->classes[c].npad = 32 * ((int)c + 1);
      s->classes[c].frag = real_frag_bytes(cfg->prec, (int)c + 1);
    }
    if (!ok) {
      pim_server_destroy(s);
      return fail(PIM_ERR_NOMEM, "server set-up failed");
    }
    *out = s;
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_server_create");
  }
}

pim_status pim_server_submit(pim_server* s, int32_t count, const uint32_t* ids, const int32_t* ns,
                             const double* const* J, const double* const* h, int32_t* admitted) {
  try {
    if (!s || !ids || !ns || !J || !admitted) return fail(PIM_ERR_INVALID, "NULL argument");
    *admitted = 0;
    for (int r = 0; r < count; ++r) {
      const int n = ns[r];
      if (n < 1 || n > s->cfg.max_n) return fail(PIM_ERR_INVALID, "request %d: n = %d outside [1, %d]", r, n, s->cfg.max_n);
      if (ids[r] >= (1u << 24)) return fail(PIM_ERR_INVALID, "request id must be < 2^24");
      const double* Jr = J[r];
      const double* hr = h ? h[r] : nullptr;
      for (int i = 0; i < n; ++i) {
        if (Jr[(size_t)i * n + i] != 0.0) return fail(PIM_ERR_INVALID, "request %d: J diagonal must be zero", r);
        if (hr && !std::isfinite(hr[i])) return fail(PIM_ERR_INVALID, "request %d: h is not finite", r);
        for (int j = 0; j < n; ++j)
          if (!std::isfinite(Jr[(size_t)i * n + j]) || Jr[(size_t)i * n + j] != Jr[(size_t)j * n + i])
            return fail(PIM_ERR_INVALID, "request %d: J must be finite and symmetric", r);
      }
      const int cls = (n + 31) / 32 - 1;
      Chunk* c = chunk_for(s, cls);
      if (!c) break;  // no slot: the caller polls and submits the rest later
      const Klass& k = s->classes[cls];
      const size_t np = k.npad, slot = c->count;
      const float scale = real_scale(Jr, (size_t)n * n, s->cfg.prec);
      pack_real_fragments(Jr, n, k.nt, s->cfg.prec, scale, c->h_frag + slot * k.frag);
      c->h_scale[slot] = scale;
      float* hf = c->h_hf + slot * np;
      double* h64 = c->h_h64 + slot * np;
      double* j64 = c->h_j64 + slot * np * np;
      std::fill(hf, hf + np, 0.0f);
      std::fill(h64, h64 + np, 0.0);
      std::fill(j64, j64 + np * np, 0.0);
      for (int i = 0; i < n; ++i) {
        if (hr) {
          hf[i] = (float)hr[i];
          h64[i] = hr[i];
        }
        std::memcpy(j64 + (size_t)i * np, Jr + (size_t)i * n, n * sizeof(double));
      }
      c->h_sid[slot] = ids[r];
      c->ids.push_back(ids[r]);
      c->ns.push_back(n);
      ++c->count;
      ++*admitted;
    }
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
    for (Klass& k : s->classes) {
      k.open = -1;
      for (Chunk* c : k.chunks) {
      if (c->launched || c->count == 0) continue;
      hipStream_t st = s->streams[s->next_stream];
      s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
      hipError_t e = launch_chunk(s, c, st);
      if (e != hipSuccess) return fail(PIM_ERR_DEVICE, "server launch failed: %s", hipGetErrorString(e));
      c->launched = true;
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
  try {
    if (!s || !ids || !done) return fail(PIM_ERR_INVALID, "NULL argument");
    *done = 0;
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
      }
      *done += c->count;
      c->count = 0;
      c->launched = false;
      c->ids.clear();
      c->ns.clear();
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
  for (hipStream_t q : s->streams) (void)hipStreamDestroy(q);
  dev_free(s->d_thtab, nullptr);
  dev_free(s->d_zero, nullptr);
  dev_free(s->d_cancel, nullptr);
  delete s;
}

}  // extern "C"
