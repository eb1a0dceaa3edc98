// Internal declarations shared by the host library and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "pim.h"

namespace pim {

// ---- errors / allocation (pim_api.cpp) ------------------------------------
pim_status fail(pim_status st, const char* fmt, ...);
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

// Runs fn(lo, hi) over [0, n) in chunks of at least `grain` items on up to
// hardware_concurrency threads (host).
template <typename F>
void parallel_for(int n, F&& fn, int grain = 256) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::min(hw, std::max(1, n / std::max(1, grain)));
  if (nt <= 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> pool;
  const int chunk = (n + nt - 1) / nt;
  for (int k = 0; k < nt; ++k) {
    const int lo = k * chunk, hi = std::min(n, lo + chunk);
    if (lo < hi) pool.emplace_back([&fn, lo, hi] { fn(lo, hi); });
  }
  for (auto& th : pool) th.join();
}

// ---- update-rule constants of one instance --------------------------------
constexpr int kNoiseBits = 8;              // B
constexpr int kNoiseVals = 1 << kNoiseBits;
constexpr int kTabEntries = kNoiseVals * 2;  // theta-by-noise table over (u, s)
constexpr int kFieldLimit = 32766;           // |I| bound that keeps thresholds in int16
constexpr int kMaxLevels = 16;

struct Rule {
  bool real = false;         // real-valued couplings (binary64 J, h)
  int n = 0;
  double c = 0, xi = 0;
  int levels = 0;
  int noise = 0;
  std::vector<double> ztab;  // 2^B non-decreasing
  uint32_t stream = 0;
  bool same_table_class(const Rule& o) const {
    return real == o.real && c == o.c && xi == o.xi && levels == o.levels && ztab == o.ztab;
  }
};

// ---- schedule compiler (schedule.cpp) -------------------------------------
// theta[j-1], j = 1..L-1: smallest integer I with fl(fl(beta*c) * I) >= b_j,
// clamped to [-32768, 32767].  umin[2k + (s<0)]: smallest u in [0, 2^B) with
// s(t+1) = +1 for LUT bin k and current spin s; 2^B if none.
void compile_step(const Rule& r, double beta, double eta, int32_t* theta, int32_t* umin);
// Field threshold per (u, s): s(t+1) = +1  <=>  I >= tab[kNoiseVals + (u ^ s)],
// s = +-1 as a two's-complement int (u ^ 1 for s = +1, ~u for s = -1).
void theta_by_noise(const int32_t* theta, const int32_t* umin, int levels, int16_t* tab);
// Real-valued fields: theta[j-1] is the smallest float x with
// fl(fl(beta*c) * x) >= b_j (-inf: every finite field, +inf: none); umin as above.
void compile_step_real(const Rule& r, double beta, double eta, float* theta, int32_t* umin);
// Float field threshold per (u, s): s(t+1) = +1  <=>  I >= tab[kNoiseVals + (u ^ m)]
// with m = 0 for s = +1 and m = -1 for s = -1 (index u, resp. ~u).
void theta_by_noise_real(const float* theta, const int32_t* umin, int levels, float* tab);
// Built-in quantile table of a noise law; false if unknown.
bool builtin_noise_table(int noise, std::vector<double>& out);

// ---- device argument blocks ----------------------------------------------
struct SweepArgs {
  const int8_t* jfrag;       // [count][NT*NT][64][16] MFMA A fragments
  int8_t* trace;             // [count][R][T+1][npad] every state s(t), or nullptr
  const int32_t* h;          // [count][npad] or nullptr
  const int16_t* thtab;      // [classes][T][kTabEntries]
  const int32_t* inst_class; // [count]
  const uint32_t* inst_stream;  // [count]
  const int32_t* target;     // [count] or nullptr
  const int8_t* init;        // [count][R][npad] or nullptr
  int8_t* final_s;           // [count][R][npad]
  int8_t* best_s;            // [count][R][npad]
  int32_t* e_best;           // [count][R]
  int32_t* t_best;
  int32_t* first_hit;
  int32_t* e_final;
  int32_t* steps_done;
  const volatile int32_t* cancel;
  int32_t n, npad, R, T, start_step;
  uint32_t k0, k1;
  int32_t waves;             // waves (32-trial blocks) per workgroup: 1, 2 or 4
  int32_t count;             // instances
};

// Real-valued instances: spins and states as in SweepArgs; energies binary32
// (stored in the int32 stat arrays as their bit patterns).
struct SweepRealArgs {
  const uint8_t* jfrag;      // [count][frag bytes] quantised couplings in fragment order
  const float* scale;        // [count]
  const float* h;            // [count][npad] or nullptr
  const float* thtab;        // [classes][T][kTabEntries]
  const int32_t* inst_class; // [count]
  const uint32_t* inst_stream;  // [count]
  const float* target;       // [count] or nullptr
  const int8_t* init;        // [count][R][npad] or nullptr
  int8_t* final_s;           // [count][R][npad]
  int8_t* best_s;            // [count][R][npad]
  float* e_best;             // [count][R]
  int32_t* t_best;
  int32_t* first_hit;
  float* e_final;
  int32_t* steps_done;
  const volatile int32_t* cancel;
  int32_t n, npad, R, T, start_step;
  uint32_t k0, k1;
};

// Sequential (conventional) PIM: same fields as SweepArgs with row-major J.
struct SeqArgs {
  const int8_t* j8pad;       // [count][npad][npad] int8 J, zero-padded rows
  const int32_t* h;          // [count][npad] or nullptr
  const int16_t* thtab;      // [classes][T][kTabEntries]
  const int32_t* inst_class;
  const uint32_t* inst_stream;
  const int32_t* target;
  const int8_t* init;
  int8_t* final_s;
  int8_t* best_s;
  int32_t* e_best;
  int32_t* t_best;
  int32_t* first_hit;
  int32_t* e_final;
  int32_t* steps_done;
  const volatile int32_t* cancel;
  int32_t n, npad, R, T, start_step;
  uint32_t k0, k1;
};

struct PlainArgs {
  const float* jf32;         // [npad][jstride] of one instance, zero-padded
  const int32_t* h;          // [n] or nullptr (integer instances)
  const float* hf;           // [n] or nullptr (real instances)
  const int32_t* steptab;    // [T][(L-1) + 2L] theta (int32, or float bits) then umin
  const int8_t* init;        // [R][npad] or nullptr
  int8_t* final_s;           // [R][npad]
  int8_t* best_s;
  int32_t* e_best;
  int32_t* t_best;
  int32_t* first_hit;
  int32_t* e_final;
  int32_t* steps_done;
  const volatile int32_t* cancel;
  int32_t n, npad, jstride, R, T, start_step, levels, use_target, target;
  uint32_t stream, k0, k1;
};

struct EnergyArgs {
  const float* jf32;   // [>= n][jstride] (integer instances)
  const int32_t* h;    // [n] or nullptr
  const double* jf64;  // [n][n] (real instances; then jf32 / h unused)
  const double* hf64;  // [n] or nullptr
  const int8_t* spins; // [count][stride]
  double* out;         // [count]
  int32_t n, jstride, stride, count;
};

struct RerankArgs {
  const int8_t* const* j8;     // [count] device pointers to each instance's int8 J (n x n)
  const int32_t* const* h;     // [count] device pointers to h, or nullptr (no fields)
  const double* const* j64;    // real instances: [count] binary64 J (n x n); then j8 / h unused
  const double* const* h64;    // real instances: [count] binary64 h, or nullptr
  const int8_t* best_s;        // [count][R][npad]
  const int32_t* t_best;       // [count][R]
  const int32_t* e_best;       // [count][R]
  double* energy;              // [count][R] binary64 re-evaluation
  int8_t* out_spins;           // [count][npad]
  double* out_energy;          // [count]
  int32_t* out_trial;          // [count]
  int32_t* out_step;           // [count]
  int32_t* out_tracked;        // [count]
  int32_t n, npad, R, count;
};

hipError_t launch_rerank_select(const RerankArgs& a, hipStream_t s);
hipError_t launch_sweep_mfma(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s);
// The same on e2m1 (FP4) operands (couplings in {0, +-1, +-2, +-3, +-4, +-6}):
// a.jfrag holds pack_f4_fragments output; no state recording.
hipError_t launch_sweep_mfma4(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s);
hipError_t launch_sweep_plain(const PlainArgs& a, bool real, hipStream_t s);
// 256 < N <= 1024: couplings streamed from global memory, spins in LDS.
hipError_t launch_sweep_big(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s);
int big_tiles(int n);  // row tiles of the streamed kernel: ceil(n / 32)
// The same range on e2m1 (FP4) operands, for couplings in {0, +-1, +-2, +-3,
// +-4, +-6} (exact): a.jfrag holds pack_f4_fragments output.
hipError_t launch_sweep_big4(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s);
// Several batches (parts) of the streamed kernels in one launch, all on e2m1
// operands (launch_sweep_big4_multi) or all on int8 (launch_sweep_big_multi):
// parts[p] holds part p's arguments and row tile count; work[b] = (part,
// instance, trial block, 0), or part -1 for an empty workgroup.  LDS is sized for the largest tile
// count.  With has_h every part's a.h is non-null (zeros where a part has no
// fields).
// The run's scalars (seed words, steps, first counter step, whether targets
// are tracked) replace those in the parts' arguments.
struct MultiPart {
  SweepArgs a;
  int32_t nt, pad[3];
};
struct MultiRun {
  uint32_t k0, k1;
  int32_t T, start_step, use_target;
};
hipError_t launch_sweep_big4_multi(const MultiPart* d_parts, const int4* d_work, int nwork, int nt_max, bool has_h,
                                   const MultiRun& run, hipStream_t s);
double big4_step_cost(int nt);  // relative workgroup time per step, for ordering work
hipError_t launch_sweep_big_multi(const MultiPart* d_parts, const int4* d_work, int nwork, int nt_max, bool has_h,
                                  const MultiRun& run, hipStream_t s);
double big_step_cost(int nt);  // the same for the int8 streamed kernel
bool f4_couplings(const int8_t* J, size_t count);  // every value e2m1-exact
size_t f4_frag_bytes(int nt);                      // per instance: nt x ceil(nt/2) fragments of 1 KB
void pack_f4_fragments(const int8_t* J, int n, int nt, uint8_t* out);
hipError_t launch_sweep_seq(const SeqArgs& a, int count, int nt, bool has_h, hipStream_t s);
hipError_t launch_sweep_real(const SweepRealArgs& a, int count, int nt, int prec, bool has_h, hipStream_t s);
size_t real_frag_bytes(int prec, int nt);
// Device-side quantisation of real instances (request server).
struct RealPackArgs {
  const double* j64;   // [count][npad][npad] binary64 J, zero-padded
  const double* h64;   // [count][npad]
  uint8_t* frag;       // [count][frag_bytes]
  float* hf;           // [count][npad]
  float* scale;        // [count]
  double* pmax;        // [count][kPackSlices] scratch: max |J| of each slice of J
  size_t frag_bytes;
  int32_t npad, count;
};
constexpr int kPackSlices = 16;
hipError_t launch_pack_real(const RealPackArgs& a, int prec, hipStream_t s);
// Device-side MIMO mapping (mimo_map.hip): per request the Ising instance of
// pim_mimo_ising, written zero-padded into j64 / h64, and x_m.
struct MimoSlot {
  int32_t nr, nt, qam, map;  // map: pim_mimo_map
  double esn0;               // Es/N0 (linear), used by the DI mapping
  int64_t hy_off;            // offset (doubles) of the request's H then y in hy
};
struct MimoMapArgs {
  const MimoSlot* slots;     // [count]
  const double* hy;          // H (nr x nt complex, interleaved, row-major) then y (nr complex)
  double* j64;               // [count][npad][npad]
  double* h64;               // [count][npad]
  double* xm;                // [count][xm_stride]
  int32_t npad, xm_stride, count;
};
hipError_t launch_mimo_map(const MimoMapArgs& a, size_t max_work, size_t max_hy, hipStream_t s);
// bytes from src to dst by a kernel on stream s (either side may be pinned,
// device-mapped host memory given by its device address); both 16-byte aligned
hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);
size_t mimo_map_work_doubles(int nr, int nt);
hipError_t launch_energy_f64(const EnergyArgs& a, hipStream_t s);

// Neighbour-triggered flip counts of one instance's recorded states.
struct FlipRateArgs {
  const int8_t* trace;         // [R][T+1][npad] of the instance
  const int8_t* j8;            // [n][n]
  unsigned long long* num;     // [T]
  unsigned long long* den;     // [T]
  int32_t n, npad, R, T;
};
hipError_t launch_flip_rate(const FlipRateArgs& a, hipStream_t s);

// Host packing of J into the MFMA fragment order (sweep_mfma.hip, sweep_real.hip).
void pack_mfma_fragments(const int8_t* J, int n, int nt, int8_t* out);
void pack_real_fragments(const double* J, int n, int nt, int prec, float scale, uint8_t* out);

// ---- quantisation (quant.cpp) ---------------------------------------------
uint8_t fp8_e4m3_rne(double x);
double fp8_e4m3_value(uint8_t c);
uint16_t bf16_rne(double x);
double bf16_value(uint16_t c);
float real_scale(const double* J, size_t count, int prec);
double quantized_value(double x, int prec, float scale);

}  // namespace pim

// ---- handles ------------------------------------------------------------
struct pim_instance {
  pim::Rule rule;                 // rule.real: real-valued instance
  int prec = 0;                   // real instances: PIM_PREC_*
  float scale = 1.0f;             // real instances: J ~ scale * q
  int npad = 0, nt = 0;
  int jstride = 0;                // row stride of d_jf32: n rounded up to 4
  size_t frag_bytes = 0;
  bool has_h = false;
  uint8_t* d_arena = nullptr;     // one allocation holding every buffer below
  int8_t* d_jfrag = nullptr;      // int8, FP8 or BF16 MFMA fragments
  uint8_t* d_jfrag4 = nullptr;    // e2m1 fragments (integer instances with e2m1-exact J) or NULL
  size_t frag4_bytes = 0;
  float* d_jf32 = nullptr;        // [npad][jstride] FP32 J, zero-padded
  int8_t* d_j8 = nullptr;         // row-major int8 J (re-rank; integer instances)
  int32_t* d_h = nullptr;         // [npad] (integer instances)
  float* d_hf = nullptr;          // [npad] fl32(h) (real instances)
  double* d_j64 = nullptr;        // [n][n] binary64 J (real instances)
  double* d_h64 = nullptr;        // [n] binary64 h (real instances)
};

struct pim_batch {
  std::vector<pim_instance*> insts;
  int count = 0, R = 0, n = 0, npad = 0, nt = 0;
  bool real = false;
  int prec = 0;
  size_t frag_bytes = 0;          // per instance
  bool has_h = false;
  hipStream_t stream = nullptr;
  // device buffers: d_arena holds the fixed-size ones (fragments .. selection
  // outputs); the step tables, trajectories and padded int8 J are separate
  uint8_t* d_arena = nullptr;
  int8_t* d_jfrag = nullptr;      // concatenated fragments of all instances
  uint8_t* d_jfrag4 = nullptr;    // concatenated e2m1 fragments, when every instance has them
  size_t frag4_bytes = 0;         // per instance
  int8_t* d_j8pad = nullptr;      // [count][npad][npad] row-major int8 J (sequential kernel)
  int8_t* d_trace = nullptr;      // [count][R][T+1][npad] recorded states (diagnostics)
  size_t trace_bytes = 0;
  bool recorded = false;          // the last run recorded its states
  int32_t* d_h = nullptr;         // [count][npad] int32 (integer) or float (real) fields
  float* d_scale = nullptr;       // [count] (real)
  int8_t* d_init = nullptr;
  int8_t* d_final = nullptr;
  int8_t* d_best = nullptr;
  int32_t* d_stats = nullptr;     // 5 x [count][R]: e_best, t_best, first_hit, e_final, steps_done
  int32_t* d_class = nullptr;
  uint32_t* d_stream_ids = nullptr;
  int32_t* d_target = nullptr;    // int32 (integer) or float (real) targets
  double* d_rerank = nullptr;     // [count][R]
  // per-instance selection (device, then one readback): ptr tables + outputs
  const int8_t** d_jptrs = nullptr;
  const int32_t** d_hptrs = nullptr;
  const double** d_j64ptrs = nullptr;
  const double** d_h64ptrs = nullptr;
  int8_t* d_sel_spins = nullptr;  // [count][npad]
  double* d_sel_e = nullptr;      // [count]
  int32_t* d_sel_i = nullptr;     // [count][3]: trial, step, tracked energy
  std::vector<int8_t> h_sel_spins;
  std::vector<double> h_sel_e;
  std::vector<int32_t> h_sel_i;
  void* d_thtab = nullptr;        // int16 (integer) or float (real) step tables
  size_t thtab_bytes = 0;
  int32_t* d_steptab = nullptr;
  size_t steptab_bytes = 0;
  // schedule the (u, s) step tables in d_thtab were compiled from: a run with
  // the same beta and eta (bit for bit) reuses them without compiling or
  // uploading again
  bool tab_valid = false;
  std::vector<double> tab_beta, tab_eta;
  int32_t* h_cancel = nullptr;    // pinned, host-mapped (a slot of a shared slab)
  int32_t* d_cancel = nullptr;    // device view of h_cancel
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // host-side class bookkeeping
  std::vector<int> inst_class;
  std::vector<int> class_rep;     // representative instance of each class
  int waves = 4;                  // int8 MFMA kernel: 32-trial waves per workgroup (1, 2, 4)
  // uneven N: one part (a simple batch) per padded size, launched together as
  // the parallel branches of one captured graph
  std::vector<pim_batch*> parts;
  std::vector<int> part_of, local_of;  // instance -> part, index inside the part
  std::vector<hipStream_t> fork;       // one per part (default priority)
  std::vector<hipEvent_t> join;
  hipEvent_t fork_ev = nullptr;
  hipStream_t cap = nullptr;           // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // e2m1 parts run as one launch: part arguments then the work list on the
  // device, and the host copy last uploaded (re-uploaded only when it changes)
  uint8_t* d_multi = nullptr;
  size_t multi_cap = 0;
  std::vector<uint8_t> h_multi;
  // run state
  bool ran = false, reranked = false, sticky_error = false;
  int last_T = 0, last_start = 0;
  int cancelled_checked = -1;     // -1 unknown, 0 complete, 1 cancelled
};
