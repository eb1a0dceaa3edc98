/*
 * pim.h -- C ABI of the MI355X PIMI sweep library (libpim.so).
 *
 * The library runs the fully parallel, synchronous p-bit update with inertia
 * (PIMI, Eq. (4) and Box 1 of Zhu et al., "A fully parallel densely connected
 * probabilistic Ising machine with inertia for real-time applications") on
 * dense integer Ising instances, many trials and instances per launch, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Sec. II, Eq. (1)): minimise
 *     H(s) = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i,   s_i in {-1, +1},
 * for a symmetric J with zero diagonal.  A *trial* starts from an initial
 * configuration and applies T update steps, producing one candidate; the
 * host keeps the lowest-energy candidate (Box 1; Suppl. "PIMI FPGA
 * implementation for Max-cut and SK-1", "Output handling and solution
 * selection").
 *
 * Update rule evaluated for every spin i of every trial at step t:
 *     I_i(t)   = sum_j J_ij s_j(t) + h_i                          (Eq. (2))
 *     s_i(t+1) = sign[ LUT_L( (beta(t) * c) * I_i(t) ) + xi * s_i(t)
 *                      + eta(t) * Z[u_i(t)] ]                      (Eq. (4))
 * where
 *   - c is the coupling normalisation (2/sqrt(N) for Max-Cut, 1/sqrt(N) for
 *     SK-1: Suppl. "Max-Cut instance generation" / "SK-1 instance
 *     generation", Preprocessing), applied to the accumulated integer field
 *     (Suppl. "Quantization scheme");
 *   - LUT_L is the L-level tanh table (Suppl. "Quantization scheme",
 *     Algorithm "LUT-based tanh approximation"): breakpoints b_k = (2k-L)/L,
 *     levels (2k-(L-1))/(L-1), saturating outside [-1, 1], x = 1 -> top level;
 *   - u_i(t) is a B-bit uniform integer (B = 8) from Philox4x32-10 with key
 *     (seed low 32 bits, seed high 32 bits) and counter
 *     (i / 16, start_step + t, trial, rng_stream); value i % 16 is byte i % 16
 *     of the 128-bit output read little-endian;
 *   - Z is a non-decreasing table of 2^B noise quantiles (Gaussian N(0,1) for
 *     PIMI; uniform U(-1,1) for the conventional PIM of Eq. (3));
 *   - every real operation is IEEE binary64 in the order written; an argument
 *     of sign that is exactly zero keeps s_i(t).
 * The library compiles these binary64 decisions, per step, into integer
 * thresholds on the exact integer field and the noise index, so every kernel
 * reproduces them bit for bit.  The conventional fully parallel PIM (Box 1,
 * middle) is the same rule with xi = 0 and uniform noise.
 *
 * Initial spins: caller-supplied, or s_i(0) = (u >= 128) ? +1 : -1 with u from
 * the same generator and counter (i / 16, 0, trial, (1 << 24) | rng_stream).
 *
 * Conventions common to every entry point
 *   - Every function returns a pim_status; a non-OK status leaves a
 *     thread-local message readable through pim_last_error().  No C++
 *     exception crosses this boundary.
 *   - "host" pointers are ordinary CPU memory owned by the caller; the
 *     library copies what it needs before returning (or, for asynchronous
 *     calls, before the call returns to the caller).
 *   - Device memory is obtained only through the allocator registered with
 *     pim_set_allocator (hipMalloc/hipFree when none is registered) and is
 *     owned by the handle that allocated it.
 *   - `stream` arguments are hipStream_t values owned by the caller (NULL =
 *     the default stream).  pim_run is asynchronous on its stream; pim_best,
 *     pim_trials and pim_energy synchronise the stream they use.  The result
 *     calls of a batch (pim_best, pim_trials, pim_states, pim_flip_counts)
 *     run on the stream of its last pim_run, which must therefore stay valid
 *     until the batch's last such call; a later pim_run on another stream and
 *     pim_batch_destroy wait for the last run through an event of the batch
 *     and never touch that stream.
 *   - Handles are not thread-safe; distinct handles may be used from
 *     distinct threads.
 */
#ifndef PIM_H
#define PIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIM_ABI_VERSION 2

/* Largest N accepted by pim_create (integer instances). */
#define PIM_MAX_N 1024
/* Largest N of the kernels that keep an instance's couplings in LDS: the
 * plain FP32 and sequential kernels, real-valued instances and state
 * recording.  Integer batches with larger N run the int8 MFMA sweep with the
 * couplings streamed from global memory. */
#define PIM_MAX_N_LDS 256

typedef enum {
  PIM_OK = 0,
  PIM_ERR_INVALID = 1,     /* argument fails validation (message says which)   */
  PIM_ERR_UNSUPPORTED = 2, /* valid request the library does not implement      */
  PIM_ERR_NOMEM = 3,       /* the allocator returned NULL                       */
  PIM_ERR_DEVICE = 4,      /* a HIP call failed; sticky on the batch            */
  PIM_ERR_STATE = 5,       /* call out of order (e.g. results before a run)     */
  PIM_ERR_CANCELLED = 6    /* the run was cancelled; results are partial        */
} pim_status;

typedef enum {
  PIM_NOISE_GAUSS = 0,   /* Z = standard normal quantiles, Eq. (4)   */
  PIM_NOISE_UNIFORM = 1  /* Z = U(-1, 1) cell midpoints, Eq. (3)     */
} pim_noise;

typedef enum {
  PIM_KERNEL_MFMA_I8 = 0,   /* persistent batched sweep on matrix cores: int8 MFMA for
                               integer instances, FP8 / BF16 MFMA for real-valued ones */
  PIM_KERNEL_PLAIN_F32 = 1, /* one instance per launch, plain FP32 dot products      */
  PIM_KERNEL_SEQ_I8 = 2,    /* conventional PIM, sequential updates (Box 1, top):
                               step t changes only spin i = (start_step + t) mod N;
                               integer instances only                               */
  PIM_KERNEL_MFMA_F4 = 3    /* as PIM_KERNEL_MFMA_I8, except that an integer batch
                               whose couplings all lie in {0, +-1, +-2, +-3, +-4,
                               +-6} runs on e2m1 (FP4) operands with binary32
                               accumulation: every product and partial sum is an
                               exact integer (|2 I| < 2^24), so results are
                               identical to int8, at twice the matrix rate; other
                               batches, and runs that record states, run the int8
                               kernel.  Integer instances only; no state recording
                               at N > 256                                           */
} pim_kernel;

/* Operand format of a real-valued instance in the batched MFMA kernel. */
typedef enum {
  PIM_PREC_FP8 = 1,   /* OCP e4m3; scale = max|J| / 448 rounded to binary32         */
  PIM_PREC_BF16 = 2   /* bfloat16; scale = the power of two with max|J|/scale in [1,2) */
} pim_prec;

/* Ising mappings of a MIMO detection problem (pim_mimo_ising). */
typedef enum {
  PIM_MIMO_ML = 0,    /* x_m = 0; T = I (4-QAM) or [2I, I] (16-QAM)                  */
  PIM_MIMO_DI = 1     /* x_m = sliced MMSE estimate; T = [I, I]                      */
} pim_mimo_map;

/* Per-instance constants of the update rule. */
typedef struct {
  int32_t n;                 /* number of spins N, 1 <= N <= PIM_MAX_N (real-valued
                                instances: N <= PIM_MAX_N_LDS)                      */
  double j_scale;            /* c > 0, finite                                      */
  double xi;                 /* inertia xi >= 0, finite                             */
  int32_t levels;            /* L, 2 <= L <= 16                                     */
  int32_t noise;             /* pim_noise                                           */
  int32_t noise_bits;        /* B; must be 8 (PIM_ERR_UNSUPPORTED otherwise): one
                                Philox4x32-10 call draws the noise of 16 spins, the
                                grain of the kernels' 16-spin tiles, and the
                                paper's own noise samples are 4-bit fixed point
                                (Suppl. "PIMI FPGA implementation for Max-cut and
                                SK-1")                                              */
  const double* noise_table; /* host, 2^B finite non-decreasing values, or NULL for
                                the built-in table of `noise` (copied at create)   */
  uint32_t rng_stream;       /* counter word 3 id, < 2^24 (request/instance id)    */
} pim_params;

/* Per-run annealing schedule (Sec. II: beta(t) up, eta(t) down; xi constant). */
typedef struct {
  int32_t steps;             /* T >= 1 update steps                                 */
  const double* beta;        /* host [T], beta(t) >= 0 finite (copied)              */
  const double* eta;         /* host [T], eta(t) >= 0 finite (copied)               */
  int32_t start_step;        /* counter step of the first update (resume), >= 0,
                                start_step + T < 2^31                               */
  int32_t kernel;            /* pim_kernel                                          */
  int32_t use_target;        /* nonzero: record first step with E <= target        */
  const double* target;      /* host [instance count] energies, or NULL; integer
                                instances compare E <= floor(target)                */
  int32_t record_states;     /* nonzero: keep every state s(t), t = 0..T, of every
                                trial on the device (diagnostics; integer instances,
                                PIM_KERNEL_MFMA_I8; count*trials*(T+1)*Npad bytes,
                                Npad = N rounded up to 32)                          */
} pim_schedule;

typedef struct pim_instance pim_instance; /* device copy of one (J, h, params)       */
typedef struct pim_batch pim_batch;       /* instances x trials + per-trial results  */

/* Device allocator hooks: alloc returns NULL on failure. */
typedef void* (*pim_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*pim_free_fn)(void* ptr, void* stream, void* user);

/* Registers the device allocator used by every later allocation (process
 * wide).  Both NULL restores hipMalloc/hipFree.  Memory allocated through one
 * allocator is freed through the same one. */
pim_status pim_set_allocator(pim_alloc_fn alloc, pim_free_fn free_fn, void* user);

/* Creates an instance from a host int8 coupling matrix J (row-major N x N,
 * symmetric, zero diagonal) and host int32 biases h (length N, NULL = zeros).
 * Rejects |sum_j |J_ij|| + |h_i| > 32766 (the integer field must fit the
 * int16 thresholds).  Copies J and h to the device on `stream`; *out owns the
 * copies.  Eq. (1)-(2). */
pim_status pim_create(const int8_t* J, const int32_t* h, const pim_params* params,
                      void* stream, pim_instance** out);

/* Creates a real-valued instance (the MIMO detection instances of Suppl.
 * "Delta-Ising MIMO (DI-MIMO) formulation"; the paper's FPGA keeps them in
 * 16-bit fixed point, Suppl. "PIMI FPGA implementation for MIMO detection").
 * J: host binary64 N x N, symmetric, zero diagonal, finite; h: host binary64
 * [N] or NULL.  `prec` (pim_prec) selects the batched kernel's operand format:
 * J is quantised once to scale * q, q in FP8 e4m3 or BF16 (round to nearest,
 * ties to even, from binary64), and that kernel forms the field in binary32 as
 *     I_i = fma(scale, sum_j q_ij s_j, fl32(h_i))   (sum on FP32-accumulating MFMA).
 * The plain kernel uses fl32(J) and fl32(h) without quantisation.  The
 * decisions are exactly Eq. (4)'s binary64 rule applied to that binary32
 * field; energies used for ranking (pim_best, pim_energy) are binary64 with
 * the original J and h.  Copies J and h; *out owns the device copies. */
pim_status pim_create_real(const double* J, const double* h, const pim_params* params, int32_t prec,
                           void* stream, pim_instance** out);

/* Host-only: the couplings the batched kernel uses for a real instance, as
 * binary64 values scale * q (J_out: N x N, may alias nothing), and the scale. */
pim_status pim_quantize(const double* J, int32_t n, int32_t prec, double* J_out, double* scale_out);

/* Groups `count` instances of one kind (all integer, or all real with one
 * pim_prec) with `trials` trials each.  Instances may have different N: the
 * batch then keeps one part per distinct N and pim_run launches the parts'
 * sweeps as one captured HIP graph (one graph launch per run): parallel
 * branches, except that the parts with N > PIM_MAX_N_LDS run as one launch
 * over a longest-first work list when there are at least two of them on one
 * operand type (e2m1 when at least two are e2m1 parts of a PIM_KERNEL_MFMA_F4
 * run, else int8), which the other parts follow when it has a workgroup for
 * every CU; init_spins then holds, instance after instance, trials x N_k
 * values.
 * init_spins:
 * host int8 [count][trials][N] of +-1, or NULL for generator-drawn initial
 * spins.  The batch keeps pointers to the instances, which must outlive it.
 * Trial a of instance k is trial id a in the generator counter. */
pim_status pim_batch_create(pim_instance* const* insts, int32_t count, int32_t trials,
                            const int8_t* init_spins, void* stream, pim_batch** out);

/* Runs T steps of Eq. (4) on every trial of every instance of the batch
 * (PIM_KERNEL_SEQ_I8: T single-spin steps of the same rule, spin
 * (start_step + t) mod N at step t, noise u = byte i % 16 of the Philox block
 * (i / 16, start_step + t, trial, rng_stream); the conventional PIM of Eq. (3)
 * is this rule with xi = 0 and uniform noise),
 * asynchronously on `stream`.  Compiles the schedule on the host, uploads the
 * tables and launches the sweep (PIM_KERNEL_MFMA_I8: one launch for the whole
 * batch; PIM_KERNEL_PLAIN_F32: one launch per instance).  The MFMA and
 * sequential kernels' tables stay on the device: a run whose beta and eta
 * equal (bit for bit, same T) those of the batch's previous such run reuses
 * them without compiling or uploading.  The host waits for the table upload
 * before returning; the sweep itself runs asynchronously.  A run on another
 * stream than the batch's previous call first waits on the host for the work
 * on that stream, since the two runs share the batch's buffers.  Tracks, over the
 * energies E(t) of s(t) for t = 0..T (counter steps start_step..start_step+T):
 * the lowest energy and its earliest step, the state there, and the first step
 * with E <= target.  Resuming: pass the previous final spins as init_spins of a
 * new batch and start_step = previous start_step + T. */
pim_status pim_run(pim_batch* batch, const pim_schedule* sched, uint64_t seed, void* stream);

/* Picks, for every distinct N of an integer batch, the number of 32-trial
 * waves per workgroup of the int8 MFMA kernel (4, 2 or 1: trials per
 * workgroup and hence workgroups per compute unit) by timing two runs of
 * `steps` steps (beta = 1, eta = 0.5) with each choice; later runs use the
 * fastest.  Overwrites the batch's results.  waves_out: host [number of
 * distinct N, ascending], or NULL.  Synchronises. */
pim_status pim_tune(pim_batch* batch, int32_t steps, void* stream, int32_t* waves_out);

/* Requests cancellation of the batch's current run: host-callable at any time
 * from any thread; the kernel stops within 256 steps.  Results of a cancelled
 * run are partial and the result getters return PIM_ERR_CANCELLED. */
pim_status pim_cancel(pim_batch* batch);

/* Energies (Eq. (1)) of `count` configurations spins[count][N] (+-1), in
 * binary64 on the device; out: host double[count].  `spins` is either host
 * memory (validated: every value must be +-1, else PIM_ERR_INVALID) or device
 * memory of the current device, which the runtime identifies as such and the
 * kernel reads in place without validation (values other than +-1 give
 * meaningless energies).  Synchronises `stream`. */
pim_status pim_energy(const pim_instance* inst, const int8_t* spins, int32_t count,
                      double* out, void* stream);

/* Size in bytes of the device scratch array behind pim_energy_noalloc (one
 * per GPU, held until the process ends). */
#define PIM_NOALLOC_SCRATCH_BYTES 1048576

/* pim_energy for callers that cannot allocate device memory (code that must
 * not call hipMalloc, tight serving loops, harnesses that forbid allocation):
 * the same arguments, validation, results and synchronisation, but no device
 * allocation of any kind.  The energies, and host spins staged for the
 * kernel, live in the library's fixed per-GPU scratch array of
 * PIM_NOALLOC_SCRATCH_BYTES bytes: 8 * count rounded up to 256, plus
 * count * N for host spins (device spins are read in place), must fit, else
 * PIM_ERR_INVALID.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (from several host threads, on any streams) race and
 * must be serialised by the caller.  Not for stream capture (it
 * synchronises). */
pim_status pim_energy_noalloc(const pim_instance* inst, const int8_t* spins, int32_t count,
                              double* out, void* stream);

/* Best candidate of instance `inst` after a run: re-evaluates every trial's
 * best state in binary64 on the device (once per run), takes the lowest
 * energy (ties: lowest trial id) and returns its state (host int8[N]), energy,
 * trial id and the step at which it occurred.  Any output may be NULL.
 * For integer instances the tracked integer energy must equal the binary64
 * value (PIM_ERR_DEVICE otherwise).  Synchronises the batch's stream. */
pim_status pim_best(pim_batch* batch, int32_t inst, int8_t* spins_out, double* e_out,
                    int32_t* trial_out, int32_t* step_out);

/* Per-trial results of instance `inst` (host arrays of length `trials`, or
 * trials*N for spins; any may be NULL): best energy, its step, first step at
 * or below target (-1 = never), final energy E(T), best and final states.
 * Energies are the ones the kernel tracked: exact integers for integer
 * instances, binary32 field energies for real ones.  Synchronises. */
pim_status pim_trials(pim_batch* batch, int32_t inst, double* best_e, int32_t* best_step,
                      int32_t* first_hit, double* final_e, int8_t* best_spins,
                      int8_t* final_spins);

/* Recorded trajectory of one trial (the last run had record_states set):
 * states: host int8 [(T+1)][N], s(t) at row t (rows after a cancellation are
 * unspecified).  Synchronises. */
pim_status pim_states(pim_batch* batch, int32_t inst, int32_t trial, int8_t* states);

/* Neighbour-triggered flip counts of instance `inst` over the recorded run
 * (Suppl. "Quantifying coupled oscillatory dynamics via neighbor-triggered
 * flip rates"): for t = 0..T-1, den[t] = #{(i, trial): some j with J_ij != 0
 * flips between s(t) and s(t+1)}, num[t] = those of them where i flips too;
 * P_NT(t) = num[t] / den[t].  Computed on the device; num, den: host [T].
 * Synchronises. */
pim_status pim_flip_counts(pim_batch* batch, int32_t inst, int64_t* num, int64_t* den);

/* Duration in milliseconds of the sweep kernel(s) of the last pim_run,
 * measured with HIP events on the run's stream.  Synchronises. */
pim_status pim_kernel_time(pim_batch* batch, float* ms);

/* Host-only: the integer thresholds the library compiles for one step t of a
 * schedule (no device work).  theta: int32[L-1], the smallest integer field
 * I with LUT bin index >= j (j = 1..L-1), clamped to [-32768, 32767];
 * u_min: int32[2*L], for LUT bin k and current spin s (index 2k + (s < 0)),
 * the smallest noise index u giving s(t+1) = +1 (2^B = never). */
pim_status pim_compile_step(const pim_params* params, double beta, double eta,
                            int32_t* theta, int32_t* u_min);

/* Host-only: the 512-entry table the MFMA kernel uses for one step:
 * s(t+1) = +1 iff I >= table[256 + (u ^ s)] with s = +-1 as a two's-complement
 * int (index 256 + (u ^ 1) for s = +1, 255 - u for s = -1).  table: int16[512]. */
pim_status pim_compile_table(const pim_params* params, double beta, double eta, int16_t* table);

/* Host-only: the 512-entry table of a real-valued batch's MFMA kernel for one
 * step: s(t+1) = +1 iff I >= table[256 + (u ^ m)], m = 0 for s = +1 and -1 for
 * s = -1 (index 256 + u, resp. 255 - u); entries are the smallest binary32
 * field x with fl(fl(beta*c) * x) >= b_j for the bin that decides, or -inf
 * (always +1) / +inf (never).  table: float[512]. */
pim_status pim_compile_table_real(const pim_params* params, double beta, double eta, float* table);

/* Ising instance of one uplink MIMO detection problem y = H x + n (Suppl.
 * "MIMO problem definition", "Real-Valued equivalent", "Delta-Ising MIMO
 * (DI-MIMO) formulation").  H: host complex [nr][nt] and y: complex [nr], both
 * as interleaved (re, im) binary64.  qam: 4 or 16.  map: pim_mimo_map; the DI
 * mapping's MMSE estimate uses the regulariser 1 / esn0 (Es/N0, linear).
 * With the real-valued model (Hr, yr) and x = x_m + T s:
 *     J = -2 zeroDiag(T^T Hr^T Hr T)   (Eq. (1) counts each pair once),
 *     h = 2 T^T Hr^T (yr - Hr x_m),
 * so E(s) of Eq. (1) = ||yr - Hr(x_m + T s)||^2 - const.  Outputs (host,
 * binary64): J [n][n], h [n], x_m [2 nt] (real parts then imaginary parts);
 * *n_out = 2 nt (ML, 4-QAM) or 4 nt.  Buffers must hold 4 nt x 4 nt, 4 nt and
 * 2 nt values; 4 nt <= PIM_MAX_N_LDS. */
pim_status pim_mimo_ising(const double* H, const double* y, int32_t nr, int32_t nt, int32_t qam, int32_t map,
                          double esn0, double* J, double* h, double* xm, int32_t* n_out);

/* pim_mimo_ising computed on the device (the request server's mapping
 * kernel, one workgroup, binary64): same arguments and outputs, plus the
 * stream it runs on (synchronised before returning).  nr <= PIM_MAX_N_LDS / 2.
 * The sums run in the host function's order, so the results are expected to
 * be identical to it. */
pim_status pim_mimo_ising_device(const double* H, const double* y, int32_t nr, int32_t nt, int32_t qam,
                                 int32_t map, double esn0, double* J, double* h, double* xm, int32_t* n_out,
                                 void* stream);

/* Detected symbols of a spin vector s (host int8 [n] of +-1) under the same
 * mapping: x = slice(x_m + T s), each real component sliced to the nearest
 * odd-integer level (2 floor(v/2) + 1, clipped).  x: host complex [nt] as
 * interleaved (re, im) binary64. */
pim_status pim_mimo_decode(const double* xm, const int8_t* s, int32_t nt, int32_t qam, int32_t map, double* x);

/* ---- request server with continuous batching -----------------------------
 * For streams of small real-valued requests (MIMO detection: Suppl. "PIMI
 * FPGA implementation for MIMO detection", host-side task scheduling).  Every
 * request is one Ising instance (binary64 J, h, N <= max_n) solved with the
 * server's fixed rule and schedule by `trials` trials on the FP8 / BF16 MFMA
 * sweep, then re-ranked in binary64; the result is the best state and its
 * energy.  The noise counter stream of a request is its id, so its result is
 * the same whatever else is in flight.
 *
 * Device memory: per N class (N rounded up to 32) up to slots_per_class slots,
 * allocated in chunks of max_batch as requests arrive, while the total stays
 * within hbm_budget bytes (0 = unbounded).  A chunk is one launch.  Its
 * host staging and result blocks are pinned, coherent and mapped into the
 * device's address space, and copy kernels on the chunk's stream move them, so
 * a chunk's whole sequence (upload, quantisation, sweep, re-rank, readback)
 * runs in order on one compute queue and never waits on a copy engine.  The
 * HIP runtime multiplexes the server's streams onto GPU_MAX_HW_QUEUES hardware
 * queues (4 unless the environment sets it before the runtime starts); mixes
 * with long requests need as many queues as streams to overlap chunks. */
typedef struct pim_server pim_server;
typedef struct {
  int32_t max_n;             /* largest request N, <= PIM_MAX_N_LDS                  */
  int32_t slots_per_class;   /* >= max_batch                                          */
  int32_t max_batch;         /* requests per launch and class, 1..65535              */
  int32_t trials;            /* trials per request                                    */
  int32_t steps;             /* T                                                      */
  const double* beta;        /* host [steps] (copied)                                 */
  const double* eta;         /* host [steps] (copied)                                 */
  double j_scale;            /* c                                                      */
  double xi;
  int32_t levels;
  int32_t noise;             /* pim_noise                                              */
  const double* noise_table; /* host [256] or NULL (copied)                            */
  int32_t prec;              /* pim_prec                                               */
  int32_t streams;           /* concurrent launch streams, 1..16                       */
  uint64_t seed;
  size_t hbm_budget;         /* bytes, 0 = no limit                                    */
  double max_wait_us;        /* pim_server_flush holds a partly filled chunk, while an
                                earlier chunk of its class is in flight, until its
                                first request has waited this long (0 = never)      */
  int32_t prealloc_chunks;   /* chunks allocated at creation per class up to max_n
                                (within slots_per_class and hbm_budget)             */
} pim_server_config;

pim_status pim_server_create(const pim_server_config* cfg, pim_server** out);

/* Admits up to `count` requests in order: ids[r] < 2^24 (also the noise
 * stream), ns[r], host J[r] (ns[r] x ns[r] binary64, symmetric, zero diagonal)
 * and h[r] (NULL for zeros).  Validates them and copies them into pinned
 * staging (quantisation happens on the device at launch); *admitted is how
 * many were taken (fewer when no slot or budget is free: poll, then submit
 * the rest).  An invalid request returns PIM_ERR_INVALID; the requests before
 * it are admitted and counted in *admitted.  Large submissions are validated
 * and staged by the server's host worker threads.  No device work. */
pim_status pim_server_submit(pim_server* server, int32_t count, const uint32_t* ids, const int32_t* ns,
                             const double* const* J, const double* const* h, int32_t* admitted);

/* Launches staged requests, one launch per chunk, on a server stream whose
 * previous launch has finished if there is one, else on the next stream in
 * turn (upload, sweep, re-rank and readback are asynchronous), and returns:
 * full chunks always; partly filled ones at once when no chunk of their class
 * is in flight (launched and not yet collected by a poll), else once their
 * first request has waited max_wait_us.  *launched: requests launched. */
pim_status pim_server_flush(pim_server* server, int32_t* launched);

/* Collects up to `max` finished requests without blocking: ids [max], states
 * (host int8 [max][PIM_MAX_N_LDS], first N entries used; may be NULL),
 * binary64 energies [max] (may be NULL); *done: how many. */
pim_status pim_server_poll(pim_server* server, int32_t max, uint32_t* ids, int8_t* states, double* energies,
                           int32_t* done);

/* pim_server_poll that also reports, per returned request, three times in
 * seconds of the host's monotonic clock (CLOCK_MONOTONIC on Linux):
 * times[3r] its admission by pim_server_submit, times[3r+1] the
 * pim_server_flush call that launched its chunk, times[3r+2] this poll,
 * which found the chunk's work finished (times: host [max][3], or NULL). */
pim_status pim_server_poll_times(pim_server* server, int32_t max, uint32_t* ids, int8_t* states,
                                 double* energies, double* times, int32_t* done);

/* A server for MIMO detection requests given as the detection problem
 * itself (Suppl. "Throughput requirement for LTE/5G systems": one instance
 * per data-bearing OFDM symbol): each request is (H, y, modulation, mapping,
 * Es/N0), and the Ising instance of pim_mimo_ising (J, h and x_m in binary64)
 * is built on the device at launch, so the host stages only H and y.  Same
 * configuration, slots, launches and results as pim_server_create; such a
 * server takes pim_server_submit_mimo only (pim_server_submit returns
 * PIM_ERR_STATE), and pim_server_poll_mimo also returns each request's x_m. */
pim_status pim_server_create_mimo(const pim_server_config* cfg, pim_server** out);

/* Admits up to `count` MIMO requests in order: ids[r] < 2^24 (also the noise
 * stream); dims[4r .. 4r+3] = (nr, nt, qam, map) with qam 4 or 16, map a
 * pim_mimo_map, 1 <= nt <= PIM_MAX_N_LDS / 4, N = 2 nt (ML, 4-QAM) or 4 nt
 * <= max_n, and 1 <= 2 nr <= N rounded up to 32; esn0[r] (linear Es/N0, > 0
 * for the DI mapping); H[r]: host complex [nr][nt] and y[r]: complex [nr],
 * interleaved (re, im) binary64, finite.  Copies H and y into pinned staging;
 * *admitted: how many were taken (fewer when no slot or budget is free).  An
 * invalid request returns PIM_ERR_INVALID with the ones before it admitted.
 * No device work.  A request whose MMSE system is not positive definite in
 * binary64 finishes with energy NaN. */
pim_status pim_server_submit_mimo(pim_server* server, int32_t count, const uint32_t* ids, const int32_t* dims,
                                  const double* esn0, const double* const* H, const double* const* y,
                                  int32_t* admitted);

/* pim_server_poll_times that also returns, for MIMO requests, x_m (host
 * [max][PIM_MAX_N_LDS / 2] binary64, first 2 nt entries used: real parts then
 * imaginary parts; may be NULL): the detected symbols are
 * pim_mimo_decode(x_m, state, nt, qam, map). */
pim_status pim_server_poll_mimo(pim_server* server, int32_t max, uint32_t* ids, int8_t* states, double* energies,
                                double* xm, double* times, int32_t* done);

/* Requests staged but not launched, and launched but not yet polled. */
pim_status pim_server_pending(pim_server* server, int32_t* staged, int32_t* in_flight);

/* Waits for launched work and frees everything. */
void pim_server_destroy(pim_server* server);

void pim_batch_destroy(pim_batch* batch);
void pim_destroy(pim_instance* inst);

/* Text of the last non-OK status on this thread ("" if none). */
const char* pim_last_error(void);

/* PIM_ABI_VERSION of the loaded library. */
int32_t pim_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PIM_H */
