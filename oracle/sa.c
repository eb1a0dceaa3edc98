/*
 * Simulated-annealing reference energies for dense integer Ising instances.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Loaded by oracle/sa.py,
 * which only tests/, the tests/golden/ writer scripts and the CPU-baseline
 * leg of the benchmark import.  Shares no code with the HIP library.
 *
 * Follows the paper's ground-truth recipe for SK-1 (Suppl. "SK-1 instance
 * generation", "Ground-truth computation"): single-spin-flip Metropolis
 * updates from a random configuration, temperature lowered geometrically
 * from T_init to T_final by a factor alpha after a fixed number of proposed
 * flips, several independent runs, the lowest energy met in any run kept.
 *
 * Energy (Eq. (1)): H(s) = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i, kept
 * exactly in int64.  Flipping spin k changes it by dE = 2 s_k I_k with
 * I_k = sum_j J_kj s_j + h_k (Eq. (2)); a proposal is accepted when dE <= 0,
 * else with probability exp(-c dE / T), c being the coupling normalisation
 * the instance is annealed under (the SK-1 preprocessing scales J by
 * 1/sqrt(N)).
 *
 * Random draws: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written
 * here from its published definition, key = (seed low, seed high), counter
 * (block low, block high, run, (domain << 24) | stream).  One block serves two
 * proposals: word 0 picks the site (multiply-shift into [0, N)), word 1 the
 * uniform (w + 0.5) / 2^32; words 2 and 3 the next proposal.  Domain 4 holds
 * the proposals, domain 5 the random initial configurations (spin i: bit
 * i % 32 of word (i / 32) % 4 of block i / 128, set = +1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SA_DOMAIN_MOVE 4u
#define SA_DOMAIN_INIT 5u

void sa_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Number of temperatures T_k = T_init * alpha^k (k = 0, 1, ...) with
 * T_k >= T_final, each formed by repeated multiplication as the anneal does. */
int64_t sa_count_temperatures(double t_init, double t_final, double alpha) {
  if (!(t_init > 0) || !(t_final > 0) || !(alpha > 0) || !(alpha < 1)) return -1;
  int64_t k = 0;
  for (double t = t_init; t >= t_final; t *= alpha) ++k;
  return k;
}

static void random_config(int n, uint64_t seed, uint32_t stream, uint32_t run, int8_t* s) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int b = 0; b * 128 < n; ++b) {
    uint32_t ctr[4] = {(uint32_t)b, 0u, run, (SA_DOMAIN_INIT << 24) | stream};
    uint32_t x[4];
    sa_philox4x32_10(ctr, key, x);
    for (int q = 0; q < 128 && b * 128 + q < n; ++q)
      s[b * 128 + q] = ((x[q / 32] >> (q % 32)) & 1u) ? 1 : -1;
  }
}

static int64_t energy_of(int n, const int32_t* J, const int32_t* h, const int8_t* s) {
  int64_t e = 0;
  for (int i = 0; i < n; ++i) {
    int64_t row = 0;
    for (int j = i + 1; j < n; ++j) row += (int64_t)J[(size_t)i * n + j] * s[j];
    e -= row * s[i];
    e -= (int64_t)h[i] * s[i];
  }
  return e;
}

/* Fields I = J s + h (int64: no overflow for any int32 instance). */
static void fields_of(int n, const int32_t* J, const int32_t* h, const int8_t* s, int64_t* I) {
  for (int i = 0; i < n; ++i) {
    int64_t a = h[i];
    for (int j = 0; j < n; ++j) a += (int64_t)J[(size_t)i * n + j] * s[j];
    I[i] = a;
  }
}

static int check_instance(int n, const int32_t* J) {
  if (n < 1 || n > 65536) return 1;
  for (int i = 0; i < n; ++i) {
    if (J[(size_t)i * n + i] != 0) return 2;
    for (int j = 0; j < i; ++j)
      if (J[(size_t)i * n + j] != J[(size_t)j * n + i]) return 3;
  }
  return 0;
}

/* One proposal stream: draws pairs (site, uniform) from consecutive Philox
 * blocks of domain 4 for run `run`. */
typedef struct {
  uint32_t key[2];
  uint32_t run, stream;
  uint64_t block;
  uint32_t x[4];
  int half;
} moves;

static void moves_init(moves* m, uint64_t seed, uint32_t stream, uint32_t run) {
  m->key[0] = (uint32_t)seed;
  m->key[1] = (uint32_t)(seed >> 32);
  m->run = run;
  m->stream = stream;
  m->block = 0;
  m->half = 2;
}

static inline void moves_next(moves* m, int n, int* site, double* u) {
  if (m->half == 2) {
    uint32_t ctr[4] = {(uint32_t)m->block, (uint32_t)(m->block >> 32), m->run,
                       (SA_DOMAIN_MOVE << 24) | m->stream};
    sa_philox4x32_10(ctr, m->key, m->x);
    m->block++;
    m->half = 0;
  }
  uint32_t ws = m->x[2 * m->half], wu = m->x[2 * m->half + 1];
  m->half++;
  *site = (int)(((uint64_t)ws * (uint64_t)n) >> 32);
  *u = ((double)wu + 0.5) * (1.0 / 4294967296.0);
}

/*
 * Anneals `runs` independent runs of the recipe above and returns, over every
 * configuration visited in every run, the lowest energy (best_e) and one
 * configuration that has it (best_state, the first met; may be NULL).
 * run_best[r] (may be NULL) is the lowest energy of run r.  hist (may be
 * NULL; N <= 20 only) counts, over every run, the configuration held after
 * each proposal, indexed by sum_i [s_i = +1] 2^i: with t_init = t_final it is
 * the visit histogram of fixed-temperature Metropolis.  J: int32 N x N
 * row-major, symmetric, zero diagonal; h: int32 [N] or NULL.  Returns 0, or a
 * positive code for invalid arguments.
 */
int sa_anneal(int n, const int32_t* J, const int32_t* h, double c, double t_init, double t_final,
              double alpha, int64_t flips_per_temp, int runs, uint64_t seed, uint32_t stream,
              int64_t* best_e, int8_t* best_state, int64_t* run_best, int64_t* hist) {
  int bad = check_instance(n, J);
  if (bad) return bad;
  if (!(c > 0) || flips_per_temp < 1 || runs < 1 || stream >= (1u << 24)) return 10;
  if (hist && n > 20) return 13;
  if (sa_count_temperatures(t_init, t_final, alpha) < 1) return 11;
  int32_t* hz = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  int8_t* s = (int8_t*)malloc((size_t)n);
  int32_t* I = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* Jt = (int32_t*)malloc((size_t)n * n * sizeof(int32_t));
  if (!hz || !s || !I || !Jt) {
    free(hz); free(s); free(I); free(Jt);
    return 12;
  }
  if (h) memcpy(hz, h, (size_t)n * sizeof(int32_t));
  memcpy(Jt, J, (size_t)n * n * sizeof(int32_t));
  /* largest possible uphill step, for the per-temperature acceptance table
   * (also bounds the fields: |I_i| <= dmax / 2, so int32 fields suffice) */
  int64_t dmax = 0;
  for (int i = 0; i < n; ++i) {
    int64_t a = llabs((int64_t)hz[i]);
    for (int j = 0; j < n; ++j) a += llabs((int64_t)Jt[(size_t)i * n + j]);
    if (2 * a > dmax) dmax = 2 * a;
  }
  double* acc = dmax < ((int64_t)1 << 30) ? (double*)malloc((size_t)(dmax + 1) * sizeof(double)) : NULL;
  if (!acc) {
    free(hz); free(s); free(I); free(Jt);
    return 12;
  }
  if (hist) memset(hist, 0, ((size_t)1 << n) * sizeof(int64_t));
  int64_t best = INT64_MAX;
  for (int r = 0; r < runs; ++r) {
    random_config(n, seed, stream, (uint32_t)r, s);
    uint32_t idx = 0;
    for (int i = 0; hist && i < n; ++i) idx |= (s[i] > 0 ? 1u : 0u) << i;
    {
      int64_t* I64 = (int64_t*)malloc((size_t)n * sizeof(int64_t));
      if (!I64) {
        free(acc); free(hz); free(s); free(I); free(Jt);
        return 12;
      }
      fields_of(n, Jt, hz, s, I64);
      for (int i = 0; i < n; ++i) I[i] = (int32_t)I64[i]; /* |I_i| <= dmax / 2 < 2^29 */
      free(I64);
    }
    int64_t e = energy_of(n, Jt, hz, s);
    int64_t rb = e;
    if (e < best) {
      best = e;
      if (best_state) memcpy(best_state, s, (size_t)n);
    }
    moves mv;
    moves_init(&mv, seed, stream, (uint32_t)r);
    for (double t = t_init; t >= t_final; t *= alpha) {
      for (int64_t d = 0; d <= dmax; ++d) acc[d] = exp(-c * (double)d / t);
      for (int64_t f = 0; f < flips_per_temp; ++f) {
        int k;
        double u;
        moves_next(&mv, n, &k, &u);
        int64_t dE = 2 * (int64_t)s[k] * I[k];
        if (dE > 0 && !(u < acc[dE])) {
          if (hist) hist[idx]++;
          continue;
        }
        /* accept: s_k -> -s_k, every field moves by J_ik (s_k,new - s_k,old) */
        int32_t delta = -2 * (int32_t)s[k];
        const int32_t* col = Jt + (size_t)k * n; /* row k = column k (symmetric) */
        for (int i = 0; i < n; ++i) I[i] += delta * col[i];
        s[k] = (int8_t)-s[k];
        e += dE;
        if (hist) {
          idx ^= 1u << k;
          hist[idx]++;
        }
        if (e < rb) rb = e;
        if (e < best) {
          best = e;
          if (best_state) memcpy(best_state, s, (size_t)n);
        }
      }
    }
    if (run_best) run_best[r] = rb;
  }
  *best_e = best;
  free(acc); free(hz); free(s); free(I); free(Jt);
  return 0;
}
