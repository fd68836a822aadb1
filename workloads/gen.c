/*
 * Seeded synthetic input generators.
 *
 * This file holds no reduction arithmetic: it only turns (seed, element
 * index) into input values.  Both the CPU oracle and the GPU library consume
 * the bytes it writes; neither links it.
 *
 * Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) used in counter form, i.e. draw i of a
 * stream with seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15).  Any range of
 * draws can therefore be produced independently and in parallel.
 *
 *  - bounded integers: Lemire's multiply-shift map of the high 32 bits onto
 *    [lo, hi] (no rejection; bias below range / 2^32);
 *  - normals: Box-Muller in double precision on draw pairs (2q, 2q+1),
 *    then rounded to float (round to nearest even, the C default);
 *  - bf16: the float normal rounded to bfloat16 with round-to-nearest-even.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <string.h>

#define SM64_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * SM64_GAMMA;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline double unit_open_closed(uint64_t u) { /* (0, 1] */
  return ((double)(u >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}
static inline double unit_closed_open(uint64_t u) { /* [0, 1) */
  return (double)(u >> 11) * (1.0 / 9007199254740992.0);
}

/* Normal draw for element i of the stream (pairs share one Box-Muller step). */
static inline double normal_at(uint64_t seed, uint64_t i) {
  uint64_t q = i >> 1;
  double u1 = unit_open_closed(sm64_at(seed, 2 * q));
  double u2 = unit_closed_open(sm64_at(seed, 2 * q + 1));
  double r = sqrt(-2.0 * log(u1));
  double a = 6.283185307179586476925286766559 * u2;
  return (i & 1) ? r * sin(a) : r * cos(a);
}

static inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t b;
  memcpy(&b, &f, 4);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) /* NaN */
    return (uint16_t)((b >> 16) | 0x40);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

enum { K_U64 = 0, K_I32 = 1, K_F32N = 2, K_BF16N = 3, K_F64N = 4 };

typedef struct {
  int kind;
  uint64_t seed, start, n;
  int32_t lo, hi;
  void* out;
} job_t;

static void run_job(const job_t* j) {
  uint64_t k;
  switch (j->kind) {
    case K_U64: {
      uint64_t* o = (uint64_t*)j->out;
      for (k = 0; k < j->n; ++k) o[k] = sm64_at(j->seed, j->start + k);
    } break;
    case K_I32: {
      int32_t* o = (int32_t*)j->out;
      uint64_t range = (uint64_t)((int64_t)j->hi - (int64_t)j->lo + 1);
      for (k = 0; k < j->n; ++k) {
        uint64_t u = sm64_at(j->seed, j->start + k) >> 32;
        o[k] = (int32_t)((int64_t)j->lo + (int64_t)((u * range) >> 32));
      }
    } break;
    case K_F32N: {
      float* o = (float*)j->out;
      for (k = 0; k < j->n; ++k) o[k] = (float)normal_at(j->seed, j->start + k);
    } break;
    case K_BF16N: {
      uint16_t* o = (uint16_t*)j->out;
      for (k = 0; k < j->n; ++k)
        o[k] = f32_to_bf16_rne((float)normal_at(j->seed, j->start + k));
    } break;
    case K_F64N: {
      double* o = (double*)j->out;
      for (k = 0; k < j->n; ++k) o[k] = normal_at(j->seed, j->start + k);
    } break;
  }
}

static void* thread_main(void* p) {
  run_job((const job_t*)p);
  return NULL;
}

static size_t elem_size(int kind) {
  switch (kind) {
    case K_U64: case K_F64N: return 8;
    case K_I32: case K_F32N: return 4;
    default: return 2;
  }
}

/* Fill out[0..n) with draws start..start+n of the given kind, on `threads`
 * host threads.  Returns 0 on success. */
int gen_fill(int kind, uint64_t seed, uint64_t start, uint64_t n, int32_t lo, int32_t hi,
             void* out, int threads) {
  if (kind < K_U64 || kind > K_F64N || (kind == K_I32 && hi < lo)) return -1;
  if (threads < 1) threads = 1;
  if (threads > 64) threads = 64;
  if (n < (uint64_t)threads * 65536u) threads = 1;
  pthread_t th[64];
  job_t jobs[64];
  uint64_t per = (n + (uint64_t)threads - 1) / (uint64_t)threads;
  size_t es = elem_size(kind);
  int t, started = 0;
  for (t = 0; t < threads; ++t) {
    uint64_t b = per * (uint64_t)t;
    uint64_t e = b + per > n ? n : b + per;
    jobs[t].kind = kind;
    jobs[t].seed = seed;
    jobs[t].start = start + b;
    jobs[t].n = e > b ? e - b : 0;
    jobs[t].lo = lo;
    jobs[t].hi = hi;
    jobs[t].out = (char*)out + b * es;
  }
  for (t = 1; t < threads; ++t) {
    if (pthread_create(&th[t], NULL, thread_main, &jobs[t]) != 0) break;
    started = t;
  }
  run_job(&jobs[0]);
  for (t = started + 1; t < threads; ++t) run_job(&jobs[t]); /* threads that failed to start */
  for (t = 1; t <= started; ++t) pthread_join(th[t], NULL);
  return 0;
}
