/*
 * Reference oracle for nested multi-level reductions -- TEST INFRASTRUCTURE.
 * See oracle.h for the definition it follows and the readings it takes.
 *
 * Plain sequential nested loops in the order of the definition: for every
 * output, level p collects the results of its e_p children in ascending t,
 * each child being the same reduction one level further in (paper, section 2:
 * one task per level gathers its siblings' results; section 3.7: partial
 * results are summed over siblings in sibling order).  No blocking, no
 * reordering, no vectorisation tricks.  Built with gcc -O2, no fast-math.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_DEPTH 8

typedef struct {
  int d, p, dtype;
  int64_t e[OR_MAX_DEPTH];
  int64_t stride[OR_MAX_DEPTH];
  int op[OR_MAX_DEPTH];
  int64_t block; /* elements reduced into one output */
  const void* in;
} nest_t;

static int setup(nest_t* n, int depth, const int64_t* extents, const int* ops, int dtype,
                 const void* in) {
  int m;
  if (depth < 1 || depth > OR_MAX_DEPTH) return -1;
  if (dtype != OR_I32 && dtype != OR_F32 && dtype != OR_BF16) return -1;
  n->d = depth;
  n->dtype = dtype;
  n->in = in;
  n->p = depth;
  for (m = 0; m < depth; ++m) {
    if (extents[m] < 1) return -1;
    if (ops[m] < OR_NONE || ops[m] > OR_ARGMAX) return -1;
    n->e[m] = extents[m];
    n->op[m] = ops[m];
    if (ops[m] != OR_NONE && n->p == depth) n->p = m;
    if (ops[m] == OR_NONE && n->p != depth) return -1; /* NONE must be a prefix */
    if (dtype != OR_I32 && ops[m] != OR_NONE && ops[m] != OR_SUM) return -1;
    if ((ops[m] == OR_ARGMIN || ops[m] == OR_ARGMAX) && extents[m] > 2147483647LL) return -1;
  }
  n->stride[depth - 1] = 1;
  for (m = depth - 2; m >= 0; --m) n->stride[m] = n->stride[m + 1] * n->e[m + 1];
  n->block = 1;
  for (m = n->p; m < depth; ++m) n->block *= n->e[m];
  return 0;
}

/* ---- floating point: double precision, Neumaier-compensated ------------ */

typedef struct {
  double s, c;
} nsum_t;

static inline void nsum_add(nsum_t* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static inline double elem_f(const nest_t* n, int64_t off) {
  if (n->dtype == OR_F32) return (double)((const float*)n->in)[off];
  {
    uint32_t u = (uint32_t)((const uint16_t*)n->in)[off] << 16; /* bf16 -> fp32 is exact */
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
  }
}

/* R_m of the block starting at element `off`; with `absval`, sum of |a|. */
static double eval_f(const nest_t* n, int m, int64_t off, int absval) {
  nsum_t acc = {0.0, 0.0};
  int64_t t, e = n->e[m], st = n->stride[m];
  if (m == n->d - 1) {
    for (t = 0; t < e; ++t) {
      double x = elem_f(n, off + t);
      nsum_add(&acc, absval ? fabs(x) : x);
    }
  } else {
    for (t = 0; t < e; ++t) nsum_add(&acc, eval_f(n, m + 1, off + t * st, absval));
  }
  return acc.s + acc.c;
}

/* ---- integers: exact ---------------------------------------------------- */

static int64_t eval_i(const nest_t* n, int m, int64_t off);

static inline int64_t child_i(const nest_t* n, int m, int64_t off, int64_t t) {
  if (m == n->d - 1) return (int64_t)((const int32_t*)n->in)[off + t];
  return eval_i(n, m + 1, off + t * n->stride[m]);
}

static int64_t eval_i(const nest_t* n, int m, int64_t off) {
  int64_t t, e = n->e[m];
  switch (n->op[m]) {
    case OR_SUM: {
      uint64_t s = 0; /* two's-complement wrap, well defined */
      for (t = 0; t < e; ++t) s += (uint64_t)child_i(n, m, off, t);
      return (int64_t)s;
    }
    case OR_MIN: {
      int64_t v = child_i(n, m, off, 0);
      for (t = 1; t < e; ++t) {
        int64_t x = child_i(n, m, off, t);
        if (x < v) v = x;
      }
      return v;
    }
    case OR_MAX: {
      int64_t v = child_i(n, m, off, 0);
      for (t = 1; t < e; ++t) {
        int64_t x = child_i(n, m, off, t);
        if (x > v) v = x;
      }
      return v;
    }
    case OR_ARGMIN: {
      int64_t v = child_i(n, m, off, 0), best = 0;
      for (t = 1; t < e; ++t) {
        int64_t x = child_i(n, m, off, t);
        if (x < v) { /* strict: the first occurrence is kept */
          v = x;
          best = t;
        }
      }
      return best;
    }
    case OR_ARGMAX: {
      int64_t v = child_i(n, m, off, 0), best = 0;
      for (t = 1; t < e; ++t) {
        int64_t x = child_i(n, m, off, t);
        if (x > v) {
          v = x;
          best = t;
        }
      }
      return best;
    }
  }
  return 0;
}

static int kind_of(const nest_t* n) {
  int m;
  if (n->dtype != OR_I32) return OR_OUT_F64;
  for (m = n->p; m < n->d; ++m) {
    if (n->op[m] == OR_SUM) return OR_OUT_I64;
    if (n->op[m] == OR_ARGMIN || n->op[m] == OR_ARGMAX) return OR_OUT_I32;
  }
  return OR_OUT_I32; /* MIN/MAX down to the elements, or no reducing level */
}

int oracle_out_kind(int depth, const int64_t* extents, const int* ops, int dtype) {
  nest_t n;
  if (setup(&n, depth, extents, ops, dtype, NULL) != 0) return -1;
  return kind_of(&n);
}

int64_t oracle_n_out(int depth, const int64_t* extents, const int* ops) {
  nest_t n;
  int64_t k = 1;
  int m;
  if (setup(&n, depth, extents, ops, OR_I32, NULL) != 0) return -1;
  for (m = 0; m < n.p; ++m) k *= n.e[m];
  return k;
}

typedef struct {
  const nest_t* n;
  void* out;
  int64_t b, e, base;
  int mode; /* 0: reduce, 1: abs sum */
} part_t;

static void run_part(const part_t* q) {
  const nest_t* n = q->n;
  int kind = kind_of(n);
  int64_t o;
  for (o = q->b; o < q->e; ++o) {
    int64_t off = o * n->block, k = o - q->base;
    if (q->mode == 1) {
      ((double*)q->out)[k] = n->p == n->d ? fabs(elem_f(n, off)) : eval_f(n, n->p, off, 1);
    } else if (kind == OR_OUT_F64) {
      ((double*)q->out)[k] = n->p == n->d ? elem_f(n, off) : eval_f(n, n->p, off, 0);
    } else {
      int64_t v = n->p == n->d ? (int64_t)((const int32_t*)n->in)[off] : eval_i(n, n->p, off);
      if (kind == OR_OUT_I64)
        ((int64_t*)q->out)[k] = v;
      else
        ((int32_t*)q->out)[k] = (int32_t)v;
    }
  }
}

static void* part_main(void* p) {
  run_part((const part_t*)p);
  return NULL;
}

static int run_range(const nest_t* n, void* out, int64_t ob, int64_t oe, int threads, int mode) {
  pthread_t th[256];
  part_t parts[256];
  int64_t cnt = oe - ob, per;
  int t, started = 0;
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if (cnt < threads) threads = cnt > 0 ? (int)cnt : 1;
  per = (cnt + threads - 1) / threads;
  for (t = 0; t < threads; ++t) {
    parts[t].n = n;
    parts[t].out = out;
    parts[t].base = ob;
    parts[t].b = ob + per * t;
    parts[t].e = ob + per * (t + 1) > oe ? oe : ob + per * (t + 1);
    if (parts[t].b > parts[t].e) parts[t].b = parts[t].e;
    parts[t].mode = mode;
  }
  for (t = 1; t < threads; ++t) {
    if (pthread_create(&th[t], NULL, part_main, &parts[t]) != 0) break;
    started = t;
  }
  run_part(&parts[0]);
  for (t = started + 1; t < threads; ++t) run_part(&parts[t]);
  for (t = 1; t <= started; ++t) pthread_join(th[t], NULL);
  return 0;
}

int oracle_reduce_range(int depth, const int64_t* extents, const int* ops, int dtype,
                        const void* in, void* out, int64_t o_begin, int64_t o_end, int threads) {
  nest_t n;
  int64_t nout = 1;
  int m;
  if (setup(&n, depth, extents, ops, dtype, in) != 0 || !in || !out) return -1;
  for (m = 0; m < n.p; ++m) nout *= n.e[m];
  if (o_begin < 0 || o_end > nout || o_begin > o_end) return -1;
  return run_range(&n, out, o_begin, o_end, threads, 0);
}

int oracle_reduce(int depth, const int64_t* extents, const int* ops, int dtype, const void* in,
                  void* out, int threads) {
  int64_t nout = oracle_n_out(depth, extents, ops);
  if (nout < 0) return -1;
  return oracle_reduce_range(depth, extents, ops, dtype, in, out, 0, nout, threads);
}

int oracle_abs_sum_range(int depth, const int64_t* extents, const int* ops, int dtype,
                         const void* in, double* out, int64_t o_begin, int64_t o_end, int threads) {
  nest_t n;
  int64_t nout = 1;
  int m;
  if (setup(&n, depth, extents, ops, dtype, in) != 0 || !in || !out) return -1;
  if (dtype == OR_I32) return -1;
  for (m = 0; m < n.p; ++m) nout *= n.e[m];
  if (o_begin < 0 || o_end > nout || o_begin > o_end) return -1;
  return run_range(&n, out, o_begin, o_end, threads, 1);
}

/* ---- ordered products ------------------------------------------------------ */

typedef struct {
  uint64_t v[4];
} elem_t; /* affine: v[0] = a, v[1] = b; mat2: row-major m00 m01 m10 m11 */

typedef struct {
  int d, p, dtype, width; /* width: uint64 words per element */
  int64_t e[OR_MAX_DEPTH];
  int64_t stride[OR_MAX_DEPTH];
  const uint64_t* in;
} pnest_t;

static elem_t p_identity(int dtype) {
  elem_t r;
  memset(&r, 0, sizeof r);
  r.v[0] = 1;
  if (dtype == OR_MAT2) r.v[3] = 1;
  return r;
}

/* x * y: x first, y second */
static elem_t p_mul(int dtype, elem_t x, elem_t y) {
  elem_t r;
  memset(&r, 0, sizeof r);
  if (dtype == OR_AFFINE) {
    r.v[0] = x.v[0] * y.v[0];
    r.v[1] = y.v[0] * x.v[1] + y.v[1];
  } else {
    r.v[0] = x.v[0] * y.v[0] + x.v[1] * y.v[2];
    r.v[1] = x.v[0] * y.v[1] + x.v[1] * y.v[3];
    r.v[2] = x.v[2] * y.v[0] + x.v[3] * y.v[2];
    r.v[3] = x.v[2] * y.v[1] + x.v[3] * y.v[3];
  }
  return r;
}

static elem_t p_load(const pnest_t* n, int64_t off) {
  elem_t r;
  int k;
  memset(&r, 0, sizeof r);
  for (k = 0; k < n->width; ++k) r.v[k] = n->in[off * n->width + k];
  return r;
}

/* R_m at element offset off: children t = 0..e_m-1 multiplied left to right */
static elem_t p_eval(const pnest_t* n, int m, int64_t off) {
  elem_t acc = p_identity(n->dtype);
  int64_t t;
  if (m == n->d) return p_load(n, off);
  for (t = 0; t < n->e[m]; ++t) acc = p_mul(n->dtype, acc, p_eval(n, m + 1, off + t * n->stride[m]));
  return acc;
}

typedef struct {
  const pnest_t* n;
  uint64_t* out;
  int64_t b, e, base, block;
} ppart_t;

static void* p_part(void* arg) {
  const ppart_t* q = (const ppart_t*)arg;
  int64_t o;
  int k;
  for (o = q->b; o < q->e; ++o) {
    elem_t r = p_eval(q->n, q->n->p, o * q->block);
    for (k = 0; k < q->n->width; ++k) q->out[(o - q->base) * q->n->width + k] = r.v[k];
  }
  return NULL;
}

int oracle_prod_range(int depth, const int64_t* extents, const int* ops, int dtype, const void* in,
                      void* out, int64_t o_begin, int64_t o_end, int threads) {
  pnest_t n;
  pthread_t th[256];
  ppart_t parts[256];
  int64_t nout = 1, block = 1, cnt, per;
  int m, t, started = 0;
  if (depth < 1 || depth > OR_MAX_DEPTH || !in || !out) return -1;
  if (dtype != OR_AFFINE && dtype != OR_MAT2) return -1;
  n.d = depth;
  n.dtype = dtype;
  n.width = dtype == OR_AFFINE ? 2 : 4;
  n.in = (const uint64_t*)in;
  n.p = depth;
  for (m = 0; m < depth; ++m) {
    if (extents[m] < 1) return -1;
    if (ops[m] != OR_NONE && ops[m] != OR_PROD) return -1;
    if (ops[m] == OR_PROD && n.p == depth) n.p = m;
    if (ops[m] == OR_NONE && n.p != depth) return -1;
    n.e[m] = extents[m];
  }
  n.stride[depth - 1] = 1;
  for (m = depth - 2; m >= 0; --m) n.stride[m] = n.stride[m + 1] * n.e[m + 1];
  for (m = 0; m < n.p; ++m) nout *= n.e[m];
  for (m = n.p; m < depth; ++m) block *= n.e[m];
  if (o_begin < 0 || o_end > nout || o_begin > o_end) return -1;
  cnt = o_end - o_begin;
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if (cnt < threads) threads = cnt > 0 ? (int)cnt : 1;
  per = (cnt + threads - 1) / threads;
  for (t = 0; t < threads; ++t) {
    parts[t].n = &n;
    parts[t].out = (uint64_t*)out;
    parts[t].base = o_begin;
    parts[t].block = block;
    parts[t].b = o_begin + per * t;
    parts[t].e = o_begin + per * (t + 1) > o_end ? o_end : o_begin + per * (t + 1);
    if (parts[t].b > parts[t].e) parts[t].b = parts[t].e;
  }
  for (t = 1; t < threads; ++t) {
    if (pthread_create(&th[t], NULL, p_part, &parts[t]) != 0) break;
    started = t;
  }
  p_part(&parts[0]);
  for (t = started + 1; t < threads; ++t) p_part(&parts[t]);
  for (t = 1; t <= started; ++t) pthread_join(th[t], NULL);
  return 0;
}

/* ---- stencils -------------------------------------------------------------- */

int oracle_stencil(int64_t rows, int64_t cols, int steps, double c0, double c1, const float* in, double* out) {
  int64_t i, j, n;
  int s;
  double *a, *b;
  if (rows < 1 || cols < 1 || steps < 0 || !in || !out) return -1;
  n = rows * cols;
  a = (double*)malloc((size_t)n * sizeof(double));
  b = (double*)malloc((size_t)n * sizeof(double));
  if (!a || !b) {
    free(a);
    free(b);
    return -1;
  }
  for (i = 0; i < n; ++i) a[i] = (double)in[i];
  for (s = 0; s < steps; ++s) {
    for (i = 0; i < rows; ++i)
      for (j = 0; j < cols; ++j) {
        const int64_t k = i * cols + j;
        if (i == 0 || i == rows - 1 || j == 0 || j == cols - 1)
          b[k] = a[k];
        else
          b[k] = c0 * a[k] + c1 * ((a[k - cols] + a[k + cols]) + (a[k - 1] + a[k + 1]));
      }
    {
      double* t = a;
      a = b;
      b = t;
    }
  }
  memcpy(out, a, (size_t)n * sizeof(double));
  free(a);
  free(b);
  return 0;
}
