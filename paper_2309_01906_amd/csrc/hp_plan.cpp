// Level-mapping planner (host only; no HIP calls, so it also runs without a GPU).
//
// Follows the paper's section 3: explicit level selection with collapse (3.1),
// selection by property for the automatic map (3.2: reductions need a shuffle at
// the wavefront, a barrier and local memory at the workgroup; the grid has no
// barrier, so its partials are folded by a second kernel after the launch), the
// reserve rule that makes maps monotone (3.3),
// strip-mining every level once all units are started (3.4, SPMD mode), static /
// masked schedules (3.5) and splitting a hardware level between nested loops (3.8).
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "hp_internal.h"

namespace hp {

static thread_local char g_err[512];

hp_status fail(hp_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

void clear_error() { g_err[0] = 0; }

static inline bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
static inline uint64_t pow2ceil(uint64_t x) {
  uint64_t r = 1;
  while (r < x) r <<= 1;
  return r;
}
static inline int log2u(uint64_t x) {
  int r = 0;
  while ((1ull << r) < x) ++r;
  return r;
}
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int lowbit(uint32_t s) { return __builtin_ctz(s); }
static inline int highbit(uint32_t s) { return 31 - __builtin_clz(s); }
// Every level is strip-mined once its units are exhausted, so an L bit next to
// other scopes only states that strips are expected; for the nesting order it is
// the other scopes that count.  A level on L alone is serial in one lane.
static inline int nest_high(uint32_t s) { return s == HP_SCOPE_L ? highbit(s) : highbit(s & ~(uint32_t)HP_SCOPE_L); }

static int elem_bytes(int dt) { return dt == HP_BF16 ? 2 : 4; }

// Magic numbers of FastDiv for a divisor 1 <= d < 2^31.
static FastDiv fastdiv(uint64_t d) {
  const int l = log2u(d);  // ceil(log2 d)
  const uint32_t s = 31u + (uint32_t)l;
  const uint64_t m = ((uint64_t)1 << s) / d + (((uint64_t)1 << s) % d != 0);
  return FastDiv{(uint32_t)m, s};
}

// gfx950's hardware levels (vendor figures; 256 compute units in 8 XCDs).
static const hp_level_props kLevels[] = {
    {HP_SCOPE_G, 0, HP_LP_ATOMIC | HP_LP_DYNAMIC, 0},
    {HP_SCOPE_X, 8, HP_LP_SHARED_CACHE, 4ll << 20},
    {HP_SCOPE_W, kMaxWaves, HP_LP_BARRIER | HP_LP_LOCALMEM | HP_LP_ATOMIC | HP_LP_DYNAMIC, 64ll << 10},
    {HP_SCOPE_V, kWave, HP_LP_SHUFFLE | HP_LP_LOCKSTEP, 0},
    {HP_SCOPE_L, 0, 0, 0},
};
static constexpr int kLevelRows = (int)(sizeof kLevels / sizeof kLevels[0]);
static constexpr int64_t kFillWorkgroups = 256 * 8;  // compute units x 8

static const hp_level_props& level_of(uint32_t scope) {
  for (const hp_level_props& l : kLevels)
    if (l.scope == scope) return l;
  return kLevels[kLevelRows - 1];
}
// the innermost level that offers `need` (all bits) among the wavefront, workgroup
// and grid: where a reduction's units can be combined
static uint32_t combine_scope(uint32_t need) {
  for (int i = kLevelRows - 1; i >= 0; --i)
    if ((kLevels[i].props & need) == need && kLevels[i].scope != HP_SCOPE_L) return kLevels[i].scope;
  return HP_SCOPE_G;
}

// Automatic map: NONE levels on the grid; reducing levels fill the lanes of a
// wavefront from the innermost level outward (shuffles are the cheapest combine),
// then the waves of a workgroup (LDS + barrier), then, when the outputs alone do
// not give the chip enough workgroups, the outermost reducing level is also split
// over the grid (partials folded by a second kernel).
static void auto_map(const hp_nest* n, int p, int chunk_last, hp_level_map* m, int force_nw) {
  const int d = n->depth;
  memset(m, 0, sizeof *m);
  for (int l = 0; l < p; ++l) m->scopes[l] = HP_SCOPE_G;
  if (p == d) {
    if (force_nw > 1) {  // a copy in a batch: the innermost level also takes the waves
      m->scopes[d - 1] = HP_SCOPE_G | HP_SCOPE_W;
      m->units[d - 1][HP_AXIS_W] = (uint32_t)force_nw;
    }
    return;
  }
  int64_t block = 1;
  for (int k = p; k < d; ++k) block *= n->extent[k];
  const int64_t bytes = block * elem_bytes(n->dtype);
  // Small blocks and many outputs: one output needs fewer lanes than a wave has, so
  // the innermost output level also takes the rest of the lanes and the waves, and
  // strips of it give every workgroup a useful amount of input.
  if (p >= 1 && bytes < (16 << 10) && n->extent[p - 1] > 1) {
    uint64_t pw = 1;
    for (int k = d - 1; k >= p; --k) pw *= pow2ceil((uint64_t)cdiv(n->extent[k], k == d - 1 ? chunk_last : 1));
    if (pw < (uint64_t)kWave) {
      int lanes = (int)pw;
      for (int k = d - 1; k >= p; --k) {
        uint64_t f = pow2ceil((uint64_t)cdiv(n->extent[k], k == d - 1 ? chunk_last : 1));
        if (f > (uint64_t)lanes || k == p) f = (uint64_t)lanes;
        m->scopes[k] = HP_SCOPE_V;
        m->units[k][HP_AXIS_V] = (uint32_t)f;
        lanes /= (int)f;
      }
      const int64_t eo = n->extent[p - 1];
      const int64_t parts = kWave / (int64_t)pw;
      int64_t nw = force_nw > 0 ? force_nw : (int64_t)pow2ceil((uint64_t)cdiv(eo, parts));
      if (nw > 4) nw = 4;
      const int64_t per_pass = parts * nw;
      // outputs per workgroup: about 32 KiB of input, but at least 1024 workgroups
      // for a single nest (a batch fills the chip with other nests' tasks)
      int64_t opt = ((32 << 10) / (bytes > 0 ? bytes : 1)) / per_pass * per_pass;
      if (force_nw == 0) {
        int64_t n_out = 1;
        for (int k = 0; k < p; ++k) n_out *= n->extent[k];
        const int64_t spread = cdiv(cdiv(n_out, 1024), per_pass) * per_pass;
        if (opt > spread) opt = spread;
      }
      if (opt < per_pass) opt = per_pass;
      m->scopes[p - 1] = HP_SCOPE_G | HP_SCOPE_W | (parts > 1 ? HP_SCOPE_V : 0u);
      m->units[p - 1][HP_AXIS_G] = (uint32_t)cdiv(eo, opt);
      m->units[p - 1][HP_AXIS_W] = (uint32_t)nw;
      if (parts > 1) m->units[p - 1][HP_AXIS_V] = (uint32_t)parts;
      return;
    }
  }
  // lanes of one wavefront, innermost reducing level first: the level whose units
  // shuffle registers (the cheapest combine, section 2)
  const uint32_t v_scope = combine_scope(HP_LP_SHUFFLE);
  int lanes_left = level_of(v_scope).units;
  int l = d - 1;
  int first_v = d;
  while (l >= p && lanes_left > 1) {
    const int64_t need = cdiv(n->extent[l], l == d - 1 ? chunk_last : 1);
    uint64_t f = pow2ceil((uint64_t)need);
    // An innermost level that is a segment of its own under another reducing level
    // is combined across its lanes after every iteration of the level above: give
    // each lane at least 4 of its chunks, so that combine runs 4 times less often.
    if (l == d - 1 && l > p) {
      const int a = n->op[l - 1], b = n->op[l];
      const bool arg = a == HP_OP_ARGMIN || a == HP_OP_ARGMAX || b == HP_OP_ARGMIN || b == HP_OP_ARGMAX;
      if ((arg || a != b) && f >= 4) f /= 4;
    }
    if (f >= (uint64_t)lanes_left || l == p) f = (uint64_t)lanes_left;
    m->scopes[l] = v_scope;
    m->units[l][HP_AXIS_V] = (uint32_t)f;
    lanes_left /= (int)f;
    first_v = l;
    --l;
  }
  if (lanes_left > 1) m->units[first_v][HP_AXIS_V] *= (uint32_t)lanes_left;
  // Waves per workgroup for the reduced block of one output.  A second wave pays
  // only when one wave's share stays large: splitting a block over waves adds an LDS
  // combine and a barrier per output, and with many outputs one-wave workgroups fill
  // the chip anyway.  Measured over 2- and 3-level nests of 4 KiB to 256 KiB blocks
  // (1,024 to 65,536 outputs): float blocks below 64 KiB and single-operator integer
  // blocks below 128 KiB were fastest on one wave (up to 2x faster than 2-4 waves).
  bool one_op = true;
  for (int k = p + 1; k < d; ++k)
    if (n->op[k] != n->op[p]) one_op = false;
  const bool flt = n->dtype != HP_I32;
  uint64_t nw_target;
  if (flt) nw_target = bytes >= (256 << 10) ? 8 : bytes >= (64 << 10) ? 4 : 1;
  else if (one_op) nw_target = bytes >= (128 << 10) ? 2 : 1;
  else nw_target = bytes >= (256 << 10) ? 8 : bytes >= (16 << 10) ? 4 : bytes >= (4 << 10) ? 2 : 1;
  // waves of one workgroup: the next level outward, or the outermost lane level
  // the next level out whose units combine through a barrier and shared memory
  const uint32_t w_scope = combine_scope(HP_LP_BARRIER | HP_LP_LOCALMEM);
  int w_level;
  int64_t per_wave_unit;
  if (l >= p) {
    w_level = l;
    m->scopes[l] = w_scope;
    per_wave_unit = n->extent[l];
    --l;
  } else {
    w_level = first_v;
    m->scopes[first_v] |= w_scope;
    per_wave_unit = cdiv(cdiv(n->extent[first_v], first_v == d - 1 ? chunk_last : 1),
                         m->units[first_v][HP_AXIS_V]);
  }
  {
    uint64_t f = pow2ceil((uint64_t)per_wave_unit);
    if (f > nw_target) f = nw_target;
    if (f > (uint64_t)level_of(w_scope).units) f = (uint64_t)level_of(w_scope).units;
    if (force_nw > 0) f = (uint64_t)force_nw;
    m->units[w_level][HP_AXIS_W] = (uint32_t)f;
  }
  // anything further out runs on the grid, one workgroup per iteration
  for (int k = p; k <= l; ++k) m->scopes[k] = HP_SCOPE_G;
  // too few outputs for the chip: split the outermost reducing level over the grid.
  // Measured: with 1,024 outputs of 256 KiB or 1 MiB a one-pass plan beat splitting
  // each output in two (int32 46.2 vs 52.1 us, fp32 156.8 vs 163.7 us), so only
  // fewer outputs than half the fill target are split.  Float splits run on twice
  // the fill target of workgroups with at most 4 waves (1 to 512 outputs over 1 GiB:
  // 162-169 us against 166-190 us on the fill target with 8 waves); integer splits
  // on the fill target (8 or 64 outputs over 256 MiB: 50 us against 54-55 us on
  // twice as many).
  int64_t n_out = 1;
  for (int k = 0; k < p; ++k) n_out *= n->extent[k];
  bool split = false;
  if (l < p) {
    if (n_out < kFillWorkgroups / 2) {
      if (flt && force_nw == 0 && m->units[w_level][HP_AXIS_W] > 4) m->units[w_level][HP_AXIS_W] = 4;
      const int64_t per = p == d - 1 ? cdiv(n->extent[p], chunk_last) : n->extent[p];
      const int64_t in_wg = (int64_t)(m->units[p][HP_AXIS_V] ? m->units[p][HP_AXIS_V] : 1) *
                            (int64_t)(m->units[p][HP_AXIS_W] ? m->units[p][HP_AXIS_W] : 1);
      int64_t gf = cdiv(flt ? 2 * kFillWorkgroups : kFillWorkgroups, n_out);
      const int64_t useful = cdiv(per, in_wg);
      const int64_t by_bytes = bytes / (64 << 10);  // keep >= 64 KiB of input per workgroup
      if (gf > useful) gf = useful;
      if (gf > by_bytes) gf = by_bytes;
      if (gf > 1) {
        m->scopes[p] |= HP_SCOPE_G;
        m->units[p][HP_AXIS_G] = (uint32_t)gf;
        split = true;
      }
    }
  }
  // Up to half the fill target of unsplit float outputs with blocks of 256 KiB to
  // 384 KiB: 2 waves per workgroup.  Measured on 1,024 outputs of 256 KiB: fp32 44.8
  // us on 2 waves against 53.8 on 8, bf16 44.4 against 56.7; with blocks of 384 KiB
  // and more, or 4,096 outputs, 8 waves were as fast or faster.
  if (flt && force_nw == 0 && !split && n_out <= kFillWorkgroups / 2 && bytes >= (256 << 10) &&
      bytes < (384 << 10) && m->units[w_level][HP_AXIS_W] > 2)
    m->units[w_level][HP_AXIS_W] = 2;
}

// Ordered products (HP_OP_PROD over AFFINE64 / MAT2X2_64 elements).  The reduced
// block of an output is contiguous; it is cut into gsplit chunks of ord_span
// elements, one wavefront each.  Lane l of the wave takes the l-th 64th of the
// chunk, K elements (one 128-byte line) at a time, into a running product; an
// order-keeping butterfly multiplies the 64 lane products once per chunk.  Chunks
// are folded in order by a second kernel.
static constexpr int kOrdWaves = 4;  // waves per workgroup (independent workers)

static hp_status lower_ordered(const hp_nest* n, const hp_level_map* map_in, uint32_t flags, Lowered* out,
                               int force_nw) {
  const int d = n->depth;
  if (map_in) return fail(HP_EUNSUPPORTED, "ordered products take the planner's map only");
  if (force_nw) return fail(HP_EUNSUPPORTED, "ordered products are not batched");
  if (flags & ~(uint32_t)HP_FLAG_NO_XCD) return fail(HP_EINVAL, "flag bits 0x%x do not apply to ordered products", flags);
  int p = d;
  int64_t total = 1;
  for (int l = 0; l < d; ++l) {
    const int64_t e = n->extent[l];
    const int op = n->op[l];
    if (e < 1) return fail(HP_EINVAL, "extent[%d] = %lld < 1", l, (long long)e);
    if (op != HP_OP_NONE && op != HP_OP_PROD)
      return fail(HP_EUNSUPPORTED, "ordered-product elements take PROD levels only (level %d)", l);
    if (op == HP_OP_NONE && p != d) return fail(HP_EINVAL, "NONE at level %d after a reducing level", l);
    if (op != HP_OP_NONE && p == d) p = l;
    if (total > (int64_t(1) << 58) / e) return fail(HP_EUNSUPPORTED, "nest has more than 2^58 elements");
    total *= e;
  }
  const int es = n->dtype == HP_AFFINE64 ? 16 : 32;
  const int K = 128 / es;  // elements per lane run: one 128-byte line (8 affine maps, 4 matrices)
  DevPlan dp;
  memset(&dp, 0, sizeof dp);
  dp.depth = d;
  dp.p = p;
  dp.dtype = n->dtype;
  dp.flags = (int32_t)flags;
  dp.chunk = K;
  dp.nw = kOrdWaves;
  dp.kernel = HP_KERNEL_ORDERED;
  dp.in_elems = total;
  int64_t n_out = 1, block = 1;
  for (int l = 0; l < p; ++l) n_out *= n->extent[l];
  for (int l = p; l < d; ++l) block *= n->extent[l];
  dp.n_out = n_out;
  dp.ord_block = block;
  // chunks: enough wave units to fill the chip several times over, each at least
  // 4 tiles
  const int64_t tile = (int64_t)kWave * K;
  int64_t C = 1;
  if (p < d) {
    C = cdiv(16384, n_out);
    const int64_t by_len = cdiv(block, 4 * tile);
    if (C > by_len) C = by_len;
    if (C > 4096) C = 4096;
    if (C < 1) C = 1;
  }
  int64_t span = cdiv(cdiv(block, C), tile) * tile;
  if (span < 1) span = 1;
  C = cdiv(block, span);
  dp.ord_span = span;
  dp.gsplit = C;
  dp.gmode = C > 1 ? GCOMB_UNIFORM : GCOMB_NONE;
  const int64_t units = n_out * C;
  int64_t grid = cdiv(units, kOrdWaves);
  if (grid > 2048) grid = 2048;  // wave workers walk the units grid-stride
  dp.grid = grid;
  dp.out_kind = n->dtype;
  hp_plan_info& I = out->info;
  memset(&I, 0, sizeof I);
  I.depth = d;
  I.out_dtype = n->dtype;
  I.n_out = n_out;
  I.out_bytes = (size_t)n_out * es;
  I.in_elems = total;
  I.in_bytes = (size_t)total * es;
  I.grid = grid;
  I.waves = kOrdWaves;
  I.chunk = K;
  I.gsplit = C;
  I.workspace_bytes = C > 1 ? (size_t)n_out * C * es : 0;
  I.lds_bytes = (size_t)kOrdWaves * 64 * (K * es + 16);  // one staged tile per wave
  for (int l = 0; l < d; ++l) {
    I.scopes[l] = l < p ? HP_SCOPE_G : (l == p ? (HP_SCOPE_G | HP_SCOPE_W | HP_SCOPE_V | HP_SCOPE_L) : HP_SCOPE_L);
    I.units[l][HP_AXIS_G] = l < p ? (uint32_t)n->extent[l] : (l == p ? (uint32_t)C : 1u);
    I.units[l][HP_AXIS_W] = l == p ? (uint32_t)kOrdWaves : 1u;
    I.units[l][HP_AXIS_V] = l == p ? (uint32_t)kWave : 1u;
    I.strips[l] = l == p ? cdiv(span, tile) : 1;
  }
  I.nseg = p < d ? 1 : 0;
  I.kernel = HP_KERNEL_ORDERED;
  out->dp = dp;
  return HP_OK;
}

bool flat_candidate(const hp_nest* n, int* p_out, int64_t* block, int* vec) {
  if (n->dtype != HP_I32 && n->dtype != HP_F32 && n->dtype != HP_BF16) return false;
  const int d = n->depth;
  int p = d;
  for (int l = 0; l < d; ++l)
    if (n->op[l] != HP_OP_NONE) {
      p = l;
      break;
    }
  if (p == d) return false;
  const int op = n->op[p];
  if (op != HP_OP_SUM && op != HP_OP_MIN && op != HP_OP_MAX) return false;
  int64_t b = 1;
  for (int l = p; l < d; ++l) {
    if (n->op[l] != op || n->extent[l] < 1) return false;
    b *= n->extent[l];
  }
  const int c = 16 / elem_bytes(n->dtype);
  if (b < 2 * c - 1) return false;  // too short for an aligned vector inside every block
  *p_out = p;
  *block = b;
  *vec = c;
  return true;
}

// The aligned interior of a flat block of b elements whose start may sit anywhere
// inside a vector of c elements (any start when b % c != 0, else vector-aligned):
// the largest multiple of `unit` (itself a multiple of c) that fits after the up to
// c - 1 elements that precede the first aligned vector.
int64_t flat_interior(int64_t b, int c, int64_t unit) {
  const int64_t hmax = (b % c) ? c - 1 : 0;
  return (b - hmax) / unit * unit;
}

}  // namespace hp

extern "C" hp_status hp_level_table(hp_level_props* out, int32_t cap, int32_t* n, int64_t* fill_workgroups) {
  if (!out || !n || !fill_workgroups || cap < 1) return hp::fail(HP_EINVAL, "null pointer or cap < 1");
  const int k = cap < hp::kLevelRows ? cap : hp::kLevelRows;
  for (int i = 0; i < k; ++i) out[i] = hp::kLevels[i];
  *n = hp::kLevelRows;
  *fill_workgroups = hp::kFillWorkgroups;
  return HP_OK;
}

namespace hp {

hp_status lower(const hp_nest* n, const hp_level_map* map_in, uint32_t flags, Lowered* out, int force_nw,
                int64_t flat_block) {
  if (!n || !out) return fail(HP_EINVAL, "null argument");
  const int d = n->depth;
  if (d < 1 || d > kMaxDepth) return fail(HP_EINVAL, "depth %d outside [1, %d]", d, kMaxDepth);
  if (n->dtype == HP_AFFINE64 || n->dtype == HP_MAT2X2_64) return lower_ordered(n, map_in, flags, out, force_nw);
  if (flags & ~(uint32_t)(HP_FLAG_OUT_F32 | HP_FLAG_SCALAR | HP_FLAG_NO_XCD | HP_FLAG_GENERIC))
    return fail(HP_EINVAL, "unknown flag bits 0x%x", flags);
  if (n->dtype != HP_I32 && n->dtype != HP_F32 && n->dtype != HP_BF16)
    return fail(HP_EINVAL, "input dtype %d is not I32, F32 or BF16", n->dtype);
  const bool is_float = n->dtype != HP_I32;
  int p = d;
  int64_t total = 1;
  for (int l = 0; l < d; ++l) {
    const int64_t e = n->extent[l];
    const int op = n->op[l];
    if (e < 1) return fail(HP_EINVAL, "extent[%d] = %lld < 1", l, (long long)e);
    if (op == HP_OP_PROD) return fail(HP_EUNSUPPORTED, "PROD needs AFFINE64 or MAT2X2_64 elements (level %d)", l);
    if (op < HP_OP_NONE || op > HP_OP_ARGMAX) return fail(HP_EINVAL, "op[%d] = %d unknown", l, op);
    if (op == HP_OP_NONE && p != d) return fail(HP_EINVAL, "NONE at level %d after a reducing level", l);
    if (op != HP_OP_NONE && p == d) p = l;
    if (is_float && op != HP_OP_NONE && op != HP_OP_SUM)
      return fail(HP_EUNSUPPORTED, "float inputs support SUM only (level %d)", l);
    if ((op == HP_OP_ARGMIN || op == HP_OP_ARGMAX) && e > 2147483647LL)
      return fail(HP_EUNSUPPORTED, "ARG level %d longer than 2^31-1", l);
    if (total > (int64_t(1) << 62) / e) return fail(HP_EUNSUPPORTED, "nest has more than 2^62 elements");
    total *= e;
  }
  // innermost chunk: as many elements as one 16-byte load holds, if the extent allows
  int chunk_last = 1;
  if (p < d && !(flags & HP_FLAG_SCALAR)) {
    // the kernels are built for a full 16-byte chunk or single elements
    const int c = 16 / elem_bytes(n->dtype);
    chunk_last = (n->extent[d - 1] % c == 0) ? c : 1;
  }
  // A single reduction whose rows are not vector multiples, planned automatically:
  // view each output's block as one contiguous run and map its aligned interior,
  // so that the stream keeps 16-byte loads (section 3.5's schedule(none) masking
  // shrinks to the few elements before and after the interior).
  if (!map_in && !flat_block && chunk_last == 1 && !(flags & HP_FLAG_SCALAR)) {
    int fp, c;
    int64_t b;
    if (flat_candidate(n, &fp, &b, &c) && flat_interior(b, c, c) >= c) {
      hp_nest v;
      memset(&v, 0, sizeof v);
      v.dtype = n->dtype;
      v.depth = fp + 1;
      for (int l = 0; l < fp; ++l) {
        v.extent[l] = n->extent[l];
        v.op[l] = HP_OP_NONE;
      }
      v.extent[fp] = flat_interior(b, c, c);
      v.op[fp] = n->op[fp];
      hp_status s = lower(&v, nullptr, flags, out, force_nw, b);
      if (s != HP_OK) return s;
      // An interior that ends inside a strip would send every strip down the masked
      // path; shrink it to whole strips and leave the rest (under one strip) to the
      // threads' scalar pass.
      const DevLevel& L = out->dp.lv[fp];
      if (L.ragged && v.extent[fp] >= L.span && L.span % c == 0) {
        Lowered whole;
        v.extent[fp] = v.extent[fp] / L.span * L.span;
        if (lower(&v, nullptr, flags, &whole, force_nw, b) == HP_OK) *out = whole;
      }
      return HP_OK;
    }
  }
  int64_t flat_e = 0;
  if (flat_block) {
    // the nest is the interior view of blocks of flat_block elements
    const int c = 16 / elem_bytes(n->dtype);
    flat_e = 1;
    for (int l = p; l < d; ++l) flat_e *= n->extent[l];
    const int op = p < d ? n->op[p] : HP_OP_NONE;
    bool one = p < d && (op == HP_OP_SUM || op == HP_OP_MIN || op == HP_OP_MAX);
    for (int l = p; l < d && one; ++l) one = n->op[l] == op;
    if (!one || chunk_last != c || flat_e < c || flat_e > flat_interior(flat_block, c, c))
      return fail(HP_EINVAL, "flat view: %lld interior elements do not fit blocks of %lld", (long long)flat_e,
                  (long long)flat_block);
    total = total / flat_e * flat_block;
  }

  hp_level_map m;
  if (map_in) {
    m = *map_in;
  } else {
    auto_map(n, p, chunk_last, &m, force_nw);
  }
  // ---- the XCD scope: 8 grid units on the outermost grid digit, which the
  // XCD-aware workgroup numbering makes the XCD index
  int xlevel = -1;
  for (int l = 0; l < d; ++l) {
    if (!(m.scopes[l] & HP_SCOPE_X)) continue;
    if (xlevel >= 0) return fail(HP_EINVAL, "levels %d and %d both use the XCD scope X", xlevel, l);
    if (m.scopes[l] & HP_SCOPE_G) return fail(HP_EINVAL, "level %d uses both X and G", l);
    for (int k = 0; k < l; ++k)
      if (m.scopes[k] & (HP_SCOPE_G | HP_SCOPE_X))
        return fail(HP_EINVAL, "X at level %d: level %d outside it already uses the grid", l, k);
    if (m.units[l][HP_AXIS_G] && m.units[l][HP_AXIS_G] != 8)
      return fail(HP_EINVAL, "X at level %d has 8 units, not %u", l, m.units[l][HP_AXIS_G]);
    if (flags & HP_FLAG_NO_XCD) return fail(HP_EINVAL, "X at level %d with HP_FLAG_NO_XCD", l);
    m.scopes[l] = (m.scopes[l] & ~(uint32_t)HP_SCOPE_X) | HP_SCOPE_G;
    m.units[l][HP_AXIS_G] = 8;
    xlevel = l;
  }
  // ---- validate the map
  for (int l = 0; l < d; ++l) {
    const uint32_t s = m.scopes[l];
    if (s == 0 || (s & ~0xFu)) return fail(HP_EINVAL, "scopes[%d] = 0x%x is not a non-empty scope set", l, s);
    const uint32_t run = s >> lowbit(s);
    if (run & (run + 1)) return fail(HP_EINVAL, "scopes[%d] = 0x%x is not a run of adjacent scopes", l, s);
    for (int a = 0; a < 3; ++a) {
      if (m.units[l][a] && !(s & (1u << a)))
        return fail(HP_EINVAL, "units[%d][%d] set for a scope the level does not use", l, a);
    }
    if (m.units[l][HP_AXIS_W] && (!is_pow2(m.units[l][HP_AXIS_W]) || m.units[l][HP_AXIS_W] > kMaxWaves))
      return fail(HP_EINVAL, "W units of level %d must be a power of two <= %d", l, kMaxWaves);
    if (m.units[l][HP_AXIS_V] && (!is_pow2(m.units[l][HP_AXIS_V]) || m.units[l][HP_AXIS_V] > kWave))
      return fail(HP_EINVAL, "V units of level %d must be a power of two <= %d", l, kWave);
  }
  for (int l = 0; l < d; ++l)
    for (int k = 0; k < l; ++k)
      if (lowbit(m.scopes[l]) < nest_high(m.scopes[k]))
        return fail(HP_EINVAL, "map not monotone: level %d uses a scope outer to level %d's", l, k);

  DevPlan dp;
  memset(&dp, 0, sizeof dp);
  dp.depth = d;
  dp.p = p;
  dp.dtype = n->dtype;
  dp.flags = (int32_t)flags;
  dp.in_elems = total;
  for (int l = 0; l < d; ++l) {
    DevLevel& L = dp.lv[l];
    L.e = n->extent[l];
    L.op = n->op[l];
    L.chunk = (l == d - 1) ? chunk_last : 1;
    L.gf = 1;
    L.wf = 1;
    L.vf = 1;
    L.seg = -1;
  }
  dp.lv[d - 1].stride = 1;
  for (int l = d - 2; l >= 0; --l)
    dp.lv[l].stride = (flat_block && l == p - 1) ? flat_block : dp.lv[l + 1].stride * dp.lv[l + 1].e;
  dp.chunk = chunk_last;
  dp.flat_b = flat_block;
  dp.flat_e = flat_e;

  // ---- V axis: 64 lanes split between the levels that use it (outer = high bits)
  {
    uint64_t fixed = 1;
    int n_auto = 0, outer_auto = -1;
    for (int l = 0; l < d; ++l)
      if (m.scopes[l] & HP_SCOPE_V) {
        if (m.units[l][HP_AXIS_V]) fixed *= m.units[l][HP_AXIS_V];
        else {
          ++n_auto;
          if (outer_auto < 0) outer_auto = l;
        }
      }
    if (fixed > (uint64_t)kWave) return fail(HP_EINVAL, "V units multiply to %llu > 64", (unsigned long long)fixed);
    uint64_t left = kWave / fixed;
    for (int l = d - 1; l >= 0; --l) {
      if (!(m.scopes[l] & HP_SCOPE_V)) continue;
      uint64_t f = m.units[l][HP_AXIS_V];
      if (!f) {
        if (l == outer_auto) f = left;
        else {
          f = pow2ceil((uint64_t)cdiv(dp.lv[l].e, dp.lv[l].chunk));
          if (f > left) f = left;
        }
        left /= f;
      }
      dp.lv[l].vf = (int32_t)f;
    }
    int sh = 0;
    for (int l = d - 1; l >= 0; --l)
      if (m.scopes[l] & HP_SCOPE_V) {
        dp.lv[l].vsh = sh;
        sh += log2u(dp.lv[l].vf);
      }
    dp.idle_vmask = (sh >= 6) ? 0u : (0xFFFFFFFFu << sh) & 0x3Fu;
  }
  // ---- W axis: waves per workgroup
  {
    uint64_t fixed = 1;
    for (int l = 0; l < d; ++l)
      if ((m.scopes[l] & HP_SCOPE_W) && m.units[l][HP_AXIS_W]) fixed *= m.units[l][HP_AXIS_W];
    if (fixed > (uint64_t)kMaxWaves)
      return fail(HP_EINVAL, "W units multiply to %llu > %d", (unsigned long long)fixed, kMaxWaves);
    uint64_t left = 4 / (fixed < 4 ? fixed : 4);  // default budget for levels left to the planner
    if (left < 1) left = 1;
    for (int l = d - 1; l >= 0; --l) {
      if (!(m.scopes[l] & HP_SCOPE_W)) continue;
      uint64_t f = m.units[l][HP_AXIS_W];
      if (!f) {
        int64_t per = cdiv(dp.lv[l].e, (int64_t)dp.lv[l].chunk * dp.lv[l].vf);
        f = pow2ceil((uint64_t)per);
        if (f > left) f = left;
        left /= f;
        if (left < 1) left = 1;
      }
      dp.lv[l].wf = (int32_t)f;
    }
    int sh = 0;
    for (int l = d - 1; l >= 0; --l)
      if (m.scopes[l] & HP_SCOPE_W) {
        dp.lv[l].wsh = sh;
        sh += log2u(dp.lv[l].wf);
      }
    dp.nw = 1 << sh;
    if (dp.nw > kMaxWaves) return fail(HP_EINVAL, "more than %d waves per workgroup", kMaxWaves);
    if (force_nw > 0 && dp.nw != force_nw)
      return fail(HP_EUNSUPPORTED, "batched plans use %d waves per workgroup, this map gives %d", force_nw, dp.nw);
    dp.idle_wmask = 0;
  }
  // ---- segments of reducing levels
  dp.nseg = 0;
  for (int l = p; l < d; ++l) {
    const int op = dp.lv[l].op;
    const bool arg = op == HP_OP_ARGMIN || op == HP_OP_ARGMAX;
    const bool joins = l > p && dp.lv[l - 1].op == op && !arg;
    if (!joins) {
      DevSeg& S = dp.seg[dp.nseg];
      memset(&S, 0, sizeof S);
      S.first = l;
      S.op = op;
      ++dp.nseg;
    }
    dp.seg[dp.nseg - 1].last = l;
    dp.lv[l].seg = dp.nseg - 1;
  }
  // ---- G axis
  {
    // which segment is the innermost one with grid units (requested or planned)
    int gq = -1;
    for (int l = p; l < d; ++l)
      if ((m.scopes[l] & HP_SCOPE_G) && (m.units[l][HP_AXIS_G] != 1)) gq = dp.lv[l].seg;
    for (int l = 0; l < d; ++l) {
      if (!(m.scopes[l] & HP_SCOPE_G)) continue;
      uint64_t f = m.units[l][HP_AXIS_G];
      DevLevel& L = dp.lv[l];
      const int64_t inner_units = (int64_t)L.wf * L.vf * L.chunk;
      if (l < p) {
        if (!f) f = (uint64_t)cdiv(L.e, inner_units);
      } else if (L.seg < gq) {
        // reducing level outside the innermost grid-spanning segment: it must
        // finish on the grid in one strip, so that its operator is applied after
        // the cross-workgroup combine of the segment inside it
        const uint64_t need = (uint64_t)cdiv(L.e, inner_units);
        if (!f) f = need;
        if (f < need)
          return fail(HP_EUNSUPPORTED,
                      "level %d reduces outside a grid-spanning segment and needs >= %llu grid units",
                      l, (unsigned long long)need);
      } else {
        if (!f) {
          // planner's choice for an explicit G scope without units: fill the machine
          int64_t outs = 1;
          for (int k = 0; k < p; ++k) outs *= dp.lv[k].e;
          int64_t want = cdiv(2048, outs);
          int64_t useful = cdiv(L.e, inner_units);
          f = (uint64_t)(want < useful ? want : useful);
          if (f < 1) f = 1;
        }
      }
      if (f > 0x7FFFFFFFull) return fail(HP_EUNSUPPORTED, "level %d asks for more than 2^31 workgroups", l);
      L.gf = (uint32_t)f;
    }
    // reducing grid product
    uint64_t gs = 1;
    for (int l = p; l < d; ++l) {
      gs *= dp.lv[l].gf;
      if (gs > (1ull << 24)) return fail(HP_EUNSUPPORTED, "more than 2^24 workgroups per output");
    }
    dp.gsplit = (int64_t)gs;
    // cap the grid: NONE levels give up units (and take strips) from the outermost inward
    const uint64_t block_threads = (uint64_t)dp.nw * kWave;
    const uint64_t max_grid = ((1ull << 31) / block_threads);
    uint64_t grid = gs;
    for (int l = 0; l < p; ++l) grid *= dp.lv[l].gf;
    for (int l = 0; l < p && grid > max_grid; ++l) {
      if (!(m.scopes[l] & HP_SCOPE_G) || m.units[l][HP_AXIS_G]) continue;
      uint64_t others = grid / dp.lv[l].gf;
      uint64_t f = max_grid / others;
      if (f < 1) f = 1;
      dp.lv[l].gf = (uint32_t)f;
      grid = others * f;
    }
    if (grid > max_grid) return fail(HP_EUNSUPPORTED, "grid of %llu workgroups exceeds the launch limit",
                                     (unsigned long long)grid);
    dp.grid = (int64_t)grid;
    uint64_t div = 1;
    for (int l = d - 1; l >= 0; --l) {
      dp.lv[l].gdiv = (uint32_t)div;
      div *= dp.lv[l].gf;
    }
  }
  // ---- per-level strips
  dp.none_iters = 1;
  dp.red_iters = 1;
  for (int l = 0; l < d; ++l) {
    DevLevel& L = dp.lv[l];
    L.span = (int64_t)L.gf * L.wf * L.vf * L.chunk;
    L.strips = cdiv(L.e, L.span);
    L.sstride = L.span * L.stride;
    L.ragged = (L.strips * L.span != L.e) ? 1 : 0;
    if (l < p) dp.none_iters *= L.strips;
    else dp.red_iters *= L.strips;
  }
  {
    int64_t os = 1;
    for (int l = p - 1; l >= 0; --l) {
      dp.lv[l].ostride = os;
      os *= dp.lv[l].e;
    }
    dp.n_out = os;
  }
  // ---- divisions the kernels make by plan constants
  for (int l = 0; l < d; ++l) {
    DevLevel& L = dp.lv[l];
    L.fd_gdiv = fastdiv((uint64_t)L.gdiv);
    L.fd_gf = fastdiv((uint64_t)L.gf);
    L.fd_span = (L.e + L.span < ((int64_t)1 << 31)) ? fastdiv((uint64_t)L.span) : FastDiv{0u, 0u};
    L.csh = log2u((uint64_t)L.chunk);
    L.pad_ = 0;
  }
  // ---- segment masks and the grid-combine mode
  dp.red_vmask = dp.red_wmask = 0;
  uint32_t outer_v = 0;
  for (int l = 0; l < p; ++l) outer_v |= (uint32_t)(dp.lv[l].vf - 1) << dp.lv[l].vsh;
  dp.lds_slot_lanes = 1;
  int gq = -1;
  for (int j = 0; j < dp.nseg; ++j) {
    DevSeg& S = dp.seg[j];
    S.vmask = S.wmask = 0;
    S.gunits = 1;
    S.wlo = 31;
    for (int l = S.first; l <= S.last; ++l) {
      const DevLevel& L = dp.lv[l];
      S.vmask |= (uint32_t)(L.vf - 1) << L.vsh;
      S.wmask |= (uint32_t)(L.wf - 1) << L.wsh;
      if (L.wf > 1 && L.wsh < S.wlo) S.wlo = L.wsh;
      S.gunits *= L.gf;
    }
    if (S.wlo == 31) S.wlo = 0;
    S.nwu = 1 << __builtin_popcount(S.wmask);
    S.lds_lanes = outer_v;
    if (S.wmask && outer_v) dp.lds_slot_lanes = kWave;
    outer_v |= S.vmask;
    dp.red_vmask |= S.vmask;
    dp.red_wmask |= S.wmask;
    if (S.gunits > 1) gq = j;
  }
  // Steps whose lower lane bits are all reduced by the time they run: bits of the
  // segment itself (steps go lowest bit first) and bits of inner segments (their
  // combines leave every lane of a group with the group's value).
  {
    uint32_t inner_v = 0;
    for (int j = dp.nseg - 1; j >= 0; --j) {
      DevSeg& S = dp.seg[j];
      S.ufast = 0;
      for (int b = 0; b < 6; ++b) {
        const uint32_t lower = (1u << b) - 1u;
        if (((S.vmask >> b) & 1u) && ((inner_v | S.vmask) & lower) == lower) S.ufast |= 1u << b;
      }
      inner_v |= S.vmask;
    }
  }
  if (gq < 0) {
    dp.gmode = GCOMB_NONE;
    dp.gsplit = 1;
  } else {
    // every reducing level before segment gq must finish in one strip (enforced above for
    // explicit units; also true for planner-chosen ones)
    for (int l = p; l < dp.seg[gq].first; ++l)
      if (dp.lv[l].strips != 1)
        return fail(HP_EUNSUPPORTED, "level %d must complete in one strip on the grid", l);
    dp.gmode = gq == 0 ? GCOMB_UNIFORM : GCOMB_NESTED;
  }
  dp.gq = gq < 0 ? 0 : gq;
  // innermost-segment stream description
  dp.a = dp.nseg > 0 ? dp.seg[dp.nseg - 1].first : d;
  dp.nid = 0;
  dp.inner_iters = 1;
  dp.outer_iters = 1;
  dp.last_dim_is_last_level = 0;
  for (int l = p; l < d; ++l) {
    if (l < dp.a) {
      dp.outer_iters *= dp.lv[l].strips;
    } else {
      dp.inner_iters *= dp.lv[l].strips;
      if (dp.lv[l].strips > 1) {
        dp.id_strips[dp.nid] = dp.lv[l].strips;
        dp.id_sstride[dp.nid] = dp.lv[l].sstride;
        dp.id_level[dp.nid] = l;
        dp.id_ragged[dp.nid] = dp.lv[l].ragged;
        if (l == d - 1) dp.last_dim_is_last_level = 1;
        ++dp.nid;
      }
    }
  }
  for (int l = 0; l < d; ++l)
    if (dp.lv[l].strips > 0x7FFFFFFFll)
      return fail(HP_EUNSUPPORTED, "level %d needs more than 2^31 strips; give it more units", l);
  dp.xcd = (!(flags & HP_FLAG_NO_XCD) && dp.grid % 8 == 0 && dp.grid >= 16) ? 1 : 0;
  // a grid of exactly 8 needs no renumbering: workgroup b already runs on XCD b
  if (xlevel >= 0 && (!(dp.xcd || dp.grid == 8) || (int64_t)dp.lv[xlevel].gdiv * 8 != dp.grid))
    return fail(HP_EUNSUPPORTED, "X at level %d needs a grid that is 8 or a multiple of 8 of at least 16 (it has %lld)",
                xlevel, (long long)dp.grid);
  // ---- output kind
  if (is_float) {
    dp.out_kind = (flags & HP_FLAG_OUT_F32) ? OUT_F32 : OUT_F64;
  } else {
    dp.out_kind = OUT_I32;
    for (int l = p; l < d; ++l) {
      if (dp.lv[l].op == HP_OP_SUM) { dp.out_kind = OUT_I64; break; }
      if (dp.lv[l].op == HP_OP_ARGMIN || dp.lv[l].op == HP_OP_ARGMAX) { dp.out_kind = OUT_I32; break; }
    }
  }
  // ---- lane spread of a wave: lane 0 has every V digit at 0, so it holds the
  // wave's lowest address and the others lie at most this far above it
  {
    int64_t vspan = 0;
    for (int l = 0; l < d; ++l) vspan += (int64_t)(dp.lv[l].vf - 1) * dp.lv[l].chunk * dp.lv[l].stride;
    if (flat_block) vspan += dp.chunk;  // each lane's interior starts up to a vector later
    dp.vlane32 = vspan * elem_bytes(n->dtype) < ((int64_t)1 << 31) ? 1 : 0;
  }
  // ---- flat blocks: the threads that share one output (they spread the elements
  // outside the interior between them)
  if (flat_block) {
    if (dp.nseg != 1 || dp.outer_iters != 1) return fail(HP_EINVAL, "flat view needs one reducing segment");
    int64_t u = 1;
    for (int l = p; l < d; ++l) u *= (int64_t)dp.lv[l].gf * dp.lv[l].wf * dp.lv[l].vf;
    dp.flat_units = u;
  }
  // ---- kernel variant
  if (is_float) {
    const int vec = n->dtype == HP_BF16 ? 8 : 4;
    if (d <= 4 && dp.nid <= 1 && dp.nw <= 8 && dp.chunk == vec && dp.vlane32 && !(flags & HP_FLAG_GENERIC))
      dp.kernel = HP_KERNEL_LEAN;
    else dp.kernel = d <= 4 ? HP_KERNEL_GENERIC4 : HP_KERNEL_GENERIC8;
  } else {
    // The flat and segmented kernels carry one 64-bit key per lane, which packs an
    // ARG level's (value, index) only when its child values fit in 32 bits: the
    // input, MIN / MAX of 32-bit values, or an inner ARG level's index.  An ARG over
    // an int64 SUM goes to the general kernel and its (value, index) pairs.
    bool narrow = true;  // the child values of segment j fit in 32 bits
    bool keys = true;
    for (int j = dp.nseg - 1; j >= 0; --j) {
      const int op = dp.seg[j].op;
      const bool arg = op == HP_OP_ARGMIN || op == HP_OP_ARGMAX;
      if (arg && !narrow) keys = false;
      narrow = arg || ((op == HP_OP_MIN || op == HP_OP_MAX) && narrow);
    }
    if (keys && d <= 4 && dp.nseg <= 1) dp.kernel = HP_KERNEL_INT_FLAT;
    else if (keys && d <= 4 && dp.nseg <= 3) dp.kernel = HP_KERNEL_INT_SEG;
    else dp.kernel = HP_KERNEL_INT_DEEP;
    // The chain kernel: every reducing level a segment of its own, nothing masked,
    // the NONE levels on the grid alone, the innermost level on lanes with at most
    // four 16-byte chunks per lane, and in three-level chains the middle level on
    // lanes too.
    if (dp.kernel == HP_KERNEL_INT_SEG && dp.nseg == d - p && dp.chunk == 4 && !flat_block &&
        dp.gmode != GCOMB_NESTED) {
      bool ok = true;
      for (int l = 0; l < d; ++l) {
        const DevLevel& L = dp.lv[l];
        if (L.ragged) ok = false;
        if (l < p && (L.wf != 1 || L.vf != 1)) ok = false;
      }
      const DevLevel& LL = dp.lv[d - 1];
      if (LL.gf != 1 || LL.wf != 1 || LL.strips > 4 || LL.chunk != 4) ok = false;
      if (dp.nseg == 3 && (dp.lv[d - 2].gf != 1 || dp.lv[d - 2].wf != 1)) ok = false;
      if (ok) dp.kernel = HP_KERNEL_INT_CHAIN;
    }
  }
  // ---- info
  hp_plan_info& I = out->info;
  memset(&I, 0, sizeof I);
  I.depth = d;
  I.out_dtype = dp.out_kind;
  I.n_out = dp.n_out;
  const size_t osz = (dp.out_kind == OUT_I32 || dp.out_kind == OUT_F32) ? 4 : 8;
  I.out_bytes = (size_t)dp.n_out * osz;
  I.in_elems = total;
  I.in_bytes = (size_t)total * elem_bytes(n->dtype);
  I.grid = dp.grid;
  I.waves = dp.nw;
  I.chunk = chunk_last;
  I.gsplit = dp.gsplit;
  I.workspace_bytes = dp.gsplit > 1 ? (size_t)dp.n_out * dp.gsplit * kSlotBytes : 0;
  {
    size_t slots = (size_t)dp.nw * dp.lds_slot_lanes * kSlotBytes;
    size_t gcomb = (size_t)dp.nw * 32;
    I.lds_bytes = (slots > gcomb ? slots : gcomb) + 16;
  }
  for (int l = 0; l < d; ++l) {
    I.scopes[l] = m.scopes[l] | (l == xlevel ? (uint32_t)HP_SCOPE_X : 0u);
    I.units[l][HP_AXIS_G] = dp.lv[l].gf;
    I.units[l][HP_AXIS_W] = (uint32_t)dp.lv[l].wf;
    I.units[l][HP_AXIS_V] = (uint32_t)dp.lv[l].vf;
    I.strips[l] = dp.lv[l].strips;
  }
  I.nseg = dp.nseg;
  I.kernel = dp.kernel;
  I.flat_block = flat_block;
  out->dp = dp;
  // A float nest is a sum of sums (floats take SUM only), so each output's block is
  // one contiguous run.  When the automatic plan iterates more than one level inside
  // a thread it runs on the general kernel; the same block as one level may fit the
  // lean kernel, which then takes it (3- and 4-level nests of 128-256 MiB: 1.04-1.5x
  // faster in fp32, 1.14-2x in bf16, none slower).
  if (is_float && !map_in && !flat_block && force_nw == 0 && dp.kernel != HP_KERNEL_LEAN && d - p >= 2 &&
      chunk_last == 16 / elem_bytes(n->dtype) && !(flags & (HP_FLAG_GENERIC | HP_FLAG_SCALAR))) {
    hp_nest v = *n;
    v.depth = p + 1;
    for (int l = p + 1; l < d; ++l) v.extent[p] *= n->extent[l];
    Lowered one;
    if (lower(&v, nullptr, flags, &one, 0, 0) == HP_OK && one.dp.kernel == HP_KERNEL_LEAN) *out = one;
  }
  return HP_OK;
}

}  // namespace hp

extern "C" const char* hp_last_error(void) { return hp::g_err; }

extern "C" const char* hp_status_str(hp_status s) {
  switch (s) {
    case HP_OK: return "HP_OK";
    case HP_EINVAL: return "HP_EINVAL";
    case HP_EUNSUPPORTED: return "HP_EUNSUPPORTED";
    case HP_ENOMEM: return "HP_ENOMEM";
    case HP_EDEVICE: return "HP_EDEVICE";
    case HP_EAGAIN: return "HP_EAGAIN";
    case HP_ETOOBIG: return "HP_ETOOBIG";
    case HP_ENOTREADY: return "HP_ENOTREADY";
    case HP_ECANCELED: return "HP_ECANCELED";
    case HP_ESTATE: return "HP_ESTATE";
  }
  return "unknown status";
}

extern "C" hp_status hp_plan_inspect(const hp_nest* nest, const hp_level_map* map, uint32_t flags,
                                     hp_plan_info* info) {
  if (!info) return hp::fail(HP_EINVAL, "null info");
  hp::Lowered L;
  hp_status s = hp::lower(nest, map, flags, &L);
  if (s != HP_OK) return s;
  *info = L.info;
  return HP_OK;
}
