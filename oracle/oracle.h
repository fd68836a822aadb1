/*
 * Reference oracle for nested multi-level reductions -- TEST INFRASTRUCTURE.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may call this code.  It shares nothing with the GPU library (no header, no
 * helper, no table) and the GPU library never calls it.
 *
 * What it computes (the recursive reduction of the paper's section 2, where on
 * every level one task collects the results of all its siblings):
 *
 *   nest A with extents e[0..d), ops o[0..d); o[0..p) are NONE (the output
 *   prefix), o[p..d) reduce.
 *     R_d(i_0..i_{d-1}) = A[i_0, ..., i_{d-1}]          (row-major storage)
 *     R_m(i_0..i_{m-1}) = OP_{o_m} over t = 0..e_m-1 of R_{m+1}(i_0..i_{m-1}, t)
 *     out[i_0..i_{p-1}] = R_p(i_0..i_{p-1})              (row-major output)
 *
 * Operators (readings of points the paper leaves open):
 *   SUM on integers : int64, wrapping modulo 2^64;
 *   SUM on floats   : double precision with Neumaier compensation over the
 *                     exact double images of the fp32 / bf16 inputs;
 *   MIN / MAX       : exact, integer inputs only;
 *   ARGMIN / ARGMAX : the smallest t attaining the extremum (first occurrence
 *                     wins); the index t is the value passed to the enclosing
 *                     level; integer inputs only.
 * Output type: float nests give double.  For integer nests the type T(m)
 * of R_m is: T(d) = int32 (an element); T(m) = int64 for SUM, int32 for
 * ARGMIN/ARGMAX (an index), T(m+1) for MIN/MAX.  The output has type T(p).
 */
#ifndef HP_ORACLE_H
#define HP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_I32 = 0, OR_F32 = 1, OR_BF16 = 2 };
enum { OR_NONE = 0, OR_SUM = 1, OR_MIN = 2, OR_MAX = 3, OR_ARGMIN = 4, OR_ARGMAX = 5 };
enum { OR_OUT_I32 = 0, OR_OUT_I64 = 1, OR_OUT_F64 = 2 };

/* Output kind of a nest, or -1 if the nest is not one the oracle defines. */
int oracle_out_kind(int depth, const int64_t* extents, const int* ops, int dtype);

/* Number of outputs (product of the NONE-prefix extents), or -1. */
int64_t oracle_n_out(int depth, const int64_t* extents, const int* ops);

/* Compute outputs [o_begin, o_end) of the nest.  `in` is the whole input
 * (row-major), `out` receives o_end - o_begin values of the output kind.
 * Outputs are split over `threads` host threads (each output is computed by
 * one thread in the same order, so the result does not depend on it).
 * Returns 0, or -1 for an invalid nest or range. */
int oracle_reduce_range(int depth, const int64_t* extents, const int* ops, int dtype,
                        const void* in, void* out, int64_t o_begin, int64_t o_end, int threads);

/* oracle_reduce_range over all outputs. */
int oracle_reduce(int depth, const int64_t* extents, const int* ops, int dtype,
                  const void* in, void* out, int threads);

/* Sum of |a| over the reduced block of each output in [o_begin, o_end)
 * (double, Neumaier), for float nests: the scale of the error bound. */
int oracle_abs_sum_range(int depth, const int64_t* extents, const int* ops, int dtype,
                         const void* in, double* out, int64_t o_begin, int64_t o_end, int threads);

/* ---- ordered products (associative, not commutative) ----------------------
 *
 * The paper notes that OpenMP reductions must be commutative; the recursive
 * definition above only needs associativity if the siblings are combined in
 * sibling order.  An ordered product level OR_PROD takes, for t = 0..e_m-1 in
 * ascending order,
 *     R_m = R_{m+1}(t=0) * R_{m+1}(t=1) * ... * R_{m+1}(t=e_m-1)
 * (left to right, never reordered).  Two element types, both with arithmetic
 * modulo 2^64 (unsigned wrap), so every result is exact:
 *   OR_AFFINE : an element is (a, b), two uint64, the map x -> a x + b;
 *               (a1, b1) * (a2, b2) = (a1 a2, a2 b1 + b2), i.e. the first map
 *               applied first (the step of a linear recurrence x <- a x + b);
 *               identity (1, 0).
 *   OR_MAT2   : an element is a 2x2 matrix of uint64, row-major (m00 m01 m10 m11);
 *               * is the matrix product; identity the unit matrix.
 * Every reducing level of such a nest is OR_PROD; the output holds one element
 * (16 or 32 bytes) per output index.  Returns 0, or -1 for an invalid nest. */
enum { OR_AFFINE = 5, OR_MAT2 = 6 };
enum { OR_PROD = 6 };
int oracle_prod_range(int depth, const int64_t* extents, const int* ops, int dtype, const void* in,
                      void* out, int64_t o_begin, int64_t o_end, int threads);

/* ---- stencils ----------------------------------------------------------------
 *
 * The paper's second class of multi-level algorithms: a stencil whose input
 * region per unit fits that level's local memory, with a ghost surface of
 * neighbours around it.  This one is the 2-D five-point Jacobi sweep on a
 * rows x cols row-major array, repeated `steps` times:
 *   B[i][j] = c0 A[i][j] + c1 ((A[i-1][j] + A[i+1][j]) + (A[i][j-1] + A[i][j+1]))
 * for interior cells (1 <= i <= rows-2, 1 <= j <= cols-2); boundary cells keep
 * their input value.  Computed in double precision from the float input; out
 * receives rows*cols doubles.  Returns 0, or -1 for bad arguments. */
int oracle_stencil(int64_t rows, int64_t cols, int steps, double c0, double c1, const float* in, double* out);

#ifdef __cplusplus
}
#endif
#endif
