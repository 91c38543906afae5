/*
 * qubo_bf.h -- exhaustive QUBO solving in Gray-code order on MI355X (gfx950).
 *
 * Problem (Sec. 1, Eq. 1): for an upper-triangular Q in R^{n x n} (or Z^{n x n})
 * and x in {0,1}^n,
 *
 *     f_Q(x) = x^T Q x = sum_{i <= j} Q_ij x_i x_j .
 *
 * The library visits all 2^n vectors (Sec. 2.2: reflected Gray code, bit CTZ(t)
 * flipped at step t; Sec. 3.1: independent sub-walks under fixed prefix bits,
 * min-combined) and returns the k lowest states.  The paper returns the single
 * minimiser and its value (Algorithm 1); k > 1, batching and the log-partition
 * function with its gradient are extensions with plain definitions given below.
 *
 * Conventions shared by every entry point:
 *   - A state is a uint64 mask with bit i = x_i (0-based; x_1 of the paper is
 *     bit 0), as in the decoding of Sec. 3.
 *   - Only entries with i <= j are read (Eq. 1, right-hand side); the lower
 *     triangle is ignored.  Q is row-major with leading dimension ldq.
 *   - The zero vector is a candidate with value 0 (Sec. 2.1).
 *   - Results are ordered by (energy, mask) ascending: equal energies go to the
 *     lower natural mask (a reading; the paper does not state a tie rule).
 *   - All array arguments are DEVICE pointers owned by the caller.  The library
 *     allocates no device memory per call: scratch comes from the caller's
 *     workspace `ws` of `ws_bytes` bytes (query the size first), which must stay
 *     untouched until the call's work on `hip_stream` has completed.
 *   - Every call only enqueues work on `hip_stream` (a hipStream_t; NULL = the
 *     default stream) and returns without synchronising, so calls can be
 *     captured into a HIP graph.  The return value reports host-checkable
 *     errors only; conditions detected on the device are written to `status`
 *     (int32 per instance, device memory) once the stream reaches that point.
 *   - Calls that share a workspace must not overlap in time.
 *   - qubo_last_error() describes the last non-OK return of the calling thread.
 *
 * Float semantics (float32 and float64 Q): every block of 64 states is
 * screened against the current threshold -- by default in packed float16 on
 * scaled values, with a margin that keeps every block a float32 screen would
 * keep (QUBO_TUNE_HALF_SCREEN = -1 selects the float32 / float64 screens;
 * results are identical) -- and the blocks that pass are replayed with
 * float64 keys.  The K' >= k best candidates are rescored in float64 in a
 * fixed order (row i ascending: Q_ii, then Q_ij for set j > i in ascending j;
 * rows summed in ascending i) and selected by (float64 energy, mask).  A
 * certificate proves that no state outside the candidates can rank among the
 * k best: every discarded state's exact value is at least the K'-th key
 * minus eps, eps = 3 * 2^-24 * R_I + 2^-36 * sum |Q_ij| for float32 Q (R_I:
 * sum |Q_ij| over the six lowest rows) and 2^-36 * sum |Q_ij| for float64 Q,
 * 0 for integer-valued Q within the exact range (sum |Q_ij| <= 2^24 float32,
 * 2^50 float64).  When it fails the outputs are still written and `status`
 * is QUBO_ERR_UNCERTAIN (qubo_bf_solve_kp with kprime = 64 gives it more
 * room).
 * Integer semantics: int32 and int64 Q, int64 energies, bit-exact results.
 * int32 Q screens in exact int16 where the six lowest rows allow it, else in
 * int32; an instance with sum |Q_ij| > 2^28 is walked on float64 tables,
 * still exactly (every int32 Q has sum |Q_ij| < 2^50).  int64 Q is walked on
 * float64 tables, exact for sum |Q_ij| <= 2^50 (else status QUBO_ERR_RANGE).
 * Floating-point and integer walks take about the same time per state.
 */
#ifndef QUBO_BF_H
#define QUBO_BF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The two range enumerators make every int a valid value of the type, so
 * that an unknown value passed from C is rejected (QUBO_ERR_INVALID_ARG)
 * rather than being undefined in the C++ implementation. */
typedef enum {
  QUBO_F32 = 0,
  QUBO_I32 = 1,
  QUBO_F64 = 2,
  QUBO_I64 = 3,
  QUBO_DTYPE_RANGE_LO_ = -0x7fffffff - 1,
  QUBO_DTYPE_RANGE_HI_ = 0x7fffffff
} qubo_dtype;

enum {
  QUBO_OK = 0,
  QUBO_ERR_INVALID_ARG = -1, /* bad argument (host) or bad n in ns (device status) */
  QUBO_ERR_NONFINITE = -2,   /* Q (or beta) holds inf or NaN (device status) */
  QUBO_ERR_WORKSPACE = -3,   /* ws_bytes smaller than the workspace query */
  QUBO_ERR_HIP = -4,         /* a HIP launch or runtime call failed */
  QUBO_ERR_UNCERTAIN = -5,   /* float certificate failed (device status) */
  QUBO_ERR_RANGE = -6,       /* int64 Q whose sum |Q_ij| exceeds 2^50 (device status) */
  QUBO_ERR_OVERFLOW = -7     /* internal slot overflow (device status; a bug) */
};

/* ------------------------------------------------------------------ top-k */

/* Workspace bytes needed by qubo_bf_solve(n, k, dt); 0 for invalid arguments.
 * Depends only on the arguments and the current tuning (qubo_bf_set_tuning). */
size_t qubo_bf_workspace_size(int n, int k, qubo_dtype dt);

/*
 * The k lowest states of one QUBO (Algorithm 1 generalised from k = 1).
 *   Q         device, n x n (ldq >= n), of the type dt: float32, int32,
 *             float64 or int64
 *   n         1 .. 63
 *   k         1 .. 64 (int32, int64), 1 .. 56 (float32, float64)
 *   energies  device, k entries: double (QUBO_F32, QUBO_F64) or int64_t
 *             (QUBO_I32, QUBO_I64); slots beyond 2^n hold +inf / INT64_MAX
 *   masks     device, k entries; slots beyond 2^n hold ~0
 *   status    device, 1 int32: QUBO_OK, QUBO_ERR_NONFINITE, QUBO_ERR_RANGE or
 *             QUBO_ERR_UNCERTAIN
 * Returns QUBO_OK, QUBO_ERR_INVALID_ARG, QUBO_ERR_WORKSPACE or QUBO_ERR_HIP.
 */
int qubo_bf_solve(const void* Q, int n, int64_t ldq, qubo_dtype dt, int k, void* energies, uint64_t* masks,
                  int32_t* status, void* ws, size_t ws_bytes, void* hip_stream);

/*
 * qubo_bf_solve with the length K' of the candidate lists given: kprime in
 * [k, 64], or 0 for the default (max(2k, k + 3) capped at 64 for float Q, k
 * for integer Q).  A longer list gives the float certificate more room above
 * the k-th value (a solve whose status was QUBO_ERR_UNCERTAIN can be repeated
 * with kprime = 64), at a larger workspace: qubo_bf_workspace_size_kp, 0 for
 * invalid arguments.  The results of a certified solve do not depend on K'.
 * Unlike the process-wide QUBO_TUNE_KPRIME knob this affects only the call.
 * Returns as qubo_bf_solve (QUBO_ERR_INVALID_ARG for a bad kprime).
 */
size_t qubo_bf_workspace_size_kp(int n, int k, int kprime, qubo_dtype dt);
int qubo_bf_solve_kp(const void* Q, int n, int64_t ldq, qubo_dtype dt, int k, int kprime, void* energies,
                     uint64_t* masks, int32_t* status, void* ws, size_t ws_bytes, void* hip_stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: qubo_bf_solve
 * without a workspace argument.  The workspace is a library-owned static
 * device array of QUBO_NOALLOC_SCRATCH_BYTES (16 MiB), one per GPU, held until
 * the process ends; it covers every single solve (n <= 63, any k, any tuning).
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); on its first call on a device it looks up that device's copy of
 * the array (hipGetSymbolAddress) and keeps the address.
 *   Arguments, outputs, status and return codes as qubo_bf_solve; a
 *   workspace need above the array's size returns QUBO_ERR_WORKSPACE.
 * Every call on one GPU shares that GPU's array, and the array keeps the last
 * call's contents (each call resets what it reads before reading it): calls
 * that overlap in time on one GPU -- from other threads, or on other streams
 * without ordering -- race and must not be issued.
 */
#define QUBO_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int qubo_bf_solve_noalloc(const void* Q, int n, int64_t ldq, qubo_dtype dt, int k, void* energies,
                          uint64_t* masks, int32_t* status, void* hip_stream);

/* Workspace bytes for qubo_bf_solve_batched with every n_b <= nmax. */
size_t qubo_bf_batched_workspace_size(int batch, int nmax, int k, qubo_dtype dt);

/*
 * Independent solves of `batch` QUBOs of uneven size in one launch sequence.
 *   Q         device, [batch][nmax][nmax]; instance b uses its leading
 *             ns[b] x ns[b] block (row stride nmax)
 *   nmax      1 .. 40
 *   ns        device, [batch] sizes, 1 .. nmax (others: status INVALID_ARG)
 *   energies  device, [batch][k]: double or int64_t (as qubo_bf_solve)
 *   masks     device, [batch][k]
 *   status    device, [batch]
 * Returns as qubo_bf_solve.
 */
int qubo_bf_solve_batched(int batch, const void* Q, int nmax, const int32_t* ns, qubo_dtype dt, int k,
                          void* energies, uint64_t* masks, int32_t* status, void* ws, size_t ws_bytes,
                          void* hip_stream);

/* --------------------------------------------------- prefix-range solves */

/* Workspace bytes for qubo_bf_solve_range with these n, k, dt and p_bits (any
 * range); 0 for invalid arguments. */
size_t qubo_bf_range_workspace_size(int n, int k, qubo_dtype dt, int p_bits);

/*
 * Part of one solve, for long enumerations cut into resumable pieces: the k
 * lowest states among the masks whose top p_bits bits (p = mask >> (n - p_bits))
 * lie in [p_begin, p_end) -- the fixed-prefix sub-walks of Sec. 3.1, each a
 * contiguous block of masks.  Arguments, outputs and status as qubo_bf_solve;
 * the result is exact (and, for float Q, certified) for that range, so the
 * k lowest of the union of the results of disjoint ranges (qubo_bf_merge_topk)
 * is the result of qubo_bf_solve.
 *   p_bits   1 .. n - 12 (a range of one prefix holds 2^(n - p_bits) masks)
 *   p_begin, p_end   0 <= p_begin < p_end <= 2^p_bits
 */
int qubo_bf_solve_range(const void* Q, int n, int64_t ldq, qubo_dtype dt, int k, int p_bits, int64_t p_begin,
                        int64_t p_end, void* energies, uint64_t* masks, int32_t* status, void* ws,
                        size_t ws_bytes, void* hip_stream);

/*
 * The k lowest (energy, mask) pairs of `count` result lists of k_in entries
 * each (device, [count][k_in], energies double for QUBO_F32 / QUBO_F64, int64_t
 * for QUBO_I32 / QUBO_I64, masks uint64), as written by qubo_bf_solve_range for disjoint
 * ranges of one instance; sentinel entries are skipped and missing outputs
 * hold the sentinels.  k: 1 .. 64.  One launch on hip_stream, no workspace.
 */
int qubo_bf_merge_topk(int count, int k_in, const void* energies_in, const uint64_t* masks_in, qubo_dtype dt,
                       int k, void* energies, uint64_t* masks, void* hip_stream);

/* ------------------------------------------------------- log-partition */

/* Workspace bytes for qubo_logz_fwd / qubo_logz_bwd (the larger of the two). */
size_t qubo_logz_workspace_size(int batch, int nmax);

/*
 * logZ_b = log sum_x exp(-beta_b f_{Q_b}(x)), natural log, float64 result.
 *   Q      device, [batch][nmax][nmax] float32, sizes ns (device, [batch])
 *   nmax   1 .. 32
 *   beta   device, [batch] float32, any finite value (else that instance's
 *          status is QUBO_ERR_NONFINITE and its logz NaN)
 *   logz   device, [batch] double
 *   status device, [batch]
 */
int qubo_logz_fwd(int batch, const float* Q, int nmax, const int32_t* ns, const float* beta, double* logz,
                  int32_t* status, void* ws, size_t ws_bytes, void* hip_stream);

/*
 * Adjoint of qubo_logz_fwd, by re-enumeration:
 *   grad_Q[b][i][j] = grad_logz[b] * (-beta_b) * E_p[x_i x_j]  for i <= j < n_b,
 *   0 elsewhere (lower triangle and padding), p(x) = exp(-beta f(x) - logZ);
 *   grad_beta[b] = grad_logz[b] * (-E_p[f])  (skipped when grad_beta is NULL).
 *   logz   device, [batch] double, the forward result for the same inputs
 *   grad_logz device, [batch] float32
 *   grad_Q device, [batch][nmax][nmax] float32 (fully written)
 */
int qubo_logz_bwd(int batch, const float* Q, int nmax, const int32_t* ns, const float* beta, const double* logz,
                  const float* grad_logz, float* grad_Q, float* grad_beta, int32_t* status, void* ws,
                  size_t ws_bytes, void* hip_stream);

/*
 * Second moments of p(x) = exp(-beta f(x) - logZ), by the same re-enumeration
 * as qubo_logz_bwd (an extension with a plain definition):
 *   moments[b][i][j] = E_p[x_i x_j]  for i <= j < n_b (E_p[x_i] on the
 *                      diagonal: the marginals), 0 elsewhere; float64
 *   mean_energy[b]   = E_p[f]  (device, [batch] double; may be NULL)
 *   logz   device, [batch] double, the forward result for the same inputs
 * Other arguments and the workspace as qubo_logz_bwd.
 */
int qubo_logz_moments(int batch, const float* Q, int nmax, const int32_t* ns, const float* beta,
                      const double* logz, double* moments, double* mean_energy, int32_t* status, void* ws,
                      size_t ws_bytes, void* hip_stream);

/* Workspace bytes for qubo_logz_sample; 0 for invalid sizes. */
size_t qubo_logz_sample_workspace_size(int batch, int nmax);

/*
 * Exact samples of p(x) = exp(-beta f(x) - logZ) (an extension with a plain
 * definition): for each instance b and uniform u = u[b][s] in [0, 1), the
 * mask m with F(m - 1) <= u < F(m), where F(m) = sum_{x <= m} p(x) runs over
 * the masks in natural (integer) order -- inversion of the exact cumulative
 * distribution.  The uniforms are inputs, so a caller owns the random stream
 * and results are reproducible; values outside [0, 1) are clamped into it.
 * Weights are evaluated in float32 per state and summed in float64, so a u
 * within about 1e-5 of a boundary F(m) may return the neighbouring mask.
 *   Q, ns, beta, nmax   as qubo_logz_fwd (nmax 1 .. 32)
 *   nsamples  samples per instance, >= 1
 *   u         device, [batch][nsamples] double
 *   masks     device, [batch][nsamples] uint64 (all ones for an instance
 *             whose status is not QUBO_OK)
 *   logz      device, [batch] double: log Z, written as by qubo_logz_fwd
 *   status    device, [batch]
 *   ws        device workspace of qubo_logz_sample_workspace_size bytes
 * One forward enumeration, then one wave per sample re-walks the sampled
 * work unit's lane; all on hip_stream.
 */
int qubo_logz_sample(int batch, const float* Q, int nmax, const int32_t* ns, const float* beta, int nsamples,
                     const double* u, uint64_t* masks, double* logz, int32_t* status, void* ws, size_t ws_bytes,
                     void* hip_stream);

/* ------------------------------------------------------------ utilities */

/* Thread-local description of the last non-OK return (never NULL). */
const char* qubo_last_error(void);
/* Library version string. */
const char* qubo_version(void);

/*
 * Tuning knobs (process-wide; 0 restores the default).  They change the
 * workspace size, so query it again after a change.
 *   QUBO_TUNE_SINGLE_OUTER_BITS   max outer (Gray-walked) bits per work unit, single solve
 *   QUBO_TUNE_SINGLE_UNIT_BITS    prefix bits reserved for work units, single solve
 *                                 (upper bound, default 14; n <= 32 reserves
 *                                 min(11, max(8, n - 18)), 12 in place of 11
 *                                 and 13 in place of 14 for walks other than
 *                                 the float32 half screen; int32 Q under the
 *                                 half screen reserves 12 at n = 32..35 and 13
 *                                 from n = 36)
 *   QUBO_TUNE_BATCHED_OUTER_BITS  max outer bits per work unit, batched / logZ
 *   QUBO_TUNE_WAVES_PER_CU        resident waves per compute unit of the walk grid
 *                                 (0, the default, reads back as 0 and means
 *                                 16 for the half-screen walks (float16
 *                                 screen: float32, float64, int64 Q; int16
 *                                 screen: int32 Q), 12 otherwise); never
 *                                 more than the walk kernel keeps resident
 *   QUBO_TUNE_KPRIME              candidate list length override (float path;
 *                                 values below k make the certificate fail)
 *   QUBO_TUNE_CHUNK_SINGLE        work units per queue pull, single solve
 *   QUBO_TUNE_CHUNK_BATCHED       work units per queue pull, batched / logZ
 *   QUBO_TUNE_DYNAMIC_QUEUE       1: atomic work queue; -1: static assignment
 *   QUBO_TUNE_LOGZ_FACTORED       1: log-partition walks may use the factored
 *                                 form (one multiply-add per state), the
 *                                 gradient walk its nested form where a unit's
 *                                 step factors allow; 2: the factored form
 *                                 with per-state products in the gradient
 *                                 walk; -1: always one exp per state (same
 *                                 results within rounding)
 *   QUBO_TUNE_SEED_SWEEPS         steepest descents (1 .. 64, default 4) of
 *                                 the per-instance threshold seed before a
 *                                 top-k walk, spread over the instance's waves
 *                                 (one in a batch, four for a single solve);
 *                                 -1: no seeding (speed only: results are
 *                                 identical)
 *   QUBO_TUNE_HALF_SCREEN         top-k walks: 1 screens each block of 64
 *                                 states of float32, float64 and int64 Q in
 *                                 packed float16 (with a margin that keeps
 *                                 every block a float32 / float64 screen
 *                                 passes); int32 instances whose inner rows
 *                                 sum to at most 32767 in |Q| screen in exact
 *                                 int16; -1: float32 / int32 / float64 screens
 *                                 (results are identical: passing blocks are
 *                                 replayed exactly)
 * Environment variables of the same names (QUBO_BF_SINGLE_OUTER_BITS, ...)
 * set the initial values.  Returns QUBO_OK or QUBO_ERR_INVALID_ARG.
 */
enum {
  QUBO_TUNE_SINGLE_OUTER_BITS = 1,
  QUBO_TUNE_SINGLE_UNIT_BITS = 2,
  QUBO_TUNE_BATCHED_OUTER_BITS = 3,
  QUBO_TUNE_WAVES_PER_CU = 4,
  QUBO_TUNE_KPRIME = 5,
  QUBO_TUNE_CHUNK_SINGLE = 6,
  QUBO_TUNE_CHUNK_BATCHED = 7,
  QUBO_TUNE_DYNAMIC_QUEUE = 8,
  QUBO_TUNE_LOGZ_FACTORED = 9,
  QUBO_TUNE_SEED_SWEEPS = 10,
  QUBO_TUNE_HALF_SCREEN = 11
};
int qubo_bf_set_tuning(int knob, int value);
int qubo_bf_get_tuning(int knob);

/*
 * Kernel timing for measurement: while enabled, the library records a HIP
 * event pair around each launch of its enumeration kernels on the call's
 * stream.  qubo_prof_collect waits for the recorded events, returns the summed
 * milliseconds and launch count of the kernel `name` ("walk_topk", "walk_exp",
 * "walk_grad") and clears the records of that kernel.
 */
int qubo_prof_enable(int on);
int qubo_prof_collect(const char* name, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* QUBO_BF_H */
