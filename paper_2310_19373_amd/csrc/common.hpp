// Shared device/host definitions of the gfx950 QUBO enumeration library.
//
// Bit layout of a state (mask bit i = x_i, 0-based):
//
//   [0, B)              inner bits   j   : enumerated from a per-lane table
//   [B, B+no)           outer bits   o   : walked in reflected Gray-code order
//   [B+no, B+no+L)      lane bits        : one value per wavefront lane
//   [B+no+L, n)         tile bits        : one value per work unit (wave task)
//
// The lane and tile bits together are the fixed prefix of Sec. 3.1: every
// (unit, lane) pair owns an independent sub-walk over the lower bits.  The
// energy of Eq. 1 splits exactly into
//
//   f(x) = C'(lane; j) + T'(o; j) + KE(lane; o)
//     C'  = E_I(j) + X_PI(p, j)      per lane, fixed for the unit  (table)
//     T'  = X_IO(j, o)                uniform over lanes, per step  (table)
//     KE  = E_P(p) + X_PO(p, o) + E_O(o)   per lane, per step (scalar)
//
// where E_A is the objective restricted to the bits of group A and X_AB the
// cross terms between groups A and B.  KE follows the Gray walk with the O(1)
// update of Eq. 2 (Sec. 2.1) restricted to the prefix/outer cross terms; the inner bits
// are never walked, each inner state costs one table addition.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qbf {

constexpr int kWave = 64;
constexpr int kInner = 6;                 // inner bits of the top-k / logZ-forward walks
constexpr int kInnerStates = 1 << kInner;  // 64 table entries per lane
constexpr int kMaxOuter = 12;              // outer bits per work unit (upper bound); keeps
                                           // the per-wave LDS rows below at 20, so that
                                           // four 4-wave blocks (40 KB each) fit per CU
// Per-wave LDS table of the walks, rows of 64 lane entries: rows [0, no) hold
// the outer cross fields c_l, rows kCIRow.. the six inner cross fields, row
// kTileRow the per-unit tile sums exchanged between lanes.
constexpr int kCIRow = kMaxOuter;
constexpr int kTileRow = kMaxOuter + 6;
constexpr int kWaveRows = kMaxOuter + 8;
constexpr int kLaneRec = 24;               // words per lane record of the lane table
constexpr int kBlock = 256;                // threads per block of the walk kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxKPrime = 64;             // candidate list length (one entry per lane)
constexpr int32_t kIntInvalid = 1 << 30;   // table sentinel of the int32 path
constexpr int64_t kIntSumLimit = int64_t(1) << 28;  // int32 path: sum |Q| bound
constexpr int32_t kInt16Limit = 32767;               // int16 screen: inner bound R_I
// float64 walk: with sum |Q| <= 2^50 every intermediate of integer data (table
// values, the running threshold offset, replay keys: at most 5 sum |Q| in
// magnitude) is an integer below 2^53, so the walk is exact
constexpr double kWideSumLimit = 1125899906842624.0;  // 2^50

// input types (mirrors qubo_dtype of include/qubo_bf.h).  F32 walks in float32
// and rescores in float64; I32 walks in int32; F64 and I64 walk in float64
// (five inner bits: 32 table entries per lane), I64 exactly for sum |Q| <= 2^50.
constexpr int kDtF32 = 0;
constexpr int kDtI32 = 1;
constexpr int kDtF64 = 2;
constexpr int kDtI64 = 3;
__host__ __device__ inline bool dt_exact(int dt) { return dt == kDtI32 || dt == kDtI64; }
__host__ __device__ inline bool dt_wide(int dt) { return dt == kDtF64 || dt == kDtI64; }
constexpr int kInnerWide = 5;               // inner bits of the float64 walk

// status codes (mirrors include/qubo_bf.h)
constexpr int32_t kOk = 0;
constexpr int32_t kErrArg = -1;
constexpr int32_t kErrNonfinite = -2;
constexpr int32_t kErrUncertain = -5;
constexpr int32_t kErrRange = -6;
constexpr int32_t kErrOverflow = -7;

// One instance of a (batched) call, written by the planner.
struct Inst {
  int32_t n, B, L, no, tb;  // bit split (see above)
  int32_t kprime;           // candidate list length
  int32_t status;           // device-detected status, 0 = OK
  int32_t seed_fix;         // top bits the threshold seed keeps at the range's first prefix
  int32_t wide;             // int32 Q beyond the int32 walk's range (sum |Q| > 2^28): the
                            // instance's tables are float64 and it walks the half screen
  int32_t pad_;
  int64_t units;            // 2^tb work units
  int64_t unit_begin;       // first global unit index
  int64_t local_off;        // tile value of the first unit (prefix-range solves; else 0)
  int64_t tab_off;          // first step of this instance's tables
  int64_t slot_off;         // first candidate-list slot
  int64_t slot_cap;         // candidate-list slots available
  double sumabs;            // sum |Q_ij| over i <= j
  double big;               // threshold that no state exceeds
  double eps;               // bound on |f32 walk value - exact value| (float path)
  double sign;              // +1, or -1 when the walk runs on -Q
  // half-width screen.  float32 / float64 / int64 Q: table values are scaled
  // by hscale (a power of two putting the inner bound R_I in [2^12, 2^13))
  // and the screen's threshold is raised by hmargin (scaled units).  int32 Q:
  // hscale = 1 when R_I <= 32767 (every screened value is an exact int16),
  // else 0 (the instance keeps the int32 screen).
  double hscale;
  double hmargin;
};

// Work-queue segments: the unit range is cut into kXcds contiguous pieces, one
// per XCD (the dispatcher places workgroup i on XCD i mod 8), so the waves of
// one XCD walk neighbouring units -- mostly the same instances -- and their
// step tables stay in that XCD's L2.  One counter per 128-byte line.
constexpr int kXcds = 8;
struct alignas(128) QueueSeg {
  uint64_t next;  // next unit to hand out
  uint64_t end;   // one past the segment's last unit
};

// Per-call header at the start of the workspace.
struct Header {
  uint64_t total_units;
  int64_t total_steps;
  int64_t total_slots;
  int32_t batch;
  int32_t nmax;
  int32_t waves;          // waves of the persistent walk grid
  int32_t chunk;          // largest run of work units per queue pull
  uint64_t direct_count;  // log-partition: units deferred to the direct-form pass
  QueueSeg seg[kXcds];    // persistent work queue
};

// Per-step uniform data of the outer walk.
// One outer step of a half-width screen (64 bytes, read with scalar loads):
// the inner 6 bits j = b | a << 4 split into 4 + 2, and T'(j) = Tb(b) + Ta(a)
// (T' is linear in the inner bits).  tb[k] holds (Tb(2k), Tb(2k + 1)), ta[a]
// holds (Ta(a), Ta(a + 2)).  float32 / float64 / int64 Q: float16 of the
// scaled values, and tau = hscale * E_O(g(t)) - hmargin; int32 Q: exact int16
// values, and neo = -E_O(g(t)).
struct HalfRow {
  uint32_t tb[8];
  uint32_t ta[2];
  int32_t neo;
  uint32_t pad0;
  double tau;
  uint32_t pad1[2];
};
static_assert(sizeof(HalfRow) == 64, "HalfRow is one 64-byte scalar load");
// The int16 rows sit in the int32 rows' 256-byte step slots (only their first
// 64 bytes used), so that in a batch instances with either screen share one
// table layout; the float32 walk's float16 rows are packed at 64 bytes.
constexpr int kInt16RowStride = 4;  // in HalfRow units

struct StepRec {
  double eo;      // E_O(g(t))
  double h[6];    // H_u(g(t)) = sum_{v in O} S_uv x_v, u < 6
  int32_t neo;    // -E_O(g(t)) for the int32 path
  int32_t pad;
};

struct Slot {
  double key;
  uint64_t mask;
};

// Ordered encoding: a < b  <=>  enc(a) < enc(b) (for non-NaN doubles).
__host__ __device__ inline uint64_t enc_key(double v) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__host__ __device__ inline double dec_key(uint64_t u) {
  uint64_t v = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
  return __builtin_bit_cast(double, v);
}

__host__ __device__ inline uint64_t gray(uint64_t t) { return t ^ (t >> 1); }

// Global-memory pointers.  Pointers taken out of a by-value argument struct are
// generic to the compiler; re-qualifying them lets it use global / scalar loads
// and keep loop bounds loaded from them in SGPRs.
#define QBF_GLOBAL __attribute__((address_space(1)))
template <class T>
using gptr = T QBF_GLOBAL*;
template <class T>
__device__ __forceinline__ gptr<T> gp(T* p) {
  return (gptr<T>)p;
}

}  // namespace qbf
