// C ABI of the library: argument validation (before any HIP call), workspace
// layout, tuning, kernel launch composition on the caller's stream.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "launch.hpp"
#include "qubo_bf.h"

using namespace qbf;

namespace {

thread_local std::string g_err = "";

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(QUBO_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------ tuning

constexpr int kMaxGridWaves = 8192;  // sizing bound of the persistent grid

struct Tuning {
  int single_outer = 12;
  int single_unit = 14;
  int batched_outer = 9;
  int waves_per_cu = 0;  // 0: 16 for the half-screen walks, 12 for the others
  int kprime = 0;
  int chunk_single = 2;
  int chunk_batched = 2;
  int dyn = 1;
  int logz_factored = 1;
  int seed_sweeps = 4;
  int half_screen = 1;
};

int env_int(const char* name, int dflt) {
  const char* s = getenv(name);
  if (!s || !*s) return dflt;
  return atoi(s);
}

Tuning& tuning() {
  static Tuning t = [] {
    Tuning d;
    d.single_outer = env_int("QUBO_BF_SINGLE_OUTER_BITS", d.single_outer);
    d.single_unit = env_int("QUBO_BF_SINGLE_UNIT_BITS", d.single_unit);
    d.batched_outer = env_int("QUBO_BF_BATCHED_OUTER_BITS", d.batched_outer);
    d.waves_per_cu = env_int("QUBO_BF_WAVES_PER_CU", d.waves_per_cu);
    d.kprime = env_int("QUBO_BF_KPRIME", d.kprime);
    d.chunk_single = env_int("QUBO_BF_CHUNK_SINGLE", d.chunk_single);
    d.chunk_batched = env_int("QUBO_BF_CHUNK_BATCHED", d.chunk_batched);
    d.dyn = env_int("QUBO_BF_DYNAMIC_QUEUE", d.dyn);
    d.logz_factored = env_int("QUBO_BF_LOGZ_FACTORED", d.logz_factored);
    d.seed_sweeps = env_int("QUBO_BF_SEED_SWEEPS", d.seed_sweeps);
    d.seed_sweeps = d.seed_sweeps < 0 ? 0 : (d.seed_sweeps > 64 ? 64 : d.seed_sweeps);
    d.half_screen = env_int("QUBO_BF_HALF_SCREEN", d.half_screen);
    return d;
  }();
  return t;
}

int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Candidate list length: k for the exact paths (int32, int64), else at least
// 2k and k + 3 so that the certificate has room above the k-th value (it
// fails only when the k-th to (k + 3)-th candidates lie within the error
// bound of one another).  Every list entry costs replays and insertions while
// the walk's thresholds settle: the 4096-instance k = 1 batch took 3.60 ms
// at K' = 9 (k + 8) and 3.45 ms at K' = 4.
int kprime_for(int k, bool exact) {
  if (exact) return k;
  const int o = tuning().kprime;
  if (o > 0) return clampi(o, 1, kMaxKPrime);
  int kp = 2 * k > k + 3 ? 2 * k : k + 3;
  return kp > kMaxKPrime ? kMaxKPrime : kp;
}

int device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cache[dev]) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cache[dev] = c;
  }
  return cache[dev];
}

// Waves of a persistent grid: the knob, else `auto_per_cu` per CU, never
// more than the kernel keeps resident (`blocks_per_cu` workgroups of
// kWavesPerBlock waves per CU).
int grid_waves(int auto_per_cu, int blocks_per_cu) {
  int per_cu = tuning().waves_per_cu > 0 ? tuning().waves_per_cu : auto_per_cu;
  if (per_cu > blocks_per_cu * kWavesPerBlock) per_cu = blocks_per_cu * kWavesPerBlock;
  long w = (long)device_cus() * clampi(per_cu, 1, 32);
  if (w > kMaxGridWaves) w = kMaxGridWaves;
  return (int)(w - w % kWavesPerBlock);
}

// ------------------------------------------------------------- profiling

struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

struct ProfScope {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  const char* name;
  ProfScope(const char* nm, hipStream_t st) : s(st), name(nm) {
    if (!g_prof_on) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      a = b = nullptr;
      return;
    }
    hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a) return;
    hipEventRecord(b, s);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back({name, a, b});
  }
};

// ------------------------------------------------------------- workspace

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct SplitH {
  int B, L, no, tb;
};

SplitH split_host(int n, const PlanParams& pp) {
  SplitH s;
  s.B = n < pp.inner ? n : pp.inner;
  s.L = (n - s.B) < pp.lane_bits ? (n - s.B) : pp.lane_bits;
  const int rest = n - s.B - s.L;
  s.no = clampi(rest - (pp.ub_min > pp.range_bits ? pp.ub_min : pp.range_bits), 0, pp.no_max);
  s.tb = rest - s.no;
  return s;
}

struct Layout {
  size_t hdr, inst, gthr, flush, qs, ei, tab, rec, eod, eoi, slots, part, lt, umap, etab, tref, dlist, total;
  int64_t umap_cap;
};

constexpr int64_t kUnitMapMax = int64_t(1) << 24;  // unit -> instance map entries

// Worst case over n <= nmax (steps and units grow with n).
Layout make_layout(int batch, int nmax, const PlanParams& pp, int64_t part_per_unit, int64_t part_per_inst,
                   bool exp_tables = false) {
  const SplitH s = split_host(nmax, pp);
  const int64_t steps = int64_t(1) << s.no;
  const int64_t units = int64_t(1) << s.tb;
  const int64_t slots = units < kMaxGridWaves ? units : kMaxGridWaves;
  const int width = 1 << pp.inner;
  Layout L;
  size_t o = 0;
  L.hdr = o;
  o += al(sizeof(Header));
  L.inst = o;
  o += al(sizeof(Inst) * (size_t)batch);
  L.gthr = o;
  o += al(8 * (size_t)batch);
  L.flush = o;
  o += al(4 * (size_t)batch);
  L.qs = o;
  o += al(8 * (size_t)batch * nmax * nmax);
  L.ei = o;
  o += al(8 * (size_t)batch * 64);
  L.tab = o;
  o += al((size_t)(pp.tab_elem > 0 ? pp.tab_elem : 4) * batch * steps * width);
  L.rec = o;
  o += al(sizeof(StepRec) * (size_t)batch * steps);
  L.eod = o;
  o += al(8 * (size_t)batch * steps);
  L.eoi = o;
  o += al(4 * (size_t)batch * steps);
  L.slots = o;
  o += al(sizeof(Slot) * (size_t)batch * slots * pp.kprime);
  L.part = o;
  o += al(8 * (size_t)batch * (units * part_per_unit + part_per_inst));
  L.lt = o;
  o += al(8 * (size_t)batch * 64 * kLaneRec);
  L.umap = o;
  L.umap_cap = (batch > 1 && (int64_t)batch * units <= kUnitMapMax) ? (int64_t)batch * units : 0;
  o += al(4 * (size_t)L.umap_cap);
  L.etab = L.tref = L.dlist = 0;
  if (exp_tables) {
    L.etab = o;
    o += al(4 * (size_t)batch * steps * width);
    L.tref = o;
    o += al(8 * (size_t)batch * steps);
    L.dlist = o;
    o += al(8 * (size_t)batch * units);
  }
  L.total = o;
  return L;
}

Views make_views(void* ws, const Layout& L, int batch, int nmax) {
  char* p = (char*)ws;
  Views v;
  v.hdr = (Header*)(p + L.hdr);
  v.inst = (Inst*)(p + L.inst);
  v.gthr = (uint64_t*)(p + L.gthr);
  v.flushcnt = (uint32_t*)(p + L.flush);
  v.qs = p + L.qs;
  v.ei = p + L.ei;
  v.tab = p + L.tab;
  v.rec = (StepRec*)(p + L.rec);
  v.eod = (double*)(p + L.eod);
  v.eoi = (int32_t*)(p + L.eoi);
  v.slots = (Slot*)(p + L.slots);
  v.part = (double*)(p + L.part);
  v.lt = p + L.lt;
  v.umap = L.umap_cap > 0 ? (uint32_t*)(p + L.umap) : nullptr;
  v.umap_cap = L.umap_cap;
  v.etab = L.etab ? (void*)(p + L.etab) : nullptr;
  v.tref = L.tref ? (double*)(p + L.tref) : nullptr;
  v.dlist = L.dlist ? (uint64_t*)(p + L.dlist) : nullptr;
  v.lanepart = nullptr;
  v.factor = L.etab ? clampi(tuning().logz_factored, 0, 2) : 0;
  v.seed_sweeps = tuning().seed_sweeps;
  v.batch = batch;
  v.nmax = nmax;
  v.dyn = tuning().dyn != 0;
  v.h16 = 0;
  return v;
}

PlanParams single_params(int kp, int n, int dt) {
  const Tuning& t = tuning();
  PlanParams pp{};
  pp.no_max = clampi(t.single_outer, 0, kMaxOuter);
  // unit bits reserved before outer bits are granted: the knob, lowered for
  // mid-size n so that units keep a useful number of Gray steps, and raised
  // from n = 33 so that a grid of ~3000 waves gets several units each.
  // Measured with the float32 walk's half screen: n=24 -> 8, n=28 -> 10,
  // n=30..32 -> 11, n=33..36 -> 14 (n=38 is flat; n=40 reaches 16 unit bits
  // either way).  The walks with a costlier step (the float32 and int32
  // screens) do best with one bit fewer: n=32 -> 12, n=34 -> 13.  int32 Q
  // under the half screen (the int16 screen where its values fit) gains from
  // more, shorter units from n = 32: 12 up to n = 35 (n=32: 0.31 ms per call
  // against 0.35 at 11; n=33: 0.42 against 0.50 at 14), 13 from n = 36.
  const bool half = t.half_screen > 0;
  const int mid_cap = half ? 11 : 12, big = half ? 14 : 13;
  int want = n >= 33 ? big : (n - 18 > mid_cap ? mid_cap : (n - 18 > 8 ? n - 18 : 8));
  if (half && dt == kDtI32 && n >= 32) want = n >= 36 ? 13 : 12;
  pp.ub_min = clampi(t.single_unit < want ? t.single_unit : want, 0, 62);
  pp.inner = kInner;
  pp.kprime = kp;
  pp.waves = kMaxGridWaves;  // replaced by the real grid at launch
  pp.lane_bits = 6;
  pp.chunk_cap = clampi(t.chunk_single, 1, 1 << 20);
  return pp;
}

PlanParams batched_params(int kp) {
  const Tuning& t = tuning();
  PlanParams pp{};
  pp.no_max = clampi(t.batched_outer, 0, kMaxOuter);
  pp.ub_min = 0;
  pp.inner = kInner;
  pp.kprime = kp;
  pp.waves = kMaxGridWaves;
  pp.lane_bits = 6;
  pp.chunk_cap = clampi(t.chunk_batched, 1, 1 << 20);
  return pp;
}

PlanParams grad_params() {
  PlanParams pp{};
  pp.no_max = 8;
  pp.ub_min = 0;
  pp.inner = 5;
  pp.kprime = 1;
  pp.waves = kMaxGridWaves;
  pp.lane_bits = 6;
  pp.chunk_cap = clampi(tuning().chunk_batched, 1, 1 << 20);
  return pp;
}

// Sampling: the forward's plan with at most 8 outer bits (a lane's block
// weights by outer value fit in LDS); per unit 1 + 64 + 1 doubles of
// partial results (unit sum, lane sums, running sum).
PlanParams sample_params() {
  PlanParams pp = batched_params(1);
  pp.no_max = 8;
  return pp;
}
constexpr int64_t kSamplePart = 66;

int logz_npairs(int nmax) { return nmax * (nmax + 1) / 2; }

bool valid_dtype(qubo_dtype dt) { return dt == QUBO_F32 || dt == QUBO_I32 || dt == QUBO_F64 || dt == QUBO_I64; }

int check_k(int k, bool exact) {
  if (k < 1 || k > kMaxKPrime) return fail(QUBO_ERR_INVALID_ARG, "k=%d outside [1, %d]", k, kMaxKPrime);
  if (!exact && k > kMaxKPrime - 8)
    return fail(QUBO_ERR_INVALID_ARG, "k=%d outside [1, %d] for float Q", k, kMaxKPrime - 8);
  return QUBO_OK;
}

// The float64 walk (float64 and int64 Q) takes five inner bits and 8-byte
// table entries.
PlanParams with_dt(PlanParams pp, qubo_dtype dt) {
  if (dt_wide(dt) && tuning().half_screen <= 0) {
    pp.inner = kInnerWide;
    pp.tab_elem = 8;
  } else {
    pp.tab_elem = 4;  // float32 / int32 rows, or the half screen's (float64 and int64 Q too)
  }
  return pp;
}

// Enqueue plan -> prep -> tables -> walk -> finalize for a top-k call.
int run_topk(const Views& v0, const void* Q, int64_t ldq, int64_t stride, const int32_t* ns, int n_single,
             int dt, int k, PlanParams pp, int64_t units_hint, int64_t steps_hint, void* energies,
             uint64_t* masks, int32_t* status, int fin_waves, hipStream_t s, bool prof = true) {
  Views v = v0;
  // float32, float64 and int64 Q screen blocks in packed float16 (the step
  // tables then hold HalfRow rows, 64 of the 256 bytes a float32 row takes);
  // int32 instances screen in exact int16 where their inner bound allows
  // (HalfRow rows in the int32 rows' 256-byte slots, so both kinds share one
  // layout in a batch)
  const bool half = tuning().half_screen > 0 && pp.inner == kInner;
  v.h16 = half ? 1 : 0;
  // the half-screen walk (float32, float64 and int64 Q) runs 4 waves per SIMD
  int waves = grid_waves(v.h16 ? 16 : 12, walk_topk_blocks_per_cu(dt, v.h16));
  if (units_hint > 0 && units_hint < waves) {
    waves = (int)units_hint;
    waves += (kWavesPerBlock - waves % kWavesPerBlock) % kWavesPerBlock;
  }
  pp.waves = waves;
  HIPCHK(launch_plan(v, ns, n_single, nullptr, pp, s));
  HIPCHK(launch_prep_inst(v, Q, ldq, stride, dt, pp.inner, s));
  // single small instances: the walk is shorter than the seed's latency
  // (measured crossover: n = 15 for float Q, whose longer K' lists start colder,
  // n = 19 for integer Q).  A prefix-range solve seeds inside its range (the
  // planner's seed_fix).
  const bool seed = ns != nullptr || n_single >= (dt_exact(dt) ? 19 : 15);
  HIPCHK(launch_prep_walk(v, dt, pp.inner, steps_hint, seed, s));
  if (prof) {
    ProfScope ps("walk_topk", s);
    HIPCHK(launch_walk_topk(v, dt, waves, s));
  } else {
    HIPCHK(launch_walk_topk(v, dt, waves, s));
  }
  HIPCHK(launch_finalize_topk(v, Q, ldq, stride, dt, k, energies, masks, status, fin_waves, s));
  return QUBO_OK;
}

// ------------------------------------------------- no-allocation solves
//
// Workspace of qubo_bf_solve_noalloc: a library-owned device array.  Every GPU
// the library runs on holds its own copy, at its own address, until the
// process ends.  In host code the array's name is only a stand-in for the
// device symbol, never a device address: the address comes from
// hipGetSymbolAddress, once per device with that device current, and host
// code uses only that pointer (kernel arguments, views of the workspace).
constexpr size_t kScratchBytes = QUBO_NOALLOC_SCRATCH_BYTES;  // covers every single solve, n <= 63, k <= 64
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up on the first call on
// that device.  Returns QUBO_OK or QUBO_ERR_HIP.
int scratch_ptr(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(QUBO_ERR_HIP, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(QUBO_ERR_HIP, "hipGetSymbolAddress(scratch) returned null on device %d", dev);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QUBO_OK;
}

}  // namespace

extern "C" {

const char* qubo_last_error(void) { return g_err.c_str(); }

const char* qubo_version(void) { return "qubo_bf 0.1.0 gfx950"; }

int qubo_bf_set_tuning(int knob, int value) {
  Tuning& t = tuning();
  const Tuning d;
  switch (knob) {
    case QUBO_TUNE_SINGLE_OUTER_BITS: t.single_outer = value > 0 ? clampi(value, 0, kMaxOuter) : d.single_outer; break;
    case QUBO_TUNE_SINGLE_UNIT_BITS: t.single_unit = value > 0 ? clampi(value, 0, 62) : d.single_unit; break;
    case QUBO_TUNE_BATCHED_OUTER_BITS: t.batched_outer = value > 0 ? clampi(value, 0, kMaxOuter) : d.batched_outer; break;
    case QUBO_TUNE_WAVES_PER_CU: t.waves_per_cu = value > 0 ? clampi(value, 1, 32) : d.waves_per_cu; break;
    case QUBO_TUNE_KPRIME: t.kprime = value > 0 ? clampi(value, 1, kMaxKPrime) : 0; break;
    case QUBO_TUNE_CHUNK_SINGLE: t.chunk_single = value > 0 ? value : d.chunk_single; break;
    case QUBO_TUNE_CHUNK_BATCHED: t.chunk_batched = value > 0 ? value : d.chunk_batched; break;
    case QUBO_TUNE_DYNAMIC_QUEUE: t.dyn = value > 0 ? 1 : (value < 0 ? 0 : d.dyn); break;
    case QUBO_TUNE_LOGZ_FACTORED: t.logz_factored = value > 0 ? clampi(value, 1, 2) : (value < 0 ? 0 : d.logz_factored); break;
    case QUBO_TUNE_SEED_SWEEPS: t.seed_sweeps = value > 0 ? clampi(value, 1, 64) : (value < 0 ? 0 : d.seed_sweeps); break;
    case QUBO_TUNE_HALF_SCREEN: t.half_screen = value > 0 ? 1 : (value < 0 ? 0 : d.half_screen); break;
    default: return fail(QUBO_ERR_INVALID_ARG, "unknown tuning knob %d", knob);
  }
  return QUBO_OK;
}

int qubo_bf_get_tuning(int knob) {
  const Tuning& t = tuning();
  switch (knob) {
    case QUBO_TUNE_SINGLE_OUTER_BITS: return t.single_outer;
    case QUBO_TUNE_SINGLE_UNIT_BITS: return t.single_unit;
    case QUBO_TUNE_BATCHED_OUTER_BITS: return t.batched_outer;
    case QUBO_TUNE_WAVES_PER_CU: return t.waves_per_cu;
    case QUBO_TUNE_KPRIME: return t.kprime;
    case QUBO_TUNE_CHUNK_SINGLE: return t.chunk_single;
    case QUBO_TUNE_CHUNK_BATCHED: return t.chunk_batched;
    case QUBO_TUNE_DYNAMIC_QUEUE: return t.dyn;
    case QUBO_TUNE_LOGZ_FACTORED: return t.logz_factored;
    case QUBO_TUNE_SEED_SWEEPS: return t.seed_sweeps;
    case QUBO_TUNE_HALF_SCREEN: return t.half_screen;
    default: return fail(QUBO_ERR_INVALID_ARG, "unknown tuning knob %d", knob);
  }
}

int qubo_prof_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = on != 0;
  return QUBO_OK;
}

int qubo_prof_collect(const char* name, double* total_ms, int64_t* launches) {
  if (!name || !total_ms || !launches) return fail(QUBO_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> g(g_prof_mu);
  double ms = 0.0;
  int64_t cnt = 0;
  std::vector<ProfRec> keep;
  for (auto& r : g_prof) {
    if (r.name != name) {
      keep.push_back(r);
      continue;
    }
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
      return fail(QUBO_ERR_HIP, "event timing failed");
    ms += t;
    ++cnt;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  g_prof.swap(keep);
  *total_ms = ms;
  *launches = cnt;
  return QUBO_OK;
}

// Candidate list length of a single solve: kprime (k .. 64) when given,
// else the default for k; -1 (with the error set) for a bad kprime.
static int kprime_arg(int k, int kprime, bool exact) {
  if (kprime == 0) return kprime_for(k, exact);
  if (kprime < k || kprime > kMaxKPrime)
    return fail(QUBO_ERR_INVALID_ARG, "kprime=%d outside [k=%d, %d]", kprime, k, kMaxKPrime), -1;
  return kprime;
}

size_t qubo_bf_workspace_size_kp(int n, int k, int kprime, qubo_dtype dt) {
  if (n < 1 || n > 63 || !valid_dtype(dt)) return 0;
  const bool exact = dt_exact(dt);
  if (check_k(k, exact) != QUBO_OK) return 0;
  const int kp = kprime_arg(k, kprime, exact);
  if (kp < 0) return 0;
  return make_layout(1, n, with_dt(single_params(kp, n, dt), dt), 0, 0).total;
}

size_t qubo_bf_workspace_size(int n, int k, qubo_dtype dt) { return qubo_bf_workspace_size_kp(n, k, 0, dt); }

int qubo_bf_solve(const void* Q, int n, int64_t ldq, qubo_dtype dt, int k, void* energies, uint64_t* masks,
                  int32_t* status, void* ws, size_t ws_bytes, void* hip_stream) {
  return qubo_bf_solve_kp(Q, n, ldq, dt, k, 0, energies, masks, status, ws, ws_bytes, hip_stream);
}

int qubo_bf_solve_kp(const void* Q, int n, int64_t ldq, qubo_dtype dt, int k, int kprime, void* energies,
                     uint64_t* masks, int32_t* status, void* ws, size_t ws_bytes, void* hip_stream) {
  if (!Q || !energies || !masks || !status || !ws) return fail(QUBO_ERR_INVALID_ARG, "null pointer argument");
  if (n < 1 || n > 63) return fail(QUBO_ERR_INVALID_ARG, "n=%d outside [1, 63]", n);
  if (ldq < n) return fail(QUBO_ERR_INVALID_ARG, "ldq=%lld < n=%d", (long long)ldq, n);
  if (!valid_dtype(dt)) return fail(QUBO_ERR_INVALID_ARG, "unknown dtype %d", (int)dt);
  const bool exact = dt_exact(dt);
  if (int rc = check_k(k, exact)) return rc;
  const int kp = kprime_arg(k, kprime, exact);
  if (kp < 0) return QUBO_ERR_INVALID_ARG;
  const PlanParams pp = with_dt(single_params(kp, n, dt), dt);
  const Layout L = make_layout(1, n, pp, 0, 0);
  if (ws_bytes < L.total)
    return fail(QUBO_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, L.total);
  const Views v = make_views(ws, L, 1, n);
  const SplitH sh = split_host(n, pp);
  return run_topk(v, Q, ldq, 0, nullptr, n, dt, k, pp, int64_t(1) << sh.tb, int64_t(1) << sh.no, energies,
                  masks, status, 16, (hipStream_t)hip_stream);
}

int qubo_bf_solve_noalloc(const void* Q, int n, int64_t ldq, qubo_dtype dt, int k, void* energies,
                          uint64_t* masks, int32_t* status, void* hip_stream) {
  if (!Q || !energies || !masks || !status) return fail(QUBO_ERR_INVALID_ARG, "null pointer argument");
  if (n < 1 || n > 63) return fail(QUBO_ERR_INVALID_ARG, "n=%d outside [1, 63]", n);
  if (ldq < n) return fail(QUBO_ERR_INVALID_ARG, "ldq=%lld < n=%d", (long long)ldq, n);
  if (!valid_dtype(dt)) return fail(QUBO_ERR_INVALID_ARG, "unknown dtype %d", (int)dt);
  const bool exact = dt_exact(dt);
  if (int rc = check_k(k, exact)) return rc;
  const int kp = kprime_for(k, exact);
  const PlanParams pp = with_dt(single_params(kp, n, dt), dt);
  const Layout L = make_layout(1, n, pp, 0, 0);
  if (L.total > kScratchBytes)
    return fail(QUBO_ERR_WORKSPACE, "n=%d, k=%d needs a %zu-byte workspace, above the %zu-byte static scratch", n, k,
                L.total, kScratchBytes);
  void* ws = nullptr;
  if (int rc = scratch_ptr(&ws)) return rc;
  const Views v = make_views(ws, L, 1, n);
  const SplitH sh = split_host(n, pp);
  return run_topk(v, Q, ldq, 0, nullptr, n, dt, k, pp, int64_t(1) << sh.tb, int64_t(1) << sh.no, energies,
                  masks, status, 16, (hipStream_t)hip_stream, false);
}

static int check_range(int n, int p_bits, int64_t p_begin, int64_t p_end) {
  if (p_bits < 1 || p_bits > n - 12)
    return fail(QUBO_ERR_INVALID_ARG, "p_bits=%d outside [1, n - 12] for n=%d", p_bits, n);
  if (p_begin < 0 || p_end <= p_begin || p_end > (int64_t(1) << p_bits))
    return fail(QUBO_ERR_INVALID_ARG, "prefix range [%lld, %lld) outside [0, 2^%d)", (long long)p_begin,
                (long long)p_end, p_bits);
  return QUBO_OK;
}

static PlanParams range_params(int kp, int n, int dt, int p_bits, int64_t p_begin, int64_t p_end) {
  PlanParams pp = single_params(kp, n, dt);
  pp.range_bits = p_bits;
  pp.range_begin = p_begin;
  pp.range_end = p_end;
  return pp;
}

size_t qubo_bf_range_workspace_size(int n, int k, qubo_dtype dt, int p_bits) {
  if (n < 1 || n > 63 || !valid_dtype(dt) || p_bits < 1 || p_bits > n - 12) return 0;
  const bool exact = dt_exact(dt);
  if (check_k(k, exact) != QUBO_OK) return 0;
  return make_layout(1, n, with_dt(range_params(kprime_for(k, exact), n, dt, p_bits, 0, 1), dt), 0, 0).total;
}

int qubo_bf_solve_range(const void* Q, int n, int64_t ldq, qubo_dtype dt, int k, int p_bits, int64_t p_begin,
                        int64_t p_end, void* energies, uint64_t* masks, int32_t* status, void* ws,
                        size_t ws_bytes, void* hip_stream) {
  if (!Q || !energies || !masks || !status || !ws) return fail(QUBO_ERR_INVALID_ARG, "null pointer argument");
  if (n < 1 || n > 63) return fail(QUBO_ERR_INVALID_ARG, "n=%d outside [1, 63]", n);
  if (ldq < n) return fail(QUBO_ERR_INVALID_ARG, "ldq=%lld < n=%d", (long long)ldq, n);
  if (!valid_dtype(dt)) return fail(QUBO_ERR_INVALID_ARG, "unknown dtype %d", (int)dt);
  const bool exact = dt_exact(dt);
  if (check_k(k, exact) != QUBO_OK) return QUBO_ERR_INVALID_ARG;
  if (check_range(n, p_bits, p_begin, p_end) != QUBO_OK) return QUBO_ERR_INVALID_ARG;
  const int kp = kprime_for(k, exact);
  const PlanParams pp = with_dt(range_params(kp, n, dt, p_bits, p_begin, p_end), dt);
  const Layout L = make_layout(1, n, pp, 0, 0);
  if (ws_bytes < L.total) return fail(QUBO_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, L.total);
  const Views v = make_views(ws, L, 1, n);
  const SplitH sh = split_host(n, pp);
  const int64_t units = (p_end - p_begin) << (sh.tb - p_bits);
  return run_topk(v, Q, ldq, 0, nullptr, n, dt, k, pp, units, int64_t(1) << sh.no, energies, masks, status,
                  16, (hipStream_t)hip_stream);
}

int qubo_bf_merge_topk(int count, int k_in, const void* energies_in, const uint64_t* masks_in, qubo_dtype dt,
                       int k, void* energies, uint64_t* masks, void* hip_stream) {
  if (!energies_in || !masks_in || !energies || !masks) return fail(QUBO_ERR_INVALID_ARG, "null pointer argument");
  if (count < 1 || k_in < 1 || k < 1 || k > kMaxKPrime)
    return fail(QUBO_ERR_INVALID_ARG, "count=%d, k_in=%d, k=%d: need count, k_in >= 1 and k in [1, %d]", count,
                k_in, k, kMaxKPrime);
  if (!valid_dtype(dt)) return fail(QUBO_ERR_INVALID_ARG, "unknown dtype %d", (int)dt);
  HIPCHK(launch_merge_topk(count, k_in, energies_in, masks_in, dt, k, energies, masks,
                           (hipStream_t)hip_stream));
  return QUBO_OK;
}

size_t qubo_bf_batched_workspace_size(int batch, int nmax, int k, qubo_dtype dt) {
  if (batch < 1 || nmax < 1 || nmax > 40 || !valid_dtype(dt)) return 0;
  const bool exact = dt_exact(dt);
  if (check_k(k, exact) != QUBO_OK) return 0;
  return make_layout(batch, nmax, with_dt(batched_params(kprime_for(k, exact)), dt), 0, 0).total;
}

int qubo_bf_solve_batched(int batch, const void* Q, int nmax, const int32_t* ns, qubo_dtype dt, int k,
                          void* energies, uint64_t* masks, int32_t* status, void* ws, size_t ws_bytes,
                          void* hip_stream) {
  if (!Q || !ns || !energies || !masks || !status || !ws) return fail(QUBO_ERR_INVALID_ARG, "null pointer argument");
  if (batch < 1) return fail(QUBO_ERR_INVALID_ARG, "batch=%d < 1", batch);
  if (nmax < 1 || nmax > 40) return fail(QUBO_ERR_INVALID_ARG, "nmax=%d outside [1, 40]", nmax);
  if (!valid_dtype(dt)) return fail(QUBO_ERR_INVALID_ARG, "unknown dtype %d", (int)dt);
  const bool exact = dt_exact(dt);
  if (int rc = check_k(k, exact)) return rc;
  const int kp = kprime_for(k, exact);
  const PlanParams pp = with_dt(batched_params(kp), dt);
  const Layout L = make_layout(batch, nmax, pp, 0, 0);
  if (ws_bytes < L.total)
    return fail(QUBO_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, L.total);
  const Views v = make_views(ws, L, batch, nmax);
  const SplitH sh = split_host(nmax, pp);
  const int64_t steps_bound = (int64_t)batch << sh.no;
  return run_topk(v, Q, nmax, (int64_t)nmax * nmax, ns, 0, dt, k, pp, 0, steps_bound, energies, masks,
                  status, 1, (hipStream_t)hip_stream);
}

size_t qubo_logz_workspace_size(int batch, int nmax) {
  if (batch < 1 || nmax < 1 || nmax > 32) return 0;
  const size_t f = make_layout(batch, nmax, batched_params(1), 1, 0, true).total;
  const size_t g = make_layout(batch, nmax, grad_params(), logz_npairs(nmax), 0, true).total;
  return f > g ? f : g;
}

int qubo_logz_fwd(int batch, const float* Q, int nmax, const int32_t* ns, const float* beta, double* logz,
                  int32_t* status, void* ws, size_t ws_bytes, void* hip_stream) {
  if (!Q || !ns || !beta || !logz || !status || !ws) return fail(QUBO_ERR_INVALID_ARG, "null pointer argument");
  if (batch < 1) return fail(QUBO_ERR_INVALID_ARG, "batch=%d < 1", batch);
  if (nmax < 1 || nmax > 32) return fail(QUBO_ERR_INVALID_ARG, "nmax=%d outside [1, 32]", nmax);
  const size_t need = qubo_logz_workspace_size(batch, nmax);
  if (ws_bytes < need) return fail(QUBO_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
  PlanParams pp = batched_params(1);
  const Layout L = make_layout(batch, nmax, pp, 1, 0, true);
  const Views v = make_views(ws, L, batch, nmax);
  hipStream_t s = (hipStream_t)hip_stream;
  const int waves = grid_waves(12, walk_exp_blocks_per_cu());
  pp.waves = waves;
  const SplitH sh = split_host(nmax, pp);
  const int64_t steps_bound = (int64_t)batch << sh.no;
  HIPCHK(launch_plan(v, ns, 0, beta, pp, s));
  HIPCHK(launch_prep_inst(v, Q, nmax, (int64_t)nmax * nmax, kDtF32, kInner, s));
  HIPCHK(launch_prep_walk(v, kDtF32, kInner, steps_bound, false, s));
  HIPCHK(launch_prep_exp_tables(v, beta, kInner, steps_bound, s));
  {
    ProfScope ps("walk_exp", s);
    HIPCHK(launch_walk_exp(v, beta, waves, s));
  }
  HIPCHK(launch_finalize_logz(v, beta, logz, status, s));
  return QUBO_OK;
}

// Adjoint walk shared by qubo_logz_bwd and qubo_logz_moments.
static int run_moment_walk(int batch, const float* Q, int nmax, const int32_t* ns, const float* beta,
                           const double* logz, const float* grad_logz, float* grad_Q, float* grad_beta,
                           double* moments, double* mean, int32_t* status, void* ws, size_t ws_bytes,
                           void* hip_stream) {
  if (batch < 1) return fail(QUBO_ERR_INVALID_ARG, "batch=%d < 1", batch);
  if (nmax < 1 || nmax > 32) return fail(QUBO_ERR_INVALID_ARG, "nmax=%d outside [1, 32]", nmax);
  const size_t need = qubo_logz_workspace_size(batch, nmax);
  if (ws_bytes < need) return fail(QUBO_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
  PlanParams pp = grad_params();
  const int np = logz_npairs(nmax);
  const Layout L = make_layout(batch, nmax, pp, np, 0, true);
  const Views v = make_views(ws, L, batch, nmax);
  hipStream_t s = (hipStream_t)hip_stream;
  const int waves = grid_waves(12, walk_grad_blocks_per_cu());
  pp.waves = waves;
  const SplitH sh = split_host(nmax, pp);
  const int64_t steps_bound = (int64_t)batch << sh.no;
  HIPCHK(launch_plan(v, ns, 0, beta, pp, s));
  HIPCHK(launch_prep_inst(v, Q, nmax, (int64_t)nmax * nmax, kDtF32, pp.inner, s));
  HIPCHK(launch_prep_walk(v, kDtF32, pp.inner, steps_bound, false, s));
  HIPCHK(launch_prep_exp_tables(v, beta, pp.inner, steps_bound, s));
  {
    ProfScope ps("walk_grad", s);
    HIPCHK(launch_walk_grad(v, beta, logz, waves, np, s));
  }
  HIPCHK(launch_finalize_grad(v, Q, beta, grad_logz, grad_Q, grad_beta, moments, mean, status, np, s));
  return QUBO_OK;
}

int qubo_logz_bwd(int batch, const float* Q, int nmax, const int32_t* ns, const float* beta, const double* logz,
                  const float* grad_logz, float* grad_Q, float* grad_beta, int32_t* status, void* ws,
                  size_t ws_bytes, void* hip_stream) {
  if (!Q || !ns || !beta || !logz || !grad_logz || !grad_Q || !status || !ws)
    return fail(QUBO_ERR_INVALID_ARG, "null pointer argument");
  return run_moment_walk(batch, Q, nmax, ns, beta, logz, grad_logz, grad_Q, grad_beta, nullptr, nullptr, status,
                         ws, ws_bytes, hip_stream);
}

int qubo_logz_moments(int batch, const float* Q, int nmax, const int32_t* ns, const float* beta,
                      const double* logz, double* moments, double* mean_energy, int32_t* status, void* ws,
                      size_t ws_bytes, void* hip_stream) {
  if (!Q || !ns || !beta || !logz || !moments || !status || !ws)
    return fail(QUBO_ERR_INVALID_ARG, "null pointer argument");
  return run_moment_walk(batch, Q, nmax, ns, beta, logz, nullptr, nullptr, nullptr, moments, mean_energy, status,
                         ws, ws_bytes, hip_stream);
}

size_t qubo_logz_sample_workspace_size(int batch, int nmax) {
  if (batch < 1 || nmax < 1 || nmax > 32) return 0;
  return make_layout(batch, nmax, sample_params(), kSamplePart, 0, true).total;
}

int qubo_logz_sample(int batch, const float* Q, int nmax, const int32_t* ns, const float* beta, int nsamples,
                     const double* u, uint64_t* masks, double* logz, int32_t* status, void* ws, size_t ws_bytes,
                     void* hip_stream) {
  if (!Q || !ns || !beta || !u || !masks || !logz || !status || !ws)
    return fail(QUBO_ERR_INVALID_ARG, "null pointer argument");
  if (batch < 1) return fail(QUBO_ERR_INVALID_ARG, "batch=%d < 1", batch);
  if (nmax < 1 || nmax > 32) return fail(QUBO_ERR_INVALID_ARG, "nmax=%d outside [1, 32]", nmax);
  if (nsamples < 1) return fail(QUBO_ERR_INVALID_ARG, "nsamples=%d < 1", nsamples);
  const size_t need = qubo_logz_sample_workspace_size(batch, nmax);
  if (ws_bytes < need) return fail(QUBO_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
  PlanParams pp = sample_params();
  const Layout L = make_layout(batch, nmax, pp, kSamplePart, 0, true);
  Views v = make_views(ws, L, batch, nmax);
  const SplitH sh = split_host(nmax, pp);
  const int64_t units_bound = (int64_t)batch << sh.tb;
  v.lanepart = v.part + units_bound;
  double* cum = v.part + units_bound * (kSamplePart - 1);
  hipStream_t s = (hipStream_t)hip_stream;
  const int waves = grid_waves(12, walk_exp_blocks_per_cu());
  pp.waves = waves;
  const int64_t steps_bound = (int64_t)batch << sh.no;
  HIPCHK(launch_plan(v, ns, 0, beta, pp, s));
  HIPCHK(launch_prep_inst(v, Q, nmax, (int64_t)nmax * nmax, kDtF32, kInner, s));
  HIPCHK(launch_prep_walk(v, kDtF32, kInner, steps_bound, false, s));
  HIPCHK(launch_prep_exp_tables(v, beta, kInner, steps_bound, s));
  HIPCHK(launch_walk_exp(v, beta, waves, s));
  HIPCHK(launch_finalize_logz(v, beta, logz, status, s));
  HIPCHK(launch_sample(v, beta, logz, cum, nsamples, u, masks, waves, s));
  return QUBO_OK;
}

}  // extern "C"
