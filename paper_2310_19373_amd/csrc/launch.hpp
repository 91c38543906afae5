// Host-side launchers of the kernels (one translation unit each); the C ABI
// in abi.hip composes them on the caller's stream.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace qbf {

// Device views of one call's workspace.
struct Views {
  Header* hdr;
  Inst* inst;
  uint64_t* gthr;
  uint32_t* flushcnt;
  void* qs;        // [batch][nmax][nmax] double (float walks) or int64 (int32 walk)
  void* ei;        // [batch][64] double or int64
  void* tab;       // [total_steps][2^inner] float, int32 or double, row-broadcast layout
  StepRec* rec;    // [total_steps]
  double* eod;     // [total_steps] E_O(g(t)), dense (float path)
  int32_t* eoi;    // [total_steps] -E_O(g(t)), dense (int path)
  Slot* slots;     // [total_slots][kprime]
  double* part;    // per-unit partial sums (logZ forward) / per-wave moments (gradient)
  void* lt;        // [batch][64][kLaneRec] lane table (double or int64), see launch_prep_walk
  uint32_t* umap;  // [umap_cap] work unit -> instance, or null (binary search)
  void* etab;      // log-partition: factor table b(t, j), layout of tab (float), or null
  double* tref;    // log-partition: min_j T'(g(t); j) + E_O(g(t)) per step, or null
  int factor;      // log-partition: 0 direct form only; 1 factored form (the adjoint nested
                   // where the factor rows allow); 2 factored form, per-state products
  uint64_t* dlist; // log-partition: units deferred to the direct-form pass, or null
  double* lanepart;  // sampling: per unit and lane, log2 of the lane's sum (forward walk output), or null
  int seed_sweeps; // steepest descents per instance of the threshold seed (0: no seeding)
  int64_t umap_cap;
  int batch, nmax;
  int dyn;         // 1: atomic work queue, 0: static round-robin of chunks
  int h16;         // float32 top-k walk: 1 = half-precision screen (tab holds HalfRow rows)
};

struct PlanParams {
  int no_max;    // outer bits per unit, upper bound
  int ub_min;    // unit bits wanted before outer bits are granted
  int inner;     // inner bits of the walk (6 for top-k and logZ forward, 5 for the gradient)
  int kprime;    // candidate list length
  int waves;     // waves of the persistent walk grid
  int lane_bits; // lane bits wanted (6 normally)
  int chunk_cap; // largest queue chunk (the planner picks <= this from the unit count)
  // prefix-range solve (single instance): only masks whose top range_bits bits
  // lie in [range_begin, range_end); range_bits = 0: every mask
  int range_bits;
  int64_t range_begin, range_end;
  int tab_elem;  // bytes per step-table entry (0: 4)
};

// plan: bit split, unit/table/slot offsets, counters.  ns == nullptr: one
// instance of size n_single.  beta (may be null): instance sign = sign(beta).
hipError_t launch_plan(const Views& v, const int32_t* ns, int n_single, const float* beta,
                       const PlanParams& pp, hipStream_t s);
// prep: symmetric Q, sums, E_I table, float/int validation.
// dt: one of kDt* (the log-partition paths pass kDtF32).
hipError_t launch_prep_inst(const Views& v, const void* q, int64_t ldq, int64_t inst_stride, int dt,
                            int inner, hipStream_t s);
// the per-instance inputs of the walks, after prep_inst, in one launch: the
// lane table (contributions of the lane bits to E_P and to the inner / outer
// cross fields, for each of the 64 lane values), the per-step tables of the
// outer walk and, when `seed`, the a-priori threshold from a greedy descent.
// steps_bound >= total steps of the plan (sizes the grid only: the kernel
// reads the exact counts from the instances).
hipError_t launch_prep_walk(const Views& v, int dt, int inner, int64_t steps_bound, bool seed, hipStream_t s);
// persistent top-k walk.
hipError_t launch_walk_topk(const Views& v, int dt, int waves, hipStream_t s);
// Workgroups of a persistent walk that one compute unit holds at once (the
// occupancy of the kernel launch_walk_topk / launch_walk_exp /
// launch_walk_grad picks).  A persistent grid never exceeds it: a workgroup
// that is not resident from the start would only begin once others have
// finished, and a wave's first run of units is assigned to it statically.
int walk_topk_blocks_per_cu(int dt, int h16);
int walk_exp_blocks_per_cu();
int walk_grad_blocks_per_cu();
// merge candidate lists, rescore in float64 / int64, certificate, outputs.
hipError_t launch_finalize_topk(const Views& v, const void* q, int64_t ldq, int64_t inst_stride, int dt,
                                int k, void* energies, uint64_t* masks, int32_t* status, int waves_per_inst,
                                hipStream_t s);

// merge of top-k lists from disjoint prefix ranges of one instance (one wave).
hipError_t launch_merge_topk(int count, int k_in, const void* ein, const uint64_t* min, int dt, int k, void* eout,
                             uint64_t* mout, hipStream_t s);
// log-partition: factor tables (after launch_prep_walk), forward walk, finalize.
hipError_t launch_prep_exp_tables(const Views& v, const float* beta, int inner, int64_t steps_bound,
                                 hipStream_t s);
hipError_t launch_walk_exp(const Views& v, const float* beta, int waves, hipStream_t s);
hipError_t launch_finalize_logz(const Views& v, const float* beta, double* logz, int32_t* status, hipStream_t s);
// Boltzmann samples by inversion in natural mask order (after a forward walk
// that wrote part and lanepart over a plan with at most 8 outer bits).
hipError_t launch_sample(const Views& v, const float* beta, const double* logz, double* cum, int nsamples,
                         const double* u, uint64_t* masks, int waves, hipStream_t s);
// log-partition backward: moment walk (inner = 5) then assembly.
hipError_t launch_walk_grad(const Views& v, const float* beta, const double* logz, int64_t total_waves,
                            int n_moments, hipStream_t s);
hipError_t launch_finalize_grad(const Views& v, const float* q, const float* beta, const float* grad_logz,
                                float* grad_q, float* grad_beta, double* moments, double* mean, int32_t* status,
                                int n_moments, hipStream_t s);

}  // namespace qbf
