// Log-partition function and its gradient by exhaustive enumeration.
//
//   logZ(beta) = log sum_x exp(-beta f(x))
//   d logZ / d Q_ij = -beta E_p[x_i x_j],  p(x) = exp(-beta f(x) - logZ)
//
// Both walks reuse the block-table enumeration of the top-k kernel: per lane
// a table C'(j) of the inner states, per outer Gray step a uniform table
// T'(g(t); j) and the per-lane scalar KE.  The instance is walked on sign(beta)*Q
// with |beta|, so the exponents stay bounded for any sign of beta.
//
// Forward: a streaming log-sum-exp, no separate minimum pass.  Each lane keeps
// a reference energy r and the sum s = sum 2^(-bb (f - r)) of its states
// (bb = |beta| log2 e), rebasing r when a block lies far below it.  A work
// unit reduces its lanes to log2 of its sum; the finalize merges the units by
// log-sum-exp in float64.  Two forms of the per-state work:
//   * factored (units whose per-lane inner range bb (max C' - min C') is at
//     most kSafeExp2): the weight of state (t, j) splits as
//       a_j * b(t, j) * 2^(c_t),  a_j = 2^(-bb (C'(j) - min C')),
//       b(t, j) = 2^(-bb (T'(g(t); j) - min_j T'(g(t); .))),
//     so a lane's sum is sum_j a_j U_j with U_j = sum_t 2^(c_t) b(t, j): per
//     wave a matrix product of the step rows and the lanes' step weights, on
//     the matrix cores (one multiply-add per state), and one exp per step.
//     The range bound keeps the block's
//     largest product above 2^-kSafeExp2, so float32 underflow only drops
//     terms below 2^-126 of an already represented block sum;
//   * direct (other units): e_j = C'(j) + T'(g(t); j), the block minimum
//     rebases r, and every state takes one exp2.
//
// Backward: each state's weight w = p(x) = 2^(-|beta| log2(e) (e_j + KE) -
// logZ log2(e)).  Per lane and unit the walk accumulates
//   W[j]          = sum_t w(t, j)                (inner x inner moments)
//   A[o][0]       = sum_t x_o(t) s(t),  s = sum_j w(t, j)
//   A[o][1+a]     = sum_t x_o(t) v_a(t), v_a = sum_j w(t, j) j_a
//   Bo[o1][o2]    = sum_t x_o1(t) x_o2(t) s(t)
// (x_o(t) = bit o of g(t), uniform across lanes) and at the end of the unit
// assembles the n(n+1)/2 moments sum w x_i x_j for the unit, the prefix bits
// entering through the lane's own bits and the unit's tile bits.  In the
// factored form W comes from the matrix cores as in the forward (W = a_j U_j),
// and s, v_a are nested multiply-adds over the inner bits where a step's row
// factors into per-bit terms (block_nested).
#include "dpp.hpp"
#include "walk.hpp"

namespace qbf {

namespace {

constexpr double kLog2e = 1.4426950408889634074;
constexpr int kGradInner = 5;
constexpr int kGradStates = 1 << kGradInner;
constexpr int kGradMaxOuter = 8;
constexpr int kSampleOuter = 8;  // outer bits of the sampling plan (block weights fit in LDS)

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Exchanges the upper 32 lanes of x with the lower 32 lanes of y:
//   x <- [x(0..31), y(0..31)],  y <- [x(32..63), y(32..63)].
// Written as inline asm: this compiler's __builtin_amdgcn_permlane32_swap can
// hand back the first result for both.  The nops cover the VALU-write /
// permlane-read and permlane-write / VALU-or-MFMA-read hazards.
__device__ __forceinline__ void half_swap(float& x, float& y) {
  asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1\n\ts_nop 1" : "+v"(x), "+v"(y));
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// ------------------------------------------------------------ exp-sum walk

// bb (max C' - min C') bound of the factored form (see the file comment).
constexpr float kSafeExp2 = 84.f;
// A block whose lower bound lies more than 2^kRebase below the lane's
// reference energy moves the reference there.
constexpr double kRebase = 32.0;

// acc[Q&3] += 2^(fma(C'(16K+Q) + T'(16K+Q), nb, cst)) for Q = 0..15.
template <int K, int Q>
__device__ __forceinline__ void block_exp(float (&acc)[4], float t, const float* C, float nb, float cst) {
  const float e = row_bcast<Q>(t) + C[16 * K + Q];
  acc[Q & 3] += exp2_fast(__builtin_fmaf(e, nb, cst));
  if constexpr (Q + 1 < 16) block_exp<K, Q + 1>(acc, t, C, nb, cst);
}

// Per-lane range of the finite entries of C' and the factored-form decision
// (uniform: every valid lane must satisfy the bound).
template <int NB>
__device__ __forceinline__ bool factor_ok(const float (&C)[NB], float bbf, bool valid, float& cmin) {
  float lo = __builtin_inff(), hi = -__builtin_inff();
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (C[j] < __builtin_inff()) {
      lo = fminf(lo, C[j]);
      hi = fmaxf(hi, C[j]);
    }
  }
  cmin = lo < __builtin_inff() ? lo : 0.f;  // a lane without states: all factors 0, any finite cmin
  return ballot(valid && !(bbf * (hi - lo) <= kSafeExp2)) == 0;
}

// C'(j) -> a_j = 2^(-bb (C'(j) - cmin)), 0 for the sentinel entries.
template <int NB>
__device__ __forceinline__ void to_factors(float (&C)[NB], float bbf, float cmin) {
#pragma unroll
  for (int j = 0; j < NB; ++j)
    C[j] = C[j] < __builtin_inff() ? exp2_fast(-bbf * (C[j] - cmin)) : 0.f;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
  return x;
}

// log2 of sum over lanes of 2^l (l = -inf for empty lanes), float64.
__device__ __forceinline__ double wave_lse2(double l) {
  const double m = wave_max(l);
  if (!(m > -__builtin_inf())) return m;
  const double t = l > -__builtin_inf() ? exp2(l - m) : 0.0;
  return m + log2(wave_sum(t));
}

// Units of the two passes.  Pass 0 (factored) walks the queue's units and
// sends a unit that fails the factored-form bound -- or every unit when the
// factored form is switched off -- to a list; pass 1 (direct) strides over
// that list.  Each pass is its own kernel, so each gets its own register
// budget; the list is usually empty and pass 1 then ends at once.
template <int PASS>
struct PassUnits {
  WorkIter it;
  uint64_t i, count, stride;
  __device__ PassUnits(const Views& v, uint64_t total_units)
      : it(v, total_units),
        i((uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)),
        count(PASS == 1 ? uniform_u64(gp((const Header*)v.hdr)->direct_count) : 0),
        stride((uint64_t)gridDim.x * kWavesPerBlock) {}
  __device__ __forceinline__ bool next(const Views& v, int lane, uint64_t& u) {
    if constexpr (PASS == 0) {
      return it.next(v, lane, u);
    } else {
      if (i >= count) return false;
      u = uniform_u64(gp(v.dlist)[i]);
      i += stride;
      return true;
    }
  }
};

// Appends unit u to the direct pass's list (all lanes call; lane 0 adds).
__device__ __forceinline__ void defer_unit(const Views& v, uint64_t u, int lane) {
  const uint64_t idx = uniform_u64(
      atomicAdd((unsigned long long*)&v.hdr->direct_count, lane == 0 ? 1ull : 0ull));
  if (lane == 0) gp(v.dlist)[idx] = u;
}

template <int PASS>
__device__ __forceinline__ void walk_exp_body(const Views& v, const float* beta) {
  __shared__ double ctab[kWavesPerBlock][kWaveRows * kWave];
  const int lane = threadIdx.x & 63;
  double* myc = ctab[threadIdx.x >> 6];
  const uint64_t total_units = uniform_u64(gp((const Header*)v.hdr)->total_units);
  PassUnits<PASS> units(v, total_units);
  uint64_t u;
  while (units.next(v, lane, u)) {
    const int b = v.batch == 1 ? 0 : find_unit(v, u);
    const InstU I = load_inst(v, b);
    if (I.status != 0) {
      if (lane == 0) gp(v.part)[u] = -__builtin_inf();
      continue;
    }
    const uint64_t local = u - (uint64_t)I.unit_begin;
    const bool valid = lane < (1 << I.L);
    float C[kInnerStates];
    const double EP = lane_init<float, kInnerStates>(v, b, I, local, valid, myc, lane, C);
    const double bb = fabs((double)gp(beta)[b]) * kLog2e;
    const float bbf = (float)bb;
    const uint32_t steps = 1u << I.no;
    const int qoff = (lane & 15) * 16;
    double K = EP;  // E_P + X_PO(p, g(t)): the lane's share of the step's constant
    double r = 0.0, S = 0.0;
    double lbias = 0.0;  // the lane's sum is S * 2^-lbias
    if constexpr (PASS == 0) {
      float cmin = 0.f;
      if (!(v.factor && factor_ok(C, bbf, valid, cmin))) {
        defer_unit(v, u, lane);
        continue;
      }
      to_factors(C, bbf, cmin);
      // The step sums are a matrix product on the matrix cores.  With g(l, t) =
      // 2^(ntau(t) + P_l(t)) the lane's weight of step t, the lane's sum is
      //   S_l = sum_j a(l, j) U(l, j),   U(l, j) = sum_t g(l, t) b(t, j),
      // and U^T (64 inner states x 64 lanes) += B_t^T G_t over pairs of steps
      // is four v_mfma_f32_32x32x2_f32 (inner half r x lane half c).  Result
      // layout: lane q, register e of tile (c, r) holds U(32c + q%32, 32r + i)
      // with i = (e%4) + 4 (q/32) + 8 (e/4).  Every 16 steps, at a reference
      // move and at the unit's end, U is folded into S: lane q multiplies its
      // entries by the matching a(l, j) (held in the same layout, AD) and
      // swaps halves with lane q^32 to collect its own row.
      const __amdgpu_buffer_rsrc_t brs = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(gp((const float*)v.etab) + I.tab_off * kInnerStates), (short)0,
          (int)(steps * (uint32_t)(kInnerStates * sizeof(float))), 0x00020000);
      // AD[c][r][e] = a(32c + lane%32, 32r + i(e, lane)): the pair (a(j0), a(j0 + 4))
      // of every lane, swapped across the wave halves
      float AD[2][2][16];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int j0 = 32 * r + (e & 3) + 8 * (e >> 2);
          AD[0][r][e] = C[j0];
          AD[1][r][e] = C[j0 + 4];
          half_swap(AD[0][r][e], AD[1][r][e]);
        }
      }
      // Exponents in units of bb: step t's weight is 2^(ntau(t) + P), ntau(t) =
      // -bb (min_j T' + E_O)(t) from the table, P = -bb (cm + K) + R the lane's
      // part, R = bb r the lane's reference; a flip of outer bit l moves K by
      // +-c_l, so P by -+bb c_l (the first three bits' products held in
      // registers).  U holds at most 16 steps of weights (each at most
      // 2^kRebase) before it is folded into the float64 sum.
      const gptr<const double> ntau = gp(v.tref) + I.tab_off;
      const double cm = (double)cmin;
      const double nt0 = ntau[0];
      double R = bb * (cm + EP) - nt0;  // so that the first block's exponent is 0
      double P = -nt0;
      const double bc0 = I.no > 0 ? bb * myc[lane] : 0.0;
      const double bc1 = I.no > 1 ? bb * myc[kWave + lane] : 0.0;
      const double bc2 = I.no > 2 ? bb * myc[2 * kWave + lane] : 0.0;
      f32x16 U[2][2];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 2; ++r) U[c][r] = f32x16{};
      auto fold = [&]() {
        // four chains of 8 products per lane half, summed pairwise
        float pa[2][4] = {};
#pragma unroll
        for (int r = 0; r < 2; ++r) {
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            pa[0][e & 3] = __builtin_fmaf(AD[0][r][e], U[0][r][e], pa[0][e & 3]);
            pa[1][e & 3] = __builtin_fmaf(AD[1][r][e], U[1][r][e], pa[1][e & 3]);
          }
        }
        float p0 = (pa[0][0] + pa[0][1]) + (pa[0][2] + pa[0][3]);
        float p1 = (pa[1][0] + pa[1][1]) + (pa[1][2] + pa[1][3]);
        half_swap(p0, p1);
        S += (double)(p0 + p1);
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int r = 0; r < 2; ++r) U[c][r] = f32x16{};
      };
      // The step's exponent after its flip.  A lane more than 2^kRebase above
      // its reference first folds U (all lanes, uniform), then moves the
      // reference by the exponent; `shift` returns that move (0 for the other
      // lanes), by which a weight computed earlier but not yet in U is scaled.
      auto expo = [&](double nt, double& shift) -> double {
        double ct = nt + P;
        shift = 0.0;
        if (__builtin_expect(ballot(ct > kRebase) != 0, 0)) {
          fold();
          if (ct > kRebase) {
            S *= (double)exp2_fast((float)-ct);
            R -= ct;
            P -= ct;
            shift = ct;
            ct = 0.0;
          }
        }
        return ct;
      };
      // A operand of a pair of steps t0, t0 + 1: lane q holds b(t0 + q/32, 32r + q%32);
      // entry j of a row sits at position 4 (j % 16) + j / 16
      const int jl = lane & 31, tk = lane >> 5;
      // lanes 32..63 read the pair's second row; both rows lie inside the
      // table (t0 + 1 < steps, or a one-step walk, whose second row is its first)
      const int boff0 = (4 * (jl & 15) + (jl >> 4)) * 4 + (steps > 1 ? tk * 256 : 0), boff1 = boff0 + 8;
      auto loadb = [&](uint32_t t0, float& b0, float& b1) {
        const int so = (int)((t0 + 1 < steps ? t0 : 0u) * 256u);
        b0 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(brs, boff0, so, 0));
        b1 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(brs, boff1, so, 0));
      };
      // one pair: the B operands (weights of both steps for the two lane
      // halves) by a half swap, then the four MFMAs
      auto mma = [&](float g0, float g1, float b0, float b1) {
        float G0 = g0, G1 = g1;
        half_swap(G0, G1);
        U[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(b0, G0, U[0][0], 0, 0, 0);
        U[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(b1, G0, U[0][1], 0, 0, 0);
        U[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(b0, G1, U[1][0], 0, 0, 0);
        U[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(b1, G1, U[1][1], 0, 0, 0);
      };
      auto weight = [&](double ct) { return valid ? exp2_fast((float)ct) : 0.f; };
      if (steps < 8) {
        // pairs of steps; the second step of a one-step walk has weight 0
        for (uint32_t t = 0; t < steps; t += 2) {
          float b0, b1;
          loadb(t, b0, b1);
          if (t) {
            const int l = __builtin_ctz(t);
            P = __builtin_fma(((t >> (l + 1)) & 1) ? bb : -bb, myc[l * kWave + lane], P);
          }
          double sh0, sh1;
          const double ct0 = expo(ntau[t], sh0);
          float g0 = weight(ct0), g1 = 0.f;
          if (t + 1 < steps) {
            P = __builtin_fma((((t + 1) >> 1) & 1) ? bb : -bb, myc[lane], P);  // t + 1 flips bit 0
            const double ct1 = expo(ntau[t + 1], sh1);
            g0 = weight(ct0 - sh1);
            g1 = weight(ct1);
          }
          mma(g0, g1, b0, b1);
        }
        fold();
      } else {
        // groups of eight steps t = 8q + r: bit 0 turns on at r = 1, 5 and off
        // at 3, 7; bit 1 on at 2, off at 6; bit 2 at 4 (off for odd q); bit
        // 3 + CTZ(q) at r = 0 (q > 0).  Four pairs per group; U is folded every
        // second group and at the end.
        const uint32_t groups = steps >> 3;
        auto flip = [&](int r, uint32_t q) {
          if (r == 0) {
            if (q) {
              const int l = 3 + __builtin_ctz(q);
              P = __builtin_fma(((q >> (l - 2)) & 1) ? bb : -bb, myc[l * kWave + lane], P);
            }
          } else if (r == 1 || r == 5) {
            P -= bc0;
          } else if (r == 3 || r == 7) {
            P += bc0;
          } else if (r == 2) {
            P -= bc1;
          } else if (r == 6) {
            P += bc1;
          } else {
            P += (q & 1) ? bc2 : -bc2;
          }
        };
        float bn0, bn1;
        loadb(0, bn0, bn1);
        double nA = ntau[0], nB = ntau[1];
        for (uint32_t q = 0; q < groups; ++q) {
#pragma unroll
          for (int pr = 0; pr < 4; ++pr) {
            const uint32_t t0 = 8 * q + 2 * pr;
            const float b0 = bn0, b1 = bn1;
            const double n0 = nA, n1 = nB;
            loadb(t0 + 2, bn0, bn1);  // the next pair's rows (rows 0, 1 past the end)
            const uint32_t tn = t0 + 2 < steps ? t0 + 2 : steps - 2;
            nA = ntau[tn];
            nB = ntau[tn + 1];
            double sh0, sh1;
            flip(2 * pr, q);
            const double ct0 = expo(n0, sh0);
            flip(2 * pr + 1, q);
            const double ct1 = expo(n1, sh1);
            mma(weight(ct0 - sh1), weight(ct1), b0, b1);
          }
          if ((q & 1) || q + 1 == groups) fold();
        }
      }
      lbias = R;
    } else {
      // direct form.  beta = 0: a tiny negative slope keeps the sentinel entries (+inf) at
      // weight 0 without changing any valid weight.
      const float nb = bb > 0.0 ? -bbf : -1e-30f;
      const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(gp((const float*)v.tab) + I.tab_off * kInnerStates), (short)0,
          (int)(steps * (uint32_t)(kInnerStates * sizeof(float))), 0x00020000);
      bool first = true;
      f32x4 tn = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(trs, qoff, 0, 0));
      const gptr<const double> eod = gp((const double*)v.eod) + I.tab_off;
      double eon = eod[0];
      for (uint32_t t = 0; t < steps; ++t) {
        const f32x4 tc = tn;
        const double eoc = eon;
        const uint32_t tt = t + 1 < steps ? t + 1 : t;
        tn = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(trs, qoff, (int)(tt * 256u), 0));
        eon = eod[tt];
        if (t) {
          const int l = __builtin_ctz(t);
          K = __builtin_fma(((t >> (l + 1)) & 1) ? -1.0 : 1.0, myc[l * kWave + lane], K);
        }
        float bm = __builtin_inff();
        block_min<0, 0>(bm, tc.x, C);
        block_min<1, 0>(bm, tc.y, C);
        block_min<2, 0>(bm, tc.z, C);
        block_min<3, 0>(bm, tc.w, C);
        const double lt = (double)bm + K + eoc;
        if (first || -bb * (lt - r) > kRebase) {
          S = first ? 0.0 : S * (double)exp2_fast((float)(-bb * (r - lt)));
          r = lt;
          first = false;
        }
        const float cst = (float)(-bb * (K + eoc - r));
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        block_exp<0, 0>(acc, tc.x, C, nb, cst);
        block_exp<1, 0>(acc, tc.y, C, nb, cst);
        block_exp<2, 0>(acc, tc.z, C, nb, cst);
        block_exp<3, 0>(acc, tc.w, C, nb, cst);
        S += (double)((acc[0] + acc[1]) + (acc[2] + acc[3]));
      }
    }
    // log2 of the lane's sum: log2 S - bb r
    if constexpr (PASS == 1) lbias = bb * r;
    const double l = (valid && S > 0.0) ? log2(S) - lbias : -__builtin_inf();
    const double lu = wave_lse2(l);
    if (lane == 0) gp(v.part)[u] = lu;
    if (v.lanepart) gp(v.lanepart)[u * kWave + lane] = l;
  }
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) walk_exp_fac_kernel(Views v,
                                                                                            const float* beta) {
  walk_exp_body<0>(v, beta);
}
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) walk_exp_direct_kernel(Views v,
                                                                                               const float* beta) {
  walk_exp_body<1>(v, beta);
}

// One thread per instance: log-sum-exp of its units' log2 sums (in unit order).
__global__ void finalize_logz_kernel(Views v, const float* beta, double* logz, int32_t* status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= v.batch) return;
  const Inst* I = &v.inst[b];
  int32_t st = I->status;
  double out = __builtin_nan("");
  if (st == 0) {
    const double* pu = v.part + I->unit_begin;
    double m = -__builtin_inf();
    for (int64_t u = 0; u < I->units; ++u) m = fmax(m, pu[u]);
    double S = 0.0;
    for (int64_t u = 0; u < I->units; ++u) S += exp2(pu[u] - m);
    out = (m + log2(S)) / kLog2e;
  }
  logz[b] = out;
  status[b] = st;
}

// Factor tables of the forward and adjoint walks: per step, b(t, j) =
// 2^(-bb (T'(g(t); j) - min_j T')) in the layout of T', and
// tref(t) = min_j T'(g(t); j) + E_O(g(t)).  blockIdx.x: instance; blockIdx.y:
// chunk of 64 of its steps; one wave per step, lane = table entry.
__global__ void __launch_bounds__(256) prep_exp_tables_kernel(Views v, const float* beta, int inner) {
  const int b = blockIdx.x;
  const Inst* I = &v.inst[b];
  if (I->status != 0) return;
  const int64_t steps = int64_t(1) << I->no;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int width = 1 << inner;
  const double bb = fabs((double)beta[b]) * kLog2e;
  const float bbf = (float)bb;
  const float* tab = (const float*)v.tab + I->tab_off * width;
  float* etab = (float*)v.etab + I->tab_off * width;
  const int64_t c0 = (int64_t)blockIdx.y * 64;
  // the wave's 16 steps c0 + w + 4i: all rows and offsets loaded first (their
  // latencies overlap), then per step one wave minimum (DPP, no LDS) and one
  // exp per entry
  constexpr int kPer = 16;
  float tv[kPer];
  double eo[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int64_t t = c0 + w + 4 * i;
    const bool ok = t < steps;
    tv[i] = ok && lane < width ? tab[t * width + lane] : __builtin_inff();
    eo[i] = ok ? v.eod[I->tab_off + t] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int64_t t = c0 + w + 4 * i;
    if (t >= steps) break;
    const float m = wave_min_f32(tv[i]);
    if (lane < width) etab[t * width + lane] = exp2_fast(-bbf * (tv[i] - m));
    if (lane == 0) v.tref[I->tab_off + t] = -bb * ((double)m + eo[i]);
  }
}

// ------------------------------------------------------------ moment walk

template <int K, int Q>
__device__ __forceinline__ void block_w(float (&w)[kGradStates], float t, const float* C, float nb, float cst) {
  const float e = row_bcast<Q>(t) + C[16 * K + Q];
  w[16 * K + Q] = exp2_fast(__builtin_fmaf(e, nb, cst));
  if constexpr (Q + 1 < 16) block_w<K, Q + 1>(w, t, C, nb, cst);
}

// w(16K+Q) = b(16K+Q) * a(16K+Q) for Q = H*8 .. H*8+7, b broadcast from lane Q
// of each 16-lane row (v_mul_f32 with a DPP row broadcast; written out because
// the compiler leaves the broadcast as a separate move here).  s_nop: two wait
// states between a VALU write of t and its DPP read.
#define QBF_STR2(x) #x
#define QBF_STR(x) QBF_STR2(x)
template <int K, int H>
__device__ __forceinline__ void block_prod8(float (&w)[kGradStates], float t, const float* A) {
  constexpr int b0 = 16 * K + 8 * H;
  if constexpr (H == 0) {
#define QS0 "0"
#define QS1 "1"
#define QS2 "2"
#define QS3 "3"
#define QS4 "4"
#define QS5 "5"
#define QS6 "6"
#define QS7 "7"
    asm("s_nop 1\n"
      "v_mul_f32_dpp %0, %8, %9 row_newbcast:" QS0 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %1, %8, %10 row_newbcast:" QS1 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %2, %8, %11 row_newbcast:" QS2 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %3, %8, %12 row_newbcast:" QS3 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %4, %8, %13 row_newbcast:" QS4 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %5, %8, %14 row_newbcast:" QS5 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %6, %8, %15 row_newbcast:" QS6 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %7, %8, %16 row_newbcast:" QS7 " row_mask:0xf bank_mask:0xf\n"
        : "=&v"(w[b0]), "=&v"(w[b0 + 1]), "=&v"(w[b0 + 2]), "=&v"(w[b0 + 3]), "=&v"(w[b0 + 4]), "=&v"(w[b0 + 5]),
          "=&v"(w[b0 + 6]), "=&v"(w[b0 + 7])
        : "v"(t), "v"(A[b0]), "v"(A[b0 + 1]), "v"(A[b0 + 2]), "v"(A[b0 + 3]), "v"(A[b0 + 4]), "v"(A[b0 + 5]),
          "v"(A[b0 + 6]), "v"(A[b0 + 7]));
#undef QS0
#undef QS1
#undef QS2
#undef QS3
#undef QS4
#undef QS5
#undef QS6
#undef QS7
  } else {
#define QS0 "8"
#define QS1 "9"
#define QS2 "10"
#define QS3 "11"
#define QS4 "12"
#define QS5 "13"
#define QS6 "14"
#define QS7 "15"
    asm("s_nop 1\n"
      "v_mul_f32_dpp %0, %8, %9 row_newbcast:" QS0 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %1, %8, %10 row_newbcast:" QS1 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %2, %8, %11 row_newbcast:" QS2 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %3, %8, %12 row_newbcast:" QS3 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %4, %8, %13 row_newbcast:" QS4 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %5, %8, %14 row_newbcast:" QS5 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %6, %8, %15 row_newbcast:" QS6 " row_mask:0xf bank_mask:0xf\n"
      "v_mul_f32_dpp %7, %8, %16 row_newbcast:" QS7 " row_mask:0xf bank_mask:0xf\n"
        : "=&v"(w[b0]), "=&v"(w[b0 + 1]), "=&v"(w[b0 + 2]), "=&v"(w[b0 + 3]), "=&v"(w[b0 + 4]), "=&v"(w[b0 + 5]),
          "=&v"(w[b0 + 6]), "=&v"(w[b0 + 7])
        : "v"(t), "v"(A[b0]), "v"(A[b0 + 1]), "v"(A[b0 + 2]), "v"(A[b0 + 3]), "v"(A[b0 + 4]), "v"(A[b0 + 5]),
          "v"(A[b0 + 6]), "v"(A[b0 + 7]));
#undef QS0
#undef QS1
#undef QS2
#undef QS3
#undef QS4
#undef QS5
#undef QS6
#undef QS7
  }
}

// s = sum_j w_j and v_a = sum_j w_j j_a (a < 5), every sum a pairwise tree:
// level a + 1 adds the pairs of level a (p, q, r, h), and v_a sums the odd
// members of level a.  57 adds, at most five deep.
template <int N>
__device__ __forceinline__ float tree_sum(const float* x) {
  if constexpr (N == 1) return x[0];
  else return tree_sum<N / 2>(x) + tree_sum<N / 2>(x + N / 2);
}
__device__ __forceinline__ void block_moments(const float (&w)[kGradStates], float& s, float (&va)[kGradInner]) {
  static_assert(kGradInner == 5, "five inner bits");
  float p[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    p[i] = w[2 * i] + w[2 * i + 1];
    o[i] = w[2 * i + 1];
  }
  va[0] = tree_sum<16>(o);
  float q[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    q[i] = p[2 * i] + p[2 * i + 1];
    o[i] = p[2 * i + 1];
  }
  va[1] = tree_sum<8>(o);
  float r[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r[i] = q[2 * i] + q[2 * i + 1];
    o[i] = q[2 * i + 1];
  }
  va[2] = tree_sum<4>(o);
  const float h0 = r[0] + r[1], h1 = r[2] + r[3];
  va[3] = r[1] + r[3];
  va[4] = h1;
  s = h0 + h1;
}

// Nested form of the same sums.  Where a step's factor row is a product over
// the inner bits, b(t, j) = b(t, 0) prod_{u in j} beta_u(t), the block sums are
// b(t, 0) times s = sum_j a_j prod_{u in j} beta_u and v_a = sum_j a_j j_a
// prod_{u in j} beta_u: multilinear polynomials in beta with the lane's a_j
// as coefficients.  Level u pairs the states that differ in bit u (c_i =
// c_2i + beta_u c_2i+1), and v_u is beta_u times the odd members of level u
// evaluated over the bits above u.  62 multiply-adds, every operand in a
// register, against 32 broadcast products and 57 adds.
template <int U, int N>
__device__ __forceinline__ float poly_eval(const float* c, const float (&be)[kGradInner]) {
  if constexpr (N == 1) {
    return c[0];
  } else {
    float d[N / 2];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) d[i] = __builtin_fmaf(be[U], c[2 * i + 1], c[2 * i]);
    return poly_eval<U + 1, N / 2>(d, be);
  }
}
__device__ __forceinline__ void block_nested(const float (&a)[kGradStates], const float (&be)[kGradInner], float& s,
                                             float (&va)[kGradInner]) {
  float p[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    p[i] = __builtin_fmaf(be[0], a[2 * i + 1], a[2 * i]);
    o[i] = a[2 * i + 1];
  }
  va[0] = be[0] * poly_eval<1, 16>(o, be);
  float q[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    q[i] = __builtin_fmaf(be[1], p[2 * i + 1], p[2 * i]);
    o[i] = p[2 * i + 1];
  }
  va[1] = be[1] * poly_eval<2, 8>(o, be);
  float r[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r[i] = __builtin_fmaf(be[2], q[2 * i + 1], q[2 * i]);
    o[i] = q[2 * i + 1];
  }
  va[2] = be[2] * poly_eval<3, 4>(o, be);
  const float h0 = __builtin_fmaf(be[3], r[1], r[0]), h1 = __builtin_fmaf(be[3], r[3], r[2]);
  va[3] = be[3] * __builtin_fmaf(be[4], r[3], r[1]);
  va[4] = be[4] * h1;
  s = __builtin_fmaf(be[4], h1, h0);
}

// The nested form needs b(t, 0) >= 2^-40 at every step of the unit: then
// beta_u = b(t, 2^u) / b(t, 0) <= 2^40 and so is every partial product.
constexpr float kNestedMinB0 = 0x1p-40f;
// Steps of the adjoint's table rows in flight ahead of the step being summed.
constexpr int kPrefetch = 2;

__device__ __forceinline__ int pidx(int n, int i, int j) { return i * n - (i * (i - 1)) / 2 + (j - i); }

// The moments of a unit in the order the adjoint sums them: pairs of positions
// (kind, index) with kind 0 an inner bit, 1 an outer bit, 2 a lane bit; kind 3
// is the unit's total (kept for the pairs of two tile bits).  The table holds
// every pair the largest plan has; a unit skips the ones its plan lacks.
struct MomentSlot {
  signed char k1, i1, k2, i2;
};
constexpr int kMomentSlots =
    kGradInner * (kGradInner + 1) / 2 + kGradMaxOuter * kGradInner + kGradMaxOuter * (kGradMaxOuter + 1) / 2 +
    6 * (kGradInner + kGradMaxOuter) + 21 + 1;
constexpr int kTotalSlot = 31;  // stash slot of the total (positions use 0 .. 19)
struct MomentTable {
  MomentSlot s[kMomentSlots];
};
constexpr MomentTable make_moment_table() {
  MomentTable t{};
  int k = 0;
  auto put = [&](int k1, int i1, int k2, int i2) {
    t.s[k++] = MomentSlot{(signed char)k1, (signed char)i1, (signed char)k2, (signed char)i2};
  };
  for (int a = 0; a < kGradInner; ++a)
    for (int a2 = a; a2 < kGradInner; ++a2) put(0, a, 0, a2);
  for (int o = 0; o < kGradMaxOuter; ++o) {
    for (int a = 0; a < kGradInner; ++a) put(0, a, 1, o);
    for (int o2 = o; o2 < kGradMaxOuter; ++o2) put(1, o, 1, o2);
  }
  for (int ll = 0; ll < 6; ++ll) {
    for (int a = 0; a < kGradInner; ++a) put(0, a, 2, ll);
    for (int o = 0; o < kGradMaxOuter; ++o) put(1, o, 2, ll);
    for (int l2 = 0; l2 <= ll; ++l2) put(2, l2, 2, ll);
  }
  put(3, 0, 3, 0);
  return t;
}
constexpr MomentTable kMomentTable = make_moment_table();
static_assert(kMomentTable.s[kMomentSlots - 1].k1 == 3 && kMomentTable.s[kMomentSlots - 2].k1 == 2,
              "the table fills every slot");
__constant__ MomentTable kMomentTableDev = kMomentTable;

// f(std::integral_constant<int, S>) for S = 0 .. N-1, in order.
template <int N, int S = 0>
struct Unrolled {
  template <class F>
  static __device__ __forceinline__ void run(F&& f) {
    if constexpr (S < N) {
      f(std::integral_constant<int, S>{});
      Unrolled<N, S + 1>::run(f);
    }
  }
};

template <int PASS>
__device__ __forceinline__ void walk_grad_body(const Views& v, const float* beta, const double* logz, int npairs) {
  __shared__ __attribute__((aligned(16))) double ctab[kWavesPerBlock][kWaveRows * kWave];
  const int lane = threadIdx.x & 63;
  double* myc = ctab[threadIdx.x >> 6];
  const uint64_t total_units = uniform_u64(gp((const Header*)v.hdr)->total_units);
  PassUnits<PASS> units(v, total_units);
  uint64_t u;
  while (units.next(v, lane, u)) {
    const int b = v.batch == 1 ? 0 : find_unit(v, u);
    const InstU I = load_inst(v, b);
    const gptr<double> out = gp(v.part) + (int64_t)u * npairs;
    if (I.status != 0) continue;
    const uint64_t local = u - (uint64_t)I.unit_begin;
    const bool valid = lane < (1 << I.L);
    const uint64_t p = (local << I.L) | (uint64_t)lane;
    float C[kGradStates];
    const double EP = lane_init<float, kGradStates>(v, b, I, local, valid, myc, lane, C);
    const double bb = fabs((double)gp(beta)[b]) * kLog2e;
    const float bbf = (float)bb;
    const double lz2 = uniform_f64(gp(logz)[b]) * kLog2e;
    const uint32_t steps = 1u << I.no;
    const int qoff = (lane & 15) * 8;
    float cmin = 0.f;
    constexpr bool fac = PASS == 0;  // pass 0: factored form; pass 1: direct form
    if constexpr (PASS == 0) {
      if (!(v.factor && factor_ok(C, bbf, valid, cmin))) {
        defer_unit(v, u, lane);
        continue;
      }
      to_factors(C, bbf, cmin);
    }
    // factored: b(t, j) rows and tref; direct: T' rows and E_O
    const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(gp((const float*)(fac ? v.etab : v.tab)) + I.tab_off * kGradStates), (short)0,
        (int)(steps * (uint32_t)(kGradStates * sizeof(float))), 0x00020000);
    const gptr<const double> tref = gp(v.tref) + I.tab_off;

    // inner x inner: the direct form sums W[j] = sum_t w(t, j) per lane; the
    // factored form sums U(j, l) = sum_t g(l, t) b(t, j) on the matrix cores
    // (W = a_j U at the end, as in the forward): U^T (32 inner states x 64
    // lanes, two 32 x 32 tiles, one per lane half) += B^T G over pairs of
    // steps, with v_mfma_f32_32x32x2_f32.  Tile c, lane q, element e holds
    // inner state (e%4) + 4 (q/32) + 8 (e/4) of lane 32 c + q%32.
    float W[kGradStates];
#pragma unroll
    for (int j = 0; j < kGradStates; ++j) W[j] = 0.f;
    f32x16 U[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 16; ++e) U[c][e] = 0.f;
    // A[o][0] = sum_t x_o(t) s(t), A[o][1 + a] = sum_t x_o(t) v_a(t),
    // Bo[hi (hi - 1) / 2 + lo] = sum_t x_lo(t) x_hi(t) s(t)
    float A[kGradMaxOuter][kGradInner + 1];
    float Bo[kGradMaxOuter * (kGradMaxOuter - 1) / 2];
#pragma unroll
    for (int o = 0; o < kGradMaxOuter; ++o)
#pragma unroll
      for (int c = 0; c <= kGradInner; ++c) A[o][c] = 0.f;
#pragma unroll
    for (int i = 0; i < kGradMaxOuter * (kGradMaxOuter - 1) / 2; ++i) Bo[i] = 0.f;

    // Direct form: K = E_P + X_PO(p, g(t)), moved along the walk.  Factored
    // form: the exponent -bb (cm + K) - logZ log2(e) of the step factor g,
    // moved the same way (a flip of outer bit l moves K by +-c_l); the table
    // holds the step's -bb (min_j T' + E_O).
    const double cm = (double)cmin;
    double K = EP;
    // a lane without states (beyond the instance's lane bits) gets g = 0
    double Pg = valid ? -bb * (cm + EP) - lz2 : -__builtin_inf();
    // Block sums of one step: y[0] = s = sum_j w(t, j), y[1 + a] = v_a =
    // sum_j w(t, j) j_a; direct form: W[j] += w(t, j); factored form: the
    // step factor g in gs.  The caller has moved K / Pg to step t.
    const float nb = bb > 0.0 ? -bbf : -1e-30f;  // see walk_exp_body
    // fc: 0 direct form, 1 factored form with per-state products, 2 factored
    // form nested (its operands broadcast from the step row tc)
    auto block = [&](auto fc, const f32x2& tc, double sc, float (&y)[kGradInner + 1], float& gs) {
      float w[kGradStates];
      float va[kGradInner];
      if constexpr (decltype(fc)::value == 2) {
        const float g = exp2_fast((float)(sc + Pg));
        gs = g;
        // b(t, 0) and b(t, 2^u) broadcast from lanes 0, 1, 2, 4, 8 (x) and 0 (y)
        // of each row
        const float b0 = row_bcast<0>(tc.x), rb = __builtin_amdgcn_rcpf(b0);
        const float be[kGradInner] = {row_bcast<1>(tc.x) * rb, row_bcast<2>(tc.x) * rb, row_bcast<4>(tc.x) * rb,
                                      row_bcast<8>(tc.x) * rb, row_bcast<0>(tc.y) * rb};
        block_nested(C, be, y[0], va);
        const float gh = g * b0;
        y[0] *= gh;
#pragma unroll
        for (int c = 0; c < kGradInner; ++c) y[1 + c] = va[c] * gh;
      } else if constexpr (decltype(fc)::value == 1) {
        // sc = -bb (min_j T' + E_O)(t); weight = g * a_j * b(t, j) <= 1, g <= 2^kSafeExp2
        const float g = exp2_fast((float)(sc + Pg));
        gs = g;
        block_prod8<0, 0>(w, tc.x, C);
        block_prod8<0, 1>(w, tc.x, C);
        block_prod8<1, 0>(w, tc.y, C);
        block_prod8<1, 1>(w, tc.y, C);
        block_moments(w, y[0], va);
        y[0] *= g;
#pragma unroll
        for (int c = 0; c < kGradInner; ++c) y[1 + c] = va[c] * g;
      } else {
        // sc = E_O(g(t))
        gs = 0.f;
        const float cst = (float)(-bb * (K + sc) - lz2);
        block_w<0, 0>(w, tc.x, C, nb, cst);
        block_w<1, 0>(w, tc.y, C, nb, cst);
#pragma unroll
        for (int j = 0; j < kGradStates; ++j) W[j] += w[j];
        block_moments(w, y[0], va);
#pragma unroll
        for (int c = 0; c < kGradInner; ++c) y[1 + c] = va[c];
      }
    };
    const gptr<const double> scal = fac ? tref : gp((const double*)v.eod) + I.tab_off;
    f32x2 tn = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(trs, qoff, 0, 0));
    double sn = scal[0];
    // operands of step t (clamped to the last step, loads unconditional)
    auto fetch = [&](uint32_t t, f32x2& tv, double& sv) {
      const uint32_t tt = t < steps ? t : steps - 1;
      tv = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(trs, qoff, (int)(tt * 128u), 0));
      sv = scal[tt];
    };
    auto kflip = [&](int l, bool off) {
      if constexpr (fac) Pg = __builtin_fma(off ? bb : -bb, myc[l * kWave + lane], Pg);
      else K = __builtin_fma(off ? -1.0 : 1.0, myc[l * kWave + lane], K);
    };
    // b(t, q%32) in lane q: the step row holds b(t, Q) and b(t, 16 + Q) in
    // lane Q = q%16 (the DPP broadcast layout)
    auto bsel = [&](const f32x2& tc) { return (lane & 16) ? tc.y : tc.x; };
    // U^T += B^T G for steps t0, t0 + 1: the A operand (32 x 2) takes
    // b(t0 + q/32, q%32) in lane q, the B operand (2 x 32) of tile c takes
    // g(t0 + q/32) of lane 32 c + q%32, which one half-wave swap of (g0, g1)
    // gives for both tiles.
    auto mma = [&](float b0, float b1, float g0, float g1) {
      const float av = (lane & 32) ? b1 : b0;
      half_swap(g0, g1);
      U[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, g0, U[0], 0, 0, 0);
      U[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, g1, U[1], 0, 0, 0);
    };

    auto walk = [&](auto fc) {
      if (steps < 8) {
        // short walks: every step adds into the moments of its set bits; a
        // one-step walk pairs its step with a zero factor
        float be = 0.f, ge = 0.f;
        for (uint32_t t = 0; t < steps; ++t) {
          const f32x2 tc = tn;
          const double sc = sn;
          fetch(t + 1, tn, sn);
          if (t) {
            const int l = __builtin_ctz(t);
            kflip(l, (t >> (l + 1)) & 1);
          }
          float y[kGradInner + 1], g;
          block(fc, tc, sc, y, g);
          if constexpr (fac) {
            const float bv = bsel(tc);
            if (t & 1) {
              mma(be, bv, ge, g);
            } else if (t + 1 == steps) {
              mma(bv, bv, g, 0.f);
            } else {
              be = bv;
              ge = g;
            }
          }
          const uint32_t o = (uint32_t)gray(t);
  #pragma unroll
          for (int a = 0; a < 3; ++a) {
            if ((o >> a) & 1) {
  #pragma unroll
              for (int c = 0; c <= kGradInner; ++c) A[a][c] += y[c];
  #pragma unroll
              for (int a2 = a + 1; a2 < 3; ++a2)
                if ((o >> a2) & 1) Bo[a2 * (a2 - 1) / 2 + a] += y[0];
            }
          }
        }
      } else {
        // Groups of 8 steps t = 8q + r.  Within a group, bit 0 of g(t) is set
        // for r in {1,2,5,6} and bit 1 for r in {2,3,4,5}; bit 2 is set for
        // r >= 4 (q even) or r < 4 (q odd), so it takes the half-group sums F
        // (r < 4) and H (r >= 4); bits 3 and up equal those of g(q) and change
        // only between groups, where bit 3 + CTZ(q) flips.  Moments of the high
        // bits use on-intervals over groups: TG[c] sums the group totals y_c and
        // TL[lo] the group sums of s over the steps with low bit lo set, over
        // the groups before the current one; a high bit turning on opens
        // (A -= TG, pairs -= TG / TL), turning off closes (+=).
        float TG[kGradInner + 1], TL[3];
  #pragma unroll
        for (int c = 0; c <= kGradInner; ++c) TG[c] = 0.f;
  #pragma unroll
        for (int i = 0; i < 3; ++i) TL[i] = 0.f;
        auto flip_high = [&](auto lc, float sgn, uint32_t gq) {
          constexpr int l = decltype(lc)::value;  // 3 .. 7
  #pragma unroll
          for (int c = 0; c <= kGradInner; ++c) A[l][c] = __builtin_fmaf(sgn, TG[c], A[l][c]);
  #pragma unroll
          for (int h = 3; h < kGradMaxOuter; ++h) {
            if (h == l) continue;
            const int hi = h > l ? h : l, lo = h > l ? l : h;
            const float m = ((gq >> (h - 3)) & 1) ? sgn : 0.f;
            Bo[hi * (hi - 1) / 2 + lo] = __builtin_fmaf(m, TG[0], Bo[hi * (hi - 1) / 2 + lo]);
          }
  #pragma unroll
          for (int lo = 0; lo < 3; ++lo) Bo[l * (l - 1) / 2 + lo] = __builtin_fmaf(sgn, TL[lo], Bo[l * (l - 1) / 2 + lo]);
        };
        const uint32_t groups = steps >> 3;
        f32x2 tq[kPrefetch];
        double sq[kPrefetch];
        tq[0] = tn;
        sq[0] = sn;
#pragma unroll
        for (int d = 1; d < kPrefetch; ++d) fetch(d, tq[d], sq[d]);
        for (uint32_t q = 0; q < groups; ++q) {
          const bool qodd = q & 1;
          if (q) {
            const int lq = __builtin_ctz(q), l = 3 + lq;
            const bool off = (q >> (lq + 1)) & 1;
            const float sgn = off ? 1.f : -1.f;
            const uint32_t gq = (uint32_t)gray(q);
            switch (l) {
              case 3: flip_high(std::integral_constant<int, 3>{}, sgn, gq); break;
              case 4: flip_high(std::integral_constant<int, 4>{}, sgn, gq); break;
              case 5: flip_high(std::integral_constant<int, 5>{}, sgn, gq); break;
              case 6: flip_high(std::integral_constant<int, 6>{}, sgn, gq); break;
              default: flip_high(std::integral_constant<int, 7>{}, sgn, gq); break;
            }
          }
          float F[kGradInner + 1], H[kGradInner + 1];
  #pragma unroll
          for (int c = 0; c <= kGradInner; ++c) F[c] = H[c] = 0.f;
          float s0f = 0.f, s0h = 0.f, s1f = 0.f, s1h = 0.f;  // s over bit-0 / bit-1 steps per half
          float be = 0.f, ge = 0.f;                          // even step of the pair
  #pragma unroll
          for (int r = 0; r < 8; ++r) {
            const uint32_t t = 8 * q + r;
            // operands kPrefetch steps ahead (the loads' latency exceeds a step)
            const f32x2 tc = tq[0];
            const double sc = sq[0];
#pragma unroll
            for (int d = 0; d + 1 < kPrefetch; ++d) {
              tq[d] = tq[d + 1];
              sq[d] = sq[d + 1];
            }
            fetch(t + kPrefetch, tq[kPrefetch - 1], sq[kPrefetch - 1]);
            if (r == 0) {
              if (q) kflip(3 + __builtin_ctz(q), (q >> (__builtin_ctz(q) + 1)) & 1);
            } else if (r == 4) {
              kflip(2, qodd);  // bit 2 turns off for odd q
            } else {
              const int l = (r & 1) ? 0 : 1;
              kflip(l, r == 3 || r == 7 || r == 6);
            }
            float y[kGradInner + 1], g;
            block(fc, tc, sc, y, g);
            if constexpr (fac) {
              const float bv = bsel(tc);
              if (r & 1) {
                mma(be, bv, ge, g);
              } else {
                be = bv;
                ge = g;
              }
            }
            const bool b0 = r == 1 || r == 2 || r == 5 || r == 6;
            const bool b1 = r >= 2 && r <= 5;
  #pragma unroll
            for (int c = 0; c <= kGradInner; ++c) {
              if (b0) A[0][c] += y[c];
              if (b1) A[1][c] += y[c];
              if (r < 4) F[c] += y[c];
              else H[c] += y[c];
            }
            if (b0 && b1) Bo[0] += y[0];
            if (b0) {
              if (r < 4) s0f += y[0];
              else s0h += y[0];
            }
            if (b1) {
              if (r < 4) s1f += y[0];
              else s1h += y[0];
            }
          }
          // bit 2 (set in the first half for odd q) and the group totals
  #pragma unroll
          for (int c = 0; c <= kGradInner; ++c) {
            A[2][c] += qodd ? F[c] : H[c];
            TG[c] += F[c] + H[c];
          }
          Bo[1] += qodd ? s0f : s0h;  // pair (0, 2)
          Bo[2] += qodd ? s1f : s1h;  // pair (1, 2)
          TL[0] += s0f + s0h;
          TL[1] += s1f + s1h;
          TL[2] += qodd ? F[0] : H[0];
        }
        // close the intervals of the high bits set in the last group
        const uint32_t gl = (uint32_t)gray(groups - 1);
  #pragma unroll
        for (int h = 3; h < kGradMaxOuter; ++h) {
          if (!((gl >> (h - 3)) & 1)) continue;
  #pragma unroll
          for (int c = 0; c <= kGradInner; ++c) A[h][c] += TG[c];
  #pragma unroll
          for (int lo = 0; lo < 3; ++lo) Bo[h * (h - 1) / 2 + lo] += TL[lo];
  #pragma unroll
          for (int h2 = h + 1; h2 < kGradMaxOuter; ++h2)
            if ((gl >> (h2 - 3)) & 1) Bo[h2 * (h2 - 1) / 2 + h] += TG[0];
        }
      }
    };
    if constexpr (fac) {
      // the nested form where the unit's factor rows allow it (every step
      // shares the check: steps <= 2^kGradMaxOuter = 4 x 64)
      static_assert(kGradMaxOuter <= 8, "four step rows per lane");
      float mb = __builtin_inff();
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t t = (uint32_t)lane + 64u * i;
        if (t < steps)
          mb = fminf(mb, __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(trs, (int)(t * 128u), 0, 0)));
      }
      if (v.factor == 1 && ballot(!(mb >= kNestedMinB0)) == 0)
        walk(std::integral_constant<int, 2>{});
      else
        walk(std::integral_constant<int, 1>{});
    } else {
      walk(std::integral_constant<int, 0>{});
    }
    if constexpr (fac) {
      // W[j] = a_j U(j, lane): a half-wave swap of the tiles' element e puts
      // inner states (e%4) + 8 (e/4) and 4 more of the lane's own column in x, y
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        float x = U[0][e], y = U[1][e];
        half_swap(x, y);
        const int j0 = (e & 3) + 8 * (e >> 2);
        W[j0] = C[j0] * x;
        W[j0 + 4] = C[j0 + 4] * y;
      }
    }

    // ---- assemble the unit's moments sum_x w x_i x_j (i <= j)
    // Each moment is the wave sum of one value per lane.  The values are summed
    // 32 at a time through this wave's lane-field table in LDS (free once the
    // walk is done): lane l stores its 32 values as row l, then sums column
    // l%32 over the rows of its half-wave, and a half-wave swap adds the two
    // halves.  Lane l%32 then looks up value l%32's pair of positions in the
    // slot table for its output index; the diagonals of the positions below
    // the tile bits and the unit's total go to a stash after the rows, for
    // the pairs with a tile bit.
    const int n = I.n, B = I.B, no = I.no, pos0 = B + no, L = I.L, m = pos0 + L;
    float st = 0.f, vt[kGradInner];
#pragma unroll
    for (int a = 0; a < kGradInner; ++a) vt[a] = 0.f;
#pragma unroll
    for (int j = 0; j < kGradStates; ++j) {
      st += W[j];
#pragma unroll
      for (int a = 0; a < kGradInner; ++a)
        if ((j >> a) & 1) vt[a] += W[j];
    }
    float* const rows = (float*)myc;
    constexpr int kStride = 36;  // row stride in floats: 16-byte aligned rows, 4 banks apart
    constexpr int kStash = kWave * kStride;
    static_assert(kStash + 32 <= 2 * kWaveRows * kWave, "the rows fit the lane-field table");
    // lane bit ll of the prefix (bit ll of the lane)
    auto lbit = [&](int ll) { return valid && ((lane >> ll) & 1); };
    float buf[32];
    // chunk ch: lane l (l < 32) writes the wave sum of value 32 ch + l
    auto flush = [&](int ch) {
      f32x4* const row = (f32x4*)(rows + lane * kStride);
#pragma unroll
      for (int i = 0; i < 8; ++i) row[i] = f32x4{buf[4 * i], buf[4 * i + 1], buf[4 * i + 2], buf[4 * i + 3]};
      float x[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) x[i] = rows[((lane & 32) + i) * kStride + (lane & 31)];
      float s = tree_sum<32>(x), t = s;
      half_swap(s, t);
      const float tot = s + t;
      const int idx = 32 * ch + (lane & 31);
      if (lane < 32 && idx < kMomentSlots) {
        const MomentSlot e = kMomentTableDev.s[idx];
        const int lim[3] = {B, no, L}, base[3] = {0, B, pos0};
        if (e.k1 == 3) {
          rows[kStash + kTotalSlot] = tot;
        } else if (e.i1 < lim[e.k1] && e.i2 < lim[e.k2]) {
          const int p1 = base[e.k1] + e.i1, p2 = base[e.k2] + e.i2;
          out[pidx(n, p1, p2)] = (double)tot;
          if (p1 == p2) rows[kStash + p1] = tot;
        }
      }
    };
    // value of slot S (the table's order), then the flush of a full chunk
    Unrolled<kMomentSlots>::run([&](auto sc) {
      constexpr int S = decltype(sc)::value;
      constexpr MomentSlot e = kMomentTable.s[S];
      float x;
      if constexpr (e.k1 == 3) {
        x = st;
      } else if constexpr (e.k1 == 0 && e.k2 == 0) {
        if constexpr (e.i1 == e.i2) {
          x = vt[e.i1];
        } else {
          x = 0.f;
#pragma unroll
          for (int j = 0; j < kGradStates; ++j)
            if (((j >> e.i1) & 1) && ((j >> e.i2) & 1)) x += W[j];
        }
      } else if constexpr (e.k1 == 0 && e.k2 == 1) {
        x = A[e.i2][1 + e.i1];
      } else if constexpr (e.k1 == 1 && e.k2 == 1) {
        if constexpr (e.i1 == e.i2) x = A[e.i1][0];
        else x = Bo[e.i2 * (e.i2 - 1) / 2 + e.i1];
      } else if constexpr (e.k1 == 0) {
        x = lbit(e.i2) ? vt[e.i1] : 0.f;
      } else if constexpr (e.k1 == 1) {
        x = lbit(e.i2) ? A[e.i1][0] : 0.f;
      } else {
        x = (lbit(e.i2) && ((lane >> e.i1) & 1)) ? st : 0.f;
      }
      buf[S & 31] = x;
      if constexpr ((S & 31) == 31 || S + 1 == kMomentSlots) flush(S >> 5);
    });
    // pairs with a tile bit: the bit is the same on every lane, so each such
    // moment is its partner's diagonal sum (or, for two tile bits, the unit's
    // total) or zero; lane i writes the pair (i, c)
    if (m < n) {
      const double dT = (double)rows[kStash + kTotalSlot];
      const double dg = (double)rows[kStash + (lane < m ? lane : 0)];
      for (int c = m; c < n; ++c) {
        const bool xc = (local >> (c - m)) & 1;
        if (lane <= c) {
          const bool xi = lane < m || ((local >> ((lane - m) & 63)) & 1);
          out[pidx(n, lane, c)] = (xc && xi) ? (lane < m ? dg : dT) : 0.0;
        }
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) walk_grad_fac_kernel(
    Views v, const float* beta, const double* logz, int npairs) {
  walk_grad_body<0>(v, beta, logz, npairs);
}
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) walk_grad_direct_kernel(
    Views v, const float* beta, const double* logz, int npairs) {
  walk_grad_body<1>(v, beta, logz, npairs);
}

// One block per instance: sum the units' moments in order, scale, write.
// Outputs (each optional): grad_q / grad_beta (adjoint of logZ, scaled by
// grad_logz), moments (E_p[x_i x_j], float64) and mean (E_p[f]).
__global__ void finalize_grad_kernel(Views v, const float* q, const float* beta, const float* grad_logz,
                                     float* grad_q, float* grad_beta, double* moments, double* mean_out,
                                     int32_t* status, int npairs) {
  __shared__ double red[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const Inst* I = &v.inst[b];
  const int nm = v.nmax;
  const int32_t st = I->status;
  const int n = I->n;
  const double g = grad_logz ? (double)grad_logz[b] : 0.0;
  const double bt = (double)beta[b];
  const float* Q = q + (int64_t)b * nm * nm;
  double mean = 0.0;
  for (int idx = tid; idx < nm * nm; idx += blockDim.x) {
    const int i = idx / nm, j = idx % nm;
    float outv = 0.f;
    double M = 0.0;
    if (st == 0 && i <= j && j < n) {
      // the units in order, eight loads in flight ahead of their additions
      const double* pu = v.part + I->unit_begin * npairs + pidx(n, i, j);
      const int64_t nu = I->units;
      int64_t u = 0;
      for (; u + 8 <= nu; u += 8) {
        double x[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) x[d] = pu[(u + d) * npairs];
#pragma unroll
        for (int d = 0; d < 8; ++d) M += x[d];
      }
      for (; u < nu; ++u) M += pu[u * npairs];
      outv = (float)(g * -bt * M);
      mean += (double)Q[(int64_t)i * nm + j] * M;
    } else if (st != 0) {
      outv = __builtin_nanf("");
      M = __builtin_nan("");
    }
    if (grad_q) grad_q[(int64_t)b * nm * nm + idx] = outv;
    if (moments) moments[(int64_t)b * nm * nm + idx] = M;
  }
  red[tid] = mean;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    if (grad_beta) grad_beta[b] = st == 0 ? (float)(-g * red[0]) : __builtin_nanf("");
    if (mean_out) mean_out[b] = st == 0 ? red[0] : __builtin_nan("");
    status[b] = st;
  }
}

// ------------------------------------------------------------ sampling

// Inclusive prefix sum over the wave (double).
__device__ __forceinline__ double wave_scan(double x, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

// One wave per instance: running sums of the units' weights
// 2^(part[u] - log2 Z), in unit order.
__global__ void __launch_bounds__(kBlock) unit_cumsum_kernel(Views v, const double* logz, double* cum) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (b >= v.batch) return;
  const Inst* I = &v.inst[b];
  if (uniform_i32(I->status) != 0) return;
  const int64_t units = (int64_t)uniform_u64((uint64_t)I->units);
  const int64_t ub = (int64_t)uniform_u64((uint64_t)I->unit_begin);
  const double lz2 = uniform_f64(logz[b]) * kLog2e;
  double carry = 0.0;
  for (int64_t u0 = 0; u0 < units; u0 += kWave) {
    const int64_t u = u0 + lane;
    const double w = u < units ? exp2(v.part[ub + u] - lz2) : 0.0;
    const double incl = wave_scan(w, lane) + carry;
    if (u < units) cum[ub + u] = incl;
    carry = readlane_f64(incl, 63);
  }
}

// First lane with a positive weight whose inclusive prefix exceeds t; if
// rounding left t at or above the total, the last lane with a positive weight.
__device__ __forceinline__ int pick_lane(double w, double incl, double t) {
  const uint64_t over = ballot(incl > t && w > 0.0);
  if (over) return __builtin_ctzll(over);
  const uint64_t pos = ballot(w > 0.0);
  return pos ? 63 - __builtin_clzll(pos) : 0;
}

// t in [0, wp) as the same fraction of a total recomputed as wc, below wc.
__device__ __forceinline__ double rescale(double t, double wp, double wc) {
  const double f = wp > 0.0 ? t / wp : 0.0;
  return (f > 0.0 ? (f < 1.0 ? f : 0x1.fffffffffffffp-1) : 0.0) * wc;
}

// One wave per sample: inverts the cumulative distribution in natural mask
// order, whose bit groups from the top are the tile bits (the work unit), the
// lane bits, the outer bits and the inner bits.  The unit comes from the
// per-unit running sums, the lane from the forward walk's per-lane sums, the
// outer value from the chosen lane's block weights (one block per outer
// value, lanes take the steps in parallel), the inner state from the chosen
// block's 64 weights in float64.  The levels evaluate their weights in
// different precisions, so the leftover of one level is carried to the next
// as a fraction of the chosen entry's weight and rescaled by the next level's
// own total: each level inverts its own distribution exactly, and the sampled
// mask differs from the exact inverse only where u lies within the weights'
// rounding of a boundary.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
sample_kernel(Views v, const float* beta, const double* logz, const double* cum, int nsamples, const double* uin,
              uint64_t* mout) {
  __shared__ double ctab[kWavesPerBlock][kWaveRows * kWave];
  __shared__ double bw[kWavesPerBlock][1 << kSampleOuter];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* myc = ctab[w];
  double* myw = bw[w];
  const int64_t total = (int64_t)v.batch * nsamples;
  for (int64_t id = (int64_t)blockIdx.x * kWavesPerBlock + w; id < total;
       id += (int64_t)gridDim.x * kWavesPerBlock) {
    const int b = (int)(id / nsamples);
    const InstU I = load_inst(v, b);
    if (I.status != 0) {
      if (lane == 0) mout[id] = ~0ull;
      continue;
    }
    const int64_t units = (int64_t)uniform_u64((uint64_t)v.inst[b].units);
    const double bb = fabs((double)beta[b]) * kLog2e;
    const double lz2 = uniform_f64(logz[b]) * kLog2e;
    double ur = uniform_f64(uin[id]);
    ur = ur > 0.0 ? (ur < 1.0 ? ur : 0x1.fffffffffffffp-1) : 0.0;  // NaN -> 0
    // 1. unit: the first whose running sum exceeds t (the last if rounding
    // left none), 64 probes per round: lane q reads the last running sum of
    // block q of the remaining range, and the first block over t is kept
    const double* cb = cum + I.unit_begin;
    double t = ur * uniform_f64(cb[units - 1]);
    int64_t lo = 0, hi = units;  // the unit lies in [lo, hi)
    while (hi - lo > 1) {
      const int64_t stride = (hi - lo + kWave - 1) / kWave;
      int64_t idx = lo + (int64_t)(lane + 1) * stride - 1;
      if (idx > hi - 1) idx = hi - 1;
      const uint64_t over = ballot(cb[idx] > t);
      const int nblk = (int)((hi - lo + stride - 1) / stride);
      const int q = over ? __builtin_ctzll(over) : nblk - 1;
      const int64_t nlo = lo + (int64_t)q * stride;
      hi = nlo + stride < hi ? nlo + stride : hi;
      lo = nlo;
    }
    const double c0 = lo > 0 ? uniform_f64(cb[lo - 1]) : 0.0;
    double wp = uniform_f64(cb[lo]) - c0;  // weight of the chosen entry
    t -= c0;
    const uint64_t u = (uint64_t)(I.unit_begin + lo);
    const uint64_t local = (uint64_t)lo;
    // 2. lane
    const double lw = exp2(gp(v.lanepart)[u * kWave + lane] - lz2);
    const double lincl = wave_scan(lw, lane);
    t = rescale(t, wp, readlane_f64(lincl, kWave - 1));
    const int ls = pick_lane(lw, lincl, t);
    t -= readlane_f64(lincl - lw, ls);
    wp = readlane_f64(lw, ls);
    // 3. outer value.  Every lane takes lane ls's C' into registers in the
    // step tables' entry order (entry 4 (j mod 16) + j / 16 holds inner state
    // j) and its outer cross fields c_l.
    const bool valid = lane < (1 << I.L);
    float C[kInnerStates];
    const double EP = lane_init<float, kInnerStates>(v, b, I, local, valid, myc, lane, C);
    float cr[kInnerStates];
    float cj = 0.f;
#pragma unroll
    for (int j = 0; j < kInnerStates; ++j) {
      const float x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(C[j]), ls));
      cr[4 * (j & 15) + (j >> 4)] = x;
      if (lane == j) cj = x;
    }
    const double EPs = readlane_f64(EP, ls);
    __builtin_amdgcn_wave_barrier();
    double cl[kSampleOuter];
#pragma unroll
    for (int l = 0; l < kSampleOuter; ++l) cl[l] = l < I.no ? myc[l * kWave + ls] : 0.0;
    const float nb = bb > 0.0 ? (float)-bb : -1e-30f;  // beta = 0: sentinels still weigh 0
    const uint32_t steps = 1u << I.no;
    const gptr<const f32x4> tab4 = gp((const f32x4*)v.tab) + I.tab_off * (kInnerStates / 4);
    const gptr<const double> eod = gp((const double*)v.eod) + I.tab_off;
    for (uint32_t st = lane; st < steps; st += kWave) {
      const uint32_t o = (uint32_t)gray(st);
      double K = EPs + eod[st];
#pragma unroll
      for (int l = 0; l < kSampleOuter; ++l)
        if ((o >> l) & 1) K += cl[l];
      const float cst = (float)(-bb * K - lz2);
      const gptr<const f32x4> row = tab4 + (int64_t)st * (kInnerStates / 4);
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < kInnerStates / 4; ++q) {
        const f32x4 tq = row[q];
        acc[0] += exp2_fast(__builtin_fmaf(cr[4 * q + 0] + tq.x, nb, cst));
        acc[1] += exp2_fast(__builtin_fmaf(cr[4 * q + 1] + tq.y, nb, cst));
        acc[2] += exp2_fast(__builtin_fmaf(cr[4 * q + 2] + tq.z, nb, cst));
        acc[3] += exp2_fast(__builtin_fmaf(cr[4 * q + 3] + tq.w, nb, cst));
      }
      myw[o] = (double)((acc[0] + acc[1]) + (acc[2] + acc[3]));
    }
    __builtin_amdgcn_wave_barrier();
    // outer values in natural order: lane q sums values q*per .. q*per+per-1
    const int per = steps >= kWave ? (int)(steps / kWave) : 1;
    double part = 0.0;
    for (int k = 0; k < per; ++k) {
      const uint32_t o = (uint32_t)lane * per + k;
      if (o < steps) part += myw[o];
    }
    const double pincl = wave_scan(part, lane);
    t = rescale(t, wp, readlane_f64(pincl, kWave - 1));
    const int q = pick_lane(part, pincl, t);
    t -= readlane_f64(pincl - part, q);
    uint32_t os = (uint32_t)q * per;
    {
      uint32_t last = os;
      bool found = false;
      for (int k = 0; k < per && !found; ++k) {
        const uint32_t o = (uint32_t)q * per + k;
        if (o >= steps) break;
        const double x = myw[o];
        if (x > 0.0) {
          last = o;
          if (t < x) {
            os = o;
            found = true;
          } else {
            t -= x;
          }
        }
      }
      if (!found) os = last;
    }
    os = (uint32_t)uniform_i32((int)os);
    wp = myw[os];
    // 4. inner state of block (ls, os), weights in float64
    uint32_t ts = os;  // step with g(ts) = os
    for (int sh = 1; sh < 32; sh <<= 1) ts ^= ts >> sh;
    double Kb = EPs + uniform_f64(eod[ts]);
#pragma unroll
    for (int l = 0; l < kSampleOuter; ++l)
      if ((os >> l) & 1) Kb += cl[l];
    const float tj = gp((const float*)v.tab)[(I.tab_off + ts) * kInnerStates + 4 * (lane & 15) + (lane >> 4)];
    const double e = (double)cj + (double)tj + Kb;
    const double wj = cj < __builtin_inff() ? exp2(-bb * e - lz2) : 0.0;
    const double jincl = wave_scan(wj, lane);
    t = rescale(t, wp, readlane_f64(jincl, kWave - 1));
    const int js = pick_lane(wj, jincl, t);
    if (lane == 0) {
      const uint64_t hi = ((local << I.L) | (uint64_t)ls) << I.no | (uint64_t)os;
      mout[id] = (hi << I.B) | (uint64_t)js;
    }
    __builtin_amdgcn_wave_barrier();  // myw / myc are rewritten by the next sample
  }
}

}  // namespace

hipError_t launch_prep_exp_tables(const Views& v, const float* beta, int inner, int64_t steps_bound,
                                 hipStream_t s) {
  const int64_t per_inst = (steps_bound + v.batch - 1) / v.batch;  // steps of one instance, bound
  const dim3 grid((unsigned)v.batch, (unsigned)((per_inst + 63) / 64 > 0 ? (per_inst + 63) / 64 : 1));
  hipLaunchKernelGGL(prep_exp_tables_kernel, grid, dim3(256), 0, s, v, beta, inner);
  return hipGetLastError();
}

namespace {
int occupancy_blocks(const void* kernel) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}
}  // namespace

int walk_exp_blocks_per_cu() {
  static int cache = 0;
  if (!cache) cache = occupancy_blocks((const void*)walk_exp_fac_kernel);
  return cache;
}

int walk_grad_blocks_per_cu() {
  static int cache = 0;
  if (!cache) cache = occupancy_blocks((const void*)walk_grad_fac_kernel);
  return cache;
}

hipError_t launch_walk_exp(const Views& v, const float* beta, int waves, hipStream_t s) {
  const int blocks = max(1, (waves + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL(walk_exp_fac_kernel, dim3(blocks), dim3(kBlock), 0, s, v, beta);
  hipLaunchKernelGGL(walk_exp_direct_kernel, dim3(blocks), dim3(kBlock), 0, s, v, beta);
  return hipGetLastError();
}

hipError_t launch_finalize_logz(const Views& v, const float* beta, double* logz, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(finalize_logz_kernel, dim3((v.batch + 255) / 256), dim3(256), 0, s, v, beta, logz, status);
  return hipGetLastError();
}

hipError_t launch_walk_grad(const Views& v, const float* beta, const double* logz, int64_t total_waves,
                            int n_moments, hipStream_t s) {
  const int64_t nb = (total_waves + kWavesPerBlock - 1) / kWavesPerBlock;
  const int blocks = nb < 1 ? 1 : (int)nb;
  hipLaunchKernelGGL(walk_grad_fac_kernel, dim3(blocks), dim3(kBlock), 0, s, v, beta, logz, n_moments);
  hipLaunchKernelGGL(walk_grad_direct_kernel, dim3(blocks), dim3(kBlock), 0, s, v, beta, logz, n_moments);
  return hipGetLastError();
}

hipError_t launch_finalize_grad(const Views& v, const float* q, const float* beta, const float* grad_logz,
                                float* grad_q, float* grad_beta, double* moments, double* mean, int32_t* status,
                                int n_moments, hipStream_t s) {
  hipLaunchKernelGGL(finalize_grad_kernel, dim3(v.batch), dim3(256), 0, s, v, q, beta, grad_logz, grad_q,
                     grad_beta, moments, mean, status, n_moments);
  return hipGetLastError();
}

}  // namespace qbf

namespace qbf {

hipError_t launch_sample(const Views& v, const float* beta, const double* logz, double* cum, int nsamples,
                         const double* u, uint64_t* masks, int waves, hipStream_t s) {
  hipLaunchKernelGGL(unit_cumsum_kernel, dim3((v.batch + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0, s,
                     v, logz, cum);
  const int blocks = max(1, (waves + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL(sample_kernel, dim3(blocks), dim3(kBlock), 0, s, v, beta, logz, cum, nsamples, u, masks);
  return hipGetLastError();
}

}  // namespace qbf
