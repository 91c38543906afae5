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
// Forward: a k = 1 top-k walk first publishes E_ref = min_x f(x) (the
// instance threshold); then every state contributes 2^a with
// a = -|beta| log2(e) (e_j + KE - E_ref) <= ~0, summed per lane in float32
// over the 64 inner states and in float64 over the steps, reduced over the
// wave and written per work unit; the finalize sums the units in order and
// returns logZ = -|beta| E_ref + ln S.
//
// Backward: each state's weight w = p(x) = 2^(-|beta| log2(e) (e_j + KE) -
// logZ log2(e)).  Per lane and unit the walk accumulates
//   W[j]          = sum_t w(t, j)                (inner x inner moments)
//   A[o][0]       = sum_t x_o(t) s(t),  s = sum_j w(t, j)
//   A[o][1+a]     = sum_t x_o(t) v_a(t), v_a = sum_j w(t, j) j_a
//   Bo[o1][o2]    = sum_t x_o1(t) x_o2(t) s(t)
// (x_o(t) = bit o of g(t), uniform across lanes) and at the end of the unit
// assembles the n(n+1)/2 moments sum w x_i x_j for the unit, the prefix bits
// entering through the lane's own bits and the unit's tile bits.
#include "walk.hpp"

namespace qbf {

namespace {

constexpr double kLog2e = 1.4426950408889634074;
constexpr int kGradInner = 5;
constexpr int kGradStates = 1 << kGradInner;
constexpr int kGradMaxOuter = 8;

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

// acc[Q&3] += 2^(fma(C'(16K+Q) + T'(16K+Q), nb, cst)) for Q = 0..15.
template <int K, int Q>
__device__ __forceinline__ void block_exp(float (&acc)[4], float t, const float* C, float nb, float cst) {
  const float e = row_bcast<Q>(t) + C[16 * K + Q];
  acc[Q & 3] += exp2_fast(__builtin_fmaf(e, nb, cst));
  if constexpr (Q + 1 < 16) block_exp<K, Q + 1>(acc, t, C, nb, cst);
}

__global__ void __launch_bounds__(kBlock) walk_exp_kernel(Views v, const float* beta) {
  __shared__ double ctab[kWavesPerBlock][kWaveRows * kWave];
  const int lane = threadIdx.x & 63;
  double* myc = ctab[threadIdx.x >> 6];
  const uint64_t total_units = uniform_u64(gp((const Header*)v.hdr)->total_units);
  WorkIter it(v, total_units);
  uint64_t u;
  while (it.next(v, lane, u)) {
    const int b = v.batch == 1 ? 0 : find_unit(v, u);
    const InstU I = load_inst(v, b);
    if (I.status != 0) {
      if (lane == 0) gp(v.part)[u] = 0.0;
      continue;
    }
    const uint64_t local = u - (uint64_t)I.unit_begin;
    const bool valid = lane < (1 << I.L);
    const uint64_t p = (local << I.L) | (uint64_t)lane;
    float C[kInnerStates];
    const double EP = lane_init<float, kInnerStates>(v, b, I, local, valid, myc, lane, C);
    const double bb = fabs((double)gp(beta)[b]) * kLog2e;
    const double eref = load_gthr(v, b);
    // beta = 0: a tiny negative slope keeps invalid table entries (+inf) at
    // weight 0 without changing any valid weight (2^cst, cst = 0).
    const float nb = bb > 0.0 ? (float)-bb : -1e-30f;
    const uint32_t steps = 1u << I.no;
    const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(gp((const float*)v.tab) + I.tab_off * kInnerStates), (short)0,
        (int)(steps * (uint32_t)(kInnerStates * sizeof(float))), 0x00020000);
    const int qoff = (lane & 15) * 16;
    const gptr<const StepRec> rec = gp((const StepRec*)v.rec) + I.tab_off;
    double K = EP;
    double S = 0.0;
    f32x4 tn = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(trs, qoff, 0, 0));
    double eon = rec[0].eo;
    for (uint32_t t = 0; t < steps; ++t) {
      const f32x4 tc = tn;
      const double eoc = eon;
      const uint32_t tt = t + 1 < steps ? t + 1 : t;
      tn = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(trs, qoff, (int)(tt * 256u), 0));
      eon = rec[tt].eo;
      if (t) {
        const int l = __builtin_ctz(t);
        K = __builtin_fma(((t >> (l + 1)) & 1) ? -1.0 : 1.0, myc[l * kWave + lane], K);
      }
      const float cst = (float)(-bb * (K + eoc - eref));
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      block_exp<0, 0>(acc, tc.x, C, nb, cst);
      block_exp<1, 0>(acc, tc.y, C, nb, cst);
      block_exp<2, 0>(acc, tc.z, C, nb, cst);
      block_exp<3, 0>(acc, tc.w, C, nb, cst);
      S += (double)((acc[0] + acc[1]) + (acc[2] + acc[3]));
    }
    S = wave_sum(S);
    if (lane == 0) gp(v.part)[u] = S;
  }
}

// One thread per instance: S = sum over its units (in unit order), logZ.
__global__ void finalize_logz_kernel(Views v, const float* beta, double* logz, int32_t* status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= v.batch) return;
  const Inst* I = &v.inst[b];
  int32_t st = I->status;
  double out = __builtin_nan("");
  if (st == 0) {
    double S = 0.0;
    for (int64_t u = 0; u < I->units; ++u) S += v.part[I->unit_begin + u];
    const double eref = dec_key(v.gthr[b]);
    out = -fabs((double)beta[b]) * eref + log(S);
  }
  logz[b] = out;
  status[b] = st;
}

// ------------------------------------------------------------ moment walk

template <int K, int Q>
__device__ __forceinline__ void block_w(float (&w)[kGradStates], float t, const float* C, float nb, float cst) {
  const float e = row_bcast<Q>(t) + C[16 * K + Q];
  w[16 * K + Q] = exp2_fast(__builtin_fmaf(e, nb, cst));
  if constexpr (Q + 1 < 16) block_w<K, Q + 1>(w, t, C, nb, cst);
}

// s = sum_j w_j and v_a = sum_j w_j j_a (a < 5) by a pairwise tree.
__device__ __forceinline__ void block_moments(const float (&w)[kGradStates], float& s, float (&va)[kGradInner]) {
  float lvl[16];
#pragma unroll
  for (int a = 0; a < kGradInner; ++a) va[a] = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    lvl[i] = w[2 * i] + w[2 * i + 1];
    va[0] += w[2 * i + 1];
  }
  int len = 16;
#pragma unroll
  for (int a = 1; a < kGradInner; ++a) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < len / 2) {
        va[a] += lvl[2 * i + 1];
        lvl[i] = lvl[2 * i] + lvl[2 * i + 1];
      }
    }
    len /= 2;
  }
  s = lvl[0];
}

__device__ __forceinline__ int pidx(int n, int i, int j) { return i * n - (i * (i - 1)) / 2 + (j - i); }

__global__ void __launch_bounds__(kBlock) walk_grad_kernel(Views v, const float* beta, const double* logz,
                                                          int npairs) {
  __shared__ double ctab[kWavesPerBlock][kWaveRows * kWave];
  const int lane = threadIdx.x & 63;
  double* myc = ctab[threadIdx.x >> 6];
  const uint64_t total_units = uniform_u64(gp((const Header*)v.hdr)->total_units);
  WorkIter it(v, total_units);
  uint64_t u;
  while (it.next(v, lane, u)) {
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
    const double lz2 = uniform_f64(gp(logz)[b]) * kLog2e;
    const float nb = bb > 0.0 ? (float)-bb : -1e-30f;  // see walk_exp_kernel
    const uint32_t steps = 1u << I.no;
    const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(gp((const float*)v.tab) + I.tab_off * kGradStates), (short)0,
        (int)(steps * (uint32_t)(kGradStates * sizeof(float))), 0x00020000);
    const int qoff = (lane & 15) * 8;
    const gptr<const StepRec> rec = gp((const StepRec*)v.rec) + I.tab_off;

    float W[kGradStates];
#pragma unroll
    for (int j = 0; j < kGradStates; ++j) W[j] = 0.f;
    float A[kGradMaxOuter][kGradInner + 1];
    float Bo[kGradMaxOuter * (kGradMaxOuter - 1) / 2];
#pragma unroll
    for (int o = 0; o < kGradMaxOuter; ++o)
#pragma unroll
      for (int c = 0; c <= kGradInner; ++c) A[o][c] = 0.f;
#pragma unroll
    for (int i = 0; i < kGradMaxOuter * (kGradMaxOuter - 1) / 2; ++i) Bo[i] = 0.f;

    double K = EP;
    f32x2 tn = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(trs, qoff, 0, 0));
    double eon = rec[0].eo;
    for (uint32_t t = 0; t < steps; ++t) {
      const f32x2 tc = tn;
      const double eoc = eon;
      const uint32_t tt = t + 1 < steps ? t + 1 : t;
      tn = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(trs, qoff, (int)(tt * 128u), 0));
      eon = rec[tt].eo;
      if (t) {
        const int l = __builtin_ctz(t);
        K = __builtin_fma(((t >> (l + 1)) & 1) ? -1.0 : 1.0, myc[l * kWave + lane], K);
      }
      const float cst = (float)(-bb * (K + eoc) - lz2);
      float w[kGradStates];
      block_w<0, 0>(w, tc.x, C, nb, cst);
      block_w<1, 0>(w, tc.y, C, nb, cst);
#pragma unroll
      for (int j = 0; j < kGradStates; ++j) W[j] += w[j];
      float s, va[kGradInner];
      block_moments(w, s, va);
      const uint32_t o = (uint32_t)gray(t);
#pragma unroll
      for (int a = 0; a < kGradMaxOuter; ++a) {
        if ((o >> a) & 1) {
          A[a][0] += s;
#pragma unroll
          for (int c = 0; c < kGradInner; ++c) A[a][1 + c] += va[c];
#pragma unroll
          for (int a2 = a + 1; a2 < kGradMaxOuter; ++a2)
            if ((o >> a2) & 1) Bo[a2 * (a2 - 1) / 2 + a] += s;
        }
      }
    }

    // ---- assemble the unit's moments sum_x w x_i x_j (i <= j)
    const int n = I.n, B = I.B, no = I.no, pos0 = B + no;
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
    auto put = [&](int i, int j, float x) {
      const double sum = (double)wave_sum(x);
      if (lane == 0) out[pidx(n, i, j)] = sum;
    };
    // inner x inner
#pragma unroll
    for (int a = 0; a < kGradInner; ++a) {
      if (a >= B) continue;
      put(a, a, vt[a]);
#pragma unroll
      for (int a2 = a + 1; a2 < kGradInner; ++a2) {
        if (a2 >= B) continue;
        float x = 0.f;
#pragma unroll
        for (int j = 0; j < kGradStates; ++j)
          if (((j >> a) & 1) && ((j >> a2) & 1)) x += W[j];
        put(a, a2, x);
      }
    }
    // inner x outer, outer x outer
#pragma unroll
    for (int o = 0; o < kGradMaxOuter; ++o) {
      if (o >= no) continue;
#pragma unroll
      for (int a = 0; a < kGradInner; ++a)
        if (a < B) put(a, B + o, A[o][1 + a]);
      put(B + o, B + o, A[o][0]);
#pragma unroll
      for (int o2 = o + 1; o2 < kGradMaxOuter; ++o2)
        if (o2 < no) put(B + o, B + o2, Bo[o2 * (o2 - 1) / 2 + o]);
    }
    // pairs with a prefix bit (lane or tile bits of this lane's prefix p)
    for (int c = pos0; c < n; ++c) {
      const bool xc = valid && ((p >> (c - pos0)) & 1);
#pragma unroll
      for (int a = 0; a < kGradInner; ++a)
        if (a < B) put(a, c, xc ? vt[a] : 0.f);
#pragma unroll
      for (int o = 0; o < kGradMaxOuter; ++o)
        if (o < no) put(B + o, c, xc ? A[o][0] : 0.f);
      for (int c2 = pos0; c2 <= c; ++c2) {
        const bool x2 = (p >> (c2 - pos0)) & 1;
        put(c2, c, (xc && x2) ? st : 0.f);
      }
    }
  }
}

// One block per instance: sum the units' moments in order, scale, write.
__global__ void finalize_grad_kernel(Views v, const float* q, const float* beta, const float* grad_logz,
                                     float* grad_q, float* grad_beta, int32_t* status, int npairs) {
  __shared__ double red[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const Inst* I = &v.inst[b];
  const int nm = v.nmax;
  const int32_t st = I->status;
  const int n = I->n;
  const double g = (double)grad_logz[b];
  const double bt = (double)beta[b];
  const float* Q = q + (int64_t)b * nm * nm;
  double mean = 0.0;
  for (int idx = tid; idx < nm * nm; idx += blockDim.x) {
    const int i = idx / nm, j = idx % nm;
    float outv = 0.f;
    if (st == 0 && i <= j && j < n) {
      double M = 0.0;
      for (int64_t u = 0; u < I->units; ++u) M += v.part[(I->unit_begin + u) * npairs + pidx(n, i, j)];
      outv = (float)(g * -bt * M);
      mean += (double)Q[(int64_t)i * nm + j] * M;
    } else if (st != 0) {
      outv = __builtin_nanf("");
    }
    grad_q[(int64_t)b * nm * nm + idx] = outv;
  }
  red[tid] = mean;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    if (grad_beta) grad_beta[b] = st == 0 ? (float)(-g * red[0]) : __builtin_nanf("");
    status[b] = st;
  }
}

}  // namespace

hipError_t launch_walk_exp(const Views& v, const float* beta, const double* eref, int waves, hipStream_t s) {
  (void)eref;
  const int blocks = max(1, (waves + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL(walk_exp_kernel, dim3(blocks), dim3(kBlock), 0, s, v, beta);
  return hipGetLastError();
}

hipError_t launch_finalize_logz(const Views& v, const float* beta, const double* eref, double* logz,
                                int32_t* status, hipStream_t s) {
  (void)eref;
  hipLaunchKernelGGL(finalize_logz_kernel, dim3((v.batch + 255) / 256), dim3(256), 0, s, v, beta, logz, status);
  return hipGetLastError();
}

hipError_t launch_walk_grad(const Views& v, const float* beta, const double* logz, int64_t total_waves,
                            int n_moments, hipStream_t s) {
  const int64_t nb = (total_waves + kWavesPerBlock - 1) / kWavesPerBlock;
  const int blocks = nb < 1 ? 1 : (int)nb;
  hipLaunchKernelGGL(walk_grad_kernel, dim3(blocks), dim3(kBlock), 0, s, v, beta, logz, n_moments);
  return hipGetLastError();
}

hipError_t launch_finalize_grad(const Views& v, const float* q, const float* beta, const float* grad_logz,
                                float* grad_q, float* grad_beta, int32_t* status, int n_moments, hipStream_t s) {
  hipLaunchKernelGGL(finalize_grad_kernel, dim3(v.batch), dim3(256), 0, s, v, q, beta, grad_logz, grad_q,
                     grad_beta, status, n_moments);
  return hipGetLastError();
}

}  // namespace qbf
