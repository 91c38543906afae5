// Issue cost of the VALU instruction forms the walks are built from, on the
// device the library runs on: cycles per wave64 instruction per SIMD.
//
// A measurement tool beside the library (its own shared object), not part of
// the solver: the roofline fractions divide by one wave64 instruction per
// SIMD per four cycles, and this tool measures which forms issue at that rate
// and which faster.  Each form runs as eight independent dependency chains per
// wave, enough waves per SIMD to hide latency, and a loop of 16 instructions;
// the shader clock is read in the same kernel (s_memtime against the
// constant-rate s_memrealtime), so throttling does not bias the figure.
//
// valu_rate(form, waves_per_simd, iters, &ms, &mhz, &cycles) returns 0 on
// success, -1 for an unknown form or bad argument, -2 on a HIP error.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace {

constexpr int kForms = 20;

template <int F>
__global__ __launch_bounds__(256) void rate_kernel(float* out, long long* times, int iters, int sarg) {
  float a0 = threadIdx.x * 1e-3f, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6,
        a7 = a0 + 7;
  const float b = threadIdx.x * 1e-4f, c = 0.5f;
  double d0 = a0, d1 = a1, d2 = a2, d3 = a3;
  const double db = b;
  const long long t0 = clock64(), w0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
#define EIGHT(S) S(a0) S(a1) S(a2) S(a3) S(a4) S(a5) S(a6) S(a7)
    if constexpr (F == 0) {
#define S(a) asm volatile("v_add_f32 %0, %1, %0" : "+v"(a) : "v"(b));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 1) {
#define S(a) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 2) {
#define S(a) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(a) : "v"(b), "v"(c));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 3) {
#define S(a) asm volatile("v_add_u32 %0, %1, %0" : "+v"(a) : "v"(b));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 4) {
#define S(a) asm volatile("v_add_f32 %0, %1, %0" : "+v"(a) : "s"(sarg));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 5) {
#define S(a) asm volatile("v_min_f32 %0, %1, %0" : "+v"(a) : "v"(b));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 6) {
#define S(a) asm volatile("v_min3_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 7) {  // the DPP source is never written in the loop
#define S(a) asm volatile("v_add_f32_dpp %0, %1, %0 row_newbcast:1 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "+v"(a) : "v"(b));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 8) {
#define S(a) asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:1 row_mask:0xf bank_mask:0xf" : "+v"(a) : "v"(b), "v"(c));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 9) {
#define S(a) asm volatile("v_mul_f32_dpp %0, %1, %0 row_newbcast:1 row_mask:0xf bank_mask:0xf" : "+v"(a) : "v"(b));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 10) {
#define S(a) asm volatile("v_pk_add_f16 %0, %0, %1" : "+v"(a) : "v"(b));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 11) {
#define S(a) asm volatile("v_pk_add_f16 %0, %0, %1 op_sel:[0,1] op_sel_hi:[1,1]" : "+v"(a) : "s"(sarg));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 12) {
#define S(a) asm volatile("v_pk_min_f16 %0, %0, %1" : "+v"(a) : "v"(b));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 13) {
#define S(a) asm volatile("v_pk_minimum3_f16 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 14) {
#define S(d) asm volatile("v_fmac_f64 %0, %1, %1" : "+v"(d) : "v"(db));
      S(d0) S(d1) S(d2) S(d3) S(d0) S(d1) S(d2) S(d3) S(d0) S(d1) S(d2) S(d3) S(d0) S(d1) S(d2) S(d3)
#undef S
    } else if constexpr (F == 15) {
#define S(a) asm volatile("v_exp_f32 %0, %0" : "+v"(a));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 16) {  // float32 screen: two DPP adds per three-input minimum
#define S(a) asm volatile("v_add_f32_dpp %0, %1, %0 row_newbcast:1 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "+v"(a) : "v"(b));
#define M(a) asm volatile("v_min3_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
      S(a0) S(a1) M(a2) S(a3) S(a4) M(a5) S(a6) S(a7) M(a0) S(a1) S(a2) M(a3) S(a4) S(a5) M(a6) S(a7)
#undef S
#undef M
    } else if constexpr (F == 17) {  // float16 screen: two packed adds (scalar operand) per minimum3
#define S(a) asm volatile("v_pk_add_f16 %0, %0, %1 op_sel:[0,1] op_sel_hi:[1,1]" : "+v"(a) : "s"(sarg));
#define M(a) asm volatile("v_pk_minimum3_f16 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
      S(a0) S(a1) M(a2) S(a3) S(a4) M(a5) S(a6) S(a7) M(a0) S(a1) S(a2) M(a3) S(a4) S(a5) M(a6) S(a7)
#undef S
#undef M
    } else if constexpr (F == 18) {
#define S(a) asm volatile("v_pk_add_i16 %0, %0, %1 op_sel:[0,1] op_sel_hi:[1,1]" : "+v"(a) : "s"(sarg));
      EIGHT(S) EIGHT(S)
#undef S
    } else if constexpr (F == 19) {
#define S(a) asm volatile("v_pk_min_i16 %0, %0, %1" : "+v"(a) : "v"(b));
      EIGHT(S) EIGHT(S)
#undef S
    }
#undef EIGHT
  }
  const long long t1 = clock64(), w1 = wall_clock64();
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  out[gid] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7 + (float)(d0 + d1 + d2 + d3);
  if ((threadIdx.x & 63) == 0) {
    times[2 * (gid >> 6)] = t1 - t0;
    times[2 * (gid >> 6) + 1] = w1 - w0;
  }
}

using KernelFn = void (*)(float*, long long*, int, int);

template <int F>
void fill(KernelFn* t) {
  t[F] = rate_kernel<F>;
  if constexpr (F + 1 < kForms) fill<F + 1>(t);
}

}  // namespace

extern "C" const char* valu_rate_form_name(int form) {
  static const char* names[kForms] = {
      "v_add_f32",         "v_fmac_f32",           "v_fma_f32 (VOP3)",      "v_add_u32",
      "v_add_f32 sgpr",    "v_min_f32",            "v_min3_f32",            "v_add_f32_dpp row_newbcast",
      "v_fmac_f32_dpp",    "v_mul_f32_dpp",        "v_pk_add_f16",          "v_pk_add_f16 sgpr op_sel",
      "v_pk_min_f16",      "v_pk_minimum3_f16",    "v_fmac_f64",            "v_exp_f32",
      "float32 screen mix (2 dpp add : 1 min3)",   "float16 screen mix (2 pk_add sgpr : 1 pk_minimum3)",
      "v_pk_add_i16 sgpr op_sel",                  "v_pk_min_i16"};
  return form >= 0 && form < kForms ? names[form] : nullptr;
}

extern "C" int valu_rate_forms(void) { return kForms; }

extern "C" int valu_rate(int form, int waves_per_simd, int iters, float* ms_out, double* mhz_out,
                         double* cycles_out) {
  if (form < 0 || form >= kForms || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || !ms_out ||
      !mhz_out || !cycles_out)
    return -1;
  static KernelFn table[kForms];
  if (!table[0]) fill<0>(table);
  int dev = 0, cus = 0, wclk_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -2;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -2;
  if (hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return -2;
  // one workgroup of four waves per CU per wave-per-SIMD
  const int blocks = cus * waves_per_simd, threads = blocks * 256, waves = threads / 64;
  float* out = nullptr;
  long long* times = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = -2;
  std::vector<long long> t(2 * (size_t)waves);
  float ms = 0.f;
  if (hipMalloc(&out, (size_t)threads * sizeof(float)) != hipSuccess) goto done;
  if (hipMalloc(&times, t.size() * sizeof(long long)) != hipSuccess) goto done;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up
    if (hipEventRecord(e0, nullptr) != hipSuccess) goto done;
    hipLaunchKernelGGL(table[form], dim3(blocks), dim3(256), 0, nullptr, out, times, iters, 0x3c003c00);
    if (hipGetLastError() != hipSuccess) goto done;
    if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) goto done;
  }
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) goto done;
  if (hipMemcpy(t.data(), times, t.size() * sizeof(long long), hipMemcpyDeviceToHost) != hipSuccess) goto done;
  {
    double sc = 0, sw = 0;
    for (int w = 0; w < waves; ++w) {
      sc += (double)t[2 * w];
      sw += (double)t[2 * w + 1];
    }
    const double mhz = sw > 0 ? sc / sw * wclk_khz / 1000.0 : 0.0;
    *ms_out = ms;
    *mhz_out = mhz;
    // SIMD cycles of the launch over the wave64 instructions each SIMD issued
    *cycles_out = (double)ms * 1e-3 * mhz * 1e6 * (4.0 * cus) / (16.0 * iters * waves);
    rc = 0;
  }
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  if (times) (void)hipFree(times);
  return rc;
}
