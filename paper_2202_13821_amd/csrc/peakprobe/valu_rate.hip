// valu_rate.hip -- measured VALU issue rates on gfx950, the evidence behind
// the ALU peaks used for the kernels' roofline fractions.
//
// Each lane runs 16 independent chains of one instruction form (no memory in
// the loop); the time of the second of two identical launches gives
// instructions per SIMD cycle at the 2.4 GHz peak clock and, for FMAs, flop/s:
//   vop3_fma : v_fma_f32 with scalar operands (x = x * a + b)
//   vop2_fmac: v_fmac_f32_e32, all operands in VGPRs (x += y * z)
//   vop2_mul : v_mul_f32_e32 (x *= z)
//   vop3_nfma: v_fma_f32 with a negated operand, all operands in VGPRs (x -= y * z)
//   sgpr_fmac: v_fmac_f32_e32 with one scalar operand (x += y * a)
//   lit_fmaak: v_fmaak_f32, a literal constant operand (x = x * y + K)
//   fp64_fma : v_fma_f64
// Build: python -m paper_2202_13821_amd.csrc.peakprobe (or hipcc as below);
// run the binary on the GPU; it prints one line per form and grid size.
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops -o valu_rate valu_rate.hip
#include <hip/hip_runtime.h>

#include <cstdio>

template <class T, int MODE>
__global__ __launch_bounds__(256) void chains(T* out, int iters, T a, T b) {
  constexpr int C = 16;
  T x[C], y[C];
  const T z = T(0.999) + T(1e-7) * T(threadIdx.x);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    x[c] = T(threadIdx.x + c);
    y[c] = T(1e-3) * T(c + 1) + T(1e-9) * T(threadIdx.x);
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if constexpr (MODE == 0) x[c] = x[c] * a + b;  // a, b: kernel arguments (SGPRs)
      else if constexpr (MODE == 1) {
        if constexpr (sizeof(T) == 4)
          x[c] = __builtin_fmaf(y[c], z, x[c]);
        else
          x[c] = __builtin_fma(y[c], z, x[c]);
      }
      else if constexpr (MODE == 3)
        x[c] = __builtin_fmaf(-y[c], z, x[c]);  // VOP3 (negation modifier), all VGPRs
      else if constexpr (MODE == 4)
        x[c] = __builtin_fmaf(y[c], a, x[c]);  // v_fmac_f32 with one scalar operand
      else if constexpr (MODE == 5)
        x[c] = __builtin_fmaf(x[c], y[c], T(1.2345678));  // v_fmaak_f32: literal addend
      else
        x[c] = x[c] * z;
    }
  }
  T s = T(0);
#pragma unroll
  for (int c = 0; c < C; ++c) s += x[c];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;  // out holds gridDim.x * 256 elements
}

template <class T, int MODE>
static int run(const char* name, int blocks, int iters, double flops_per_op) {
  T* out = nullptr;
  if (hipMalloc(&out, sizeof(T) * (size_t)blocks * 256) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  chains<T, MODE><<<blocks, 256>>>(out, iters, T(0.999), T(0.001));
  if (hipDeviceSynchronize() != hipSuccess) return 1;
  (void)hipEventRecord(e0);
  chains<T, MODE><<<blocks, 256>>>(out, iters, T(0.999), T(0.001));
  (void)hipEventRecord(e1);
  if (hipEventSynchronize(e1) != hipSuccess) return 1;
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  const double wave_instr = 16.0 * iters * blocks * 256 / 64.0;
  const double per_simd = wave_instr / 1024.0;  // 256 CUs x 4 SIMDs
  const double cycles = ms * 1e-3 * 2.4e9;
  printf("%-9s blocks=%5d: %.3f ms, %.2f SIMD cycles per wavefront instruction, %.1f TFLOP/s\n", name, blocks, ms,
         cycles / per_simd, flops_per_op * 16.0 * iters * blocks * 256 / (ms * 1e-3) / 1e12);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  return 0;
}

int main() {
  int rc = 0;
  for (int b : {2048, 4096, 8192}) {
    rc |= run<float, 0>("vop3_fma", b, 10000, 2.0);
    rc |= run<float, 1>("vop2_fmac", b, 10000, 2.0);
    rc |= run<float, 2>("vop2_mul", b, 10000, 1.0);
    rc |= run<float, 3>("vop3_nfma", b, 10000, 2.0);
    rc |= run<float, 4>("sgpr_fmac", b, 10000, 2.0);
    rc |= run<float, 5>("lit_fmaak", b, 10000, 2.0);
    rc |= run<double, 0>("fp64_fma", b, 5000, 2.0);
  }
  return rc;
}
