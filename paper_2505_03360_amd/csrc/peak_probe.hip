// Issue-rate probe of the FP32 vector ALU on gfx950, built as its own small
// library (libbz_peak.so) for the measurement script; not part of the
// collision library.
//
// Every thread runs eight independent dependency chains of one unpacked FP32
// operation (fma, add or mul) for `iters` rounds and stores the sum of its
// chains once, so the only memory traffic is one float per thread.  The
// library is compiled without packed FP32 instructions, like the collision
// kernels, so the rate it measures is the one those kernels can reach.
#include <hip/hip_runtime.h>
#include <cstdint>

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;

template <int KIND>
__global__ __launch_bounds__(kThreads) void k_valu_rate(float* out, int iters, float b, float c) {
  float a[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) a[i] = float(threadIdx.x + i) * 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int i = 0; i < kChains; ++i) {
        if (KIND == 0) a[i] = __builtin_fmaf(a[i], b, c);
        else if (KIND == 1) a[i] = a[i] + c;
        else if (KIND == 2) a[i] = a[i] * b;
        else a[i] = __builtin_fmaf(b, c, a[i]);  // accumulating form (v_fmac_f32)
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < kChains; ++i) s += a[i];
  out[size_t(blockIdx.x) * kThreads + threadIdx.x] = s;
}

}  // namespace

extern "C" {

// kind 0: v_fma_f32 and 3: v_fmac_f32 (2 flop each), 1: v_add_f32, 2: v_mul_f32
// (1 flop each).
// out must hold blocks * 256 floats on the current device.  Runs the kernel
// once untimed, then `reps` times between two events on the null stream, and
// returns the FP32 operations per second achieved (flop/s) through *rate and
// the average kernel time in *ms.  Returns 0, or a hipError_t value.
int bz_peak_valu(int kind, int blocks, int iters, int reps, float* out, double* rate, double* ms) {
  if (kind < 0 || kind > 3 || blocks <= 0 || iters <= 0 || reps <= 0 || !out || !rate || !ms) return -1;
  auto launch = [&]() {
    const float b = 0.9999f, c = 1e-4f;
    if (kind == 0) hipLaunchKernelGGL(k_valu_rate<0>, dim3(blocks), dim3(kThreads), 0, 0, out, iters, b, c);
    else if (kind == 1) hipLaunchKernelGGL(k_valu_rate<1>, dim3(blocks), dim3(kThreads), 0, 0, out, iters, b, c);
    else if (kind == 2) hipLaunchKernelGGL(k_valu_rate<2>, dim3(blocks), dim3(kThreads), 0, 0, out, iters, b, c);
    else hipLaunchKernelGGL(k_valu_rate<3>, dim3(blocks), dim3(kThreads), 0, 0, out, iters, b, c);
  };
  launch();
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return int(e);
  e = hipEventCreate(&e1);
  if (e != hipSuccess) { (void)hipEventDestroy(e0); return int(e); }
  (void)hipEventRecord(e0, 0);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, 0);
  e = hipEventSynchronize(e1);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e == hipSuccess) e = hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return int(e);
  const double per = double(t) / reps;
  const double ops = double(blocks) * kThreads * double(iters) * 8.0 * kChains * (kind == 0 || kind == 3 ? 2.0 : 1.0);
  *ms = per;
  *rate = ops / (per * 1e-3);
  return 0;
}

}  // extern "C"
