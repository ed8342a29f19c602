// Issue-rate probes of the FP32 vector ALU and of the LDS on gfx950, built as
// their own small library (libbz_peak.so) for the measurement script; not
// part of the collision library.
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

// LDS traffic: every thread reads (KIND 0) or writes (KIND 1) one 8-byte
// element per step, 16 steps per round at immediate offsets 2 KB apart from a
// base that moves with the round (64 consecutive lanes touch 512 consecutive
// bytes: no bank conflicts).  A read is consumed by one fma, a write stores
// one register pair per round, so the VALU issues at most one instruction per
// LDS instruction.
constexpr int kLdsElems = 8192;  // 64 KB of float2

template <int KIND>
__global__ __launch_bounds__(kThreads) void k_lds_rate(float* out, int iters) {
  __shared__ float2 buf[kLdsElems];
  const int t = threadIdx.x;
  for (int i = t; i < kLdsElems; i += kThreads) buf[i] = make_float2(float(i & 7), 1.0f);
  __syncthreads();
  float s = 0.0f;
  for (int it = 0; it < iters; ++it) {
    const int base = t + (it & 7) * 512;  // + 15 * 256 + 255 < kLdsElems
    const float2 w = make_float2(float(it), float(t));
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (KIND == 0) {
        const float2 v = buf[base + u * 256];
        s = __builtin_fmaf(v.x, v.y, s);
      } else {
        buf[base + u * 256] = w;
      }
    }
  }
  __syncthreads();
  if (KIND == 1) s = buf[t].x + buf[t + 4096].y;
  out[size_t(blockIdx.x) * kThreads + t] = s;
}

// LDS writes of one width (B = 4, 8 or 16 bytes per lane), one instruction
// each (hand-written, so that the compiler does not pair them): per round 16
// writes at offsets 256 B apart from a lane base that rotates with the round,
// all aligned and inside the 64 KB array, which is the kernel's only LDS
// allocation and so starts at LDS address 0.
typedef float v2f __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <int B>
__global__ __launch_bounds__(kThreads) void k_lds_write_width(float* out, int iters) {
  __shared__ v4f wbuf[4096];  // 64 KB
  const int t = threadIdx.x;
  for (int i = t; i < 4096; i += kThreads) wbuf[i] = v4f{1.0f, 2.0f, 3.0f, 4.0f};
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    // largest byte written: (255 + 15 * 256) * B + B - 1 = 4096 B - 1 < 65536
    const unsigned addr = unsigned(((t + (it & 3)) & 255) * B);
    const float fv = float(it);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if constexpr (B == 4) {
        asm volatile("ds_write_b32 %0, %1 offset:%2" ::"v"(addr), "v"(fv), "i"(u * 256 * B) : "memory");
      } else if constexpr (B == 8) {
        const v2f d = {fv, 1.0f};
        asm volatile("ds_write_b64 %0, %1 offset:%2" ::"v"(addr), "v"(d), "i"(u * 256 * B) : "memory");
      } else {
        const v4f d = {fv, 1.0f, 2.0f, 3.0f};
        asm volatile("ds_write_b128 %0, %1 offset:%2" ::"v"(addr), "v"(d), "i"(u * 256 * B) : "memory");
      }
    }
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __syncthreads();
  out[size_t(blockIdx.x) * kThreads + t] = wbuf[t].x + wbuf[(t + 2048) & 4095].y;
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

// kind 0: reads, 1: writes (8 bytes per lane each, paired by the compiler);
// 2, 3, 4: single ds_write_b32, _b64, _b128 (4, 8, 16 bytes per lane).  out must hold
// blocks * 256 floats on the current device.  Same protocol as bz_peak_valu;
// *rate returns LDS bytes per second over the whole device.
int bz_peak_lds(int kind, int blocks, int iters, int reps, float* out, double* rate, double* ms) {
  if (kind < 0 || kind > 4 || blocks <= 0 || iters <= 0 || reps <= 0 || !out || !rate || !ms) return -1;
  auto launch = [&]() {
    if (kind == 0) hipLaunchKernelGGL(k_lds_rate<0>, dim3(blocks), dim3(kThreads), 0, 0, out, iters);
    else if (kind == 1) hipLaunchKernelGGL(k_lds_rate<1>, dim3(blocks), dim3(kThreads), 0, 0, out, iters);
    else if (kind == 2) hipLaunchKernelGGL(k_lds_write_width<4>, dim3(blocks), dim3(kThreads), 0, 0, out, iters);
    else if (kind == 3) hipLaunchKernelGGL(k_lds_write_width<8>, dim3(blocks), dim3(kThreads), 0, 0, out, iters);
    else hipLaunchKernelGGL(k_lds_write_width<16>, dim3(blocks), dim3(kThreads), 0, 0, out, iters);
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
  const double width = kind == 2 ? 4.0 : (kind == 4 ? 16.0 : 8.0);
  const double bytes = double(blocks) * kThreads * double(iters) * 16.0 * width;
  *ms = per;
  *rate = bytes / (per * 1e-3);
  return 0;
}

}  // extern "C"
