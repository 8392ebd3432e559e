// stream_probe.hip -- bandwidth ceiling of the step kernel's memory access pattern, without
// its arithmetic.  Same plane layout as the lattice Boltzmann state (19 population planes
// read from one buffer and written to the other, 4 previous-step planes read and rewritten
// in place, 1 porosity plane read), FP32, one node per thread, 256-wide tiles.  mode 0:
// every plane read at the node itself (aligned); mode 1: the population planes read at the
// upstream node of each lattice direction (the +-1 shifted pull of the real step, interior
// only); mode 2: as mode 1 with a blocked layout, where the 19 populations of each run of
// 64 consecutive nodes of a row are stored next to each other (element (i, x, y) at
// ((y nbx + x/64) 19 + i) 64 + x%64, nbx = pitch/64), so that a wave's accesses fall in a
// few contiguous 4.75 KB regions instead of 19 separate planes.  Used by bench.py --stream-probe to place the step kernel against the ceiling of
// its own access pattern.  Not part of the solver.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t rs(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float ld(rsrc_t r, uint32_t v, uint32_t s) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
}
__device__ __forceinline__ void st(float x, rsrc_t r, uint32_t v, uint32_t s) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, 2);
}

__global__ void __launch_bounds__(256) probe_kernel(const float *src, float *dst, float *d4, const float *phi,
                                                    int nx, int ny, int pitch, int plane, int mode) {
  const int ntx = (nx + 255) / 256;
  const int t = blockIdx.x;
  const int x = (t % ntx) * 256 + threadIdx.x;
  const int y = t / ntx;
  if (x >= nx || y >= ny) return;
  const uint32_t PB = (uint32_t)plane * 4u;
  const rsrc_t rsrc = rs(src, 19u * PB), rdst = rs(dst, 19u * PB), rd4 = rs(d4, 4u * PB), rphi = rs(phi, PB);
  const uint32_t c = (uint32_t)y * pitch + x;
  // upstream node of each direction, clamped to the domain
  const int ex[19] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 0, 1, 0, -1, 0, 0, 1, 0, -1, 0};
  const int ey[19] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 0, 1, 0, -1, 0, 0, 1, 0, -1};
  float acc = ld(rphi, c * 4u, 0);
  float v[19];
  const uint32_t nbx = (uint32_t)pitch >> 6;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    int sx = x, sy = y;
    if (mode) {
      sx = min(max(x - ex[i], 0), nx - 1);
      sy = min(max(y - ey[i], 0), ny - 1);
    }
    if (mode == 2)
      v[i] = ld(rsrc, ((((uint32_t)sy * nbx + ((uint32_t)sx >> 6)) * 19u) * 64u + ((uint32_t)sx & 63u)) * 4u,
                (uint32_t)i * 256u);
    else
      v[i] = ld(rsrc, ((uint32_t)sy * pitch + sx) * 4u, (uint32_t)i * PB);
  }
  float p[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) p[k] = ld(rd4, c * 4u, (uint32_t)k * PB);
  const uint32_t cb = ((((uint32_t)y * nbx + ((uint32_t)x >> 6)) * 19u) * 64u + ((uint32_t)x & 63u)) * 4u;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    if (mode == 2)
      st(v[i] + acc * 1e-30f, rdst, cb, (uint32_t)i * 256u);
    else
      st(v[i] + acc * 1e-30f, rdst, c * 4u, (uint32_t)i * PB);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) st(p[k] + acc * 1e-30f, rd4, c * 4u, (uint32_t)k * PB);
}

}  // namespace

// Runs `reps` launches of the probe on caller-provided device buffers (src and dst: 19 planes,
// d4: 4 planes, phi: 1 plane, each plane `plane` floats) and returns the average milliseconds
// per launch, or a negative value on a HIP error.
extern "C" __attribute__((visibility("default"))) double stream_probe_run(const float *src, float *dst, float *d4,
                                                                          const float *phi, int nx, int ny, int pitch,
                                                                          int plane, int mode, int reps) {
  if (nx < 1 || ny < 1 || pitch < nx || (long long)plane < (long long)pitch * ny || reps < 1) return -1.0;
  const int ntx = (nx + 255) / 256;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -2.0;
  hipLaunchKernelGGL(probe_kernel, dim3(ntx * ny), dim3(256), 0, 0, src, dst, d4, phi, nx, ny, pitch, plane, mode);
  (void)hipEventRecord(a, 0);
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(probe_kernel, dim3(ntx * ny), dim3(256), 0, 0, src, dst, d4, phi, nx, ny, pitch, plane, mode);
  (void)hipEventRecord(b, 0);
  (void)hipEventSynchronize(b);
  float ms = 0.f;
  const hipError_t e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return e == hipSuccess ? ms / reps : -3.0;
}
