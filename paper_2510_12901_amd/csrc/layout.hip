// layout.hip -- spatial order of a resident particle set.
//
// The renderer's results do not depend on the order of the particles (every list is ordered by
// depth key, ties by index), but its memory traffic does: the projection reads every particle's
// SH coefficients component-major, and a camera sees a spatially compact subset.  With the
// particles stored along a Z-order (Morton) curve of their means, the visible ones of a view
// share cache lines, so the SH lines of invisible regions are never fetched.  The order is
// computed once per resident scene: bounding box of the finite means (two-level min/max), a
// 30-bit Morton code per particle (10 bits per axis; non-finite means last), and a stable radix
// sort of (code, index) with the library's onesweep passes.
#include "ut_internal.hpp"

namespace ut {
namespace {

constexpr int kBoxBlocks = 1024;

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// per block: min and max of each mean component over the finite means it visits
__global__ __launch_bounds__(256) void k_box_partial(const float* __restrict__ mean, int n, float* __restrict__ part) {
  __shared__ float s[6][4];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float x = mean[i], y = mean[n + i], z = mean[2 * n + i];
    if (isfinite(x) && isfinite(y) && isfinite(z)) {
      lo[0] = fminf(lo[0], x); lo[1] = fminf(lo[1], y); lo[2] = fminf(lo[2], z);
      hi[0] = fmaxf(hi[0], x); hi[1] = fmaxf(hi[1], y); hi[2] = fmaxf(hi[2], z);
    }
  }
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float a = wave_min(lo[c]), b = wave_max(hi[c]);
    if (lane == 0) { s[c][wave] = a; s[3 + c][wave] = b; }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int c = threadIdx.x;
    float v = s[c][0];
    for (int w = 1; w < 4; ++w) v = c < 3 ? fminf(v, s[c][w]) : fmaxf(v, s[c][w]);
    part[(size_t)c * kBoxBlocks + blockIdx.x] = v;
  }
}

// one block: the partial boxes -> box[6] (min x, y, z, max x, y, z)
__global__ __launch_bounds__(256) void k_box_final(const float* __restrict__ part, float* __restrict__ box) {
  __shared__ float s[6][4];
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    float v = c < 3 ? INFINITY : -INFINITY;
    for (int b = threadIdx.x; b < kBoxBlocks; b += 256) {
      const float p = part[(size_t)c * kBoxBlocks + b];
      v = c < 3 ? fminf(v, p) : fmaxf(v, p);
    }
    v = c < 3 ? wave_min(v) : wave_max(v);
    if (lane == 0) s[c][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int c = threadIdx.x;
    float v = s[c][0];
    for (int w = 1; w < 4; ++w) v = c < 3 ? fminf(v, s[c][w]) : fmaxf(v, s[c][w]);
    box[c] = v;
  }
}

// 10 bits spread to every third bit
__device__ __forceinline__ uint32_t spread10(uint32_t x) {
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ mean, int n, const float* __restrict__ box,
                                                 uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float x = mean[i], y = mean[n + i], z = mean[2 * n + i];
  uint32_t code = 0xFFFFFFFFu;   // non-finite means sort last
  if (isfinite(x) && isfinite(y) && isfinite(z)) {
    uint32_t q[3];
    const float p[3] = {x, y, z};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float ext = box[3 + c] - box[c];
      const float f = ext > 0.0f ? (p[c] - box[c]) / ext : 0.0f;
      q[c] = (uint32_t)fminf(fmaxf(f * 1023.0f, 0.0f), 1023.0f);
    }
    code = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
  }
  key[i] = code;
  val[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_copy_u32(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// dst[c][j] = src[c][perm[j]] for `rows` component rows of length n
__global__ __launch_bounds__(256) void k_gather_rows(const float* __restrict__ src, const uint32_t* __restrict__ perm,
                                                      float* __restrict__ dst, int rows, int n) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const uint32_t s = perm[j];
  for (int c = 0; c < rows; ++c) dst[(size_t)c * n + j] = src[(size_t)c * n + s];
}

}  // namespace

size_t spatial_order_ws_bytes(int n) {
  const size_t nn = (size_t)(n > 0 ? n : 1);
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  return al(4 * 6 * kBoxBlocks) + al(4 * 6) + 3 * al(4 * nn) + al(radix_ws_bytes(nn));
}

hipError_t launch_spatial_order(const ut_gaussians& g, uint32_t* perm, void* ws, hipStream_t st) {
  const int n = g.n;
  if (n == 0) return hipSuccess;
  const size_t nn = (size_t)n;
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  char* p = static_cast<char*>(ws);
  float* part = reinterpret_cast<float*>(p);
  p += al(4 * 6 * kBoxBlocks);
  float* box = reinterpret_cast<float*>(p);
  p += al(4 * 6);
  uint32_t* kA = reinterpret_cast<uint32_t*>(p);
  p += al(4 * nn);
  uint32_t* kB = reinterpret_cast<uint32_t*>(p);
  p += al(4 * nn);
  uint32_t* vB = reinterpret_cast<uint32_t*>(p);
  p += al(4 * nn);
  uint32_t* rws = reinterpret_cast<uint32_t*>(p);
  hipLaunchKernelGGL(k_box_partial, dim3(kBoxBlocks), dim3(256), 0, st, g.mean, n, part);
  hipLaunchKernelGGL(k_box_final, dim3(1), dim3(256), 0, st, part, box);
  const unsigned blocks = (unsigned)((n + 255) / 256);
  // the values start in perm (the caller's output) and the sort's result is copied there if
  // it ends in the other buffer
  hipLaunchKernelGGL(k_morton, dim3(blocks), dim3(256), 0, st, g.mean, n, box, kA, perm);
  uint32_t *kr, *vr;
  hipError_t e = radix_sort(kA, kB, perm, vB, nn, nullptr, 32, rws, st, &kr, &vr);
  if (e != hipSuccess) return e;
  if (vr != perm) hipLaunchKernelGGL(k_copy_u32, dim3(blocks), dim3(256), 0, st, vr, perm, n);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const float* src, const uint32_t* perm, float* dst, int rows, int n, hipStream_t st) {
  if (n == 0 || rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, perm, dst, rows, n);
  return hipGetLastError();
}

}  // namespace ut
