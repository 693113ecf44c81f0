// Bandwidth ceilings for the benchmark (not part of libwave's interface):
// plain streams of the step kernel's traffic shape, hand-written for gfx950.
//
//   probe_stream_3r1w: d[i] = a[i] + b[i] * c[i]   (3 reads + 1 write, like one
//                      float32 step: A^n, A^{n-1}, m read; A^{n+1} written)
//   probe_copy:        d[i] = a[i]                 (1 read + 1 write)
//   probe_stream_16bit: the 16-bit storage step's traffic: A and V read at
//                      2 B per node, m at 4 B (or 2 B as 16-bit codes),
//                      A' and V' written at 2 B; four nodes per lane (8-B
//                      accesses, like the step's 4-node lanes; 16-B lanes
//                      measured no faster)
//
// Same access policies as the step kernel: a (the A^n role) with the regular
// cache policy, b and c (read once) and the store nontemporal.  Each lane
// moves 16 B per access, a workgroup owns a contiguous block, and workgroup
// ids are remapped so each of the 8 XCDs owns a contiguous run of blocks.
// One access per lane and array (4 KB per array per workgroup, many short
// workgroups) is the fastest form measured: 6.4 TB/s for the 3r1w stream at
// 512^3 against 6.0 with four accesses per lane, and persistent grids that
// loop over blocks were slower still (5.5-6.0).
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kThreads = 256;
constexpr int kPerThread = 1;  // f4 per lane per array
constexpr size_t kBlock = size_t(kThreads) * kPerThread * 4;  // floats per workgroup

__device__ __forceinline__ size_t block_of() {
  const unsigned nwg = gridDim.x, bid = blockIdx.x;
  return static_cast<size_t>((bid & 7u) * (nwg >> 3) + (bid >> 3));
}

__global__ void __launch_bounds__(kThreads) stream_3r1w(const f4 *__restrict__ a, const f4 *__restrict__ b,
                                                         const f4 *__restrict__ c, f4 *__restrict__ d,
                                                         size_t n4) {
  const size_t base = block_of() * (kBlock / 4) + threadIdx.x;
  f4 va[kPerThread], vb[kPerThread], vc[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const size_t i = base + static_cast<size_t>(k) * kThreads;
    if (i < n4) {
      va[k] = a[i];
      vb[k] = __builtin_nontemporal_load(&b[i]);
      vc[k] = __builtin_nontemporal_load(&c[i]);
    }
  }
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const size_t i = base + static_cast<size_t>(k) * kThreads;
    if (i < n4) {
      f4 r;
      r.x = fmaf(vb[k].x, vc[k].x, va[k].x);
      r.y = fmaf(vb[k].y, vc[k].y, va[k].y);
      r.z = fmaf(vb[k].z, vc[k].z, va[k].z);
      r.w = fmaf(vb[k].w, vc[k].w, va[k].w);
      __builtin_nontemporal_store(r, &d[i]);
    }
  }
}

__global__ void __launch_bounds__(kThreads) copy_1r1w(const f4 *__restrict__ a, f4 *__restrict__ d,
                                                       size_t n4) {
  const size_t base = block_of() * (kBlock / 4) + threadIdx.x;
  f4 va[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const size_t i = base + static_cast<size_t>(k) * kThreads;
    if (i < n4) va[k] = __builtin_nontemporal_load(&a[i]);
  }
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const size_t i = base + static_cast<size_t>(k) * kThreads;
    if (i < n4) __builtin_nontemporal_store(va[k], &d[i]);
  }
}

typedef uint32_t u2 __attribute__((ext_vector_type(2)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

// one group of four nodes per lane; A with the regular policy, the rest
// nontemporal, as the step kernel; vo may be v (updated in place, as V is)
template <bool M16>
__global__ void __launch_bounds__(kThreads) stream_16bit(const u2 *__restrict__ a, const u2 *v,
                                                          const void *__restrict__ m, u2 *__restrict__ ao, u2 *vo,
                                                          size_t ng) {
  const size_t i = block_of() * kThreads + threadIdx.x;
  if (i >= ng) return;
  const u2 xa = a[i];
  const u2 xv = __builtin_nontemporal_load(&v[i]);
  u2 xm;
  if constexpr (M16) {
    xm = __builtin_nontemporal_load(&static_cast<const u2 *>(m)[i]);
  } else {
    const u4 w = __builtin_nontemporal_load(&static_cast<const u4 *>(m)[i]);
    xm = u2{w.x ^ w.z, w.y ^ w.w};
  }
  __builtin_nontemporal_store(xa ^ xm, &ao[i]);
  __builtin_nontemporal_store(xv + xm, &vo[i]);
}

unsigned grid_for(size_t n) {  // whole blocks, rounded up to a multiple of 8 (the XCD remap)
  const size_t blocks = (n + kBlock - 1) / kBlock;
  return static_cast<unsigned>((blocks + 7) / 8 * 8);
}

}  // namespace

extern "C" {

// n float32 elements (a multiple of 4, arrays 16-byte aligned); returns the
// hipError_t of the launch (0 on success).
int probe_stream_3r1w(const float *a, const float *b, const float *c, float *d, size_t n, void *stream) {
  if (n % 4 || !a || !b || !c || !d) return static_cast<int>(hipErrorInvalidValue);
  hipLaunchKernelGGL(stream_3r1w, dim3(grid_for(n)), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const f4 *>(a), reinterpret_cast<const f4 *>(b),
                     reinterpret_cast<const f4 *>(c), reinterpret_cast<f4 *>(d), n / 4);
  return static_cast<int>(hipGetLastError());
}

// n nodes (a multiple of 4): a, v, ao, vo hold n 16-bit values, m n floats
// (m16 == 0) or n 16-bit codes (m16 != 0), all 16-byte aligned; vo may be v
int probe_stream_16bit(const void *a, const void *v, const void *m, void *ao, void *vo, size_t n, int m16,
                       void *stream) {
  if (n % 4 || !a || !v || !m || !ao || !vo) return static_cast<int>(hipErrorInvalidValue);
  const size_t ng = n / 4;
  const size_t blocks = (ng + kThreads - 1) / kThreads;
  const dim3 grid(static_cast<unsigned>((blocks + 7) / 8 * 8));
  auto *A = static_cast<const u2 *>(a), *V = static_cast<const u2 *>(v);
  auto *AO = static_cast<u2 *>(ao), *VO = static_cast<u2 *>(vo);
  if (m16)
    hipLaunchKernelGGL(stream_16bit<true>, grid, dim3(kThreads), 0, static_cast<hipStream_t>(stream), A, V, m, AO,
                       VO, ng);
  else
    hipLaunchKernelGGL(stream_16bit<false>, grid, dim3(kThreads), 0, static_cast<hipStream_t>(stream), A, V, m, AO,
                       VO, ng);
  return static_cast<int>(hipGetLastError());
}

int probe_copy(const float *a, float *d, size_t n, void *stream) {
  if (n % 4 || !a || !d) return static_cast<int>(hipErrorInvalidValue);
  hipLaunchKernelGGL(copy_1r1w, dim3(grid_for(n)), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const f4 *>(a), reinterpret_cast<f4 *>(d), n / 4);
  return static_cast<int>(hipGetLastError());
}

}  // extern "C"
