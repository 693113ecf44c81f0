// gfx950 kernels of libwave other than the step kernel (whose templates
// live in step_kernels.h): the CPML boundary passes, setup, decode,
// gather/scatter, gradient and fill kernels, and the launchers.
#include "step_kernels.h"

namespace wave {
namespace {

// ------------------------------------------------------------ CPML boundary
//
// The convolutional PML the paper names as its boundary (Sec. II, Sec.
// IV-A), for the second-order acoustic equation: per axis a memory variable
// psi_a of the first derivative and zeta_a of the second,
//   psi_a^n  = b psi_a^{n-1}  + a D1_a p^n
//   zeta_a^n = b zeta_a^{n-1} + a (D2_a p^n + D1_a psi_a^n)
//   p^{n+1}  = (plain leapfrog step) + m sum_a (D1_a psi_a^n + zeta_a^n).
// Both kernels run one thread per node of the boundary shell: the planes of
// the z layers, then the rows of the y layers in the remaining planes, then
// the columns of the x layers in the remaining rows (each node once).

// Node t of the boundary shell for layers of E nodes: the planes of the z
// layers, then in the remaining planes the rows of the y layers, then in the
// remaining rows the columns of the x layers (every shell node once).  32-bit
// index arithmetic: the host keeps the shell below 2^31 nodes.
struct Shell {
  unsigned nx, ny, nz, E, cz, cy, cx, mz, my, n0, n1, n2;
  __host__ __device__ Shell(int e, int x, int y, int z) {
    nx = x;
    ny = y;
    nz = z;
    E = e;
    cz = nz < 2u * E ? nz : 2u * E;
    cy = ny < 2u * E ? ny : 2u * E;
    cx = nx < 2u * E ? nx : 2u * E;
    mz = nz - cz;
    my = ny - cy;
    n0 = cz * ny * nx;
    n1 = mz * cy * nx;
    n2 = mz * my * cx;
  }
  __host__ __device__ unsigned count() const { return n0 + n1 + n2; }
  __device__ void node(unsigned t, int &x, int &y, int &z) const {
    if (t < n0) {
      const unsigned k = t / (ny * nx), r = t - k * (ny * nx);
      z = static_cast<int>(k < E ? k : nz - cz + k);
      y = static_cast<int>(r / nx);
      x = static_cast<int>(r - (r / nx) * nx);
      return;
    }
    t -= n0;
    if (t < n1) {
      const unsigned row = t / nx, k = row % cy;
      z = static_cast<int>(E + row / cy);
      y = static_cast<int>(k < E ? k : ny - cy + k);
      x = static_cast<int>(t - row * nx);
      return;
    }
    t -= n1;
    const unsigned row = t / cx, k = t - row * cx;
    z = static_cast<int>(E + row / my);
    y = static_cast<int>(E + row % my);
    x = static_cast<int>(k < E ? k : nx - cx + k);
  }
};

// Per-axis addressing of one node: coordinate i along the axis, axis length
// n, field stride, and the node's offset in the axis' slab array without its
// slab index (plus the slab stride), 32-bit.
struct AxisAt {
  int i, n;
  unsigned stride, slab_rest, slab_stride;
};

__device__ __forceinline__ AxisAt axis_at(const CpmlArgs &c, int a, int x, int y, int z) {
  const unsigned nx = c.nx, ny = c.ny, W2 = 2u * c.W;
  AxisAt r;
  if (a == 0) {
    r = {x, c.nx, 1u, (static_cast<unsigned>(z) * ny + y) * W2, 1u};
  } else if (a == 1) {
    r = {y, c.ny, nx, static_cast<unsigned>(z) * W2 * nx + x, nx};
  } else {
    r = {z, c.nz, nx * ny, static_cast<unsigned>(y) * nx + x, ny * nx};
  }
  return r;
}

// psi_a at the node k steps along the axis (zero outside the layers).
__device__ __forceinline__ float psi_k(const CpmlArgs &c, int a, const AxisAt &A, int k) {
  const int s = slab_index(A.i + k, A.n, c.W);
  return s < 0 ? 0.f : c.psi[a][A.slab_rest + static_cast<unsigned>(s) * A.slab_stride];
}

// cur at the node k steps along the axis (zero outside the grid).
__device__ __forceinline__ float cur_k(const float *cur, unsigned o, const AxisAt &A, int k) {
  const int j = A.i + k;
  return (j < 0 || j >= A.n) ? 0.f : cur[static_cast<int>(o) + k * static_cast<int>(A.stride)];
}

// Row r of the shell's first two parts (the rows of its z-layer planes, then
// its y-layer rows in the remaining planes) as (y, z).
__device__ __forceinline__ void shell_row(const Shell &S, unsigned r, int &y, int &z) {
  const unsigned r0 = S.cz * S.ny;
  if (r < r0) {
    const unsigned k = r / S.ny;
    y = static_cast<int>(r - k * S.ny);
    z = static_cast<int>(k < S.E ? k : S.nz - S.cz + k);
    return;
  }
  r -= r0;
  const unsigned k = r / S.cy, j = r - k * S.cy;
  z = static_cast<int>(S.E + k);
  y = static_cast<int>(j < S.E ? j : S.ny - S.cy + j);
}

template <int VEC> __device__ __forceinline__ void vload(const float *p, float *v) { lds_get<VEC>(p, v); }
template <int VEC> __device__ __forceinline__ void vstore(float *p, const float *v) { lds_put<VEC>(p, v); }

// psi_a update over the rows of the first two parts of the W-node shell, VEC
// consecutive x nodes per thread (nx % VEC == 0): the y and z axes where the
// row lies in their layers (whole rows), the x axis for the nodes of the row
// in the x layers.
template <int VEC>
__global__ void __launch_bounds__(256) cpml_psi_rows_kernel(CpmlArgs c, const float *__restrict__ cur) {
  const Shell S(c.W, c.nx, c.ny, c.nz);
  const unsigned qx = static_cast<unsigned>(c.nx) / VEC;
  const unsigned t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (S.cz * S.ny + S.mz * S.cy) * qx) return;
  const unsigned r = t / qx;
  const int x = static_cast<int>((t - r * qx) * VEC);
  int y, z;
  shell_row(S, r, y, z);
  const unsigned nx = c.nx, ny = c.ny, W2 = 2u * c.W;
  const unsigned o = (static_cast<unsigned>(z) * ny + y) * nx + x;
#pragma unroll
  for (int a = 1; a < 3; ++a) {
    const int i = a == 1 ? y : z, n = a == 1 ? c.ny : c.nz;
    const int s = slab_index(i, n, c.W);
    if (s < 0) continue;
    const unsigned stride = a == 1 ? nx : nx * ny;
    float d[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) d[e] = 0.f;
#pragma unroll
    for (int m = 1; m <= R; ++m) {
      float up[VEC], dn[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) up[e] = dn[e] = 0.f;
      if (i + m < n) vload<VEC>(cur + o + m * stride, up);
      if (i - m >= 0) vload<VEC>(cur + o - m * stride, dn);
#pragma unroll
      for (int e = 0; e < VEC; ++e) d[e] = fmaf(c.d1w[a][m - 1], up[e] - dn[e], d[e]);
    }
    float *ps = c.psi[a] + (a == 1 ? (static_cast<unsigned>(z) * W2 + s) * nx : (s * ny + static_cast<unsigned>(y)) * nx) + x;
    float pv[VEC];
    vload<VEC>(ps, pv);
#pragma unroll
    for (int e = 0; e < VEC; ++e) pv[e] = fmaf(c.cb[a][i], pv[e], c.ca[a][i] * d[e]);
    vstore<VEC>(ps, pv);
  }
  if (x < c.W || x + VEC - 1 >= c.nx - c.W) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int xe = x + e;
      const int s = slab_index(xe, c.nx, c.W);
      if (s < 0) continue;
      float d = 0.f;
#pragma unroll
      for (int m = 1; m <= R; ++m) {
        const float up = xe + m < c.nx ? cur[o + e + m] : 0.f;
        const float dn = xe - m >= 0 ? cur[o + e - m] : 0.f;
        d = fmaf(c.d1w[0][m - 1], up - dn, d);
      }
      float *ps = c.psi[0] + (static_cast<unsigned>(z) * ny + y) * W2 + s;
      *ps = fmaf(c.cb[0][xe], *ps, c.ca[0][xe] * d);
    }
  }
}

// One thread per node of the W-node shell from node t0 on (the x-layer
// columns of its third part, after cpml_psi_rows_kernel; or all of it).
__global__ void __launch_bounds__(256) cpml_psi_kernel(CpmlArgs c, const float *__restrict__ cur, unsigned t0) {
  const Shell S(c.W, c.nx, c.ny, c.nz);
  const unsigned t = t0 + blockIdx.x * 256u + threadIdx.x;
  if (t >= S.count()) return;
  int x, y, z;
  S.node(t, x, y, z);
  const unsigned o = (static_cast<unsigned>(z) * c.ny + y) * c.nx + x;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const AxisAt A = axis_at(c, a, x, y, z);
    const int s = slab_index(A.i, A.n, c.W);
    if (s < 0) continue;
    float d = 0.f;
#pragma unroll
    for (int m = 1; m <= R; ++m) d = fmaf(c.d1w[a][m - 1], cur_k(cur, o, A, m) - cur_k(cur, o, A, -m), d);
    float *ps = c.psi[a] + A.slab_rest + static_cast<unsigned>(s) * A.slab_stride;
    *ps = fmaf(c.cb[a][A.i], *ps, c.ca[a][A.i] * d);
  }
}

// The y and z terms after the step with the x part fused in:
// out += m * sum_{a = y, z} (D1_a psi_a + zeta_a), zeta_a updated, over the
// rows of the first two parts of the (W + R)-node shell (the other nodes get
// no y or z term), VEC consecutive x nodes per thread (nx % VEC == 0).  Per
// node the same operations as cpml_fix_kernel with a0 = 1.
template <int VEC>
__global__ void __launch_bounds__(256) cpml_fix_yz_kernel(CpmlArgs c, const float *__restrict__ cur,
                                                          const float *__restrict__ m, float *out) {
  const Shell S(c.W + R, c.nx, c.ny, c.nz);
  const unsigned qx = static_cast<unsigned>(c.nx) / VEC;
  const unsigned t = blockIdx.x * 256u + threadIdx.x;
  if (t >= (S.cz * S.ny + S.mz * S.cy) * qx) return;
  const unsigned r = t / qx;
  const int x = static_cast<int>((t - r * qx) * VEC);
  int y, z;
  shell_row(S, r, y, z);
  const unsigned nx = c.nx, ny = c.ny, W2 = 2u * c.W;
  const unsigned o = (static_cast<unsigned>(z) * ny + y) * nx + x;
  float extra[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) extra[e] = 0.f;
#pragma unroll
  for (int a = 1; a < 3; ++a) {
    const int i = a == 1 ? y : z, n = a == 1 ? c.ny : c.nz;
    if (i >= c.W + R && i < n - c.W - R) continue;  // psi_a and zeta_a vanish this far in
    const unsigned stride = a == 1 ? nx : nx * ny;
    // slab element of slab index s: y: (z, s, x), z: (s, y, x)
    auto slab = [&](int sidx) {
      return a == 1 ? (static_cast<unsigned>(z) * W2 + static_cast<unsigned>(sidx)) * nx + x
                    : (static_cast<unsigned>(sidx) * ny + static_cast<unsigned>(y)) * nx + x;
    };
    float dpsi[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) dpsi[e] = 0.f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
      float pp[VEC], pm[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) pp[e] = pm[e] = 0.f;
      const int sp = slab_index(i + k, n, c.W), sm = slab_index(i - k, n, c.W);
      if (sp >= 0) vload<VEC>(c.psi[a] + slab(sp), pp);
      if (sm >= 0) vload<VEC>(c.psi[a] + slab(sm), pm);
#pragma unroll
      for (int e = 0; e < VEC; ++e) dpsi[e] = fmaf(c.d1w[a][k - 1], pp[e] - pm[e], dpsi[e]);
    }
    const int s = slab_index(i, n, c.W);
    if (s < 0) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) extra[e] += dpsi[e];
      continue;
    }
    float cc[VEC], d2[VEC];
    vload<VEC>(cur + o, cc);
#pragma unroll
    for (int e = 0; e < VEC; ++e) d2[e] = 0.f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {  // second differences from the centre (no large centre term)
      float up[VEC], dn[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) up[e] = dn[e] = 0.f;
      if (i + k < n) vload<VEC>(cur + o + k * stride, up);
      if (i - k >= 0) vload<VEC>(cur + o - k * stride, dn);
#pragma unroll
      for (int e = 0; e < VEC; ++e) d2[e] = fmaf(c.d2w[a][k], (up[e] - cc[e]) + (dn[e] - cc[e]), d2[e]);
    }
    float *ze = c.zeta[a] + slab(s);
    float zv[VEC];
    vload<VEC>(ze, zv);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      zv[e] = fmaf(c.cb[a][i], zv[e], c.ca[a][i] * (d2[e] + dpsi[e]));
      extra[e] += dpsi[e] + zv[e];
    }
    vstore<VEC>(ze, zv);
  }
  float mv[VEC], ov[VEC];
  vload<VEC>(m + o, mv);
  vload<VEC>(out + o, ov);
#pragma unroll
  for (int e = 0; e < VEC; ++e) ov[e] = fmaf(mv[e], extra[e], ov[e]);
  vstore<VEC>(out + o, ov);
}

// One thread per node within W + R of a face, adding the terms of axes
// a0 .. 2: a0 = 0 after the plain step (all nodes of the shell), a0 = 1 after
// the step with the x part fused in (then only the z-layer planes and the
// y-layer rows of the shell, count = its first two parts, need a term).
__global__ void __launch_bounds__(256) cpml_fix_kernel(CpmlArgs c, const float *__restrict__ cur,
                                                       const float *__restrict__ m, float *out, int a0,
                                                       unsigned count) {
  const Shell S(c.W + R, c.nx, c.ny, c.nz);
  const unsigned t = blockIdx.x * 256u + threadIdx.x;
  if (t >= count) return;
  int x, y, z;
  S.node(t, x, y, z);
  const unsigned o = (static_cast<unsigned>(z) * c.ny + y) * c.nx + x;
  float extra = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < a0) continue;
    const AxisAt A = axis_at(c, a, x, y, z);
    if (A.i >= c.W + R && A.i < A.n - c.W - R) continue;  // psi_a and zeta_a vanish this far in
    float dpsi = 0.f;
#pragma unroll
    for (int k = 1; k <= R; ++k) dpsi = fmaf(c.d1w[a][k - 1], psi_k(c, a, A, k) - psi_k(c, a, A, -k), dpsi);
    const int s = slab_index(A.i, A.n, c.W);
    if (s < 0) {
      extra += dpsi;
      continue;
    }
    const float cc = cur[o];
    float d2 = 0.f;
#pragma unroll
    for (int k = 1; k <= R; ++k) d2 = fmaf(c.d2w[a][k], (cur_k(cur, o, A, k) - cc) + (cur_k(cur, o, A, -k) - cc), d2);
    float *ze = c.zeta[a] + A.slab_rest + static_cast<unsigned>(s) * A.slab_stride;
    const float zn = fmaf(c.cb[a][A.i], *ze, c.ca[a][A.i] * (d2 + dpsi));
    *ze = zn;
    extra += dpsi + zn;
  }
  out[o] = fmaf(m[o], extra, out[o]);
}

// ------------------------------------------------------------ utilities

__global__ void init_m_kernel(const float *__restrict__ vel, float *__restrict__ m, size_t n, float dt,
                              StepState *st) {
  __shared__ float smin[4], smax[4];
  __shared__ int sbad[4];
  float lo = __builtin_huge_valf(), hi = 0.f;
  int bad = 0;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float v = vel[i];
    const float t = v * dt;
    if (m) m[i] = t * t;
    if (!(v > 0.f) || !(v < __builtin_huge_valf())) bad = 1;
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off, 64));
    hi = fmaxf(hi, __shfl_xor(hi, off, 64));
    bad |= __shfl_xor(bad, off, 64);
  }
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    smin[w] = lo;
    smax[w] = hi;
    sbad[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      lo = fminf(lo, smin[k]);
      hi = fmaxf(hi, smax[k]);
      bad |= sbad[k];
    }
    if (bad) atomicOr(&st->flags, 2u);
    if (lo > 0.f) atomicMin(&st->vmin_bits, __float_as_uint(lo));
    atomicMax(&st->vmax_bits, __float_as_uint(fmaxf(hi, 0.f)));
  }
}

__global__ void encode_m16_kernel(const float *__restrict__ vel, uint16_t *__restrict__ codes, size_t n, float dt,
                                  float m_lo, float m_step) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float t = vel[i] * dt;
    const float u = m_step > 0.f ? rintf((t * t - m_lo) / m_step) : 0.f;
    codes[i] = static_cast<uint16_t>(fminf(fmaxf(u, 0.f), 65535.f));
  }
}

// Setting a 16-bit stored field from float32 values (wave_write_field): the
// field's maximum record of step n first holds max |x| (float bits; the
// values are non-negative, so unsigned order is float order), the encode
// uses the exponent the step kernel's rule gives for that bound, and the
// record then takes the largest stored magnitude, with the exponent beside it.
__global__ void scale_record_clear_kernel(StepState *st, int v_field) {
  if (threadIdx.x == 0) (v_field ? st->amax_v : st->amax)[st->n & 3] = 0u;
}

__global__ void __launch_bounds__(256) absmax_kernel(const float *__restrict__ x, size_t n, StepState *st,
                                                     int v_field) {
  __shared__ float part[4];
  float mx = 0.f;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    mx = fmaxf(mx, fabsf(x[i]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(&(v_field ? st->amax_v : st->amax)[st->n & 3],
              __float_as_uint(fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]))));
}

template <int S>
__global__ void encode_field_kernel(const float *__restrict__ x, typename Codec<S>::raw *__restrict__ dst, size_t n,
                                    const StepState *st, int v_field) {
  const float bound = __uint_as_float((v_field ? st->amax_v : st->amax)[st->n & 3]);
  const float sc = exp2i(scale_exponent(bound));
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    dst[i] = Codec<S>::enc(x[i] * sc);
}

template <int S>
__global__ void scale_record_kernel(StepState *st, int v_field) {
  if (threadIdx.x != 0) return;
  const int slot = st->n & 3;
  uint32_t *rec = v_field ? st->amax_v : st->amax;
  const float bound = __uint_as_float(rec[slot]);
  const int e = scale_exponent(bound);
  rec[slot] = __float_as_uint(fabsf(Codec<S>::dec(Codec<S>::enc(bound * exp2i(e)))));
  (v_field ? st->exps_v : st->exps)[slot] = e;
}

__global__ void bump_kernel(StepState *st, int count) {
  if (threadIdx.x == 0) st->n += count;
}

__global__ void set_n_kernel(StepState *st, int n) {
  if (threadIdx.x == 0) st->n = n;
}

__global__ void reset_state_kernel(StepState *st) {
  const int t = threadIdx.x;
  if (t == 0) {
    st->n = 0;
    st->flags = 0u;
  }
  if (t < 4) {
    st->amax[t] = 0u;
    st->exps[t] = 0;
    st->amax_v[t] = 0u;
    st->exps_v[t] = 0;
  }
}

template <int S>
__global__ void decode_kernel(const typename Codec<S>::raw *__restrict__ f, float *__restrict__ out, size_t n,
                              const StepState *st, int slot_off, int v_field) {
  const int slot = (st->n + slot_off) & 3;
  const int e = S == kF32 ? 0 : (v_field ? st->exps_v[slot] : st->exps[slot]);
  const float inv = exp2i(-e);
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    out[i] = Codec<S>::dec(f[i]) * inv;
}

// A^{n-1} = (A^n - V^n) / g from the 16-bit velocity-form pair.
template <int S>
__global__ void decode_prev_kernel(const typename Codec<S>::raw *__restrict__ fa,
                                   const typename Codec<S>::raw *__restrict__ fv, float *__restrict__ out,
                                   const float *__restrict__ gx, const float *__restrict__ gy,
                                   const float *__restrict__ gz, int nx, int ny, int nz, const StepState *st) {
  const int slot = st->n & 3;
  const float ia = exp2i(-st->exps[slot]), iv = exp2i(-st->exps_v[slot]);
  const size_t total = static_cast<size_t>(nx) * ny * nz;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int x = static_cast<int>(i % nx);
    const int y = static_cast<int>((i / nx) % ny);
    const int z = static_cast<int>(i / (static_cast<size_t>(nx) * ny));
    const float g = gx[x] * (gy[y] * gz[z]);  // the step kernel's association
    out[i] = (Codec<S>::dec(fa[i]) * ia - Codec<S>::dec(fv[i]) * iv) / g;
  }
}

template <int S>
__global__ void gather_kernel(const typename Codec<S>::raw *__restrict__ f, const int64_t *__restrict__ lin,
                              int nrec, float *__restrict__ traces, const StepState *st, int k) {
  const int n = st->n + k;
  const int e = S == kF32 ? 0 : st->exps[(n + 1) & 3];
  const float inv = exp2i(-e);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrec) traces[static_cast<size_t>(n) * nrec + r] = Codec<S>::dec(f[lin[r]]) * inv;
}

// Adjoint injection at an irregular receiver list: one thread per distinct
// receiver node adds g m times the sum of that node's residuals, taken in
// receiver order.  Each node is written by one thread and duplicates are
// summed in a fixed order, so the result does not depend on scheduling.
__global__ void scatter_kernel(float *f, const int64_t *__restrict__ node, const int32_t *__restrict__ off,
                               const int32_t *__restrict__ ord, int nnode, int nrec, const float *__restrict__ m,
                               const float *__restrict__ gnode, const float *__restrict__ resid, int row) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nnode) return;
  const float *rr = resid + static_cast<size_t>(row) * nrec;
  float sum = 0.f;
  for (int j = off[u]; j < off[u + 1]; ++j) sum += rr[ord[j]];
  const int64_t p = node[u];
  f[p] = fmaf(gnode[u] * m[p], sum, f[p]);
}

template <int S>
__global__ void finite_kernel(const typename Codec<S>::raw *__restrict__ f, size_t n, StepState *st) {
  int bad = 0;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float v = Codec<S>::dec(f[i]);
    if (!(fabsf(v) < __builtin_huge_valf())) bad = 1;
  }
  if (bad) atomicOr(&st->flags, 1u);
}

__global__ void grad_kernel(const float *__restrict__ img, const float *__restrict__ m, float dt,
                            float *__restrict__ grad, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    grad[i] = 2.f * img[i] * dt / sqrtf(m[i]);
}

__global__ void zero_kernel(uint4 *p, size_t n16, uint8_t *tail, size_t ntail) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n16;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

unsigned grid_for(size_t n, unsigned block) {
  const size_t want = (n + block - 1) / block;
  const size_t cap = 256 * 64;  // enough workgroups to cover all CUs many times over
  return static_cast<unsigned>(want < 1 ? 1 : (want > cap ? cap : want));
}
}  // namespace

int variant_count() { return kNumVariants; }

int step_blocks_per_cu(int storage, int variant, bool cpml) {
  if (variant < 0 || variant >= kNumVariants) return 1;
  switch (storage) {
    case kF32: return blocks_variant_f32(variant, cpml);
    case kF16: return blocks_variant_f16(variant);
    case kBF16: return blocks_variant_bf16(variant);
    default: return 1;
  }
}

Variant variant_info(int v) { return kVariants[v]; }

bool variant_fuses_cpml(int v) {
  switch (v) {
#define WAVE_VARIANT_CASE(id, fam, by, ry, pd, vec) \
  case id: return fam == 0 && fuses_cpml<ry, vec>();
    WAVE_VARIANTS(WAVE_VARIANT_CASE)
#undef WAVE_VARIANT_CASE
    default: return false;
  }
}

hipError_t launch_step(int storage, int variant, bool adjoint, const StepArgs &a, hipStream_t s) {
  if (variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
  if (adjoint) {
    if (storage != kF32) return hipErrorInvalidValue;
    return launch_variant_adj(variant, a, s);
  }
  switch (storage) {
    case kF32: return launch_variant_f32(variant, a, s);
    case kF16: return a.m16 ? launch_variant_f16m(variant, a, s) : launch_variant_f16(variant, a, s);
    case kBF16: return a.m16 ? launch_variant_bf16m(variant, a, s) : launch_variant_bf16(variant, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init_m(const float *vel, float *m, size_t n, float dt, StepState *st, hipStream_t s) {
  hipLaunchKernelGGL(init_m_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, vel, m, n, dt, st);
  return hipGetLastError();
}

hipError_t launch_encode_m16(const float *vel, uint16_t *codes, size_t n, float dt, float m_lo, float m_step,
                             hipStream_t s) {
  hipLaunchKernelGGL(encode_m16_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, vel, codes, n, dt, m_lo, m_step);
  return hipGetLastError();
}

hipError_t launch_encode_field(int storage, const float *x, void *dst, size_t n, StepState *st, bool v_field,
                              hipStream_t s) {
  if (storage != kF16 && storage != kBF16) return hipErrorInvalidValue;
  const int vf = v_field ? 1 : 0;
  const dim3 g(grid_for(n, 256)), b(256);
  hipLaunchKernelGGL(scale_record_clear_kernel, dim3(1), dim3(64), 0, s, st, vf);
  hipLaunchKernelGGL(absmax_kernel, g, b, 0, s, x, n, st, vf);
  if (storage == kF16) {
    hipLaunchKernelGGL(encode_field_kernel<kF16>, g, b, 0, s, x, static_cast<uint16_t *>(dst), n, st, vf);
    hipLaunchKernelGGL(scale_record_kernel<kF16>, dim3(1), dim3(64), 0, s, st, vf);
  } else {
    hipLaunchKernelGGL(encode_field_kernel<kBF16>, g, b, 0, s, x, static_cast<uint16_t *>(dst), n, st, vf);
    hipLaunchKernelGGL(scale_record_kernel<kBF16>, dim3(1), dim3(64), 0, s, st, vf);
  }
  return hipGetLastError();
}

hipError_t launch_bump(StepState *st, int count, hipStream_t s) {
  hipLaunchKernelGGL(bump_kernel, dim3(1), dim3(64), 0, s, st, count);
  return hipGetLastError();
}

hipError_t launch_set_n(StepState *st, int n, hipStream_t s) {
  hipLaunchKernelGGL(set_n_kernel, dim3(1), dim3(64), 0, s, st, n);
  return hipGetLastError();
}

hipError_t launch_reset_state(StepState *st, hipStream_t s) {
  hipLaunchKernelGGL(reset_state_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_decode(int storage, const void *field, float *out, size_t n, const StepState *st,
                         int slot_off, bool v_field, hipStream_t s) {
  const dim3 g(grid_for(n, 256)), b(256);
  const int vf = v_field ? 1 : 0;
  switch (storage) {
    case kF32: hipLaunchKernelGGL(decode_kernel<kF32>, g, b, 0, s, (const float *)field, out, n, st, slot_off, vf); break;
    case kF16: hipLaunchKernelGGL(decode_kernel<kF16>, g, b, 0, s, (const uint16_t *)field, out, n, st, slot_off, vf); break;
    case kBF16: hipLaunchKernelGGL(decode_kernel<kBF16>, g, b, 0, s, (const uint16_t *)field, out, n, st, slot_off, vf); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_decode_prev(int storage, const void *fa, const void *fv, float *out, const float *gx,
                              const float *gy, const float *gz, int nx, int ny, int nz, const StepState *st,
                              hipStream_t s) {
  const size_t n = static_cast<size_t>(nx) * ny * nz;
  const dim3 g(grid_for(n, 256)), b(256);
  switch (storage) {
    case kF16:
      hipLaunchKernelGGL(decode_prev_kernel<kF16>, g, b, 0, s, (const uint16_t *)fa, (const uint16_t *)fv, out, gx,
                         gy, gz, nx, ny, nz, st);
      break;
    case kBF16:
      hipLaunchKernelGGL(decode_prev_kernel<kBF16>, g, b, 0, s, (const uint16_t *)fa, (const uint16_t *)fv, out,
                         gx, gy, gz, nx, ny, nz, st);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather(int storage, const void *field, const int64_t *lin, int nrec, float *traces,
                         const StepState *st, int k, hipStream_t s) {
  const dim3 g((nrec + 255) / 256), b(256);
  switch (storage) {
    case kF32: hipLaunchKernelGGL(gather_kernel<kF32>, g, b, 0, s, (const float *)field, lin, nrec, traces, st, k); break;
    case kF16: hipLaunchKernelGGL(gather_kernel<kF16>, g, b, 0, s, (const uint16_t *)field, lin, nrec, traces, st, k); break;
    case kBF16: hipLaunchKernelGGL(gather_kernel<kBF16>, g, b, 0, s, (const uint16_t *)field, lin, nrec, traces, st, k); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_scatter(float *field, const int64_t *node, const int32_t *off, const int32_t *ord, int nnode,
                          int nrec, const float *m, const float *gnode, const float *resid, int row, hipStream_t s) {
  if (nnode <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3((nnode + 255) / 256), dim3(256), 0, s, field, node, off, ord, nnode, nrec, m,
                     gnode, resid, row);
  return hipGetLastError();
}

hipError_t launch_check_finite(int storage, const void *field, size_t n, StepState *st, hipStream_t s) {
  const dim3 g(grid_for(n, 256)), b(256);
  switch (storage) {
    case kF32: hipLaunchKernelGGL(finite_kernel<kF32>, g, b, 0, s, (const float *)field, n, st); break;
    case kF16: hipLaunchKernelGGL(finite_kernel<kF16>, g, b, 0, s, (const uint16_t *)field, n, st); break;
    case kBF16: hipLaunchKernelGGL(finite_kernel<kBF16>, g, b, 0, s, (const uint16_t *)field, n, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_grad_final(const float *img, const float *m, float dt, float *grad, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(grad_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, img, m, dt, grad, n);
  return hipGetLastError();
}

hipError_t launch_cpml_psi(const CpmlArgs &c, const float *cur, hipStream_t s) {
  const Shell S(c.W, c.nx, c.ny, c.nz);
  const int vec = c.nx % 4 == 0 ? 4 : (c.nx % 2 == 0 ? 2 : 1);
  const unsigned nrow = (S.cz * S.ny + S.mz * S.cy) * (static_cast<unsigned>(c.nx) / vec);
  if (nrow > 0) {
    const dim3 g((nrow + 255) / 256), b(256);
    if (vec == 4) hipLaunchKernelGGL(cpml_psi_rows_kernel<4>, g, b, 0, s, c, cur);
    else if (vec == 2) hipLaunchKernelGGL(cpml_psi_rows_kernel<2>, g, b, 0, s, c, cur);
    else hipLaunchKernelGGL(cpml_psi_rows_kernel<1>, g, b, 0, s, c, cur);
  }
  if (S.n2 > 0)
    hipLaunchKernelGGL(cpml_psi_kernel, dim3((S.n2 + 255) / 256), dim3(256), 0, s, c, cur, S.n0 + S.n1);
  return hipGetLastError();
}

hipError_t launch_cpml_fix(const CpmlArgs &c, const float *cur, const float *m, float *out, bool yz_only,
                           hipStream_t s) {
  const Shell S(c.W + kRadius, c.nx, c.ny, c.nz);
  if (yz_only) {
    const int vec = c.nx % 4 == 0 ? 4 : (c.nx % 2 == 0 ? 2 : 1);
    const unsigned n = (S.cz * S.ny + S.mz * S.cy) * (static_cast<unsigned>(c.nx) / vec);
    if (n == 0) return hipSuccess;
    const dim3 g((n + 255) / 256), b(256);
    if (vec == 4) hipLaunchKernelGGL(cpml_fix_yz_kernel<4>, g, b, 0, s, c, cur, m, out);
    else if (vec == 2) hipLaunchKernelGGL(cpml_fix_yz_kernel<2>, g, b, 0, s, c, cur, m, out);
    else hipLaunchKernelGGL(cpml_fix_yz_kernel<1>, g, b, 0, s, c, cur, m, out);
    return hipGetLastError();
  }
  const unsigned n = S.count();
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cpml_fix_kernel, dim3((n + 255) / 256), dim3(256), 0, s, c, cur, m, out, 0, n);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  const size_t tail = bytes - n16 * 16;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n16 ? n16 : 1, 256)), dim3(256), 0, s, static_cast<uint4 *>(p), n16,
                     static_cast<uint8_t *>(p) + n16 * 16, tail);
  return hipGetLastError();
}

}  // namespace wave
