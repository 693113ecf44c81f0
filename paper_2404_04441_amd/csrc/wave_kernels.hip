// gfx950 kernels of libwave.
//
// The fused step evaluates the 25-point, 8th-order star Laplacian of Eq. 1
// (paper Sec. II) at every node and applies the leapfrog update with sponge,
// source and receivers in the same pass.  Blocking follows the 2.5D idea of
// paper Sec. IV-A (tile x and y, stream along z) redesigned for CDNA4:
//
//  * a workgroup owns a 64 x TY column of the grid (TY = BY*RY rows) over a
//    z-chunk; each 64-lane wavefront covers one 256-byte row segment, so every
//    global access of the interior is a fully coalesced row;
//  * the centre xy plane (with its radius-4 x/y halo) is staged in LDS, double
//    buffered so one barrier per plane suffices;
//  * the 9 values each thread needs along z live in a register queue that
//    shifts by one plane per iteration; A^n is read from HBM once per chunk;
//  * loads for plane z+1 are issued before the barrier of plane z, so their
//    latency overlaps the stencil arithmetic of plane z;
//  * A^{n-1}, m and A^{n+1} are touched exactly once: they use nontemporal
//    loads/stores so that L2 keeps the A^n planes the neighbours' halos need;
//  * workgroup ids are remapped so that each XCD (hardware dispatches ids
//    round-robin over the 8 XCDs) owns a contiguous run of tiles, keeping
//    y-halo re-reads inside one XCD's L2.
#include <hip/hip_runtime.h>

#include "wave_internal.h"

namespace wave {
namespace {

constexpr int R = kRadius;

__device__ __forceinline__ float exp2i(int e) {  // 2^e, e in [-126, 127]
  return __uint_as_float(static_cast<uint32_t>(e + 127) << 23);
}

// Exponent e such that B * 2^e < 2^14 (65504 is the largest half): the
// stored magnitude stays below 16384 whatever the next field's maximum is.
__device__ __forceinline__ int scale_exponent(float B) {
  if (!(B > 0.f)) return 0;
  const uint32_t bits = __float_as_uint(B);
  const int E = static_cast<int>((bits >> 23) & 0xffu) - 126;  // B < 2^E
  int e = 14 - E;
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

template <int S> struct Codec;

template <> struct Codec<kF32> {
  using raw = float;
  __device__ static float dec(raw r) { return r; }
  __device__ static raw enc(float x) { return x; }
};

template <> struct Codec<kF16> {
  using raw = uint16_t;
  __device__ static float dec(raw r) { return static_cast<float>(__builtin_bit_cast(_Float16, r)); }
  __device__ static raw enc(float x) {  // round to nearest even (v_cvt_f16_f32)
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
  }
};

template <> struct Codec<kBF16> {
  using raw = uint16_t;
  __device__ static float dec(raw r) { return __uint_as_float(static_cast<uint32_t>(r) << 16); }
  __device__ static raw enc(float x) {  // round to nearest even on the float32 bits
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<raw>((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<raw>(u >> 16);
  }
};

template <typename T> __device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T> __device__ __forceinline__ void st_stream(T v, T *p) { __builtin_nontemporal_store(v, p); }

template <int S, int BY, int RY, bool ADJ>
__global__ void __launch_bounds__(64 * BY) step_kernel(StepArgs a) {
  using C = Codec<S>;
  using raw = typename C::raw;
  constexpr int TY = BY * RY;
  constexpr int NT = 64 * BY;
  constexpr int LW = kTileX + 2 * R;
  constexpr int LH = TY + 2 * R;
  constexpr int HALO = 2 * R * kTileX + 2 * R * TY;
  constexpr int HS = (HALO + NT - 1) / NT;
  __shared__ float lds[2][LH * LW];
  __shared__ float ldsF[ADJ ? 2 : 1][ADJ ? LH * LW : 1];
  __shared__ float red[BY];

  // XCD-aware tile order: hardware id b runs on XCD b % 8.
  const int nwg = static_cast<int>(gridDim.x);
  const int bid = static_cast<int>(blockIdx.x);
  const int logical = (bid & 7) * (nwg >> 3) + (bid >> 3);
  if (logical >= a.total_tiles) return;
  const int tix = logical % a.tiles_x;
  const int rest = logical / a.tiles_x;
  const int tiy = rest % a.tiles_y;
  const int chunk = rest / a.tiles_y;
  const int x0 = tix * kTileX, y0 = tiy * TY;
  const int zb = chunk * a.zchunk;
  const int ze = min(zb + a.zchunk, a.nz);
  const int lx = static_cast<int>(threadIdx.x), ly = static_cast<int>(threadIdx.y);
  const int tid = ly * 64 + lx;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t plane = static_cast<size_t>(nx) * static_cast<size_t>(ny);
  const int x = x0 + lx;
  const bool xin = x < nx;

  // ---- step index and 16-bit field scales
  const int n = ADJ ? 0 : a.st->n + a.k;
  float inv_cur = 1.f, inv_prev = 1.f, s_next = 1.f, inv_next = 1.f;
  if (S != kF32) {
    const int ec = a.st->exps[n & 3], ep = a.st->exps[(n + 3) & 3];
    inv_cur = exp2i(-ec);
    inv_prev = exp2i(-ep);
    const float acur = __uint_as_float(a.st->amax[n & 3]) * inv_cur;
    const float aprev = __uint_as_float(a.st->amax[(n + 3) & 3]) * inv_prev;
    const float qmag = a.sx >= 0 ? fabsf(a.wavelet[n]) * a.src_scale : 0.f;
    const int e_next = scale_exponent(a.beta * acur + aprev + qmag);
    s_next = exp2i(e_next);
    inv_next = exp2i(-e_next);
    if (logical == 0 && tid == 0) {
      a.st->exps[(n + 1) & 3] = e_next;
      a.st->amax[(n + 2) & 3] = 0u;
    }
  }

  // ---- rows owned by this thread: y = y0 + ly + BY*j
  int roff[RY];
  bool rin[RY];
  float gxy[RY];
  int ryi[RY];
  int srcj = -1;
  const float gxv = xin ? a.gx[x] : 0.f;
  int rxi = -1;
  if (a.box.cnx > 0 && xin) {
    const int d = x - a.box.x0;
    if (d >= 0 && d % a.box.sx == 0 && d / a.box.sx < a.box.cnx) rxi = d / a.box.sx;
  }
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const int yj = y0 + ly + BY * j;
    rin[j] = xin && yj < ny;
    roff[j] = rin[j] ? yj * nx + x : 0;
    gxy[j] = rin[j] ? gxv * a.gy[yj] : 0.f;
    ryi[j] = -1;
    if (rxi >= 0 && rin[j]) {
      const int d = yj - a.box.y0;
      if (d >= 0 && d % a.box.sy == 0 && d / a.box.sy < a.box.cny) ryi[j] = d / a.box.sy;
    }
    if (!ADJ && a.sx >= 0 && x == a.sx && yj == a.sy) srcj = j;
  }

  // ---- halo slots: LDS offset and in-plane global offset (-1: ghost zero)
  int hl[HS], ho[HS];
#pragma unroll
  for (int s = 0; s < HS; ++s) {
    const int i = tid + s * NT;
    hl[s] = -1;
    ho[s] = -1;
    if (i < 2 * R * kTileX) {  // rows above / below the tile
      const int r = i / kTileX, c = i % kTileX;
      const int lr = r < R ? r : TY + r;
      const int gyy = y0 - R + lr, gxx = x0 + c;
      hl[s] = lr * LW + R + c;
      if (gyy >= 0 && gyy < ny && gxx < nx) ho[s] = gyy * nx + gxx;
    } else if (i < HALO) {  // columns left / right of the tile
      const int jj = i - 2 * R * kTileX;
      const int r = jj / (2 * R), c = jj % (2 * R);
      const int gxx = c < R ? x0 - R + c : x0 + kTileX + (c - R);
      const int gyy = y0 + r;
      hl[s] = (R + r) * LW + (c < R ? c : kTileX + c);
      if (gxx >= 0 && gxx < nx && gyy < ny) ho[s] = gyy * nx + gxx;
    }
  }

  const raw *U = static_cast<const raw *>(a.cur);
  const raw *P = static_cast<const raw *>(a.prev);
  raw *O = static_cast<raw *>(a.out);

  // ---- prologue: queue planes zb-4 .. zb+3, lead plane zb+4, halo/prev/m of plane zb
  float q[2 * R + 1][RY];
  float qF[ADJ ? 2 * R + 1 : 1][RY];
  float lead[RY], leadF[RY], hal[HS], halF[HS], pv[RY], mv[RY], iv[RY];
#pragma unroll
  for (int i = 0; i < 2 * R; ++i) {
    const int zz = zb - R + i;
    const bool zok = zz >= 0 && zz < nz;
    const size_t zo = zok ? static_cast<size_t>(zz) * plane : 0;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      q[i][j] = (zok && rin[j]) ? C::dec(U[zo + roff[j]]) * inv_cur : 0.f;
      if (ADJ) qF[i][j] = (zok && rin[j]) ? a.fwd[zo + roff[j]] : 0.f;
    }
  }
  {
    const int zz = zb + R;
    const bool zok = zz < nz;
    const size_t zo = zok ? static_cast<size_t>(zz) * plane : 0;
    const size_t zc = static_cast<size_t>(zb) * plane;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      lead[j] = (zok && rin[j]) ? C::dec(U[zo + roff[j]]) * inv_cur : 0.f;
      if (ADJ) leadF[j] = (zok && rin[j]) ? a.fwd[zo + roff[j]] : 0.f;
      pv[j] = rin[j] ? C::dec(ld_stream(P + zc + roff[j])) * inv_prev : 0.f;
      mv[j] = rin[j] ? ld_stream(a.m + zc + roff[j]) : 0.f;
      if (ADJ) iv[j] = rin[j] ? ld_stream(a.img + zc + roff[j]) : 0.f;
    }
#pragma unroll
    for (int s = 0; s < HS; ++s) {
      hal[s] = ho[s] >= 0 ? C::dec(U[zc + ho[s]]) * inv_cur : 0.f;
      if (ADJ) halF[s] = ho[s] >= 0 ? a.fwd[zc + ho[s]] : 0.f;
    }
  }

  const float wsrc = (!ADJ && a.sx >= 0) ? a.wavelet[n] * a.src_scale : 0.f;
  float amax_loc = 0.f;

  for (int z = zb; z < ze; ++z) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      q[2 * R][j] = lead[j];
      if (ADJ) qF[2 * R][j] = leadF[j];
    }
    float *L = lds[z & 1];
    float *LF = ldsF[ADJ ? (z & 1) : 0];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      L[(R + ly + BY * j) * LW + R + lx] = q[R][j];
      if (ADJ) LF[(R + ly + BY * j) * LW + R + lx] = qF[R][j];
    }
#pragma unroll
    for (int s = 0; s < HS; ++s) {
      if (hl[s] >= 0) {
        L[hl[s]] = hal[s];
        if (ADJ) LF[hl[s]] = halF[s];
      }
    }
    float pc[RY], mc[RY], ic[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      pc[j] = pv[j];
      mc[j] = mv[j];
      ic[j] = ADJ ? iv[j] : 0.f;
    }
    if (z + 1 < ze) {  // prefetch plane z+1 (lead plane z+1+R)
      const int zz = z + 1 + R;
      const bool zok = zz < nz;
      const size_t zo = zok ? static_cast<size_t>(zz) * plane : 0;
      const size_t zc = static_cast<size_t>(z + 1) * plane;
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        lead[j] = (zok && rin[j]) ? C::dec(U[zo + roff[j]]) * inv_cur : 0.f;
        if (ADJ) leadF[j] = (zok && rin[j]) ? a.fwd[zo + roff[j]] : 0.f;
        pv[j] = rin[j] ? C::dec(ld_stream(P + zc + roff[j])) * inv_prev : 0.f;
        mv[j] = rin[j] ? ld_stream(a.m + zc + roff[j]) : 0.f;
        if (ADJ) iv[j] = rin[j] ? ld_stream(a.img + zc + roff[j]) : 0.f;
      }
#pragma unroll
      for (int s = 0; s < HS; ++s) {
        hal[s] = ho[s] >= 0 ? C::dec(U[zc + ho[s]]) * inv_cur : 0.f;
        if (ADJ) halF[s] = ho[s] >= 0 ? a.fwd[zc + ho[s]] : 0.f;
      }
    }
    __syncthreads();

    const float gzv = a.gz[z];
    const size_t zc = static_cast<size_t>(z) * plane;
    int rzi = -1;
    if (rxi >= 0) {
      const int d = z - a.box.z0;
      if (d >= 0 && d % a.box.sz == 0 && d / a.box.sz < a.box.cnz) rzi = d / a.box.sz;
    }
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const float *row = L + (R + ly + BY * j) * LW + R + lx;
      const float c = q[R][j];
      float lap = a.c.k0 * c;
#pragma unroll
      for (int m = 1; m <= R; ++m) {
        lap = fmaf(a.c.kx[m - 1], row[m] + row[-m], lap);
        lap = fmaf(a.c.ky[m - 1], row[m * LW] + row[-m * LW], lap);
        lap = fmaf(a.c.kz[m - 1], q[R + m][j] + q[R - m][j], lap);
      }
      const bool at_rec = rzi >= 0 && ryi[j] >= 0;
      const int ridx = at_rec ? (rzi * a.box.cny + ryi[j]) * a.box.cnx + rxi : 0;
      if (ADJ && at_rec) lap += a.resid[static_cast<size_t>(a.resid_row) * a.nrec + ridx];
      const float g = gxy[j] * gzv;
      float v = fmaf(-g, pc[j], 2.f * c);
      v = fmaf(mc[j], lap, v);
      if (!ADJ && srcj == j && z == a.sz) v += wsrc;
      v *= g;
      if (rin[j]) {
        const raw r = C::enc(v * s_next);
        st_stream(r, O + zc + roff[j]);
        const float stored = C::dec(r);
        if (S != kF32) amax_loc = fmaxf(amax_loc, fabsf(stored));
        if (!ADJ && at_rec) a.traces[static_cast<size_t>(n) * a.nrec + ridx] = stored * inv_next;
        if (ADJ) {
          const float *rowF = LF + (R + ly + BY * j) * LW + R + lx;
          const float cF = qF[R][j];
          float lapF = a.c.k0 * cF;
#pragma unroll
          for (int m = 1; m <= R; ++m) {
            lapF = fmaf(a.c.kx[m - 1], rowF[m] + rowF[-m], lapF);
            lapF = fmaf(a.c.ky[m - 1], rowF[m * LW] + rowF[-m * LW], lapF);
            lapF = fmaf(a.c.kz[m - 1], qF[R + m][j] + qF[R - m][j], lapF);
          }
          st_stream(fmaf(c, lapF, ic[j]), a.img + zc + roff[j]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) {
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        q[i][j] = q[i + 1][j];
        if (ADJ) qF[i][j] = qF[i + 1][j];
      }
    }
  }

  if (S != kF32) {  // one order-independent atomic per workgroup
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax_loc = fmaxf(amax_loc, __shfl_xor(amax_loc, off, 64));
    if (lx == 0) red[ly] = amax_loc;
    __syncthreads();
    if (tid == 0) {
      float mx = red[0];
#pragma unroll
      for (int w = 1; w < BY; ++w) mx = fmaxf(mx, red[w]);
      atomicMax(&a.st->amax[(n + 1) & 3], __float_as_uint(mx));
    }
  }
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
    m[i] = t * t;
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
  }
}

template <int S>
__global__ void decode_kernel(const typename Codec<S>::raw *__restrict__ f, float *__restrict__ out, size_t n,
                              const StepState *st, int slot_off) {
  const int e = S == kF32 ? 0 : st->exps[(st->n + slot_off) & 3];
  const float inv = exp2i(-e);
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    out[i] = Codec<S>::dec(f[i]) * inv;
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

__global__ void scatter_kernel(float *f, const int64_t *__restrict__ lin, int nrec, const float *__restrict__ m,
                               const float *__restrict__ grec, const float *__restrict__ resid, int row) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrec) {
    const int64_t p = lin[r];
    atomicAdd(f + p, grec[r] * m[p] * resid[static_cast<size_t>(row) * nrec + r]);
  }
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

// (BY, RY) per variant
constexpr Variant kVariants[] = {{4, 4}, {8, 4}, {4, 2}, {8, 2}, {2, 4}, {4, 8}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int S, int BY, int RY, bool ADJ>
hipError_t launch_one(const StepArgs &a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>((a.total_tiles + 7) / 8 * 8);
  hipLaunchKernelGGL((step_kernel<S, BY, RY, ADJ>), dim3(grid), dim3(64, BY), 0, s, a);
  return hipGetLastError();
}

template <int S, bool ADJ>
hipError_t launch_variant(int v, const StepArgs &a, hipStream_t s) {
  switch (v) {
    case 0: return launch_one<S, 4, 4, ADJ>(a, s);
    case 1: return launch_one<S, 8, 4, ADJ>(a, s);
    case 2: return launch_one<S, 4, 2, ADJ>(a, s);
    case 3: return launch_one<S, 8, 2, ADJ>(a, s);
    case 4: return launch_one<S, 2, 4, ADJ>(a, s);
    case 5: return launch_one<S, 4, 8, ADJ>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int variant_count() { return kNumVariants; }

Variant variant_info(int v) { return kVariants[v]; }

hipError_t launch_step(int storage, int variant, bool adjoint, const StepArgs &a, hipStream_t s) {
  if (variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
  if (adjoint) {
    if (storage != kF32) return hipErrorInvalidValue;
    return launch_variant<kF32, true>(variant, a, s);
  }
  switch (storage) {
    case kF32: return launch_variant<kF32, false>(variant, a, s);
    case kF16: return launch_variant<kF16, false>(variant, a, s);
    case kBF16: return launch_variant<kBF16, false>(variant, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init_m(const float *vel, float *m, size_t n, float dt, StepState *st, hipStream_t s) {
  hipLaunchKernelGGL(init_m_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, vel, m, n, dt, st);
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
                         int slot_off, hipStream_t s) {
  const dim3 g(grid_for(n, 256)), b(256);
  switch (storage) {
    case kF32: hipLaunchKernelGGL(decode_kernel<kF32>, g, b, 0, s, (const float *)field, out, n, st, slot_off); break;
    case kF16: hipLaunchKernelGGL(decode_kernel<kF16>, g, b, 0, s, (const uint16_t *)field, out, n, st, slot_off); break;
    case kBF16: hipLaunchKernelGGL(decode_kernel<kBF16>, g, b, 0, s, (const uint16_t *)field, out, n, st, slot_off); break;
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

hipError_t launch_scatter(float *field, const int64_t *lin, int nrec, const float *m, const float *grec,
                          const float *resid, int row, hipStream_t s) {
  hipLaunchKernelGGL(scatter_kernel, dim3((nrec + 255) / 256), dim3(256), 0, s, field, lin, nrec, m, grec, resid, row);
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

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  const size_t tail = bytes - n16 * 16;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n16 ? n16 : 1, 256)), dim3(256), 0, s, static_cast<uint4 *>(p), n16,
                     static_cast<uint8_t *>(p) + n16 * 16, tail);
  return hipGetLastError();
}

}  // namespace wave
