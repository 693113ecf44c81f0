// Step-kernel templates of libwave (gfx950), shared by the translation
// units that instantiate them: one per storage type and one for the
// adjoint, compiled in parallel.  Included only by HIP sources.
//
//
// The fused step evaluates the 25-point, 8th-order star Laplacian of Eq. 1
// (paper Sec. II) at every node and applies the leapfrog update with sponge,
// source and receivers in the same pass.  Blocking follows the 2.5D idea of
// paper Sec. IV-A (tile x and y, stream along z) redesigned for CDNA4:
//
//  * a workgroup owns a (64*VEC) x (BY*RY) column of the grid over a z-chunk;
//    each 64-lane wavefront owns RY consecutive rows and each lane VEC
//    consecutive x nodes, so every global access of the interior is one
//    coalesced row of 256*VEC bytes;
//  * each field has one buffer resource per workgroup; the plane is the
//    scalar offset, the row and column one lane register.  Lanes outside the
//    grid use an offset past the resource's end (loads read zero, stores are
//    dropped) and the fields carry zero padding planes past nz, so the z loop
//    has no clamps, selects or store branches;
//  * the centre xy plane (with its radius-4 x/y halo) is staged in LDS, double
//    buffered so one barrier per plane suffices; x neighbours are read as one
//    aligned window per lane, y neighbours inside a wavefront's own rows come
//    from registers;
//  * the 9 values each thread needs along z live in a register queue with
//    compile-time slots; A^n is read from HBM once per chunk;
//  * loads run PD planes ahead of the plane being computed (a register
//    pipeline), so enough bytes are in flight to cover HBM latency;
//  * A^{n-1}, m and A^{n+1} are touched exactly once: they use nontemporal
//    loads/stores so that L2 keeps the A^n planes the neighbours' halos need
//    (the KEEP instances use the regular policy instead, for grids whose
//    fields fit the last-level cache);
//  * workgroup ids are remapped so that each XCD (hardware dispatches ids
//    round-robin over the 8 XCDs) owns a contiguous run of tiles, keeping
//    halo re-reads inside one XCD's L2.
//
// Beside it: the paper's 3D-blocked designs (gmem, smem) and a semi-stencil
// form for the kernel study, the CPML boundary (its x part fused into the
// step kernel, the memory-variable update and the y/z part in row kernels),
// and small utility kernels (setup, decode, gather/scatter, gradient, fills).
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "wave_internal.h"

namespace wave {
namespace {

constexpr int R = kRadius;

// f(std::integral_constant<int, 0>) ... f(std::integral_constant<int, N-1>):
// a loop whose index is a compile-time constant in every iteration.
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

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

typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 b16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));

template <> struct Codec<kF16> {
  using raw = uint16_t;
  __device__ static float dec(raw r) { return static_cast<float>(__builtin_bit_cast(_Float16, r)); }
  __device__ static raw enc(float x) {  // round to nearest even (v_cvt_f16_f32)
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
  }
  // two values, low half first: one v_cvt_pk_f16_f32 (round to nearest even)
  __device__ static uint32_t enc2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v{lo, hi}), h16x2));
  }
};

template <> struct Codec<kBF16> {
  using raw = uint16_t;
  __device__ static float dec(raw r) { return __uint_as_float(static_cast<uint32_t>(r) << 16); }
  __device__ static raw enc(float x) {  // round to nearest even: gfx950's v_cvt_pk_bf16_f32
    return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
  }
  __device__ static uint32_t enc2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v{lo, hi}), b16x2));
  }
};

template <typename T> __device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T> __device__ __forceinline__ void st_stream(T v, T *p) { __builtin_nontemporal_store(v, p); }

// ---- buffer access: raw buffer loads and stores through a resource (base
// and size in bytes) with a scalar byte offset (the plane) and a 32-bit lane
// offset (row and column).  Nothing is clamped: a node outside the grid gets
// a lane offset past the end of the resource (kOOB below), for which the
// hardware returns zero on a load and drops a store, so ghost nodes read as
// the zero-Dirichlet exterior without selects or branches.
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;  // raw (untyped) buffer, gfx9 family
constexpr int kNT = 2;                  // nontemporal cache policy bit

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), static_cast<short>(0),
                                           static_cast<int>(bytes), kRsrcWord3);
}

// ---- rows of VEC consecutive values as loaded: NB bytes in 32-bit words
// (a 16-bit value alone is zero-extended into one word).
template <int NB> struct Words {
  static constexpr int N = (NB + 3) / 4;
  uint32_t w[N];
};

template <int NB, int AUX>
__device__ __forceinline__ Words<NB> ld_words(rsrc_t r, uint32_t vo, uint32_t so) {
  Words<NB> out;
  const int v = static_cast<int>(vo), s = static_cast<int>(so);
  if constexpr (NB == 2) {
    out.w[0] = __builtin_amdgcn_raw_buffer_load_b16(r, v, s, AUX);
  } else if constexpr (NB == 4) {
    out.w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, v, s, AUX);
  } else if constexpr (NB == 8) {
    const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(r, v, s, AUX);
    out.w[0] = t.x;
    out.w[1] = t.y;
  } else {
    static_assert(NB == 16, "row width");
    const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(r, v, s, AUX);
    out.w[0] = t.x;
    out.w[1] = t.y;
    out.w[2] = t.z;
    out.w[3] = t.w;
  }
  return out;
}

template <int NB, int AUX>
__device__ __forceinline__ void st_words(const Words<NB> &in, rsrc_t r, uint32_t vo, uint32_t so) {
  const int v = static_cast<int>(vo), s = static_cast<int>(so);
  if constexpr (NB == 2) {
    __builtin_amdgcn_raw_buffer_store_b16(static_cast<uint16_t>(in.w[0]), r, v, s, AUX);
  } else if constexpr (NB == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(in.w[0], r, v, s, AUX);
  } else if constexpr (NB == 8) {
    __builtin_amdgcn_raw_buffer_store_b64(u32x2{in.w[0], in.w[1]}, r, v, s, AUX);
  } else {
    static_assert(NB == 16, "row width");
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{in.w[0], in.w[1], in.w[2], in.w[3]}, r, v, s, AUX);
  }
}

// Value i of a row of storage type S (decoded, unscaled) and the inverse.
template <int S, int NB>
__device__ __forceinline__ float row_get(const Words<NB> &r, int i) {
  if constexpr (S == kF32) {
    return __uint_as_float(r.w[i]);
  } else {
    const uint32_t h = (r.w[i >> 1] >> (16 * (i & 1))) & 0xffffu;
    return Codec<S>::dec(static_cast<uint16_t>(h));
  }
}
template <int S, int VEC>
__device__ __forceinline__ Words<VEC * (S == kF32 ? 4 : 2)> row_put(const float *v) {
  Words<VEC * (S == kF32 ? 4 : 2)> r;
  if constexpr (S == kF32) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) r.w[i] = __float_as_uint(v[i]);
  } else if constexpr (VEC == 1) {
    r.w[0] = Codec<S>::enc(v[0]);
  } else {
#pragma unroll
    for (int k = 0; k < VEC / 2; ++k) r.w[k] = Codec<S>::enc2(v[2 * k], v[2 * k + 1]);
  }
  return r;
}

// LDS rows of VEC floats at a VEC-aligned address.
template <int VEC> __device__ __forceinline__ void lds_put(float *p, const float *v) {
  if constexpr (VEC == 1) {
    p[0] = v[0];
  } else if constexpr (VEC == 2) {
    *reinterpret_cast<f32x2 *>(p) = f32x2{v[0], v[1]};
  } else {
    *reinterpret_cast<f32x4 *>(p) = f32x4{v[0], v[1], v[2], v[3]};
  }
}
template <int VEC> __device__ __forceinline__ void lds_get(const float *p, float *v) {
  if constexpr (VEC == 1) {
    v[0] = p[0];
  } else if constexpr (VEC == 2) {
    const f32x2 t = *reinterpret_cast<const f32x2 *>(p);
    v[0] = t.x;
    v[1] = t.y;
  } else {
    const f32x4 t = *reinterpret_cast<const f32x4 *>(p);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
  }
}

// Slab index along an axis of n nodes with layers of W nodes, or -1.
__device__ __forceinline__ int slab_index(int i, int n, int W) {
  if (i < 0 || i >= n) return -1;
  if (i < W) return i;
  if (i >= n - W) return i - (n - 2 * W);
  return -1;
}

// Registers one thread holds for one z-plane of the pipeline: raw loaded
// rows, so that nothing waits on a load until the plane is consumed.  Every
// vector-memory load of the z loop lives here: s_waitcnt vmcnt retires loads
// in issue order, so a load consumed in the same iteration would also wait for
// every prefetch issued before it.
template <int S, int RY, int VEC, int NYH, bool ADJ, bool CP, bool M16 = false>
struct Stage {
  static constexpr int NA = VEC * (S == kF32 ? 4 : 2);  // bytes of one A-type row
  static constexpr int NF = VEC * 4;                    // bytes of one float row
  static constexpr int NM = VEC * (M16 ? 2 : 4);        // bytes of one row of m (or of its codes)
  Words<NA> lead[RY];             // A^n at plane z+R (enters the z queue)
  Words<NA> p[RY];                // A^{n-1} (or V^n) at plane z
  Words<NM> m[RY];                // m (or its 16-bit codes) at plane z
  Words<NA> yh[NYH];              // y-halo rows of A^n at plane z owned by this wavefront
  Words<S == kF32 ? 4 : 2> xh;    // x-halo value of A^n at plane z (lanes < 8*RY)
  float gz;                       // sponge factor of plane z
  int rz;                         // receiver-box plane index of plane z, or -1
  Words<NF> leadF[ADJ ? RY : 1];  // adjoint: forward field, same roles
  Words<NF> img[ADJ ? RY : 1];    // adjoint: imaging accumulator at plane z
  Words<NF> yhF[ADJ ? NYH : 1];
  float xhF;
  float res[ADJ ? RY : 1][ADJ ? VEC : 1];  // adjoint: residual injected at receivers of plane z
  float psx[CP ? RY : 1][CP ? VEC : 1];  // CPML: psi_x at the lane's columns (0 off the x layers)
  float zex[CP ? RY : 1][CP ? VEC : 1];  // CPML: zeta_x at the lane's columns
  float psxh;                            // CPML: psi_x at this lane's x-halo node (lanes < 8*RY)
};

constexpr int kQ = 2 * R + 1;  // z-queue length (planes z-4 .. z+4)

// Lane byte offset past the end of every buffer resource the step kernel
// builds (each spans less than 2^31 bytes, and resource offset plus this
// value stays below 2^32): a load at it returns zero, a store is dropped.
constexpr uint32_t kOOB = 0x80000000u;
static_assert(kPadZ >= (kQ - 1) + kMaxPD + R, "z padding must cover the last trip's loads");

// BY wavefronts per workgroup, RY consecutive rows per wavefront, VEC
// consecutive x nodes per lane (tile 64*VEC x BY*RY), PD planes of loads in
// flight ahead of the plane being computed (PD divides 9: the z loop is
// unrolled 9 times so the queue rotates by register renaming instead of
// copies).  VEC > 1 requires nx % VEC == 0 (whole rows stay aligned).
// SEMI: the z part of the stencil as a semi-stencil (the paper's st_semi,
// Sec. IV-A): the left half sum_m kz_m A(z-m) of plane z is summed R planes
// early, at the position of plane z-R (from planes z-R .. z-1), so only planes
// z .. z+R stay live in the queue; the right half is added when z is computed.
// CP: the x part of the CPML boundary fused into the step (float32 forward;
// psi_a^n is already updated by cpml_psi_kernel).  The Laplacian is summed
// per axis, and every node adds D1_x psi_x^n + zeta_x^n, with zeta_x updated
// in place on the x layers.  Off the layers psi_x and zeta_x read as zero,
// so this needs no branch.  psi_x and zeta_x come through the prefetch
// pipeline; psi_x is staged in LDS like A^n (its x neighbours are other
// lanes' values).  The y and z parts follow in cpml_fix_kernel over the rows
// and planes within W + R of a y or z face: in the streaming kernel their
// neighbours would be loads the z loop waits on in every such row and plane.
// KEEP: the fields read or written once (float32: A^{n-1}, m, A^{n+1};
// 16-bit: V^n, m, A^{n+1}, V^{n+1}) use the regular cache policy instead of the
// nontemporal one, so that a grid whose fields fit the last-level cache stays
// there from step to step (forward; chosen by create-time tuning or the
// caller).
// M16: m is read as 16-bit codes (m = m_lo + u m_step; 16-bit storage only).
template <int S, int BY, int RY, int PD, int VEC, bool SEMI, bool ADJ, bool CP, bool KEEP, bool M16 = false>
__global__ void __launch_bounds__(64 * BY) step_kernel(StepArgs a) {
  using StageT = Stage<S, RY, VEC, (2 * R + BY - 1) / BY, ADJ, CP, M16>;
  static_assert(!M16 || (S != kF32 && !ADJ && !CP && !SEMI), "16-bit model codes: 16-bit storage forward");
  constexpr int NA = StageT::NA, NF = StageT::NF;
  constexpr int TX = kTileX * VEC;
  constexpr int TY = BY * RY;
  constexpr int LW = TX + 2 * R;
  constexpr int LH = TY + 2 * R;
  constexpr int NYH = (2 * R + BY - 1) / BY;
  constexpr uint32_t ES = S == kF32 ? 4u : 2u;
  static_assert(8 * RY <= 64, "x-halo of a wavefront's rows must fit in one load");
  static_assert(kQ % PD == 0, "pipeline depth must divide the queue length");
  static_assert(PD <= kMaxPD, "z padding assumes at most kMaxPD planes in flight");
  static_assert(VEC == 1 || VEC == 2 || VEC == 4, "lane width");
  static_assert(!(SEMI && ADJ), "the semi-stencil form is forward only");
  static_assert(!CP || (S == kF32 && !SEMI && !ADJ), "the fused CPML step is float32 forward");
  static_assert(!KEEP || (!SEMI && !ADJ && !CP), "the cached policy is for the plain forward step");
  constexpr int NTP = KEEP ? 0 : kNT;  // cache policy of the fields read or written once
  // f16 storage with 16-bit m sums the Laplacian from its centre weight (Eq. 1
  // as written) instead of as centred differences: 25 instead of 48 vector
  // operations per node, for the one form whose rate the instruction issue
  // limits.  Its float32 rounding, relative to the terms rather than to their
  // differences, stays far below the f16 rounding of the stored fields.
  constexpr bool kSumForm = M16 && S == kF16;
  // each LDS plane ends with a scratch row: halo writes of lanes or
  // wavefronts with nothing to write go there, so no write is predicated
  constexpr int LP = LH * LW + 64 * VEC;
  constexpr int DUMMY = LH * LW;
  // LEADH: the x and y halo of A^n is loaded with the lead plane z+R, when
  // the neighbouring tiles load the same lines as their own lead (so those
  // loads meet in L2), instead of R planes later at the centre plane, by
  // which time the lines have often left L2.  Planes z .. z+R then live in a
  // ring of R+2 LDS planes: iteration z writes plane z+R into slot
  // (z+R) mod 6 and reads plane z from slot z mod 6; the next iteration's
  // writes go to the slot read one iteration earlier, so one barrier per
  // plane still suffices.  Plain forward kernels whose ring fits 150 KB of
  // LDS; the others stage the centre plane double-buffered.
  constexpr bool LEADH = !ADJ && !CP && 6 * LP * 4 <= 150 * 1024;
  constexpr int NSLOT = LEADH ? R + 2 : 2;
  __shared__ __attribute__((aligned(16))) float lds[NSLOT][LP];
  __shared__ __attribute__((aligned(16))) float ldsF[ADJ ? 2 : 1][ADJ ? LP : 1];
  // CPML: psi_x rows of the tile (TY rows of LW, no y halo) and a scratch row
  constexpr int LPX = TY * LW + 64 * VEC;
  constexpr int DUMMYX = TY * LW;
  __shared__ __attribute__((aligned(16))) float ldsX[CP ? 2 : 1][CP ? LPX : 1];
  __shared__ float red[BY], redv[BY];

  // XCD-aware tile order: hardware id b runs on XCD b % 8.
  const int nwg = static_cast<int>(gridDim.x);
  const int bid = static_cast<int>(blockIdx.x);
  const int logical = (bid & 7) * (nwg >> 3) + (bid >> 3);
  if (logical >= a.total_tiles) return;
  const int tix = logical % a.tiles_x;
  const int rest = logical / a.tiles_x;
  const int tiy = rest % a.tiles_y;
  const int chunk = rest / a.tiles_y;
  const int x0 = tix * TX, y0 = tiy * TY;
  // output planes [zb, zend) of this chunk, in trips of nine planes over
  // [zb, ze); the planes of the last trip at or past zend are skipped (a
  // uniform branch), so a chunk may have any length and the chunks of a grid
  // can be equal.  Nothing is written past nz: the padding planes stay zero.
  // The fused CPML kernel, bound by instruction issue, measured 4% slower
  // with that branch between its planes: it keeps whole trips (its z-chunks
  // are multiples of nine), and its last chunk's final trip writes the zero
  // padding planes with zeros (sponge factor 0 past nz).
  constexpr bool kSkipTail = !CP;
  const int zb = chunk * a.zchunk;
  const int zend = min(zb + a.zchunk, a.nz);
  const int ze = zb + (zend - zb + kQ - 1) / kQ * kQ;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int nx = a.nx, ny = a.ny;
  const size_t plane = static_cast<size_t>(nx) * static_cast<size_t>(ny);
  const uint32_t pbytes = static_cast<uint32_t>(plane) * ES;
  const uint32_t pbytes_f = static_cast<uint32_t>(plane) * 4u;
  const int x = x0 + VEC * lane;  // first of this lane's VEC columns
  const bool xin = x < nx;        // all VEC columns (nx % VEC == 0)
  const int yb = y0 + w * RY;     // first row of this wavefront

  // ---- step index and 16-bit field scales.  16-bit storage: the exponents of
  // A^{n+1} and V^{n+1} come from bounds valid at every node,
  //   |V^{n+1}| <= max|V^n| + gamma max|A^n| + |q^n| = bV,  |A^{n+1}| <= max|A^n| + bV,
  // so each is fixed before anything is written.
  const int n = ADJ ? 0 : a.st->n + a.k;
  float inv_cur = 1.f, inv_prev = 1.f, s_next = 1.f, inv_next = 1.f, sv_next = 1.f;
  if (S != kF32) {
    const int ea = a.st->exps[n & 3], ev = a.st->exps_v[n & 3];
    inv_cur = exp2i(-ea);
    inv_prev = exp2i(-ev);
    const float a_a = __uint_as_float(a.st->amax[n & 3]) * inv_cur;
    const float a_v = __uint_as_float(a.st->amax_v[n & 3]) * inv_prev;
    const float qmag = a.sx >= 0 ? fabsf(a.wavelet[n]) * a.src_scale : 0.f;
    const float bv = a_v + a.gamma * a_a + qmag;
    const int ea_next = scale_exponent(a_a + bv), ev_next = scale_exponent(bv);
    s_next = exp2i(ea_next);
    inv_next = exp2i(-ea_next);
    sv_next = exp2i(ev_next);
    if (logical == 0 && threadIdx.x == 0) {
      a.st->exps[(n + 1) & 3] = ea_next;
      a.st->exps_v[(n + 1) & 3] = ev_next;
      a.st->amax[(n + 2) & 3] = 0u;
      a.st->amax_v[(n + 2) & 3] = 0u;
    }
  }

  // ---- buffer resources: one per field for the whole workgroup, based at
  // the first plane it touches (zlo) and spanning the planes [zlo, zhi) its
  // trips, prefetches and halo cover (the host keeps every span below 2^31
  // bytes; the fields carry kPadZ zero planes past nz).  The plane goes into
  // the scalar offset; a lane's row and column go into its vector offset,
  // which is kOOB for nodes outside the grid, so those lanes load zeros and
  // store nothing.  Planes below 0 (prologue only) use rnull (no records):
  // every load from it is zero.
  const int zlo = max(zb - R, 0);
  const int zhi = ze + PD + R;
  const uint32_t span = static_cast<uint32_t>(zhi - zlo) * pbytes;
  const uint32_t span_f = static_cast<uint32_t>(zhi - zlo) * pbytes_f;
  const size_t base = static_cast<size_t>(zlo) * plane;
  const size_t base_b = base * ES;
  const char *U = static_cast<const char *>(a.cur);
  const char *P = static_cast<const char *>(a.prev);
  char *O = static_cast<char *>(a.out);
  const rsrc_t rU = make_rsrc(U + base_b, span);
  const rsrc_t rP = make_rsrc(P + base_b, span);
  const rsrc_t rO = make_rsrc(O + base_b, span);
  const rsrc_t rVo = make_rsrc((S != kF32 ? static_cast<char *>(a.vout) : O) + base_b, span);
  const rsrc_t rM = M16 ? make_rsrc(reinterpret_cast<const char *>(a.m) + base * 2, span)
                        : make_rsrc(a.m + base, span_f);
  const rsrc_t rnull = make_rsrc(a.gz, 0u);
  const rsrc_t rF = make_rsrc((ADJ ? a.fwd : a.m) + base, span_f);
  const rsrc_t rI = make_rsrc((ADJ ? a.img : a.m) + base, ADJ ? span_f : 0u);
  auto so = [&](int z) { return static_cast<uint32_t>(z - zlo) * pbytes; };     // plane offset, A fields
  auto so_f = [&](int z) { return static_cast<uint32_t>(z - zlo) * pbytes_f; };  // plane offset, float fields

  // ---- per-row data (wavefront-uniform) and per-lane offsets
  float gxv[VEC], gyv[RY], qrow[RY];
  int ryi[RY], rxi[VEC];
  uint32_t vrow[RY], vrow_f[RY];  // lane byte offset of (x, row j) in a plane, or kOOB
#pragma unroll
  for (int i = 0; i < VEC; ++i) {
    gxv[i] = xin ? a.gx[x + i] : 0.f;
    rxi[i] = -1;
    if (a.box.cnx > 0 && xin) {
      const int d = x + i - a.box.x0;
      if (d >= 0 && d % a.box.sx == 0 && d / a.box.sx < a.box.cnx) rxi[i] = d / a.box.sx;
    }
  }
  // the source node: qrow[j] = 1 in its lane and row, its column index srci
  const int srci = (!ADJ && a.sx >= 0) ? (a.sx - x0) % VEC : 0;
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const int yj = yb + j;
    const bool ok = yj < ny && xin;
    const uint32_t e = static_cast<uint32_t>(yj) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(x);
    vrow[j] = ok ? e * ES : kOOB;
    vrow_f[j] = ok ? e * 4u : kOOB;
    gyv[j] = yj < ny ? a.gy[yj] : 0.f;
    ryi[j] = -1;
    if (a.box.cnx > 0 && yj < ny) {
      const int d = yj - a.box.y0;
      if (d >= 0 && d % a.box.sy == 0 && d / a.box.sy < a.box.cny) ryi[j] = d / a.box.sy;
    }
    qrow[j] = (!ADJ && a.sx >= 0 && a.sx >= x && a.sx < x + VEC && yj == a.sy) ? 1.f : 0.f;
  }
  // y-halo rows of this wavefront: halo row r = w + BY*i (r < R above the tile, else below)
  int yhlds[NYH];
  uint32_t vyh[NYH], vyh_f[NYH];
#pragma unroll
  for (int i = 0; i < NYH; ++i) {
    const int r = w + BY * i;
    const bool yhin = r < 2 * R;
    const int lr = r < R ? r : TY + r;
    const int gyy = y0 - R + lr;
    const bool ok = yhin && gyy >= 0 && gyy < ny && xin;
    yhlds[i] = yhin ? lr * LW + R + VEC * lane : DUMMY + VEC * lane;
    const uint32_t e = static_cast<uint32_t>(gyy) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(x);
    vyh[i] = ok ? e * ES : kOOB;
    vyh_f[i] = ok ? e * 4u : kOOB;
  }
  // x-halo: lane l < 8*RY covers row l/8 of this wavefront, column l%8
  int xhlds = DUMMY + lane, xhx = DUMMYX + lane, xh_x = -1, xh_y = 0;
  uint32_t vxh = kOOB, vxh_f = kOOB;
  if (lane < 8 * RY) {
    const int j = lane >> 3, c = lane & 7;
    const int gxx = c < R ? x0 - R + c : x0 + TX + (c - R);
    const int yj = yb + j;
    xhlds = (R + w * RY + j) * LW + (c < R ? c : TX + c);
    xhx = (w * RY + j) * LW + (c < R ? c : TX + c);
    if (yj < ny) {
      xh_x = gxx;
      xh_y = yj;
    }
    if (gxx >= 0 && gxx < nx && yj < ny) {
      const uint32_t e = static_cast<uint32_t>(yj) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(gxx);
      vxh = e * ES;
      vxh_f = e * 4u;
    }
  }

  // ---- CPML (fused x part): one resource per x slab array (the host keeps
  // it below 2^31 bytes; loads outside it read zero), the x profile at this
  // lane's columns, and whether any of those columns lies in an x layer
  const int W = CP ? a.cp.W : 0;
  const uint32_t W2 = 2u * static_cast<uint32_t>(W);
  const uint32_t uny = static_cast<uint32_t>(ny);
  rsrc_t rPX = rnull, rZX = rnull;
  float cax[CP ? VEC : 1], cbx[CP ? VEC : 1];
  bool xown = false;  // some of this lane's columns lie in an x layer
  if constexpr (CP) {
    const uint32_t bx = static_cast<uint32_t>(a.nz) * uny * W2 * 4u;
    rPX = make_rsrc(a.cp.psi[0], bx);
    rZX = make_rsrc(a.cp.zeta[0], bx);
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      cax[i] = xin ? a.cp.ca[0][x + i] : 0.f;
      cbx[i] = xin ? a.cp.cb[0][x + i] : 0.f;
    }
    xown = xin && (x < W || x + VEC - 1 >= nx - W);
  }
  // byte offset of node (c, yj) in a plane of the x slabs, or kOOB off the x layers
  auto xoff = [&](int c, int yj) {
    const int sx = slab_index(c, nx, W);
    return sx >= 0 ? (static_cast<uint32_t>(yj) * W2 + static_cast<uint32_t>(sx)) * 4u : kOOB;
  };

  auto rec_plane = [&](int z) {  // receiver-box index of plane z, or -1
    int rzi = -1;
    if (a.box.cnx > 0) {
      const int d = z - a.box.z0;
      if (d >= 0 && d % a.box.sz == 0 && d / a.box.sz < a.box.cnz) rzi = d / a.box.sz;
    }
    return rzi;
  };
  // per-plane tables, nz + kPadZ entries: the padding planes read sponge
  // factor 0 and receiver index -1
  const rsrc_t rgz = make_rsrc(a.gz, static_cast<uint32_t>(a.nz + kPadZ) * 4u);
  const rsrc_t rrz = make_rsrc(a.rz, static_cast<uint32_t>(a.nz + kPadZ) * 4u);
  // residual row of this launch (adjoint); the resource covers exactly that
  // row.  Without receivers it has no records (its loads return zero).
  const bool has_res = ADJ && a.resid != nullptr && a.nrec > 0;
  const rsrc_t rres = has_res ? make_rsrc(a.resid + static_cast<size_t>(a.resid_row) * a.nrec,
                                          static_cast<uint32_t>(a.nrec) * 4u)
                              : rnull;

  auto load_stage = [&](StageT &st, int z) {
    const uint32_t sl = so(z + R), slf = so_f(z + R);
    const uint32_t sc = so(z), scf = so_f(z);
    st.gz = __uint_as_float(ld_words<4, 0>(rgz, 0u, static_cast<uint32_t>(z) * 4u).w[0]);
    st.rz = static_cast<int>(ld_words<4, 0>(rrz, 0u, static_cast<uint32_t>(z) * 4u).w[0]);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      st.lead[j] = ld_words<NA, 0>(rU, vrow[j], sl);
      st.p[j] = ld_words<NA, NTP>(rP, vrow[j], sc);
      st.m[j] = ld_words<StageT::NM, NTP>(rM, M16 ? vrow[j] : vrow_f[j], M16 ? sc : scf);
    }
#pragma unroll
    for (int i = 0; i < NYH; ++i) st.yh[i] = ld_words<NA, 0>(rU, vyh[i], LEADH ? sl : sc);
    st.xh = ld_words<S == kF32 ? 4 : 2, 0>(rU, vxh, LEADH ? sl : sc);
    if constexpr (ADJ) {
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        st.leadF[j] = ld_words<NF, 0>(rF, vrow_f[j], slf);
        st.img[j] = ld_words<NF, kNT>(rI, vrow_f[j], scf);
      }
#pragma unroll
      for (int i = 0; i < NYH; ++i) st.yhF[i] = ld_words<NF, 0>(rF, vyh_f[i], scf);
      st.xhF = __uint_as_float(ld_words<4, 0>(rF, vxh_f, scf).w[0]);
      const int rzi = rec_plane(z);
#pragma unroll
      for (int j = 0; j < RY; ++j)
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
          const bool at = rzi >= 0 && ryi[j] >= 0 && rxi[i] >= 0;
          const uint32_t ridx =
              at ? static_cast<uint32_t>((rzi * a.box.cny + ryi[j]) * a.box.cnx + rxi[i]) * 4u : kOOB;
          st.res[j][i] = __uint_as_float(ld_words<4, 0>(rres, ridx, 0u).w[0]);
        }
    }
    if constexpr (CP) {  // x slab plane z (none past nz); zero off the x layers
      const bool zin = z < a.nz;
      const rsrc_t rp = zin ? rPX : rnull, rz = zin ? rZX : rnull;
      const uint32_t sp = zin ? static_cast<uint32_t>(z) * uny * W2 * 4u : 0u;
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        const int yj = yb + j;
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
          const uint32_t o = (xown && yj < ny) ? xoff(x + i, yj) : kOOB;
          st.psx[j][i] = __uint_as_float(ld_words<4, 0>(rp, o, sp).w[0]);
          st.zex[j][i] = __uint_as_float(ld_words<4, 0>(rz, o, sp).w[0]);
        }
      }
      st.psxh = __uint_as_float(ld_words<4, 0>(rp, xh_x >= 0 ? xoff(xh_x, xh_y) : kOOB, sp).w[0]);
    }
  };

  // ---- prologue: queue slot (p - zb + R) mod 9 holds plane p; stages hold planes zb .. zb+PD-1
  float q[kQ][RY][VEC];
  float qF[ADJ ? kQ : 1][RY][VEC];
#pragma unroll
  for (int k = 0; k < 2 * R; ++k) {
    const int zz = zb - R + k;
    const bool zok = zz >= 0;
    const rsrc_t r = zok ? rU : rnull;
    const rsrc_t rf = zok ? rF : rnull;
    const uint32_t s0 = zok ? so(zz) : 0u, s0f = zok ? so_f(zz) : 0u;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const Words<NA> t = ld_words<NA, 0>(r, vrow[j], s0);
#pragma unroll
      for (int i = 0; i < VEC; ++i) q[k][j][i] = row_get<S>(t, i) * inv_cur;
      if constexpr (ADJ) {
        const Words<NF> tf = ld_words<NF, 0>(rf, vrow_f[j], s0f);
#pragma unroll
        for (int i = 0; i < VEC; ++i) qF[k][j][i] = __uint_as_float(tf.w[i]);
      }
    }
  }
  if constexpr (LEADH) {  // ring slots 0 .. R-1: planes zb .. zb+R-1 with their halo
#pragma unroll
    for (int k = 0; k < R; ++k) {
      float *Lk = lds[k];
      const uint32_t s0 = so(zb + k);
#pragma unroll
      for (int j = 0; j < RY; ++j) lds_put<VEC>(Lk + (R + w * RY + j) * LW + R + VEC * lane, q[R + k][j]);
#pragma unroll
      for (int i = 0; i < NYH; ++i) {
        const Words<NA> t = ld_words<NA, 0>(rU, vyh[i], s0);
        float v[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = row_get<S>(t, e) * inv_cur;
        lds_put<VEC>(Lk + yhlds[i], v);
      }
      Lk[xhlds] = row_get<S>(ld_words<S == kF32 ? 4 : 2, 0>(rU, vxh, s0), 0) * inv_cur;
    }
  }
  // semi-stencil partials: slot (p - zb + R) mod 9 holds sum_m kz_m A(p-m) of plane p
  float X[SEMI ? kQ : 1][RY][VEC];
  if constexpr (SEMI) {
#pragma unroll
    for (int k = R; k < 2 * R; ++k)
#pragma unroll
      for (int j = 0; j < RY; ++j)
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
          const float c = q[k][j][i];
          float t = a.c.kz[R - 1] * (q[k - R][j][i] - c);
#pragma unroll
          for (int m = R - 1; m >= 1; --m) t = fmaf(a.c.kz[m - 1], q[k - m][j][i] - c, t);
          X[k][j][i] = t;
        }
  }
  StageT stg[PD];
#pragma unroll
  for (int s = 0; s < PD; ++s) load_stage(stg[s], zb + s);

  const float wsrc = (!ADJ && a.sx >= 0) ? a.wavelet[n] * a.src_scale : 0.f;
  // 16-bit storage: running maxima of the stored magnitudes kept as 16-bit
  // patterns with the sign cleared, both halves of a word per instruction;
  // for f16 and bf16 the magnitude order of finite values is the unsigned
  // order of those bits, so the maxima decode to max |stored| exactly
  float amax_loc = 0.f, amaxv_loc = 0.f;
  u16x2 amax_bits = {0, 0}, amaxv_bits = {0, 0};

  // Laplacian of Eq. 1 at the VEC nodes of row j of this lane: centre and z
  // neighbours from the queue Q, x neighbours from a window of the LDS row,
  // y neighbours from this lane's own rows when they lie in the strip, else
  // from the LDS rows above and below.
  // CP: also the per-axis parts lax[a] (centre weight c_0 / h_a^2 each), and
  // lap = (lax[0] + lax[1]) + lax[2].  sum_form (a compile-time flag): k0 u +
  // sum k_m (u(+m) + u(-m)) instead of the centred differences.
  auto laplacian = [&](const float (&Q)[kQ][RY][VEC], const float *Lp, int cs, int s0, int j, float *lap,
                       const float (&Xp)[SEMI ? kQ : 1][RY][VEC], float (&lax)[3][VEC], auto sum_form)
                       __attribute__((always_inline)) {
    constexpr bool kSum = decltype(sum_form)::value;
    const float *row = Lp + (R + w * RY + j) * LW + VEC * lane;  // window start: column x - R
    float win[VEC + 2 * R];
#pragma unroll
    for (int k = 0; k < (VEC + 2 * R) / VEC; ++k)
      if (VEC > 1 || k != R) lds_get<VEC>(row + VEC * k, win + VEC * k);
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      lap[i] = kSum ? a.c.k0 * Q[cs][j][i] : 0.f;
      if constexpr (CP) {  // per axis, from the centre term (the sum form; see below)
#pragma unroll
        for (int d = 0; d < 3; ++d) lax[d][i] = a.c.k0a[d] * Q[cs][j][i];
      }
    }
#pragma unroll
    for (int m = 1; m <= R; ++m) {
      float yp[VEC], ym[VEC];
      if (j + m < RY) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) yp[i] = Q[cs][(j + m) % RY][i];
      } else {
        lds_get<VEC>(row + m * LW + R, yp);
      }
      if (j - m >= 0) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) ym[i] = Q[cs][(j - m + RY) % RY][i];
      } else {
        lds_get<VEC>(row - m * LW + R, ym);
      }
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        // second differences from the centre: (u(+m) - u) + (u(-m) - u)
        const float c = Q[cs][j][i];
        const float sx = (win[R + i + m] - c) + (win[R + i - m] - c);
        const float sy = (yp[i] - c) + (ym[i] - c);
        const float sz = (Q[(s0 + R + m) % kQ][j][i] - c) + (Q[(s0 + R - m + kQ) % kQ][j][i] - c);
        if constexpr (CP) {
          // The fused CPML kernel sums c_0 u + sum_m c_m (u(+m) + u(-m)) per
          // axis: it is issue-bound (its x boundary terms on top of the
          // stencil), and the centred differences' extra 24 operations per
          // node cost it 18%; its runs are checked against the oracle at the
          // float32 tolerance
          lax[0][i] = fmaf(a.c.kx[m - 1], win[R + i + m] + win[R + i - m], lax[0][i]);
          lax[1][i] = fmaf(a.c.ky[m - 1], yp[i] + ym[i], lax[1][i]);
          lax[2][i] = fmaf(a.c.kz[m - 1], Q[(s0 + R + m) % kQ][j][i] + Q[(s0 + R - m + kQ) % kQ][j][i], lax[2][i]);
        } else if constexpr (kSum) {
          lap[i] = fmaf(a.c.kx[m - 1], win[R + i + m] + win[R + i - m], lap[i]);
          lap[i] = fmaf(a.c.ky[m - 1], yp[i] + ym[i], lap[i]);
          lap[i] = fmaf(a.c.kz[m - 1], Q[(s0 + R + m) % kQ][j][i] + Q[(s0 + R - m + kQ) % kQ][j][i], lap[i]);
        } else {
          lap[i] = fmaf(a.c.kx[m - 1], sx, lap[i]);
          lap[i] = fmaf(a.c.ky[m - 1], sy, lap[i]);
          if constexpr (!SEMI) lap[i] = fmaf(a.c.kz[m - 1], sz, lap[i]);
        }
      }
    }
    if constexpr (CP) {
#pragma unroll
      for (int i = 0; i < VEC; ++i) lap[i] = (lax[0][i] + lax[1][i]) + lax[2][i];
    }
    if constexpr (SEMI) {  // left half from the partial, right half from the queue
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        float t = Xp[cs][j][i];
#pragma unroll
        for (int m = 1; m <= R; ++m) t = fmaf(a.c.kz[m - 1], Q[(s0 + R + m) % kQ][j][i] - Q[cs][j][i], t);
        lap[i] += t;
      }
    }
  };

  for (int zs = zb; zs < ze; zs += kQ) {
    // nine planes per trip with compile-time queue slots and stage indices, so
    // the queue rotates by register renaming (a runtime index would move the
    // queue into scratch memory)
    static_for<kQ>([&](auto sc) __attribute__((always_inline)) {
      constexpr int s = decltype(sc)::value;
      const int z = zs + s;
      if (kSkipTail && z >= zend) return;  // past the chunk: the same for the whole workgroup
      constexpr int cslot = (s + R) % kQ;  // plane z
      StageT &cs = stg[s % PD];
      const int par = (z - zb) & 1;
      // L: the centre plane z (read after the barrier); Lw: the plane staged
      // in this iteration (plane z+R with LEADH, else plane z)
      float *L = lds[LEADH ? (z - zb) % NSLOT : par];
      float *Lw = LEADH ? lds[(z - zb + R) % NSLOT] : L;
      float *LF = ldsF[ADJ ? par : 0];
#pragma unroll
      for (int j = 0; j < RY; ++j) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) q[(s + 2 * R) % kQ][j][i] = row_get<S>(cs.lead[j], i) * inv_cur;
        lds_put<VEC>(Lw + (R + w * RY + j) * LW + R + VEC * lane, q[LEADH ? (s + 2 * R) % kQ : cslot][j]);
        if constexpr (SEMI) {  // left half of plane z+R from planes z .. z+R-1
#pragma unroll
          for (int i = 0; i < VEC; ++i) {
            const float c = q[(s + 2 * R) % kQ][j][i];
            float t = a.c.kz[R - 1] * (q[cslot][j][i] - c);
#pragma unroll
            for (int m = R - 1; m >= 1; --m) t = fmaf(a.c.kz[m - 1], q[(s + 2 * R - m) % kQ][j][i] - c, t);
            X[(s + 2 * R) % kQ][j][i] = t;
          }
        }
        if constexpr (ADJ) {
#pragma unroll
          for (int i = 0; i < VEC; ++i) qF[(s + 2 * R) % kQ][j][i] = __uint_as_float(cs.leadF[j].w[i]);
          lds_put<VEC>(LF + (R + w * RY + j) * LW + R + VEC * lane, qF[cslot][j]);
        }
      }
#pragma unroll
      for (int k = 0; k < NYH; ++k) {
        float t[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) t[i] = row_get<S>(cs.yh[k], i) * inv_cur;
        lds_put<VEC>(Lw + yhlds[k], t);
        if constexpr (ADJ) {
#pragma unroll
          for (int i = 0; i < VEC; ++i) t[i] = __uint_as_float(cs.yhF[k].w[i]);
          lds_put<VEC>(LF + yhlds[k], t);
        }
      }
      Lw[xhlds] = row_get<S>(cs.xh, 0) * inv_cur;
      if constexpr (ADJ) LF[xhlds] = cs.xhF;
      float *LX = ldsX[CP ? par : 0];
      float zex[CP ? RY : 1][CP ? VEC : 1];
      if constexpr (CP) {
#pragma unroll
        for (int j = 0; j < RY; ++j) {
          lds_put<VEC>(LX + (w * RY + j) * LW + R + VEC * lane, cs.psx[j]);
#pragma unroll
          for (int i = 0; i < VEC; ++i) zex[j][i] = cs.zex[j][i];
        }
        LX[xhx] = cs.psxh;
      }
      float pc[RY][VEC], mc[RY][VEC], ic[RY][VEC], rc[RY][VEC];
#pragma unroll
      for (int j = 0; j < RY; ++j)
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
          pc[j][i] = row_get<S>(cs.p[j], i) * inv_prev;
          if constexpr (M16) {
            const uint32_t u = (cs.m[j].w[i >> 1] >> (16 * (i & 1))) & 0xffffu;
            mc[j][i] = fmaf(static_cast<float>(u), a.m_step, a.m_lo);
          } else {
            mc[j][i] = __uint_as_float(cs.m[j].w[i]);
          }
          ic[j][i] = ADJ ? __uint_as_float(cs.img[ADJ ? j : 0].w[i]) : 0.f;
          rc[j][i] = ADJ ? cs.res[ADJ ? j : 0][ADJ ? i : 0] : 0.f;
        }
      const float gzv = cs.gz;
      const int rzi = ADJ ? rec_plane(z) : __builtin_amdgcn_readfirstlane(cs.rz);
      load_stage(cs, z + PD);  // past the chunk end: planes of the next chunk or padding, unused
      __syncthreads();

      const uint32_t sz0 = so(z), sz0f = so_f(z);
      const bool zin = z < a.nz;
      // source term of this plane, per column of the lane's VEC nodes
      float wsp[VEC];
#pragma unroll
      for (int i = 0; i < VEC; ++i) wsp[i] = (!ADJ && z == a.sz && i == srci) ? wsrc : 0.f;
      float outv[S == kF32 ? RY : 1][S == kF32 ? VEC : 1];  // float32: A^{n+1} of the plane's rows
      Words<NA> rkeep[S != kF32 ? RY : 1];                  // 16-bit: the stored rows (receivers)
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        float lap[VEC], lax[3][VEC];
        laplacian(q, L, cslot, s, j, lap, X, lax, std::integral_constant<bool, kSumForm>{});
        if constexpr (CP) {  // x part of the CPML terms: D1_x psi_x + zeta_x, zeta_x updated
          const int yj = yb + j;
          float ext[VEC], zn[VEC];
          // x: every lane, psi_x window (columns x-R .. x+VEC+R-1) from LDS;
          // psi_x and zeta_x are zero off the layers
          {
            float px[VEC + 2 * R];
            const float *xrow = LX + (w * RY + j) * LW + VEC * lane;
#pragma unroll
            for (int k = 0; k < (VEC + 2 * R) / VEC; ++k) lds_get<VEC>(xrow + VEC * k, px + VEC * k);
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
              float d = 0.f;
#pragma unroll
              for (int k = 1; k <= R; ++k) d = fmaf(a.cp.d1w[0][k - 1], px[R + i + k] - px[R + i - k], d);
              zn[i] = fmaf(cbx[i], zex[j][i], cax[i] * (lax[0][i] + d));
              ext[i] = d + zn[i];
            }
          }
          if (xown && zin && yj < ny) {
            const uint32_t sp = static_cast<uint32_t>(z) * uny * W2 * 4u;
#pragma unroll
            for (int i = 0; i < VEC; ++i)
              st_words<4, 0>(Words<4>{{__float_as_uint(zn[i])}}, rZX, xoff(x + i, yj), sp);
          }
#pragma unroll
          for (int i = 0; i < VEC; ++i) lap[i] += ext[i];
        }
        const float gyz = gyv[j] * gzv;
        float v[VEC], vv[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
          const float c = q[cslot][j][i];
          if (ADJ) lap[i] += rc[j][i];  // zero off the receivers
          const float g = gxv[i] * gyz;
          if (S == kF32) {  // A^{n+1} = g (2 A^n - g A^{n-1} + m L A^n + q)
            float t = fmaf(-g, pc[j][i], 2.f * c);
            t = fmaf(mc[j][i], lap[i], t);
            if (!ADJ) t = fmaf(qrow[j], wsp[i], t);
            v[i] = t * g;
          } else {  // V^{n+1} = g (V^n + m L A^n + q),  A^{n+1} = g A^n + V^{n+1}
            float t = fmaf(mc[j][i], lap[i], pc[j][i]);
            t = fmaf(qrow[j], wsp[i], t);
            vv[i] = t * g;
            v[i] = fmaf(g, c, vv[i]);
          }
        }
        if constexpr (S == kF32) {
          st_words<NA, NTP>(row_put<S, VEC>(v), rO, vrow[j], sz0);
#pragma unroll
          for (int i = 0; i < VEC; ++i) outv[j][i] = v[i];
        } else {
          float sa[VEC], sv[VEC];
#pragma unroll
          for (int i = 0; i < VEC; ++i) {
            sa[i] = v[i] * s_next;
            sv[i] = vv[i] * sv_next;
          }
          const Words<NA> ra = row_put<S, VEC>(sa), rv = row_put<S, VEC>(sv);
          st_words<NA, NTP>(ra, rO, vrow[j], sz0);
          st_words<NA, NTP>(rv, rVo, vrow[j], sz0);
#pragma unroll
          for (int k = 0; k < Words<NA>::N; ++k) {
            amax_bits = __builtin_elementwise_max(amax_bits, __builtin_bit_cast(u16x2, ra.w[k] & 0x7fff7fffu));
            amaxv_bits = __builtin_elementwise_max(amaxv_bits, __builtin_bit_cast(u16x2, rv.w[k] & 0x7fff7fffu));
          }
          rkeep[S != kF32 ? j : 0] = ra;
        }
        if constexpr (ADJ) {
          // the imaging term L(A^k), only accumulated (no recurrence runs
          // through it): summed from the centre weight, 25 instead of 48
          // operations per node
          float lapF[VEC], im[VEC], laxF[3][VEC];
          laplacian(qF, LF, cslot, s, j, lapF, X, laxF, std::integral_constant<bool, true>{});
#pragma unroll
          for (int i = 0; i < VEC; ++i) im[i] = fmaf(q[cslot][j][i], lapF[i], ic[j][i]);
          st_words<NF, kNT>(row_put<kF32, VEC>(im), rI, vrow_f[j], sz0f);
        }
      }
      // receiver samples of A^{n+1} (forward), in the plane's own uniform branch
      if (!ADJ && rzi >= 0) {
#pragma unroll
        for (int j = 0; j < RY; ++j)
#pragma unroll
          for (int i = 0; i < VEC; ++i)
            if (ryi[j] >= 0 && rxi[i] >= 0) {
              float val;
              if constexpr (S == kF32)
                val = outv[j][i];
              else
                val = row_get<S>(rkeep[j], i) * inv_next;
              a.traces[static_cast<size_t>(n) * a.nrec + (rzi * a.box.cny + ryi[j]) * a.box.cnx + rxi[i]] = val;
            }
      }
    });
  }

  if (S != kF32) {  // one order-independent atomic per workgroup and field
    amax_loc = row_get<S>(Words<2>{{static_cast<uint32_t>(amax_bits.x > amax_bits.y ? amax_bits.x : amax_bits.y)}}, 0);
    amaxv_loc = row_get<S>(Words<2>{{static_cast<uint32_t>(amaxv_bits.x > amaxv_bits.y ? amaxv_bits.x : amaxv_bits.y)}}, 0);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      amax_loc = fmaxf(amax_loc, __shfl_xor(amax_loc, off, 64));
      amaxv_loc = fmaxf(amaxv_loc, __shfl_xor(amaxv_loc, off, 64));
    }
    if (lane == 0) {
      red[w] = amax_loc;
      redv[w] = amaxv_loc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float mx = red[0], mv = redv[0];
#pragma unroll
      for (int k = 1; k < BY; ++k) {
        mx = fmaxf(mx, red[k]);
        mv = fmaxf(mv, redv[k]);
      }
      atomicMax(&a.st->amax[(n + 1) & 3], __float_as_uint(mx));
      atomicMax(&a.st->amax_v[(n + 1) & 3], __float_as_uint(mv));
    }
  }
}

// ------------------------------------------------------------ 3D-blocked kernels
//
// The two 3D-blocking designs the paper compares against 2.5D streaming
// (Sec. IV-A: "gmem" reads every stencil point from global memory, "smem"
// stages a 3D tile with its halo in shared memory), rebuilt for gfx950 with
// the same fused update, sponge, source and receivers and the same
// floating-point operation order as step_kernel, so their results are
// bitwise identical to it.  Float32 storage, forward only.  A workgroup is a
// 64 x BY x BZ block of nodes, one thread per node.

// Byte offset of node (x, y, z) in a float32 field whose resource starts at
// plane zlo, or kOOB outside the grid in x or y or below plane 0 (the
// padding planes past nz read as zeros).
__device__ __forceinline__ uint32_t node_off(int x, int y, int z, int nx, int ny, int zlo) {
  const bool ok = x >= 0 && x < nx && y >= 0 && y < ny && z >= 0;
  const uint32_t e = (static_cast<uint32_t>(z - zlo) * static_cast<uint32_t>(ny) + static_cast<uint32_t>(y)) *
                         static_cast<uint32_t>(nx) +
                     static_cast<uint32_t>(x);
  return ok ? e * 4u : kOOB;
}

// Node of this thread and the shared set-up of the 3D kernels.
template <int BY, int BZ>
struct Block3D {
  int x0, y0, z0, x, y, z, zlo;
  bool inside;
  __device__ bool init(const StepArgs &a) {
    const int nwg = static_cast<int>(gridDim.x);
    const int bid = static_cast<int>(blockIdx.x);
    const int logical = (bid & 7) * (nwg >> 3) + (bid >> 3);
    if (logical >= a.total_tiles) return false;
    const int tix = logical % a.tiles_x;
    const int rest = logical / a.tiles_x;
    const int tiy = rest % a.tiles_y;
    const int tiz = rest / a.tiles_y;
    x0 = tix * kTileX;
    y0 = tiy * BY;
    z0 = tiz * BZ;
    const int t = static_cast<int>(threadIdx.x);
    x = x0 + (t & 63);
    y = y0 + (t >> 6) % BY;
    z = z0 + t / (64 * BY);
    zlo = max(z0 - R, 0);
    inside = x < a.nx && y < a.ny && z < a.nz;
    return true;
  }
};

// The fused update of one node from its Laplacian (float32 storage), with the
// receiver sample; identical operations to step_kernel<kF32, ...>.
__device__ __forceinline__ void update_node(const StepArgs &a, int n, int x, int y, int z, bool inside, float c,
                                            float lap, float pc, float mc, float gzv, rsrc_t rO, uint32_t voff) {
  const float gxv = inside ? a.gx[x] : 0.f;
  const float gyv = inside ? a.gy[y] : 0.f;
  const float g = gxv * (gyv * gzv);
  const float wsrc = a.sx >= 0 ? a.wavelet[n] * a.src_scale : 0.f;
  const float qsel = (a.sx >= 0 && x == a.sx && y == a.sy) ? 1.f : 0.f;
  const float wsp = z == a.sz ? wsrc : 0.f;
  float t = fmaf(-g, pc, 2.f * c);
  t = fmaf(mc, lap, t);
  t = fmaf(qsel, wsp, t);
  const float v = t * g;
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rO, static_cast<int>(inside ? voff : kOOB), 0, kNT);
  if (inside && a.box.cnx > 0 && z < a.nz && a.rz[z] >= 0) {
    const int dx = x - a.box.x0, dy = y - a.box.y0;
    if (dx >= 0 && dx % a.box.sx == 0 && dx / a.box.sx < a.box.cnx && dy >= 0 && dy % a.box.sy == 0 &&
        dy / a.box.sy < a.box.cny)
      a.traces[static_cast<size_t>(n) * a.nrec + (a.rz[z] * a.box.cny + dy / a.box.sy) * a.box.cnx + dx / a.box.sx] =
          v;
  }
}

// "gmem": every one of the 25 stencil values is a load of its own; reuse
// between neighbouring threads is left to the L1 and L2 caches.
template <int BY, int BZ>
__global__ void __launch_bounds__(64 * BY * BZ) gmem_kernel(StepArgs a) {
  Block3D<BY, BZ> b;
  if (!b.init(a)) return;
  const int nx = a.nx, ny = a.ny, n = a.st->n + a.k;
  const uint32_t planes = static_cast<uint32_t>(b.z0 + BZ + R - b.zlo);
  const uint32_t bytes = planes * static_cast<uint32_t>(nx) * static_cast<uint32_t>(ny) * 4u;
  const size_t base = static_cast<size_t>(b.zlo) * nx * ny;
  const rsrc_t rU = make_rsrc(static_cast<const float *>(a.cur) + base, bytes);
  const rsrc_t rP = make_rsrc(static_cast<const float *>(a.prev) + base, bytes);
  const rsrc_t rO = make_rsrc(static_cast<float *>(a.out) + base, bytes);
  const rsrc_t rM = make_rsrc(a.m + base, bytes);
  auto U = [&](int x, int y, int z) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rU, static_cast<int>(node_off(x, y, z, nx, ny, b.zlo)),
                                                                0, 0));
  };
  const int x = b.x, y = b.y, z = b.z;
  const uint32_t own = node_off(x, y, z, nx, ny, b.zlo);
  const float c = U(x, y, z);
  float lap = 0.f;
#pragma unroll
  for (int m = 1; m <= R; ++m) {
    lap = fmaf(a.c.kx[m - 1], (U(x + m, y, z) - c) + (U(x - m, y, z) - c), lap);
    lap = fmaf(a.c.ky[m - 1], (U(x, y + m, z) - c) + (U(x, y - m, z) - c), lap);
    lap = fmaf(a.c.kz[m - 1], (U(x, y, z + m) - c) + (U(x, y, z - m) - c), lap);
  }
  const float pc = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rP, static_cast<int>(own), 0, kNT));
  const float mc = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rM, static_cast<int>(own), 0, kNT));
  const float gzv = b.inside ? a.gz[z] : 0.f;
  update_node(a, n, x, y, z, b.inside, c, lap, pc, mc, gzv, rO, own);
}

// "smem": the block's nodes and their radius-4 halo in all three directions
// are staged in LDS, (64+8) x (BY+8) x (BZ+8) values, then every stencil value
// is read from there.
template <int BY, int BZ>
__global__ void __launch_bounds__(64 * BY * BZ) smem_kernel(StepArgs a) {
  constexpr int SX = kTileX + 2 * R, SY = BY + 2 * R, SZ = BZ + 2 * R;
  __shared__ float T[SZ][SY][SX];
  Block3D<BY, BZ> b;
  if (!b.init(a)) return;
  const int nx = a.nx, ny = a.ny, n = a.st->n + a.k;
  const uint32_t planes = static_cast<uint32_t>(b.z0 + BZ + R - b.zlo);
  const uint32_t bytes = planes * static_cast<uint32_t>(nx) * static_cast<uint32_t>(ny) * 4u;
  const size_t base = static_cast<size_t>(b.zlo) * nx * ny;
  const rsrc_t rU = make_rsrc(static_cast<const float *>(a.cur) + base, bytes);
  const rsrc_t rP = make_rsrc(static_cast<const float *>(a.prev) + base, bytes);
  const rsrc_t rO = make_rsrc(static_cast<float *>(a.out) + base, bytes);
  const rsrc_t rM = make_rsrc(a.m + base, bytes);
  for (int i = static_cast<int>(threadIdx.x); i < SX * SY * SZ; i += 64 * BY * BZ) {
    const int lx = i % SX, ly = (i / SX) % SY, lz = i / (SX * SY);
    const uint32_t off = node_off(b.x0 - R + lx, b.y0 - R + ly, b.z0 - R + lz, nx, ny, b.zlo);
    T[lz][ly][lx] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rU, static_cast<int>(off), 0, 0));
  }
  __syncthreads();
  const int tx = static_cast<int>(threadIdx.x) & 63, ty = (static_cast<int>(threadIdx.x) >> 6) % BY,
            tz = static_cast<int>(threadIdx.x) / (64 * BY);
  const int cx = tx + R, cy = ty + R, cz = tz + R;
  const float c = T[cz][cy][cx];
  float lap = 0.f;
#pragma unroll
  for (int m = 1; m <= R; ++m) {
    lap = fmaf(a.c.kx[m - 1], (T[cz][cy][cx + m] - c) + (T[cz][cy][cx - m] - c), lap);
    lap = fmaf(a.c.ky[m - 1], (T[cz][cy + m][cx] - c) + (T[cz][cy - m][cx] - c), lap);
    lap = fmaf(a.c.kz[m - 1], (T[cz + m][cy][cx] - c) + (T[cz - m][cy][cx] - c), lap);
  }
  const uint32_t own = node_off(b.x, b.y, b.z, nx, ny, b.zlo);
  const float pc = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rP, static_cast<int>(own), 0, kNT));
  const float mc = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rM, static_cast<int>(own), 0, kNT));
  const float gzv = b.inside ? a.gz[b.z] : 0.f;
  update_node(a, n, b.x, b.y, b.z, b.inside, c, lap, pc, mc, gzv, rO, own);
}


// ------------------------------------------------------------ two time steps per pass
//
// Temporal blocking (the multi-step blocking the paper cites among related
// work in Sec. II): one pass over the grid advances two time steps.  A
// workgroup of 8 wavefronts covers a 64 x 32 region E (a lane per column, 4
// rows per wavefront); it computes step n+1 on all of E and step n+2 on E's
// interior O (56 x 24: E less a ring of R = 4 nodes), R planes behind in z.
// The ring's step n+1 is also computed by the neighbouring workgroups: the
// price of keeping step n+2's stencil inside the workgroup.  Per plane z:
//   * step n+1 at plane z on E: A^n from a register queue (z) and a
//     double-buffered LDS plane (x and y, with E's halo), A^{n-1} and m
//     from the prefetch stage;
//   * A^{n+1}(z) enters a second register queue and a ring of R+1 LDS
//     planes (E only), and m(z) a third queue;
//   * step n+2 at plane z-R on O: A^{n+1} from that queue and ring, A^n at
//     plane z-R (the oldest slot of the first queue) as its previous level.
// Both steps perform step_kernel's operations in its order (the Laplacian
// as centred second differences), so a pass gives the bits of two single
// steps.  The two results go to two further buffers: writing in place would
// race with neighbouring workgroups that still read the ring's inputs.
// Float32 forward without CPML.  A z-chunk of output planes [zb, ze) runs
// step n+1 over [zb-R, ze+R): 2R extra planes per chunk.
constexpr int kTbBY = 8, kTbRY = 4;                        // E: 64 x 32
constexpr int kTbEX = kTileX, kTbEY = kTbBY * kTbRY;
constexpr int kTbOX = kTbEX - 2 * R, kTbOY = kTbEY - 2 * R;  // O: 56 x 24

__global__ void __launch_bounds__(64 * kTbBY) step2_kernel(StepArgs a) {
  constexpr int BY = kTbBY, RY = kTbRY, EX = kTbEX, EY = kTbEY;
  constexpr int LW = EX + 2 * R, LH = EY + 2 * R;
  constexpr int DUMMY = LH * LW;  // scratch row for halo lanes with nothing to write
  static_assert(2 * R <= BY && 8 * RY <= 64, "one y-halo row per wavefront, x halo in one load");
  __shared__ __attribute__((aligned(16))) float ldsA[2][LH * LW + 64];
  __shared__ __attribute__((aligned(16))) float ldsB[R + 1][EY * EX];

  const int nwg = static_cast<int>(gridDim.x);
  const int bid = static_cast<int>(blockIdx.x);
  const int logical = (bid & 7) * (nwg >> 3) + (bid >> 3);
  if (logical >= a.total_tiles) return;
  const int tix = logical % a.tiles_x;
  const int rest = logical / a.tiles_x;
  const int tiy = rest % a.tiles_y;
  const int chunk = rest / a.tiles_y;
  const int ex0 = tix * kTbOX - R, ey0 = tiy * kTbOY - R;  // corner of E
  const int zb = chunk * a.zchunk;
  const int zend = min(zb + a.zchunk, a.nz);  // output planes [zb, zend)
  const int z1b = zb - R;                      // step n+1 planes [z1b, z1e), whole trips of nine
  const int z1e = z1b + (zend - zb + 2 * R + kQ - 1) / kQ * kQ;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const uint32_t pbytes = static_cast<uint32_t>(nx) * static_cast<uint32_t>(ny) * 4u;
  const int n = a.st->n + a.k;  // this pass advances steps n and n+1

  // Resources over the planes [zlo, zhi) the pass touches, cut at the end of
  // the padded allocation (loads past it read zero); planes below zlo are
  // below the grid and read zero through rnull.
  const int zlo = max(z1b - R, 0);
  const int zhi = min(z1e + R + 1, nz + kPadZ);
  const uint32_t span = zhi > zlo ? static_cast<uint32_t>(zhi - zlo) * pbytes : 0u;
  const size_t base = static_cast<size_t>(zlo) * static_cast<size_t>(nx) * static_cast<size_t>(ny);
  const rsrc_t rU = make_rsrc(static_cast<const float *>(a.cur) + base, span);
  const rsrc_t rP = make_rsrc(static_cast<const float *>(a.prev) + base, span);
  const rsrc_t rM = make_rsrc(a.m + base, span);
  const rsrc_t rO = make_rsrc(static_cast<float *>(a.out) + base, span);
  const rsrc_t rO2 = make_rsrc(static_cast<float *>(a.out2) + base, span);
  const rsrc_t rnull = make_rsrc(a.gz, 0u);
  const rsrc_t rgz = make_rsrc(a.gz, static_cast<uint32_t>(nz + kPadZ) * 4u);
  const rsrc_t rrz = make_rsrc(a.rz, static_cast<uint32_t>(nz + kPadZ) * 4u);
  auto ld = [&](const rsrc_t &r, uint32_t voff, int z, int aux) {  // float of plane z (zero below zlo)
    const bool ok = z >= zlo;
    const rsrc_t rr = ok ? r : rnull;
    const uint32_t so = ok ? static_cast<uint32_t>(z - zlo) * pbytes : 0u;
    return aux ? __uint_as_float(ld_words<4, kNT>(rr, voff, so).w[0]) : __uint_as_float(ld_words<4, 0>(rr, voff, so).w[0]);
  };
  auto tab = [&](const rsrc_t &r, int z) {  // per-plane table entry (0 below the grid)
    return ld_words<4, 0>(z >= 0 ? r : rnull, 0u, z >= 0 ? static_cast<uint32_t>(z) * 4u : 0u).w[0];
  };

  // ---- this lane's column and rows
  const int ex = ex0 + lane;
  const bool xin = ex >= 0 && ex < nx;
  const float gxv = xin ? a.gx[ex] : 0.f;
  const bool ocol = lane >= R && lane < EX - R && xin;
  int rxi = -1;
  if (a.box.cnx > 0 && ocol) {
    const int d = ex - a.box.x0;
    if (d >= 0 && d % a.box.sx == 0 && d / a.box.sx < a.box.cnx) rxi = d / a.box.sx;
  }
  float gyv[RY], qrow[RY];
  int ryi[RY];
  bool orow[RY];
  uint32_t vrow[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const int er = w * RY + j, ey = ey0 + er;
    const bool yin = ey >= 0 && ey < ny;
    vrow[j] = (xin && yin) ? (static_cast<uint32_t>(ey) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(ex)) * 4u
                           : kOOB;
    gyv[j] = yin ? a.gy[ey] : 0.f;
    orow[j] = er >= R && er < EY - R && yin;
    ryi[j] = -1;
    if (a.box.cnx > 0 && yin) {
      const int d = ey - a.box.y0;
      if (d >= 0 && d % a.box.sy == 0 && d / a.box.sy < a.box.cny) ryi[j] = d / a.box.sy;
    }
    qrow[j] = (a.sx >= 0 && a.sx == ex && a.sy == ey) ? 1.f : 0.f;
  }
  // y halo of E: wavefront w loads halo row w (rows above E first)
  const int hr = w < R ? w : EY + w;
  const int hy = ey0 - R + hr;
  const int yhlds = hr * LW + R + lane;
  const uint32_t vyh =
      (xin && hy >= 0 && hy < ny) ? (static_cast<uint32_t>(hy) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(ex)) * 4u
                                  : kOOB;
  // x halo of E: lane l < 8 RY covers row l/8 of this wavefront, column l%8
  int xhlds = DUMMY + lane;
  uint32_t vxh = kOOB;
  if (lane < 8 * RY) {
    const int j = lane >> 3, c = lane & 7;
    const int gxx = c < R ? ex0 - R + c : ex0 + EX + (c - R);
    const int yj = ey0 + w * RY + j;
    xhlds = (R + w * RY + j) * LW + (c < R ? c : EX + c);
    if (gxx >= 0 && gxx < nx && yj >= 0 && yj < ny)
      vxh = (static_cast<uint32_t>(yj) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(gxx)) * 4u;
  }

  struct Stg {
    float lead[RY], p[RY], m[RY], yh, xh, gz1, gz2;
    int rz1, rz2;
  };
  auto load_stage = [&](Stg &st, int z) {  // plane z of step n+1 (and z-R of step n+2)
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      st.lead[j] = ld(rU, vrow[j], z + R, 0);
      st.p[j] = ld(rP, vrow[j], z, 1);
      st.m[j] = ld(rM, vrow[j], z, 1);
    }
    st.yh = ld(rU, vyh, z, 0);
    st.xh = ld(rU, vxh, z, 0);
    st.gz1 = __uint_as_float(tab(rgz, z));
    st.gz2 = __uint_as_float(tab(rgz, z - R));
    st.rz1 = static_cast<int>(tab(rrz, z));
    st.rz2 = static_cast<int>(tab(rrz, z - R));
  };

  // queues: qa slot (p - z1b + R) mod 9 holds A^n of plane p; qb and qm slot
  // (p - z1b) mod 9 hold A^{n+1} and m of plane p
  float qa[kQ][RY], qb[kQ][RY], qm[kQ][RY];
#pragma unroll
  for (int k = 0; k < kQ; ++k)
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      qb[k][j] = 0.f;
      qm[k][j] = 0.f;
      qa[k][j] = k < 2 * R ? ld(rU, vrow[j], z1b - R + k, 0) : 0.f;
    }
  Stg stg;
  load_stage(stg, z1b);
  const float wsrc1 = a.sx >= 0 ? a.wavelet[n] * a.src_scale : 0.f;
  const float wsrc2 = a.sx >= 0 ? a.wavelet[n + 1] * a.src_scale : 0.f;

  for (int zs = z1b; zs < z1e; zs += kQ) {
    static_for<kQ>([&](auto sc) __attribute__((always_inline)) {
      constexpr int s = decltype(sc)::value;
      const int z = zs + s;                 // step n+1 plane
      const int z2 = z - R;                 // step n+2 plane
      constexpr int ca = (s + R) % kQ;      // qa: plane z
      constexpr int cb = (s + kQ - R) % kQ; // qb, qm: plane z - R
      float *LA = ldsA[(z - z1b) & 1];
      float *LB = ldsB[(z - z1b) % (R + 1)];
      const float *LB2 = ldsB[(z2 - z1b + R + 1) % (R + 1)];
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        qa[(s + 2 * R) % kQ][j] = stg.lead[j];
        LA[(R + w * RY + j) * LW + R + lane] = qa[ca][j];
      }
      LA[yhlds] = stg.yh;
      LA[xhlds] = stg.xh;
      float pc[RY], mc[RY];
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        pc[j] = stg.p[j];
        mc[j] = stg.m[j];
      }
      const float gz1 = stg.gz1, gz2 = stg.gz2;
      const int rz1 = __builtin_amdgcn_readfirstlane(stg.rz1), rz2 = __builtin_amdgcn_readfirstlane(stg.rz2);
      load_stage(stg, z + 1);
      __syncthreads();

      // step n+1 at plane z on E
      float v1[RY];
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        const float *row = LA + (R + w * RY + j) * LW + R + lane;
        const float c = qa[ca][j];
        float lap = 0.f;
#pragma unroll
        for (int m = 1; m <= R; ++m) {
          const float yp = (j + m < RY) ? qa[ca][(j + m) % RY] : row[m * LW];
          const float ym = (j - m >= 0) ? qa[ca][(j - m + RY) % RY] : row[-m * LW];
          const float sx = (row[m] - c) + (row[-m] - c);
          const float sy = (yp - c) + (ym - c);
          const float sz = (qa[(s + R + m) % kQ][j] - c) + (qa[(s + R - m + kQ) % kQ][j] - c);
          lap = fmaf(a.c.kx[m - 1], sx, lap);
          lap = fmaf(a.c.ky[m - 1], sy, lap);
          lap = fmaf(a.c.kz[m - 1], sz, lap);
        }
        const float g = gxv * (gyv[j] * gz1);
        float t = fmaf(-g, pc[j], 2.f * c);
        t = fmaf(mc[j], lap, t);
        t = fmaf(qrow[j], z == a.sz ? wsrc1 : 0.f, t);
        v1[j] = t * g;
        qb[s][j] = v1[j];
        qm[s][j] = mc[j];
        LB[(w * RY + j) * EX + lane] = v1[j];
      }
      const bool out1 = z >= zb && z < zend;
      if (out1) {
#pragma unroll
        for (int j = 0; j < RY; ++j)
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v1[j]), rO,
                                                static_cast<int>((ocol && orow[j]) ? vrow[j] : kOOB),
                                                static_cast<int>(static_cast<uint32_t>(z - zlo) * pbytes), kNT);
        if (rz1 >= 0 && rxi >= 0) {
#pragma unroll
          for (int j = 0; j < RY; ++j)
            if (orow[j] && ryi[j] >= 0)
              a.traces[static_cast<size_t>(n) * a.nrec + (rz1 * a.box.cny + ryi[j]) * a.box.cnx + rxi] = v1[j];
        }
      }

      // step n+2 at plane z - R on O (the ring's threads compute at the
      // nearest O node and discard the result)
      const int lc = min(max(lane, R), EX - R - 1);
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        const int er = min(max(w * RY + j, R), EY - R - 1);
        const float *row = LB2 + er * EX + lc;
        const float c = qb[cb][j];
        float lap = 0.f;
#pragma unroll
        for (int m = 1; m <= R; ++m) {
          const float sx = (row[m] - c) + (row[-m] - c);
          const float sy = (row[m * EX] - c) + (row[-m * EX] - c);
          const float sz = (qb[(cb + m) % kQ][j] - c) + (qb[(cb - m + kQ) % kQ][j] - c);
          lap = fmaf(a.c.kx[m - 1], sx, lap);
          lap = fmaf(a.c.ky[m - 1], sy, lap);
          lap = fmaf(a.c.kz[m - 1], sz, lap);
        }
        const float g = gxv * (gyv[j] * gz2);
        float t = fmaf(-g, qa[s][j], 2.f * c);  // qa slot s: A^n of plane z - R
        t = fmaf(qm[cb][j], lap, t);
        t = fmaf(qrow[j], z2 == a.sz ? wsrc2 : 0.f, t);
        const float v2 = t * g;
        if (z2 >= zb && z2 < zend) {
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v2), rO2,
                                                static_cast<int>((ocol && orow[j]) ? vrow[j] : kOOB),
                                                static_cast<int>(static_cast<uint32_t>(z2 - zlo) * pbytes), kNT);
          if (rz2 >= 0 && rxi >= 0 && orow[j] && ryi[j] >= 0)
            a.traces[static_cast<size_t>(n + 1) * a.nrec + (rz2 * a.box.cny + ryi[j]) * a.box.cnx + rxi] = v2;
        }
      }
    });
  }
}

// Kernel variants (FAMILY, BY, RY, PD, VEC).  Family 0 is the 2.5D streaming
// step_kernel (tile 64*VEC x BY*RY, PD planes in flight).  Variant 0 asks the
// runtime for its automatic choice; its row is the shape that choice falls
// back to, which variant 18 requests explicitly.  Families 1 (gmem)
// and 2 (smem) are the 3D-blocked kernels with blocks of 64 x BY x RY nodes;
// family 3 is the 2.5D kernel with the semi-stencil z sum; family 4 the
// two-steps-per-pass kernel (step2_kernel; its shape is fixed).
#define WAVE_VARIANTS(X)  \
  X(0, 0, 8, 4, 3, 1)     \
  X(1, 0, 4, 8, 1, 1)     \
  X(2, 0, 4, 4, 3, 1)     \
  X(3, 0, 8, 2, 3, 1)     \
  X(4, 0, 4, 4, 1, 1)     \
  X(5, 0, 8, 4, 1, 1)     \
  X(6, 0, 2, 8, 1, 1)     \
  X(7, 0, 4, 2, 3, 1)     \
  X(8, 0, 8, 2, 3, 2)     \
  X(9, 0, 8, 2, 1, 4)     \
  X(10, 0, 4, 4, 1, 2)    \
  X(11, 0, 8, 4, 1, 2)    \
  X(12, 0, 8, 1, 3, 4)    \
  X(13, 0, 4, 2, 3, 2)    \
  X(14, 1, 4, 4, 1, 1)    \
  X(15, 2, 4, 4, 1, 1)    \
  X(16, 3, 8, 4, 3, 1)    \
  X(17, 3, 8, 1, 3, 4)    \
  X(18, 0, 8, 4, 3, 1)     \
  X(19, 4, 8, 4, 1, 1)

#define WAVE_VARIANT_INFO(id, fam, by, ry, pd, vec) {by, ry, pd, vec, fam},
constexpr Variant kVariants[] = {WAVE_VARIANTS(WAVE_VARIANT_INFO)};
#undef WAVE_VARIANT_INFO
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Shapes with the x part of the CPML boundary fused into the step: those
// whose fused kernel fits the register file without spilling (at most two
// rows per wavefront and four nodes per thread).
template <int RY, int VEC>
constexpr bool fuses_cpml() {
  return RY <= 2 && RY * VEC <= 4;
}

template <int S, int BY, int RY, int PD, int VEC, bool SEMI, bool ADJ, bool CP = false>
int blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void *>(step_kernel<S, BY, RY, PD, VEC, SEMI, ADJ, CP, false>), 64 * BY, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <int FAM, int S, int BY, int RY, int PD, int VEC, bool ADJ>
int blocks_fam(bool cpml) {
  if constexpr (FAM == 0 && S == kF32 && !ADJ && fuses_cpml<RY, VEC>())
    if (cpml) return blocks_per_cu<S, BY, RY, PD, VEC, false, false, true>();
  if constexpr (FAM == 0) return blocks_per_cu<S, BY, RY, PD, VEC, false, ADJ>();
  if constexpr (FAM == 3 && S == kF32 && !ADJ) return blocks_per_cu<S, BY, RY, PD, VEC, true, false, false>();
  return 1;  // the 3D-blocked kernels size their grids from the block shape alone
}

template <int S, bool ADJ>
int blocks_variant(int v, bool cpml) {
  switch (v) {
#define WAVE_VARIANT_CASE(id, fam, by, ry, pd, vec) \
  case id: return blocks_fam<fam, S, by, ry, pd, vec, ADJ>(cpml);
    WAVE_VARIANTS(WAVE_VARIANT_CASE)
#undef WAVE_VARIANT_CASE
    default: return 1;
  }
}

template <int FAM, int S, int BY, int RY, int PD, int VEC, bool ADJ, bool M16 = false>
hipError_t launch_one(const StepArgs &a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>((a.total_tiles + 7) / 8 * 8);
  if constexpr (M16) {  // 16-bit storage forward with 16-bit model codes
    if constexpr (FAM != 0 || S == kF32 || ADJ) {
      return hipErrorInvalidValue;
    } else {
      if (a.keep)
        hipLaunchKernelGGL((step_kernel<S, BY, RY, PD, VEC, false, false, false, true, true>), dim3(grid),
                           dim3(64 * BY), 0, s, a);
      else
        hipLaunchKernelGGL((step_kernel<S, BY, RY, PD, VEC, false, false, false, false, true>), dim3(grid),
                           dim3(64 * BY), 0, s, a);
      return hipGetLastError();
    }
  } else if constexpr (FAM == 0) {
    if constexpr (S == kF32 && !ADJ && fuses_cpml<RY, VEC>()) {
      if (a.cpml) {
        if (a.zchunk % kQ) return hipErrorInvalidValue;  // whole trips only (no skip branch)
        hipLaunchKernelGGL((step_kernel<S, BY, RY, PD, VEC, false, false, true, false>), dim3(grid), dim3(64 * BY),
                           0, s, a);
        return hipGetLastError();
      }
    }
    if constexpr (!ADJ) {
      if (a.keep) {
        hipLaunchKernelGGL((step_kernel<S, BY, RY, PD, VEC, false, false, false, true>), dim3(grid), dim3(64 * BY),
                           0, s, a);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((step_kernel<S, BY, RY, PD, VEC, false, ADJ, false, false>), dim3(grid), dim3(64 * BY), 0, s,
                       a);
  } else if constexpr (S != kF32 || ADJ) {
    return hipErrorInvalidValue;  // the study families are float32 forward only
  } else if constexpr (FAM == 4) {
    hipLaunchKernelGGL(step2_kernel, dim3(grid), dim3(64 * kTbBY), 0, s, a);
  } else if constexpr (FAM == 3) {
    hipLaunchKernelGGL((step_kernel<S, BY, RY, PD, VEC, true, false, false, false>), dim3(grid), dim3(64 * BY), 0, s,
                       a);
  } else if constexpr (FAM == 1) {
    hipLaunchKernelGGL((gmem_kernel<BY, RY>), dim3(grid), dim3(64 * BY * RY), 0, s, a);
  } else {
    hipLaunchKernelGGL((smem_kernel<BY, RY>), dim3(grid), dim3(64 * BY * RY), 0, s, a);
  }
  return hipGetLastError();
}

template <int S, bool ADJ, bool M16 = false>
hipError_t launch_variant(int v, const StepArgs &a, hipStream_t s) {
  switch (v) {
#define WAVE_VARIANT_CASE(id, fam, by, ry, pd, vec) \
  case id: return launch_one<fam, S, by, ry, pd, vec, ADJ, M16>(a, s);
    WAVE_VARIANTS(WAVE_VARIANT_CASE)
#undef WAVE_VARIANT_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// The per-storage instantiations, each in a translation unit of its own:
// launch a step variant, and how many of its workgroups fit on one CU.
hipError_t launch_variant_f32(int v, const StepArgs &a, hipStream_t s);
hipError_t launch_variant_f16(int v, const StepArgs &a, hipStream_t s);
hipError_t launch_variant_bf16(int v, const StepArgs &a, hipStream_t s);
hipError_t launch_variant_adj(int v, const StepArgs &a, hipStream_t s);
hipError_t launch_variant_f16m(int v, const StepArgs &a, hipStream_t s);   // 16-bit model codes
hipError_t launch_variant_bf16m(int v, const StepArgs &a, hipStream_t s);
int blocks_variant_f32(int v, bool cpml);
int blocks_variant_f16(int v);
int blocks_variant_bf16(int v);

}  // namespace wave
