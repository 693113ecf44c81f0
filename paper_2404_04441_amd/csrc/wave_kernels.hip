// gfx950 kernels of libwave.
//
// The fused step evaluates the 25-point, 8th-order star Laplacian of Eq. 1
// (paper Sec. II) at every node and applies the leapfrog update with sponge,
// source and receivers in the same pass.  Blocking follows the 2.5D idea of
// paper Sec. IV-A (tile x and y, stream along z) redesigned for CDNA4:
//
//  * a workgroup owns a 64 x TY column of the grid (TY = BY*RY rows) over a
//    z-chunk; each 64-lane wavefront owns RY consecutive rows, so every global
//    access of the interior is a fully coalesced 256-byte row whose address
//    is wavefront-uniform (scalar row base + one shared lane offset);
//  * the centre xy plane (with its radius-4 x/y halo) is staged in LDS, double
//    buffered so one barrier per plane suffices; y neighbours inside a
//    wavefront's own rows come from registers instead;
//  * the 9 values each thread needs along z live in a register queue that
//    shifts by one plane per iteration; A^n is read from HBM once per chunk;
//  * loads run PD planes ahead of the plane being computed (a register
//    pipeline), so enough bytes are in flight to cover HBM latency;
//  * A^{n-1}, m and A^{n+1} are touched exactly once: they use nontemporal
//    loads/stores so that L2 keeps the A^n planes the neighbours' halos need;
//  * workgroup ids are remapped so that each XCD (hardware dispatches ids
//    round-robin over the 8 XCDs) owns a contiguous run of tiles, keeping
//    y-halo re-reads inside one XCD's L2.
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

// ---- buffer access: a per-plane resource (scalar base), a scalar byte offset
// for the row and one 32-bit lane offset; every address used is inside the
// array (rows, planes and columns are clamped), ghost values are selected
// to zero where they are consumed.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw (untyped) buffer, gfx9 family
constexpr int kNT = 2;                  // nontemporal cache policy bit

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), static_cast<short>(0),
                                           static_cast<int>(bytes), kRsrcWord3);
}

template <typename T> struct Buf;
template <> struct Buf<float> {
  template <int AUX> __device__ static float ld(rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(vo),
                                                                          static_cast<int>(so), AUX));
  }
  template <int AUX> __device__ static void st(float v, rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, static_cast<int>(vo),
                                          static_cast<int>(so), AUX);
  }
};
template <> struct Buf<uint16_t> {
  template <int AUX> __device__ static uint16_t ld(rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, static_cast<int>(vo), static_cast<int>(so), AUX);
  }
  template <int AUX> __device__ static void st(uint16_t v, rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, static_cast<int>(vo), static_cast<int>(so), AUX);
  }
};

// Registers one thread holds for one z-plane of the pipeline: raw loaded
// values, so that nothing waits on a load until the plane is consumed.  Every
// vector-memory load of the z loop lives here: s_waitcnt vmcnt retires loads
// in issue order, so a load consumed in the same iteration would also wait for
// every prefetch issued before it.
template <typename raw, int RY, int NYH, bool ADJ>
struct Stage {
  raw lead[RY];                 // A^n at plane z+R (enters the z queue)
  raw p[RY];                    // A^{n-1} at plane z
  float m[RY];                  // m at plane z
  raw yh[NYH];                  // y-halo rows of A^n at plane z owned by this wavefront
  raw xh;                       // x-halo value of A^n at plane z (lanes < 8*RY)
  float gz;                     // sponge factor of plane z
  float leadF[ADJ ? RY : 1];    // adjoint: forward field, same roles
  float res[ADJ ? RY : 1];      // adjoint: residual injected at receivers of plane z
  float yhF[ADJ ? NYH : 1];
  float xhF;
  float img[ADJ ? RY : 1];      // adjoint: imaging accumulator at plane z
};

constexpr int kQ = 2 * R + 1;  // z-queue length (planes z-4 .. z+4)

// BY wavefronts per workgroup, RY consecutive rows per wavefront (tile 64 x
// BY*RY), PD planes of loads in flight ahead of the plane being computed
// (PD divides 9: the z loop is unrolled 9 times so the queue rotates by
// register renaming instead of copies).
template <int S, int BY, int RY, int PD, bool ADJ>
__global__ void __launch_bounds__(64 * BY) step_kernel(StepArgs a) {
  using C = Codec<S>;
  using raw = typename C::raw;
  using B = Buf<raw>;
  constexpr int TY = BY * RY;
  constexpr int LW = kTileX + 2 * R;
  constexpr int LH = TY + 2 * R;
  constexpr int NYH = (2 * R + BY - 1) / BY;
  constexpr uint32_t ES = sizeof(raw);
  static_assert(8 * RY <= 64, "x-halo of a wavefront's rows must fit in one load");
  static_assert(kQ % PD == 0, "pipeline depth must divide the queue length");
  // each LDS plane ends with a 64-float scratch row: halo writes of lanes or
  // wavefronts with nothing to write go there, so no write is predicated
  constexpr int LP = LH * LW + 64;
  constexpr int DUMMY = LH * LW;
  __shared__ float lds[2][LP];
  __shared__ float ldsF[ADJ ? 2 : 1][ADJ ? LP : 1];
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
  const int x0 = tix * kTileX, y0 = tiy * TY;
  const int zb = chunk * a.zchunk;
  const int ze = min(zb + a.zchunk, a.nz);
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t plane = static_cast<size_t>(nx) * static_cast<size_t>(ny);
  const uint32_t pbytes = static_cast<uint32_t>(plane) * ES;
  const uint32_t pbytes_f = static_cast<uint32_t>(plane) * 4u;
  const int x = x0 + lane;
  const bool xin = x < nx;
  const int yb = y0 + w * RY;  // first row of this wavefront

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

  // ---- per-row data (wavefront-uniform) and per-lane data
  bool rowin[RY], ok[RY];
  float gyv[RY];
  int ryi[RY];
  uint32_t rowo[RY], rowo_f[RY];  // byte offset of the (clamped) row in a plane
  const uint32_t xl = static_cast<uint32_t>(min(x, nx - 1));
  const float gxv = xin ? a.gx[x] : 0.f;
  int rxi = -1;
  if (a.box.cnx > 0 && xin) {
    const int d = x - a.box.x0;
    if (d >= 0 && d % a.box.sx == 0 && d / a.box.sx < a.box.cnx) rxi = d / a.box.sx;
  }
  int srcj = -1;
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    const int yj = yb + j;
    rowin[j] = yj < ny;
    ok[j] = rowin[j] && xin;
    rowo[j] = static_cast<uint32_t>(min(yj, ny - 1)) * static_cast<uint32_t>(nx) * ES;
    rowo_f[j] = static_cast<uint32_t>(min(yj, ny - 1)) * static_cast<uint32_t>(nx) * 4u;
    gyv[j] = rowin[j] ? a.gy[yj] : 0.f;
    ryi[j] = -1;
    if (a.box.cnx > 0 && rowin[j]) {
      const int d = yj - a.box.y0;
      if (d >= 0 && d % a.box.sy == 0 && d / a.box.sy < a.box.cny) ryi[j] = d / a.box.sy;
    }
    if (!ADJ && a.sx >= 0 && x == a.sx && yj == a.sy) srcj = j;
  }
  const uint32_t vo = xl * ES, vo_f = xl * 4u;  // lane byte offsets
  // y-halo rows of this wavefront: halo row r = w + BY*i (r < R above the tile, else below)
  bool yhin[NYH], yhok[NYH];
  int yhlds[NYH];
  uint32_t yho[NYH], yho_f[NYH];
#pragma unroll
  for (int i = 0; i < NYH; ++i) {
    const int r = w + BY * i;
    yhin[i] = r < 2 * R;
    const int lr = r < R ? r : TY + r;
    const int gyy = y0 - R + lr;
    yhok[i] = yhin[i] && gyy >= 0 && gyy < ny && xin;
    yhlds[i] = yhin[i] ? lr * LW + R : DUMMY;
    const uint32_t row = static_cast<uint32_t>(min(max(gyy, 0), ny - 1)) * static_cast<uint32_t>(nx);
    yho[i] = row * ES;
    yho_f[i] = row * 4u;
  }
  // x-halo: lane l < 8*RY covers row l/8 of this wavefront, column l%8
  int xhlds = DUMMY + lane;
  bool xhok = false;
  uint32_t xho = 0, xho_f = 0;
  if (lane < 8 * RY) {
    const int j = lane >> 3, c = lane & 7;
    const int gxx = c < R ? x0 - R + c : x0 + kTileX + (c - R);
    const int yj = yb + j;
    xhlds = (R + w * RY + j) * LW + (c < R ? c : kTileX + c);
    xhok = gxx >= 0 && gxx < nx && yj < ny;
    const uint32_t e = static_cast<uint32_t>(min(yj, ny - 1)) * static_cast<uint32_t>(nx) +
                       static_cast<uint32_t>(min(max(gxx, 0), nx - 1));
    xho = e * ES;
    xho_f = e * 4u;
  }

  const raw *U = static_cast<const raw *>(a.cur);
  const raw *P = static_cast<const raw *>(a.prev);
  raw *O = static_cast<raw *>(a.out);

  auto rec_plane = [&](int z) {  // receiver-box index of plane z, or -1
    int rzi = -1;
    if (a.box.cnx > 0) {
      const int d = z - a.box.z0;
      if (d >= 0 && d % a.box.sz == 0 && d / a.box.sz < a.box.cnz) rzi = d / a.box.sz;
    }
    return rzi;
  };
  const rsrc_t rgz = make_rsrc(a.gz, static_cast<uint32_t>(nz) * 4u);
  // residual row of this launch (adjoint); the resource covers exactly that
  // row.  Its loads are unconditional, so without receivers it points at the
  // (always valid) z table instead.
  const bool has_res = ADJ && a.resid != nullptr && a.nrec > 0;
  const rsrc_t rres = has_res ? make_rsrc(a.resid + static_cast<size_t>(a.resid_row) * a.nrec,
                                          static_cast<uint32_t>(a.nrec) * 4u)
                              : make_rsrc(a.gz, 4u);

  using StageT = Stage<raw, RY, NYH, ADJ>;
  auto load_stage = [&](StageT &st, int z) {
    const size_t zc = static_cast<size_t>(z) * plane;
    const size_t zl = static_cast<size_t>(min(z + R, nz - 1)) * plane;
    st.gz = Buf<float>::ld<0>(rgz, 0u, static_cast<uint32_t>(z) * 4u);
    const rsrc_t rl = make_rsrc(U + zl, pbytes);
    const rsrc_t rc = make_rsrc(U + zc, pbytes);
    const rsrc_t rp = make_rsrc(P + zc, pbytes);
    const rsrc_t rm = make_rsrc(a.m + zc, pbytes_f);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      st.lead[j] = B::template ld<0>(rl, vo, rowo[j]);
      st.p[j] = B::template ld<kNT>(rp, vo, rowo[j]);
      st.m[j] = Buf<float>::ld<kNT>(rm, vo_f, rowo_f[j]);
    }
#pragma unroll
    for (int i = 0; i < NYH; ++i) st.yh[i] = B::template ld<0>(rc, vo, yho[i]);
    st.xh = B::template ld<0>(rc, xho, 0);
    if (ADJ) {
      const rsrc_t fl = make_rsrc(a.fwd + zl, pbytes_f);
      const rsrc_t fc = make_rsrc(a.fwd + zc, pbytes_f);
      const rsrc_t ri = make_rsrc(a.img + zc, pbytes_f);
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        st.leadF[j] = Buf<float>::ld<0>(fl, vo_f, rowo_f[j]);
        st.img[j] = Buf<float>::ld<kNT>(ri, vo_f, rowo_f[j]);
      }
#pragma unroll
      for (int i = 0; i < NYH; ++i) st.yhF[i] = Buf<float>::ld<0>(fc, vo_f, yho_f[i]);
      st.xhF = Buf<float>::ld<0>(fc, xho_f, 0);
      const int rzi = rec_plane(z);
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        const bool at = rzi >= 0 && ryi[j] >= 0 && rxi >= 0;
        const uint32_t ridx = at ? static_cast<uint32_t>((rzi * a.box.cny + ryi[j]) * a.box.cnx + rxi) : 0u;
        st.res[j] = Buf<float>::ld<0>(rres, ridx * 4u, 0u);
      }
    }
  };

  // ---- prologue: queue slot (p - zb + R) mod 9 holds plane p; stages hold planes zb .. zb+PD-1
  float q[kQ][RY];
  float qF[ADJ ? kQ : 1][RY];
#pragma unroll
  for (int i = 0; i < 2 * R; ++i) {
    const int zz = zb - R + i;
    const bool zok = zz >= 0 && zz < nz;
    const rsrc_t r = make_rsrc(U + static_cast<size_t>(min(max(zz, 0), nz - 1)) * plane, pbytes);
    const rsrc_t rf = make_rsrc(a.fwd + static_cast<size_t>(min(max(zz, 0), nz - 1)) * plane, pbytes_f);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const float u = C::dec(B::template ld<0>(r, vo, rowo[j])) * inv_cur;
      q[i][j] = (zok && ok[j]) ? u : 0.f;
      if (ADJ) {
        const float f = Buf<float>::ld<0>(rf, vo_f, rowo_f[j]);
        qF[i][j] = (zok && ok[j]) ? f : 0.f;
      }
    }
  }
  StageT stg[PD];
#pragma unroll
  for (int s = 0; s < PD; ++s)
    if (zb + s < ze) load_stage(stg[s], zb + s);

  const float wsrc = (!ADJ && a.sx >= 0) ? a.wavelet[n] * a.src_scale : 0.f;
  float amax_loc = 0.f, amaxv_loc = 0.f;

  for (int zs = zb; zs < ze; zs += kQ) {
    // nine planes per trip with compile-time queue slots and stage indices, so
    // the queue rotates by register renaming (a runtime index would move the
    // queue into scratch memory)
    // Positions past the chunk end (only in a trip that straddles it) run on
    // clamped in-bounds planes with their stores switched off: no position is
    // skipped, so no control-flow join makes the compiler drain the loads.
    static_for<kQ>([&](auto sc) __attribute__((always_inline)) {
      constexpr int s = decltype(sc)::value;
      const int z = min(zs + s, ze - 1);
      const bool live = zs + s < ze;
      const int cslot = (s + R) % kQ;          // plane z
      StageT &cs = stg[s % PD];
      // buffer parity follows the unclamped position: consecutive positions
      // must alternate even when the plane index is clamped
      const int par = (zs + s - zb) & 1;
      float *L = lds[par];
      float *LF = ldsF[ADJ ? par : 0];
      const bool lok = z + R < nz;
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        q[(s + 2 * R) % kQ][j] = (ok[j] && lok) ? C::dec(cs.lead[j]) * inv_cur : 0.f;
        L[(R + w * RY + j) * LW + R + lane] = q[cslot][j];
        if (ADJ) {
          qF[(s + 2 * R) % kQ][j] = (ok[j] && lok) ? cs.leadF[j] : 0.f;
          LF[(R + w * RY + j) * LW + R + lane] = qF[cslot][j];
        }
      }
#pragma unroll
      for (int i = 0; i < NYH; ++i) {
        L[yhlds[i] + lane] = yhok[i] ? C::dec(cs.yh[i]) * inv_cur : 0.f;
        if (ADJ) LF[yhlds[i] + lane] = yhok[i] ? cs.yhF[i] : 0.f;
      }
      L[xhlds] = xhok ? C::dec(cs.xh) * inv_cur : 0.f;
      if (ADJ) LF[xhlds] = xhok ? cs.xhF : 0.f;
      float pc[RY], mc[RY], ic[RY], rc[RY];
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        pc[j] = C::dec(cs.p[j]) * inv_prev;
        mc[j] = cs.m[j];
        ic[j] = ADJ ? cs.img[j] : 0.f;
        rc[j] = ADJ ? cs.res[j] : 0.f;
      }
      const float gzv = cs.gz;
      load_stage(cs, min(z + PD, ze - 1));  // past the chunk end: a repeat of the last plane, unused
      __syncthreads();

      const size_t zc = static_cast<size_t>(z) * plane;
      const rsrc_t ro = make_rsrc(O + zc, pbytes);
      const rsrc_t rvo = make_rsrc((S != kF32 ? static_cast<raw *>(a.vout) : O) + zc, pbytes);
      const int rzi = rec_plane(z);
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        const float *row = L + (R + w * RY + j) * LW + R + lane;
        const float c = q[cslot][j];
        float lap = a.c.k0 * c;
#pragma unroll
        for (int m = 1; m <= R; ++m) {
          // y neighbours come from this thread's own rows when they lie in the strip
          const float yp = (j + m < RY) ? q[cslot][(j + m) % RY] : row[m * LW];
          const float ym = (j - m >= 0) ? q[cslot][(j - m + RY) % RY] : row[-m * LW];
          lap = fmaf(a.c.kx[m - 1], row[m] + row[-m], lap);
          lap = fmaf(a.c.ky[m - 1], yp + ym, lap);
          lap = fmaf(a.c.kz[m - 1], q[(s + R + m) % kQ][j] + q[(s + R - m + kQ) % kQ][j], lap);
        }
        const bool at_rec = rzi >= 0 && ryi[j] >= 0 && rxi >= 0;
        const int ridx = at_rec ? (rzi * a.box.cny + ryi[j]) * a.box.cnx + rxi : 0;
        if (ADJ && at_rec) lap += rc[j];
        const float g = gxv * (gyv[j] * gzv);
        float v, vv = 0.f;
        if (S == kF32) {  // A^{n+1} = g (2 A^n - g A^{n-1} + m L A^n + q)
          v = fmaf(-g, pc[j], 2.f * c);
          v = fmaf(mc[j], lap, v);
          if (!ADJ && srcj == j && z == a.sz) v += wsrc;
          v *= g;
        } else {  // V^{n+1} = g (V^n + m L A^n + q),  A^{n+1} = g A^n + V^{n+1}
          vv = fmaf(mc[j], lap, pc[j]);
          if (srcj == j && z == a.sz) vv += wsrc;
          vv *= g;
          v = fmaf(g, c, vv);
        }
        if (ok[j] && live) {
          const raw r = C::enc(v * s_next);
          B::template st<kNT>(r, ro, vo, rowo[j]);
          const float stored = C::dec(r);
          if (S != kF32) {
            const raw rv = C::enc(vv * sv_next);
            B::template st<kNT>(rv, rvo, vo, rowo[j]);
            amax_loc = fmaxf(amax_loc, fabsf(stored));
            amaxv_loc = fmaxf(amaxv_loc, fabsf(C::dec(rv)));
          }
          if (!ADJ && at_rec) a.traces[static_cast<size_t>(n) * a.nrec + ridx] = stored * inv_next;
          if (ADJ) {
            const float *rowF = LF + (R + w * RY + j) * LW + R + lane;
            const float cF = qF[cslot][j];
            float lapF = a.c.k0 * cF;
#pragma unroll
            for (int m = 1; m <= R; ++m) {
              const float yp = (j + m < RY) ? qF[cslot][(j + m) % RY] : rowF[m * LW];
              const float ym = (j - m >= 0) ? qF[cslot][(j - m + RY) % RY] : rowF[-m * LW];
              lapF = fmaf(a.c.kx[m - 1], rowF[m] + rowF[-m], lapF);
              lapF = fmaf(a.c.ky[m - 1], yp + ym, lapF);
              lapF = fmaf(a.c.kz[m - 1], qF[(s + R + m) % kQ][j] + qF[(s + R - m + kQ) % kQ][j], lapF);
            }
            const rsrc_t ri = make_rsrc(a.img + zc, pbytes_f);
            Buf<float>::st<kNT>(fmaf(c, lapF, ic[j]), ri, vo_f, rowo_f[j]);
          }
        }
      }
    });
  }

  if (S != kF32) {  // one order-independent atomic per workgroup and field
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
    const float g = gx[x] * (gy[y] * gz[z]);
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

// (BY, RY, PD) per variant
constexpr Variant kVariants[] = {{8, 4, 3}, {4, 8, 1}, {4, 4, 3}, {8, 2, 3},
                                 {4, 4, 1}, {8, 4, 1}, {2, 8, 1}, {4, 2, 3}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int S, int BY, int RY, int PD, bool ADJ>
int blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(step_kernel<S, BY, RY, PD, ADJ>),
                                                   64 * BY, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <int S, bool ADJ>
int blocks_variant(int v) {
  switch (v) {
    case 0: return blocks_per_cu<S, 8, 4, 3, ADJ>();
    case 1: return blocks_per_cu<S, 4, 8, 1, ADJ>();
    case 2: return blocks_per_cu<S, 4, 4, 3, ADJ>();
    case 3: return blocks_per_cu<S, 8, 2, 3, ADJ>();
    case 4: return blocks_per_cu<S, 4, 4, 1, ADJ>();
    case 5: return blocks_per_cu<S, 8, 4, 1, ADJ>();
    case 6: return blocks_per_cu<S, 2, 8, 1, ADJ>();
    case 7: return blocks_per_cu<S, 4, 2, 3, ADJ>();
    default: return 1;
  }
}

template <int S, int BY, int RY, int PD, bool ADJ>
hipError_t launch_one(const StepArgs &a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>((a.total_tiles + 7) / 8 * 8);
  hipLaunchKernelGGL((step_kernel<S, BY, RY, PD, ADJ>), dim3(grid), dim3(64 * BY), 0, s, a);
  return hipGetLastError();
}

template <int S, bool ADJ>
hipError_t launch_variant(int v, const StepArgs &a, hipStream_t s) {
  switch (v) {
    case 0: return launch_one<S, 8, 4, 3, ADJ>(a, s);
    case 1: return launch_one<S, 4, 8, 1, ADJ>(a, s);
    case 2: return launch_one<S, 4, 4, 3, ADJ>(a, s);
    case 3: return launch_one<S, 8, 2, 3, ADJ>(a, s);
    case 4: return launch_one<S, 4, 4, 1, ADJ>(a, s);
    case 5: return launch_one<S, 8, 4, 1, ADJ>(a, s);
    case 6: return launch_one<S, 2, 8, 1, ADJ>(a, s);
    case 7: return launch_one<S, 4, 2, 3, ADJ>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int variant_count() { return kNumVariants; }

int step_blocks_per_cu(int storage, int variant) {
  if (variant < 0 || variant >= kNumVariants) return 1;
  switch (storage) {
    case kF32: return blocks_variant<kF32, false>(variant);
    case kF16: return blocks_variant<kF16, false>(variant);
    case kBF16: return blocks_variant<kBF16, false>(variant);
    default: return 1;
  }
}

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
