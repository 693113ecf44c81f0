// Internal interface between the C-ABI runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "wave.h"

namespace wave {

constexpr int kRadius = 4;   // stencil half-width (8th order)
constexpr int kTileX = 64;   // tile width in x: one wavefront row
constexpr int kMaxPD = 3;    // most z-planes of loads a step kernel keeps in flight
// Zero planes after the nz interior planes of every field the step kernel
// reads or writes: the last z-chunk's final nine-plane trip, its prefetches
// and its z halo run into them instead of past the allocation.
constexpr int kPadZ = 2 * kRadius + kMaxPD + kRadius;

// Device-resident per-run state, at the head of the workspace.
struct StepState {
  int32_t n;            // absolute index of the next step (advanced by bump kernels)
  int32_t pad0[3];
  uint32_t amax[4];     // 16-bit storage, slot k%4: max |stored raw value| of A^k (float bits)
  int32_t exps[4];      // slot k%4: scale exponent of A^k (stored = A * 2^e)
  uint32_t flags;       // WAVE_FLAG_* bits
  uint32_t vmin_bits;   // velocity range from the create pass (float bits)
  uint32_t vmax_bits;
  uint32_t amax_v[4];   // the same two records for V^k = A^k - g A^{k-1}
  int32_t exps_v[4];
  uint32_t pad1[9];
};
static_assert(sizeof(StepState) == 128, "state block layout");

// Weights of the Laplacian of Eq. 1.  The kernels evaluate it as second
// differences from the centre, sum_a sum_m k_am ((u(+m) - u) + (u(-m) - u)):
// with c0 = -2 sum_m c_m this is the same operator, but no large centre term
// is summed against its neighbours (in float32 that cancellation dominated
// the rounding error of a long run; see the tolerance notes in the tests).
// Some terms sum the operator from its centre weight instead (Eq. 1 as
// written): the step with the CPML x terms fused in, per axis from k0a; the
// f16 step with 16-bit m and the adjoint step's imaging term L(A^k), from k0
// (see step_kernel).
struct Coef {
  float kx[4];     // c_m / dx^2, m = 1..4
  float ky[4];
  float kz[4];
  float k0a[3];    // c0 / h_a^2 per axis: the fused CPML step sums each axis' second derivative
                   // from its centre term (see step_kernel)
  float k0;        // c0 (1/dx^2 + 1/dy^2 + 1/dz^2): the centre weight of the whole operator
};

// Receivers forming a regular box, listed x fastest then y then z:
// receiver (i, j, l) is node (x0 + i*sx, y0 + j*sy, z0 + l*sz), index
// (l*cny + j)*cnx + i.  cnx == 0 means the fused path is off.
struct RecBox {
  int x0, sx, cnx;
  int y0, sy, cny;
  int z0, sz, cnz;
};

enum Storage { kF32 = 0, kF16 = 1, kBF16 = 2 };

// CPML boundary (float32 forward): memory variables psi_a, zeta_a in slab
// arrays over the W-node layers of each axis -- x: [nz][ny][2W], y:
// [nz][2W][nx], z: [2W][ny][nx]; slab index s = i for i < W and
// i - (n - 2W) for i >= n - W.
struct CpmlArgs {
  float *psi[3], *zeta[3];   // x, y, z
  const float *ca[3];        // a coefficient per node along each axis (n_a entries)
  const float *cb[3];        // b coefficient
  float d1w[3][4];           // w_m / h_a (first derivative)
  float d2w[3][5];           // c_m / h_a^2 (second derivative; [0] = c_0 / h_a^2 is implied by the
                             // centred second differences and not read)
  int W;                     // layer width in nodes (2W <= every axis)
  int nx, ny, nz;
};

// Float32 storage keeps (A^n, A^{n-1}) and writes A^{n+1} over A^{n-1}.
// 16-bit storage keeps (A^n, V^n = A^n - g A^{n-1}): `prev` and `vout` both
// point at V (updated in place) and A^{n+1} goes to `out`.
struct StepArgs {
  const void *cur;    // A^n (storage type)
  const void *prev;   // A^{n-1} (float32) or V^n (16-bit)
  void *out;          // A^{n+1}; may alias prev (float32)
  void *out2;         // two-step pass: A^{n+2} (a fourth buffer)
  void *vout;         // 16-bit storage: V^{n+1} (same buffer as prev)
  const float *m;     // (v dt)^2
  const float *gx, *gy, *gz;
  const int *rz;       // per plane: receiver-box plane index, or -1
  int nx, ny, nz;
  int tiles_x, tiles_y, nchunks, zchunk, total_tiles;
  Coef c;
  int sx, sy, sz;     // source node; sx < 0: none
  float src_scale;    // dt^2 / (dx dy dz)
  const float *wavelet;
  RecBox box;
  float *traces;
  int nrec;
  StepState *st;
  int k;              // this launch advances step st->n + k
  float gamma;        // 16-bit storage: |m L A| <= gamma max|A| at every node
  // adjoint mode only
  const float *fwd;   // forward field A^k for the imaging term
  float *img;         // accumulator sum_k mu^{k+1} L(A^k)
  const float *resid; // [nt][nrec] residual, injected at receivers
  int resid_row;      // row of resid injected by this launch
  // CPML (float32 forward, 2.5D kernels): 1 = add the x part of the boundary
  // terms and update zeta_x inside the step (psi is updated by a pass before
  // it, the y and z parts by a pass after it)
  int cpml;
  CpmlArgs cp;
  // 1: the fields read or written once with the regular cache policy
  // (forward 2.5D, no CPML), for grids whose fields fit the last-level cache
  int keep;
  // 16-bit storage only: m holds 16-bit codes u, m = m_lo + u * m_step
  int m16;
  float m_lo, m_step;
};

struct Variant {
  int by;   // wavefronts per workgroup
  int ry;   // consecutive rows per wavefront (tile height = by * ry)
  int pd;   // z-planes of loads in flight ahead of the plane being computed
  int vec;  // consecutive x nodes per lane (tile width = 64 * vec); needs nx % vec == 0
  int family;  // 0: 2.5D streaming; 1: 3D blocks from global memory; 2: 3D blocks via LDS;
               // 3: 2.5D streaming with a semi-stencil z sum; 4: two time steps per
               // pass (families 1 and 2: blocks of 64 x by x ry nodes; families 1-4:
               // float32 forward only)
};

int variant_count();
Variant variant_info(int v);
// True for the float32 2.5D shapes whose step kernel has the CPML boundary fused in.
bool variant_fuses_cpml(int v);
// Workgroups of the forward step kernel that fit on one CU at once (cpml: the
// fused CPML kernel where the shape has one).
int step_blocks_per_cu(int storage, int variant, bool cpml);

// Launchers; each returns the hipError_t of the launch.
hipError_t launch_step(int storage, int variant, bool adjoint, const StepArgs &a, hipStream_t s);
// m = (v dt)^2 (skipped when m is null) and the velocity range / validity into st
hipError_t launch_init_m(const float *vel, float *m, size_t n, float dt, StepState *st, hipStream_t s);
// codes u = round(((v dt)^2 - m_lo) / m_step), clamped to [0, 65535] (0 when m_step == 0)
hipError_t launch_encode_m16(const float *vel, uint16_t *codes, size_t n, float dt, float m_lo, float m_step,
                             hipStream_t s);
hipError_t launch_bump(StepState *st, int count, hipStream_t s);
// 16-bit storage: encode float32 x into a stored field of step n (dst; the
// V field with v_field) at the exponent the bound rule gives for max |x|,
// and set that field's exponent and stored-maximum records for step n
hipError_t launch_encode_field(int storage, const float *x, void *dst, size_t n, StepState *st, bool v_field,
                              hipStream_t s);
hipError_t launch_decode(int storage, const void *field, float *out, size_t n, const StepState *st,
                         int slot_from_n_offset, bool v_field, hipStream_t s);
hipError_t launch_decode_prev(int storage, const void *a, const void *v, float *out, const float *gx,
                              const float *gy, const float *gz, int nx, int ny, int nz, const StepState *st,
                              hipStream_t s);
hipError_t launch_gather(int storage, const void *field, const int64_t *rec_lin, int nrec, float *traces,
                         const StepState *st, int k, hipStream_t s);
// field[node[u]] += g_u m (sum of the residuals of node u's receivers, summed
// in receiver order): nodes u < nnode, their receivers ord[off[u] .. off[u+1])
hipError_t launch_scatter(float *field, const int64_t *node, const int32_t *off, const int32_t *ord, int nnode,
                          int nrec, const float *m, const float *gnode, const float *resid, int row, hipStream_t s);
hipError_t launch_reset_state(StepState *st, hipStream_t s);
hipError_t launch_set_n(StepState *st, int n, hipStream_t s);
hipError_t launch_check_finite(int storage, const void *field, size_t n, StepState *st, hipStream_t s);
hipError_t launch_grad_final(const float *img, const float *m, float dt, float *grad, size_t n,
                             hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
// psi_a^n = b psi_a^{n-1} + a D1_a cur, on the W-node layers
hipError_t launch_cpml_psi(const CpmlArgs &c, const float *cur, hipStream_t s);
// out += m * sum_a (D1_a psi_a + zeta_a), zeta_a = b zeta_a + a (D2_a cur + D1_a psi_a),
// on the nodes within W + R of a face; yz_only: axes y and z only, on the
// z-layer planes and y-layer rows of that shell (the x part is fused in the step)
hipError_t launch_cpml_fix(const CpmlArgs &c, const float *cur, const float *m, float *out, bool yz_only,
                           hipStream_t s);

// wave_create with the workspace in a device's static scratch array
// (scratch_bytes long): at most one such context per device at a time
// (WAVE_ESTATE otherwise); tuning off; graph_steps must be 0.  wave_destroy
// of that context synchronises its stream and frees the device's slot.
int create_static_ctx(const wave_params *p, const float *vel_dev, void *scratch, size_t scratch_bytes,
                      void *hip_stream, wave_t *out, int device);

}  // namespace wave
