/*
 * libwave -- 3D constant-density acoustic wave propagation on one gfx950 GPU.
 *
 * The operation (paper Sec. II, Eq. 1): the 25-point, 8th-order (radius 4)
 * star Laplacian L, evaluated at every grid node in each time step to advance
 * the wavefield.  The time integrator (not named in the paper) is the
 * 2nd-order leapfrog; an exponential sponge (Cerjan) damps the outer
 * `sponge_width` nodes; a point source injects a wavelet; receivers sample
 * the field.  One step, fused into one kernel pass over the grid:
 *
 *     A^{n+1} = g * (2 A^n - g * A^{n-1} + m * L(A^n) + q^n)
 *     m       = (v dt)^2,   g = gx(x) gy(y) gz(z),
 *     q^n     = dt^2 s(t_n) / (dx dy dz) at the source node, 0 elsewhere,
 *     trace[n][r] = A^{n+1}(rec_r)
 *
 * L(u) = sum_a h_a^-2 [c0 u + sum_{m=1..4} c_m (u(+m e_a) + u(-m e_a))] with
 * (c0..c4) = (-205/72, 8/5, -1/5, 8/315, -1/560); nodes outside the grid are
 * zero.  This form is algebraically equal to damping both stored time levels
 * each step; A^{n-1} is kept undamped in the buffer.
 *
 * Layout: every grid array is float32 (or the 16-bit storage type for the
 * wavefields inside the workspace), x fastest: index = x + nx*(y + ny*z).
 *
 * Ownership: every device byte is allocated by the caller (velocity, the
 * workspace, wavelet, traces, residual, gradient).  A context borrows its
 * workspace, which must outlive it.  wave_destroy frees host memory only.
 *
 * Asynchrony: calls enqueue work on the context's HIP stream and return
 * without waiting, except wave_create (reads back the velocity range) and
 * wave_sync_status.  Argument errors are detected before anything is
 * enqueued.  One host thread per context at a time; contexts on different
 * streams run concurrently.
 *
 * Errors: every call returns WAVE_OK (0) or a negative status.  No call
 * aborts, throws or prints.
 */
#ifndef LIBWAVE_WAVE_H
#define LIBWAVE_WAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wave_ctx *wave_t;

enum wave_status {
  WAVE_OK = 0,
  WAVE_EINVAL = -1,     /* bad argument: null pointer, size < 1, node outside the grid, bad enum */
  WAVE_EUNSTABLE = -2,  /* dt exceeds the leapfrog stability limit for max(v) */
  WAVE_ENOSPC = -3,     /* workspace smaller than wave_workspace_bytes() */
  WAVE_EHIP = -4,       /* a HIP runtime call or kernel launch failed */
  WAVE_ESTATE = -5      /* call not valid for this context (e.g. no adjoint workspace) */
};

/* Float32 storage keeps (A^n, A^{n-1}).  16-bit storage keeps A^n and
 * V^n = A^n - g A^{n-1} (so the step-to-step change is rounded relative to its
 * own size), each with its own power-of-two scale, updated as
 * V^{n+1} = g (V^n + m L(A^n) + q^n), A^{n+1} = g A^n + V^{n+1} in float32. */
enum wave_storage {
  WAVE_F32 = 0,   /* float32 wavefields */
  WAVE_F16 = 1,   /* IEEE half A and V with a power-of-two scale per field, float32 arithmetic */
  WAVE_BF16 = 2   /* bfloat16 A and V, same scaling, float32 arithmetic */
};

/* Flags reported by wave_sync_status. */
enum { WAVE_FLAG_NONFINITE = 1u };

typedef struct {
  int32_t nx, ny, nz;        /* grid nodes per axis, >= 1; nx*ny <= 2^24 */
  double dx, dy, dz;         /* grid spacing (m), > 0 */
  double dt;                 /* time step (s), > 0, at most the stability limit */
  int32_t sponge_width;      /* damping strip width in nodes; 0 = zero-Dirichlet only */
  double sponge_alpha;       /* strip factor: g = exp(-(alpha (W - d))^2) for distance d < W */
  int32_t storage;           /* enum wave_storage */
  int32_t src[3];            /* source node (ix, iy, iz); src[0] < 0: no source */
  int32_t nrec;              /* number of receivers, >= 0 */
  const int32_t *rec;        /* host array of 3*nrec node coordinates (ix, iy, iz), copied at create */
  int32_t adjoint;           /* nonzero: reserve the workspace wave_adjoint needs (float32 only) */
  int32_t nt_max;            /* adjoint: largest nt wave_adjoint will be called with */
  int32_t ckpt_interval;     /* adjoint: steps between checkpoints; 0 = ceil(sqrt(nt_max)) */
  int32_t variant;           /* kernel variant, 1 .. wave_variant_count()-1 (see wave_variant_info);
                                0 = automatic (the measured-best 2.5D shape for the storage type
                                and nx).  WAVE_EINVAL: 2 or 4 x nodes per lane with nx not divisible
                                by that; a 3D-blocked family with 16-bit storage or adjoint */
  int32_t zchunk;            /* z-planes per workgroup (any length; capped so a workgroup's buffers
                                span < 2 GiB); 0 = chosen from the grid size */
  int32_t graph_steps;       /* >0: replay steps from a captured HIP graph of this many steps */
  int32_t tune;              /* 1 (the default) with variant = 0 and zchunk = 0: wave_create
                                times candidate configurations for a few steps on the fresh
                                (zero) fields: the 2.5D shapes and z-chunks, both cache policies
                                (without CPML or adjoint), and for float32 forward runs without
                                CPML or adjoint also the 3D-blocked gmem and smem shapes.  It
                                keeps the fastest (the fixed rule's choice unless another is more
                                than 3% faster).  With adjoint != 0 it also times the adjoint
                                step's shapes and z-chunks on their own and keeps the fastest the
                                same way.  The choices are cached per (nx, ny, nz, storage, CPML,
                                adjoint, cache_hint, model_bits) for the life of the process.
                                Every choice computes the same bits; wave_tiling reports the
                                forward one.  0: the fixed automatic rule (measured: 30-50%
                                slower at some sizes) */
  int32_t cpml_width;        /* >0: CPML absorbing layers of this many nodes on all six faces (the
                                boundary of paper Sec. II / IV-A; float32, forward only, needs
                                sponge_width = 0, 2*cpml_width <= nx, ny, nz, nx*ny*nz < 2^31 and
                                each memory-variable array, 4 * 2*cpml_width * (largest of nx*ny,
                                ny*nz, nx*nz) bytes, < 2^31).  2.5D shapes with at most 2 rows per
                                wavefront and 4 nodes per lane (the automatic choice is one) apply
                                the x part of the boundary terms inside the step kernel; other
                                shapes apply all of it in a correction pass.  With tune = 1 only
                                the former are timed.  0: none */
  double cpml_reflection;    /* CPML target reflection coefficient R in (0, 1] (default 1e-3):
                                d(xi) = -3 v_max ln(R) xi^2 / (2 W h) */
  double cpml_f0;            /* CPML frequency shift alpha(xi) = pi f0 (1 - xi), Hz (default 0) */
  int32_t cache_hint;        /* cache policy of the fields the forward step reads or writes once
                                (float32: A^{n-1}, m, A^{n+1}; 16-bit: V^n, m, A^{n+1}, V^{n+1}):
                                0 = nontemporal, so that the cache keeps A^n's halo planes (with
                                tune = 1 the regular policy is timed too); 1 = regular, for grids
                                whose fields fit the 256 MB last-level cache.  1 needs no CPML
                                and a 2.5D variant.  Results are the same bits either way */
  int32_t model_bits;        /* storage of m = (v dt)^2 read by every forward step: 0 or 32 = float32;
                                16 = (16-bit wavefield storage only, WAVE_EINVAL otherwise) a 16-bit
                                code u of the affine map m = m_min + u (m_max - m_min) / 65535
                                between the grid's smallest and largest m, rounded to nearest: a
                                relative error in m of at most (m_max / m_min - 1) / 131070 (6.1e-5
                                for a 1500..4500 m/s model), and a step that moves 10 instead of 12
                                bytes per node (2 + 2 + 2 read, 2 + 2 written) */
  int32_t time_block;        /* 2: advance two time steps per pass over the grid (temporal blocking,
                                the multi-step blocking of paper Sec. II's related work): the pass
                                kernel (variant family 4) computes step n+1 on 64 x 32 tiles and
                                step n+2 on their 56 x 24 interiors, R planes behind along z; A^k is
                                kept in buffer k mod 4 (two more float32 fields in the workspace).
                                Same bits as one step per pass.  Float32 forward only: needs no
                                CPML, no adjoint, cache_hint 0, variant 0 or family 4 and
                                graph_steps a multiple of 4; tune is not applied.  An odd step count
                                ends with a single step.  0 (default): one step per pass */
} wave_params;

/* Fill `p` with defaults: no source, no receivers, float32 storage,
 * alpha 0.015, unit spacings and dt (callers set the grid and dt), tune = 1. */
void wave_params_init(wave_params *p);

/* The largest stable time step for velocities up to vmax on p's grid
 * spacing (the test wave_create applies, WAVE_EUNSTABLE above it, once it has
 * read the velocity's maximum): the leapfrog of the update in paper Sec. II
 * is stable iff (vmax dt)^2 lambda_max <= 4, with lambda_max = 2048/315 *
 * sum_a h_a^-2 the largest eigenvalue magnitude of the Laplacian (Eq. 1's
 * stencil at the Nyquist wavenumber on each axis), so
 * dt_max = 2 / (vmax sqrt(2048/315 sum_a h_a^-2)).  Host only.  Errors:
 * WAVE_EINVAL (null pointer, vmax or a spacing not finite and positive). */
int wave_stable_dt(const wave_params *p, double vmax, double *dt_max);

/* Bytes of device workspace wave_create needs for `p`: m = (v dt)^2, the
 * wavefields of the update (two float32 fields, or three 16-bit fields A,
 * A', V), the sponge tables, the receiver map and, with adjoint != 0, the
 * checkpoints, the recomputation buffer and the adjoint fields.  Validates `p`
 * (WAVE_EINVAL on any bad field); touches no device. */
int wave_workspace_bytes(const wave_params *p, size_t *bytes);

/* Create a context: the setup of the update of paper Sec. II (Eq. 1 weights
 * divided by h_a^2, m = (v dt)^2, sponge tables, receiver map).
 * vel_dev: device float32 [nz][ny][nx] velocity (m/s), finite and > 0, read
 * during the call only (m is stored in the workspace).  ws_dev: device
 * workspace of ws_bytes >= wave_workspace_bytes, 256-byte aligned, owned by
 * the caller and borrowed until wave_destroy.  hip_stream: the hipStream_t all
 * work is queued on (NULL = default stream).  Synchronises that stream to read
 * back the velocity range and, with tune = 1 (a grid shape not yet tuned in
 * this process), to time a few steps of each candidate configuration on the
 * zeroed fields.  Errors: WAVE_EINVAL (bad params, pointer,
 * alignment, non-finite or non-positive velocity), WAVE_ENOSPC (workspace too
 * small), WAVE_EUNSTABLE (max(v) dt above the leapfrog stability limit
 * 2 / sqrt(2048/315 * sum_a h_a^-2)), WAVE_EHIP.  The state is reset:
 * A^0 = A^{-1} = 0, n = 0. */
int wave_create(const wave_params *p, const float *vel_dev, void *ws_dev, size_t ws_bytes,
                void *hip_stream, wave_t *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): wave_create
 * with the workspace in the library's own static device array of
 * WAVE_STATIC_BYTES bytes (64 MiB: a float32 128^3 forward shot fits) instead
 * of a caller-allocated one.  Each GPU the library runs on holds one such
 * array for the life of the process; the context uses the array of the
 * device current in the calling thread, which must be hip_stream's device.
 * The caller still passes the velocity and, to the other calls, the
 * wavelet, traces, residual and gradient.  Differences from wave_create:
 * tune is ignored (the fixed rule's shape; timing would create events) and
 * graph_steps must be 0 (WAVE_EINVAL; graph instantiation allocates).  At
 * most one static context may exist per device: a second wave_create_static
 * there returns WAVE_ESTATE until the first is destroyed; wave_destroy of a
 * static context synchronises its stream so that the next one starts on an
 * idle array.  Work from any other source that writes the array while a
 * static context's work is in flight on that device races with it.  Errors
 * as wave_create, plus WAVE_ENOSPC when wave_workspace_bytes(p) exceeds
 * WAVE_STATIC_BYTES and WAVE_ESTATE as above. */
#define WAVE_STATIC_BYTES ((size_t)64 << 20)
int wave_create_static(const wave_params *p, const float *vel_dev, void *hip_stream, wave_t *out);

/* Zero the wavefields and the step counter n (enqueued on the stream). */
int wave_reset(wave_t w);

/* Advance nsteps >= 0 steps from the current n: the per-iteration update of
 * paper Sec. II (Eq. 1 at every node, once per time step), fused with the
 * sponge, the source and the receivers as in the formula at the top.
 * wavelet_dev: device float32 s(t_k) indexed by the absolute step k since the
 * last reset (entries n..n+nsteps-1 are read; may be NULL without a source).
 * traces_dev: device float32 [k][nrec], absolute rows n..n+nsteps-1 are written
 * (may be NULL when nrec == 0); both arrays are the caller's and must stay
 * valid until the stream reaches this work.  With graph_steps > 0 the steps
 * are replayed from captured HIP graphs (bit-identical results).  For 16-bit
 * storage a trace holds the stored (rounded) value.  Errors: WAVE_EINVAL
 * (null context, nsteps < 0, a needed pointer NULL), WAVE_EHIP. */
int wave_step(wave_t w, int32_t nsteps, const float *wavelet_dev, float *traces_dev);

/* wave_reset followed by wave_step(nt): one whole forward shot. */
int wave_run(wave_t w, int32_t nt, const float *wavelet_dev, float *traces_dev);

/* Velocity gradient for subsurface imaging (the application of paper Sec. I;
 * the paper has no adjoint): for any scalar J of the traces of an nt-step
 * shot, given resid_dev = dJ/dtrace (device float32 [nt][nrec]), writes
 * grad_vel_dev (device float32 [nz][ny][nx]) = dJ/dv.  Exact discrete adjoint
 * of wave_step: a forward run storing (A^k, A^{k-1}) every ckpt_interval
 * steps, then per segment, last first, a recomputation of the segment's
 * forward fields and the backward adjoint steps with the imaging term fused
 * (mu = m g lambda; dJ/dv = (2/v) sum_n mu^{n+1} L(A^n)).  Requires
 * adjoint != 0 at create (else WAVE_ESTATE), storage == WAVE_F32 and
 * 1 <= nt <= nt_max (else WAVE_EINVAL).  Leaves the context reset (n = 0). */
int wave_adjoint(wave_t w, int32_t nt, const float *wavelet_dev, const float *resid_dev,
                 float *grad_vel_dev);

/* Copy a wavefield, decoded to float32, into out_dev [nz][ny][nx]:
 * which = 0: A^n; which = 1: A^{n-1} (undamped); which = 2 (16-bit storage
 * only, WAVE_EINVAL otherwise): the stored V^n = A^n - g A^{n-1}. */
int wave_read_field(wave_t w, int32_t which, float *out_dev);

/* Set a stored time level from in_dev (device float32 [nz][ny][nx]), so
 * that the next wave_step advances from a given state (paper Sec. II's update
 * applied to any wavefield; the inverse of wave_read_field).  Float32
 * storage: which = 0 writes A^n, which = 1 the stored (undamped) A^{n-1}.
 * 16-bit storage: which = 0 writes A^n, which = 2 the stored V^n = A^n -
 * g A^{n-1}, each rounded to nearest even at the power-of-two scale the step
 * rule gives for the field's maximum (stored magnitudes below 2^14), with the
 * field's scale and maximum records set as a step would leave them.  Other
 * values of which: WAVE_EINVAL.  The step counter is unchanged.  Non-finite
 * inputs are stored as given (the scale then falls back to 2^0 or its
 * clamp), and wave_sync_status reports them as for a run that diverged.
 * Enqueued on the context's stream; in_dev must stay valid until the stream
 * reaches it. */
int wave_write_field(wave_t w, int32_t which, const float *in_dev);

/* Host copy of the step counter n (steps since the last reset). */
int wave_time_index(wave_t w, int32_t *n);

/* The forward step configuration wave_create settled on (after tuning, if
 * asked), written to out[0..2] (caller-owned host array of 3): the kernel
 * variant (1 .. wave_variant_count()-1; see wave_variant_info), the z-chunk
 * in planes, and the cache policy (0 nontemporal, 1 regular; see
 * cache_hint).  Passing these back as variant, zchunk and cache_hint (with
 * tune = 0) reproduces the forward configuration (an adjoint context then
 * runs its adjoint step in the same shape, with the same bits).  Errors:
 * WAVE_EINVAL for a null argument. */
int wave_tiling(wave_t w, int32_t *out);

/* Shot snapshots: the complete state of a forward run after its last
 * enqueued step (step counter, both stored time levels -- A^n and A^{n-1}, or
 * A^n and V^n with 16-bit storage -- their scale records, and the CPML memory
 * variables), so that the per-iteration update of paper Sec. II continues
 * from it bit for bit.  wave_state_bytes gives the size; wave_save_state
 * copies the state to `dst_dev` (caller-owned device memory of at least that
 * size) and wave_load_state restores it into a context created with the same
 * grid, storage and boundary parameters (the same or another context, e.g. to
 * resume a preempted shot).  Both synchronise the context's stream.  Errors:
 * WAVE_EINVAL (null arguments; a snapshot from a context with other
 * parameters), WAVE_EHIP. */
int wave_state_bytes(wave_t w, size_t *bytes);
int wave_save_state(wave_t w, void *dst_dev);
int wave_load_state(wave_t w, const void *src_dev);

/* Synchronise the stream and report WAVE_FLAG_* bits for the current field
 * (WAVE_FLAG_NONFINITE: A^n holds an infinity or NaN). */
int wave_sync_status(wave_t w, uint32_t *flags);

/* Free the host context (the workspace stays the caller's). */
int wave_destroy(wave_t w);

/* Number of kernel tiling variants (valid values of wave_params.variant). */
int wave_variant_count(void);

/* Shape of kernel variant `variant` (0 .. wave_variant_count()-1), written to
 * info[0..4] (caller-owned host array of 5): family, by, ry, pd, vec.
 * Family 0 is the 2.5D blocking of paper Sec. IV-A (tile x and y, stream
 * along z): tiles of 64*vec x by*ry nodes, pd planes of loads in flight.
 * Variant 0 means "automatic"; its info is the shape that choice falls back
 * to (also available explicitly as another variant).
 * Families 1 and 2 are the paper's 3D-blocking designs of the same section
 * ("gmem": every stencil value from global memory; "smem": a 3D tile with
 * its halo staged in shared memory): blocks of 64 x by x ry nodes, float32
 * storage and forward steps only; they compute the same bits as family 0.
 * Family 3 is the 2.5D blocking with the z sum as a semi-stencil (the
 * paper's st_semi, same section): float32 forward only, the z sum in another
 * order (not bitwise equal to family 0).  Family 4 is the two-steps-per-pass
 * kernel of time_block = 2 (by, ry give its 64 x by*ry first-step tile).  Errors: WAVE_EINVAL for a null
 * `info` or an out-of-range variant. */
int wave_variant_info(int32_t variant, int32_t *info);

/* Static text for a status code. */
const char *wave_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* LIBWAVE_WAVE_H */
