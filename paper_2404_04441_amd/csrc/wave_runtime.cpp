// Host runtime of libwave: argument validation, workspace layout, FP64 host
// tables (stencil weights, sponge profiles), receiver mapping, the time loop
// with optional HIP-graph replay, and the checkpointed adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "wave.h"
#include "wave_internal.h"

using namespace wave;

namespace {

// Centred second-derivative weights, 8th order (Eq. 1 of paper Sec. II; the
// paper leaves the values unprinted): the textbook values of Fornberg (1988).
constexpr double kC[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
// Centred first-derivative weights, 8th order (the CPML memory variables):
// f'(0) ~ sum_m w_m (f(m) - f(-m)), Fornberg (1988).
constexpr double kD1[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct Layout {
  size_t st, gx, gy, gz, rz, rec_lin, rec_node, rec_off, rec_ord, grec, m, fa, fb, fc, fd, fv, ckpt, seg, mua, mub, img;
  size_t cpml_ab, cpml_slab[3], total;  // CPML: a/b tables, psi+zeta slab pair per axis
  int K, nck;
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const wave_params *p) {
  if (!p) return WAVE_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return WAVE_EINVAL;
  // at most 2^24 nodes per xy plane: a workgroup's buffer resources span its
  // z-chunk plus halo planes, and every span must stay below 2^31 bytes
  if (static_cast<int64_t>(p->nx) * p->ny > (int64_t(1) << 24)) return WAVE_EINVAL;
  if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->dz) || !finite_pos(p->dt)) return WAVE_EINVAL;
  if (p->sponge_width < 0 || !std::isfinite(p->sponge_alpha) || p->sponge_alpha < 0.0) return WAVE_EINVAL;
  if (p->cpml_width < 0) return WAVE_EINVAL;
  if (p->cpml_width > 0) {
    const int W = p->cpml_width;
    if (p->sponge_width != 0 || p->storage != WAVE_F32 || p->adjoint) return WAVE_EINVAL;
    if (2 * W > p->nx || 2 * W > p->ny || 2 * W > p->nz) return WAVE_EINVAL;
    if (!(p->cpml_reflection > 0.0 && p->cpml_reflection <= 1.0)) return WAVE_EINVAL;
    if (!std::isfinite(p->cpml_f0) || p->cpml_f0 < 0.0) return WAVE_EINVAL;
    // the boundary shell (nodes within W + R of a face) is indexed with 32 bits
    const int64_t E2 = 2 * (static_cast<int64_t>(W) + 4), nx = p->nx, ny = p->ny, nz = p->nz;
    const int64_t mz = std::max<int64_t>(nz - E2, 0), my = std::max<int64_t>(ny - E2, 0);
    const int64_t shell = std::min(E2, nz) * ny * nx + mz * std::min(E2, ny) * nx + mz * my * std::min(E2, nx);
    if (shell >= (int64_t(1) << 31)) return WAVE_EINVAL;
    if (nx * ny * nz >= (int64_t(1) << 31)) return WAVE_EINVAL;  // 32-bit node offsets in the CPML kernels
    // each psi / zeta slab array (2W x the cross-section) is one buffer resource
    const int64_t cross = std::max(ny * nx, std::max(nz * nx, nz * ny));
    if (4 * 2 * static_cast<int64_t>(W) * cross >= (int64_t(1) << 31)) return WAVE_EINVAL;
  }
  if (p->storage < WAVE_F32 || p->storage > WAVE_BF16) return WAVE_EINVAL;
  if (p->src[0] >= 0) {
    if (p->src[0] >= p->nx || p->src[1] < 0 || p->src[1] >= p->ny || p->src[2] < 0 || p->src[2] >= p->nz)
      return WAVE_EINVAL;
  }
  if (p->nrec < 0 || (p->nrec > 0 && !p->rec)) return WAVE_EINVAL;
  for (int r = 0; r < p->nrec; ++r) {
    const int32_t *c = p->rec + 3 * r;
    if (c[0] < 0 || c[0] >= p->nx || c[1] < 0 || c[1] >= p->ny || c[2] < 0 || c[2] >= p->nz) return WAVE_EINVAL;
  }
  if (p->adjoint) {
    if (p->storage != WAVE_F32 || p->nt_max < 1 || p->ckpt_interval < 0) return WAVE_EINVAL;
  }
  if (p->variant < 0 || p->variant >= variant_count()) return WAVE_EINVAL;
  if (p->variant > 0) {
    const Variant v = variant_info(p->variant);
    // a tile shape with VEC > 1 x nodes per lane needs whole vectors per row
    if (p->nx % v.vec) return WAVE_EINVAL;
    // the study families (3D-blocked, semi-stencil) are float32 forward only
    if (v.family != 0 && (p->storage != WAVE_F32 || p->adjoint)) return WAVE_EINVAL;
  }
  if (p->zchunk < 0 || p->graph_steps < 0) return WAVE_EINVAL;
  if (p->tune < 0 || p->tune > 1) return WAVE_EINVAL;
  // the cached policy exists for the 2.5D forward kernels without CPML
  if (p->cache_hint < 0 || p->cache_hint > 1) return WAVE_EINVAL;
  // two time steps per pass: float32 forward, no CPML, its own kernel (variant 0 or its family's)
  if (p->time_block != 0 && p->time_block != 2) return WAVE_EINVAL;
  if (p->time_block == 2) {
    if (p->storage != WAVE_F32 || p->cpml_width > 0 || p->adjoint || p->cache_hint != 0) return WAVE_EINVAL;
    if (p->variant > 0 && variant_info(p->variant).family != 4) return WAVE_EINVAL;
    if (p->graph_steps % 4) return WAVE_EINVAL;  // replays start at the same buffer phase (n mod 4)
  } else if (p->variant > 0 && variant_info(p->variant).family == 4) {
    return WAVE_EINVAL;
  }
  // 16-bit model codes exist for the 16-bit storage forward step only
  if (p->model_bits != 0 && p->model_bits != 32 && p->model_bits != 16) return WAVE_EINVAL;
  if (p->model_bits == 16 && p->storage == WAVE_F32) return WAVE_EINVAL;
  if (p->cache_hint == 1 && (p->cpml_width > 0 || (p->variant > 0 && variant_info(p->variant).family != 0)))
    return WAVE_EINVAL;
  return WAVE_OK;
}

int plan(const wave_params *p, Layout *L) {
  const int rc = validate(p);
  if (rc) return rc;
  const size_t N = static_cast<size_t>(p->nx) * p->ny * p->nz;
  // fields the step kernel touches carry kPadZ zero planes after the interior
  const size_t Np = static_cast<size_t>(p->nx) * p->ny * (static_cast<size_t>(p->nz) + kPadZ);
  const size_t es = p->storage == WAVE_F32 ? 4 : 2;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return at;
  };
  L->st = take(sizeof(StepState));
  L->gx = take(4 * static_cast<size_t>(p->nx));
  L->gy = take(4 * static_cast<size_t>(p->ny));
  L->gz = take(4 * (static_cast<size_t>(p->nz) + kPadZ));
  L->rz = take(4 * (static_cast<size_t>(p->nz) + kPadZ));
  L->rec_lin = take(8 * static_cast<size_t>(p->nrec));
  // the receivers grouped by node (adjoint injection): distinct nodes, the
  // offsets of each node's receivers in rec_ord, and the sponge factor per node
  L->rec_node = take(8 * static_cast<size_t>(p->nrec));
  L->rec_off = take(4 * (static_cast<size_t>(p->nrec) + 1));
  L->rec_ord = take(4 * static_cast<size_t>(p->nrec));
  L->grec = take(4 * static_cast<size_t>(p->nrec));
  L->m = take((p->model_bits == 16 ? 2 : 4) * Np);  // m: float32, or 16-bit codes
  L->fa = take(es * Np);
  L->fb = take(es * Np);
  // 16-bit storage keeps V^n = A^n - g A^{n-1} besides the A ping-pong pair
  L->fv = p->storage == WAVE_F32 ? off : take(es * Np);
  // two steps per pass: A^k in buffer k mod 4 (no pass writes a buffer it reads)
  L->fc = L->fd = off;
  if (p->time_block == 2) {
    L->fc = take(es * Np);
    L->fd = take(es * Np);
  }
  L->K = 0;
  L->nck = 0;
  L->ckpt = L->seg = L->mua = L->mub = L->img = off;
  if (p->adjoint) {
    int K = p->ckpt_interval;
    if (K <= 0) K = static_cast<int>(std::ceil(std::sqrt(static_cast<double>(p->nt_max))));
    K = std::max(1, std::min(K, p->nt_max));
    const int nseg = (p->nt_max + K - 1) / K;
    L->K = K;
    L->nck = nseg - 1;
    L->ckpt = take(4 * N * 2 * static_cast<size_t>(L->nck));  // interiors only
    L->seg = take(4 * Np * static_cast<size_t>(K + 2));
    L->mua = take(4 * Np);
    L->mub = take(4 * Np);
    L->img = take(4 * Np);
  }
  L->cpml_ab = off;
  L->cpml_slab[0] = L->cpml_slab[1] = L->cpml_slab[2] = off;
  if (p->cpml_width > 0) {
    const size_t W2 = 2 * static_cast<size_t>(p->cpml_width);
    const size_t nx = p->nx, ny = p->ny, nz = p->nz;
    L->cpml_ab = take(4 * 2 * (nx + ny + nz));
    L->cpml_slab[0] = take(4 * 2 * nz * ny * W2);
    L->cpml_slab[1] = take(4 * 2 * nz * W2 * nx);
    L->cpml_slab[2] = take(4 * 2 * W2 * ny * nx);
  }
  L->total = off;
  return WAVE_OK;
}

std::vector<float> sponge_table(int n, int width, double alpha) {
  std::vector<float> g(n);
  for (int i = 0; i < n; ++i) {
    const int d = std::min(i, n - 1 - i);
    const double t = d < width ? alpha * (width - d) : 0.0;
    g[i] = static_cast<float>(d < width ? std::exp(-t * t) : 1.0);
  }
  return g;
}

// If the receivers are a regular box listed x fastest, then y, then z, fill
// `b` and return true.
bool detect_box(const std::vector<int32_t> &rec, int nrec, RecBox *b) {
  if (nrec == 0) return false;
  auto X = [&](int r) { return rec[3 * r]; };
  auto Y = [&](int r) { return rec[3 * r + 1]; };
  auto Z = [&](int r) { return rec[3 * r + 2]; };
  int cnx = 1;
  while (cnx < nrec && Y(cnx) == Y(0) && Z(cnx) == Z(0)) ++cnx;
  const int sx = cnx > 1 ? X(1) - X(0) : 1;
  if (sx <= 0 || nrec % cnx) return false;
  int cny = 1;
  while (cny * cnx < nrec && Z(cny * cnx) == Z(0)) ++cny;
  const int sy = cny > 1 ? Y(cnx) - Y(0) : 1;
  if (sy <= 0 || nrec % (cnx * cny)) return false;
  const int cnz = nrec / (cnx * cny);
  const int sz = cnz > 1 ? Z(cnx * cny) - Z(0) : 1;
  if (sz <= 0) return false;
  for (int l = 0; l < cnz; ++l)
    for (int j = 0; j < cny; ++j)
      for (int i = 0; i < cnx; ++i) {
        const int r = (l * cny + j) * cnx + i;
        if (X(r) != X(0) + i * sx || Y(r) != Y(0) + j * sy || Z(r) != Z(0) + l * sz) return false;
      }
  *b = RecBox{X(0), sx, cnx, Y(0), sy, cny, Z(0), sz, cnz};
  return true;
}

// One tile decomposition of the grid for a step-kernel variant.
struct Tiling {
  int variant = 0, tiles_x = 0, tiles_y = 0, nchunks = 0, zchunk = 0, total_tiles = 0;
  bool keep = false;  // forward: regular cache policy for the fields streamed once
};

// Measured-best tile shapes on MI355X (variant indices of the kernel
// table): 4 x nodes per lane when rows allow it (8 wavefronts x 1 row; for
// float32 planes above 512 x 512, 8 x 4 rows of 2 nodes), else 2, else 1.
int auto_variant(const wave_params *p) {
  const int64_t plane = static_cast<int64_t>(p->nx) * p->ny;
  if (p->cpml_width > 0 && p->storage == WAVE_F32)  // shapes with the CPML terms fused into the step
    return p->nx % 4 == 0 ? 12 : (p->nx % 2 == 0 ? 8 : 3);
  if (p->nx % 4 == 0) return (p->storage == WAVE_F32 && plane > (int64_t(1) << 18)) ? 11 : 12;
  if (p->nx % 2 == 0) return 8;
  return p->storage == WAVE_F32 ? 0 : 3;
}
// The adjoint kernel keeps two z queues: its default is a one-node-per-lane
// shape that fits in registers (8 wavefronts x 4 rows, one plane in flight).
constexpr int kAdjointVariant = 5;
// The two-steps-per-pass kernel (variant family 4).
constexpr int kPairVariant = 19;

Tiling make_tiling(const wave_params *p, int variant) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  Tiling t;
  t.variant = variant;
  const Variant v = variant_info(variant);
  if (v.family == 4) {  // two steps per pass: 56 x 24 output tiles (64 x 32 for the first step)
    t.tiles_x = (nx + kTileX - 2 * kRadius - 1) / (kTileX - 2 * kRadius);
    t.tiles_y = (ny + v.by * v.ry - 2 * kRadius - 1) / (v.by * v.ry - 2 * kRadius);
    // about one workgroup per CU (its LDS and registers allow one); each
    // chunk also runs 2R planes of the first step beyond its outputs
    const int per_plane = t.tiles_x * t.tiles_y;
    int zc = p->zchunk;
    if (zc <= 0) {
      const int chunks = std::max(1, (256 + per_plane / 2) / per_plane);
      zc = std::max(std::min(nz, 27), (nz + chunks - 1) / chunks);
    }
    // a workgroup's resources span its chunk plus 2R + 9 + R + 1 planes, below 2^31 bytes
    const int64_t plane_f = 4 * static_cast<int64_t>(nx) * ny;
    const int zc_max = static_cast<int>(((int64_t(1) << 31) - 1) / plane_f) - (3 * kRadius + 10);
    zc = std::max(1, std::min(zc, zc_max));
    t.zchunk = zc;
    t.nchunks = (nz + zc - 1) / zc;
    t.total_tiles = t.tiles_x * t.tiles_y * t.nchunks;
    return t;
  }
  if (v.family == 1 || v.family == 2) {  // 3D blocks of 64 x by x ry nodes
    t.tiles_x = (nx + kTileX - 1) / kTileX;
    t.tiles_y = (ny + v.by - 1) / v.by;
    t.zchunk = v.ry;
    t.nchunks = (nz + v.ry - 1) / v.ry;
    t.total_tiles = t.tiles_x * t.tiles_y * t.nchunks;
    return t;
  }
  const int TY = v.by * v.ry;
  const int TX = kTileX * v.vec;
  t.tiles_x = (nx + TX - 1) / TX;
  t.tiles_y = (ny + TY - 1) / TY;
  // a workgroup's buffer resources span its z-chunk rounded up to whole
  // nine-plane trips, R halo planes below and kMaxPD + R prefetch and halo
  // planes above; every span (float32 fields) must stay below 2^31 bytes.
  // With at most 2^24 nodes per plane this leaves at least one trip.
  const int64_t plane_f = 4 * static_cast<int64_t>(nx) * ny;
  const int zc_max = (static_cast<int>(((int64_t(1) << 31) - 1) / plane_f) - (2 * kRadius + kMaxPD)) / 9 * 9;
  int zc = p->zchunk;
  if (zc <= 0) {
    // k equal z-chunks, k minimising the launch time in the model
    // (rounds of workgroups over the 256 CUs) x (planes per chunk + 3): the
    // 3 stands for a chunk's overlap planes and pipeline fill, so long
    // chunks win unless more of them fill the CUs' last round.  Chunks keep
    // at least 18 planes and fit the resource span.
    const int64_t per_plane = static_cast<int64_t>(t.tiles_x) * t.tiles_y;
    const int64_t cap = 256 * static_cast<int64_t>(step_blocks_per_cu(p->storage, variant, p->cpml_width > 0));
    const int k_min = (nz + zc_max - 1) / zc_max;
    int best_k = k_min;
    int64_t best_cost = -1;
    for (int k = k_min; k == k_min || (nz + k - 1) / k >= 18; ++k) {
      const int64_t rounds = (per_plane * k + cap - 1) / cap;
      const int64_t cost = rounds * ((nz + k - 1) / k + 3);
      if (best_cost < 0 || cost < best_cost) {
        best_cost = cost;
        best_k = k;
      }
    }
    zc = (nz + best_k - 1) / best_k;
  }
  if (zc > zc_max) {  // equal chunks that fit
    const int k = (nz + zc_max - 1) / zc_max;
    zc = std::min((nz + k - 1) / k, zc_max);
  }
  // the fused CPML step runs whole nine-plane trips (no skip branch)
  if (p->cpml_width > 0 && variant_fuses_cpml(variant)) zc = std::min((zc + 8) / 9 * 9, zc_max);
  t.zchunk = zc;
  t.nchunks = (nz + zc - 1) / zc;
  t.total_tiles = t.tiles_x * t.tiles_y * t.nchunks;
  return t;
}

}  // namespace

struct wave_ctx {
  wave_params p{};
  std::vector<int32_t> rec;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  Layout L{};
  StepState *st = nullptr;
  float *gx = nullptr, *gy = nullptr, *gz = nullptr, *m = nullptr, *grec = nullptr;  // grec: per receiver node
  int32_t *rz = nullptr;
  bool cpml = false;
  bool cpml_fused = false;  // the forward shape's step kernel applies the x part of the CPML terms
  CpmlArgs cp{};
  int64_t *rec_lin = nullptr;   // linear node index of each receiver (gather)
  int64_t *rec_node = nullptr;  // distinct receiver nodes, ascending (adjoint injection)
  int32_t *rec_off = nullptr, *rec_ord = nullptr;
  int nrec_nodes = 0;
  void *fa = nullptr, *fb = nullptr, *fc = nullptr, *fd = nullptr, *fv = nullptr;
  size_t N = 0;   // interior nodes
  size_t Np = 0;  // nodes of a padded field (interior + kPadZ zero planes)
  int n = 0;      // host mirror of the step counter
  Coef c{};
  float src_scale = 0.f, gamma = 0.f;
  bool m16 = false;                  // m held as 16-bit codes: m = m_lo + u * m_step
  float m_lo = 0.f, m_step = 0.f;
  RecBox box{};
  bool fused_rec = false;
  Tiling fwd{}, adj{};  // forward and adjoint step kernels
  Tiling pair{};        // time_block == 2: the two-steps-per-pass kernel
  // graph replay cache: one graph per buffer parity
  hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};  // by buffer phase
  const float *g_wavelet = nullptr;
  float *g_traces = nullptr;

  int static_dev = -1;  // >= 0: the context lives in that device's static scratch array
  ~wave_ctx() { drop_graphs(); }
  void drop_graphs() {
    for (auto &g : graph)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  }
  // A^k lives in field(k): buffer k mod 2, or k mod 4 with two steps per pass
  void *field(int k) const {
    if (p.time_block == 2) {
      void *const b[4] = {fa, fb, fc, fd};
      return b[k & 3];
    }
    return (k & 1) ? fb : fa;
  }
};

namespace {

int hip_rc(hipError_t e) { return e == hipSuccess ? WAVE_OK : WAVE_EHIP; }

StepArgs base_args(const wave_ctx *w, const Tiling &t) {
  StepArgs a{};
  a.m = w->m;
  a.gx = w->gx;
  a.gy = w->gy;
  a.gz = w->gz;
  a.rz = w->rz;
  a.nx = w->p.nx;
  a.ny = w->p.ny;
  a.nz = w->p.nz;
  a.tiles_x = t.tiles_x;
  a.tiles_y = t.tiles_y;
  a.nchunks = t.nchunks;
  a.zchunk = t.zchunk;
  a.total_tiles = t.total_tiles;
  a.keep = t.keep ? 1 : 0;
  a.c = w->c;
  a.sx = w->p.src[0] >= 0 ? w->p.src[0] : -1;
  a.sy = w->p.src[1];
  a.sz = w->p.src[2];
  a.src_scale = w->src_scale;
  a.st = w->st;
  a.gamma = w->gamma;
  a.nrec = w->p.nrec;
  a.m16 = w->m16 ? 1 : 0;
  a.m_lo = w->m_lo;
  a.m_step = w->m_step;
  return a;
}

// Enqueue `count` forward steps starting at device counter st->n (and host
// n), then advance the counter.  sample = write traces.
int enqueue_steps(wave_ctx *w, int count, const float *wavelet, float *traces, bool sample) {
  StepArgs a = base_args(w, w->fwd);
  a.wavelet = wavelet;
  a.traces = traces;
  // CPML: psi pass, step, correction pass (y and z parts only for the shapes
  // whose step applies the x part itself); the receivers are gathered after
  // the correction
  const bool fix_pass = w->cpml;
  if (w->cpml_fused) {
    a.cpml = 1;
    a.cp = w->cp;
  }
  if (sample && w->fused_rec && !fix_pass) a.box = w->box;
  const bool gather = sample && (!w->fused_rec || fix_pass) && w->p.nrec > 0;
  for (int k = 0; k < count; ++k) {
    const int nk = w->n + k;
    if (w->p.time_block == 2 && count - k >= 2) {  // steps nk and nk+1 in one pass
      StepArgs b = base_args(w, w->pair);
      b.wavelet = wavelet;
      b.traces = traces;
      if (sample && w->fused_rec) b.box = w->box;
      b.cur = w->field(nk);
      b.prev = w->field(nk + 3);
      b.out = w->field(nk + 1);
      b.out2 = w->field(nk + 2);
      b.k = k;
      int rc = hip_rc(launch_step(WAVE_F32, w->pair.variant, false, b, w->stream));
      for (int e = 0; e < 2 && !rc && gather; ++e)
        rc = hip_rc(launch_gather(w->p.storage, w->field(nk + 1 + e), w->rec_lin, w->p.nrec, traces, w->st, k + e,
                                  w->stream));
      if (rc) return rc;
      ++k;
      continue;
    }
    a.cur = w->field(nk);
    a.out = w->field(nk + 1);
    a.prev = w->p.storage == WAVE_F32 ? w->field(nk + 3) : w->fv;
    a.vout = w->fv;
    a.k = k;
    int rc = 0;
    if (w->cpml) rc = hip_rc(launch_cpml_psi(w->cp, static_cast<const float *>(a.cur), w->stream));
    if (!rc) rc = hip_rc(launch_step(w->p.storage, w->fwd.variant, false, a, w->stream));
    if (!rc && fix_pass)
      rc = hip_rc(launch_cpml_fix(w->cp, static_cast<const float *>(a.cur), w->m, static_cast<float *>(a.out),
                                  w->cpml_fused, w->stream));
    if (rc) return rc;
    if (gather) {
      rc = hip_rc(launch_gather(w->p.storage, a.out, w->rec_lin, w->p.nrec, traces, w->st, k, w->stream));
      if (rc) return rc;
    }
  }
  return hip_rc(launch_bump(w->st, count, w->stream));
}

// Replay `reps` times a captured graph of graph_steps steps (even count, so
// the buffer parity is the same at every replay).
int replay_graph(wave_ctx *w, int reps, const float *wavelet, float *traces) {
  const int K = w->p.graph_steps;
  if (w->g_wavelet != wavelet || w->g_traces != traces) {
    w->drop_graphs();
    w->g_wavelet = wavelet;
    w->g_traces = traces;
  }
  const int parity = w->p.time_block == 2 ? (w->n & 3) : (w->n & 1);
  if (!w->graph[parity]) {
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return WAVE_EHIP;
    hipGraph_t g = nullptr;
    int rc = hip_rc(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    if (!rc) {
      hipStream_t saved = w->stream;
      const int saved_n = w->n;
      w->stream = cs;
      rc = enqueue_steps(w, K, wavelet, traces, true);
      w->stream = saved;
      w->n = saved_n;
      const int rc2 = hip_rc(hipStreamEndCapture(cs, &g));
      if (!rc) rc = rc2;
    }
    if (!rc) rc = hip_rc(hipGraphInstantiate(&w->graph[parity], g, nullptr, nullptr, 0));
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (rc) return rc;
  }
  for (int r = 0; r < reps; ++r) {
    const int rc = hip_rc(hipGraphLaunch(w->graph[parity], w->stream));
    if (rc) return rc;
  }
  w->n += reps * K;
  return WAVE_OK;
}

int do_step(wave_ctx *w, int nsteps, const float *wavelet, float *traces) {
  int done = 0;
  const int K = w->p.graph_steps;
  if (K > 0 && K % 2 == 0 && nsteps >= K) {
    const int reps = nsteps / K;
    const int rc = replay_graph(w, reps, wavelet, traces);
    if (rc) return rc;
    done = reps * K;
  }
  if (nsteps - done > 0) {
    const int rc = enqueue_steps(w, nsteps - done, wavelet, traces, true);
    if (rc) return rc;
    w->n += nsteps - done;
  }
  return WAVE_OK;
}

// Bytes of the psi + zeta pair of axis a's CPML slabs.
size_t slab_bytes(const wave_ctx *w, int a) {
  const size_t W2 = 2 * static_cast<size_t>(w->p.cpml_width);
  const size_t nx = w->p.nx, ny = w->p.ny, nz = w->p.nz;
  const size_t n = a == 0 ? nz * ny * W2 : (a == 1 ? nz * W2 * nx : W2 * ny * nx);
  return 4 * 2 * n;
}

int do_reset(wave_ctx *w) {
  const size_t es = w->p.storage == WAVE_F32 ? 4 : 2;
  int rc = hip_rc(launch_fill_zero(w->fa, es * w->Np, w->stream));
  for (int a = 0; a < 3 && w->cpml && !rc; ++a)
    rc = hip_rc(launch_fill_zero(w->ws + w->L.cpml_slab[a], slab_bytes(w, a), w->stream));
  if (!rc) rc = hip_rc(launch_fill_zero(w->fb, es * w->Np, w->stream));
  if (!rc && w->fc) rc = hip_rc(launch_fill_zero(w->fc, es * w->Np, w->stream));
  if (!rc && w->fd) rc = hip_rc(launch_fill_zero(w->fd, es * w->Np, w->stream));
  if (!rc && w->fv) rc = hip_rc(launch_fill_zero(w->fv, es * w->Np, w->stream));
  if (!rc) rc = hip_rc(launch_reset_state(w->st, w->stream));
  if (!rc) w->n = 0;
  return rc;
}

// ---- shape tuning: time each candidate (2.5D shape, z-chunk) for a few
// steps on the zeroed fields and keep the fastest.  All candidates compute
// identical bits, so the choice only changes speed.
struct TuneEntry {
  int nx, ny, nz, storage, cache_hint, model_bits;
  bool cpml, adjoint;
  Tiling t, adj;  // forward step; adjoint step (adjoint contexts)
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune_cache;

int tune_forward(wave_ctx *w) {
  const wave_params &p = w->p;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const TuneEntry &e : g_tune_cache)
      if (e.nx == p.nx && e.ny == p.ny && e.nz == p.nz && e.storage == p.storage && e.cpml == w->cpml &&
          e.cache_hint == p.cache_hint && e.adjoint == (p.adjoint != 0) && e.model_bits == (p.model_bits == 16)) {
        w->fwd = e.t;
        if (p.adjoint) w->adj = e.adj;
        w->cpml_fused = w->cpml && variant_fuses_cpml(w->fwd.variant);
        return WAVE_OK;
      }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = hip_rc(hipEventCreate(&e0));
  if (!rc) rc = hip_rc(hipEventCreate(&e1));
  // no source while timing (the wavelet is not known yet); the fields stay zero
  const int src_x = w->p.src[0];
  w->p.src[0] = -1;
  const Tiling fixed = w->fwd;
  // milliseconds of 3 steps after 1 warm-up step, or a negative value on error
  auto time_one = [&](const Tiling &t) {
    w->fwd = t;
    w->cpml_fused = w->cpml && variant_fuses_cpml(t.variant);
    int r = enqueue_steps(w, 1, nullptr, nullptr, false);
    if (!r) r = hip_rc(hipEventRecord(e0, w->stream));
    if (!r) r = enqueue_steps(w, 3, nullptr, nullptr, false);
    if (!r) r = hip_rc(hipEventRecord(e1, w->stream));
    if (!r) r = hip_rc(hipEventSynchronize(e1));
    float ms = 0.f;
    if (!r) r = hip_rc(hipEventElapsedTime(&ms, e0, e1));
    if (r) rc = r;
    return r ? -1.f : ms;
  };
  // stage 1: the fixed rule's choice, then every shape at its automatic
  // z-chunk, 2.5D shapes with both cache policies where they apply (only the
  // cached one for cache_hint 1; not for adjoint contexts, whose recomputation
  // streams the checkpoint buffer through the same cache).  The 3D-blocked families compute the same
  // bits as the 2.5D shapes (float32 forward); on small grids, where
  // everything stays in cache, they can win.
  const bool blocked_ok = p.storage == WAVE_F32 && !w->cpml && !p.adjoint && p.cache_hint == 0;
  std::vector<Tiling> cands{fixed};
  for (int v = 1; v < variant_count(); ++v) {
    const Variant info = variant_info(v);
    if ((info.family == 1 || info.family == 2) && blocked_ok) {
      cands.push_back(make_tiling(&p, v));
      continue;
    }
    if (info.family != 0 || p.nx % info.vec) continue;
    if (w->cpml && !variant_fuses_cpml(v)) continue;
    wave_params q = p;
    q.variant = v;
    q.zchunk = 0;
    Tiling t = make_tiling(&q, v);
    t.keep = p.cache_hint == 1;
    cands.push_back(t);
    if (!w->cpml && p.cache_hint == 0 && !p.adjoint) {
      t.keep = true;
      cands.push_back(t);
    }
  }
  std::vector<std::pair<float, Tiling>> timed;
  for (size_t i = 0; i < cands.size() && !rc; ++i) timed.emplace_back(time_one(cands[i]), cands[i]);
  // stage 2: the z-chunk list for the four fastest 2.5D candidates of stage 1
  std::vector<std::pair<float, Tiling>> top;
  for (const auto &c : timed)
    if (variant_info(c.second.variant).family == 0) top.push_back(c);
  std::sort(top.begin(), top.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
  if (top.size() > 4) top.resize(4);
  for (const auto &c : top) {
    wave_params q = p;
    q.variant = c.second.variant;
    for (int zc : {9, 18, 27, 45, 72, 99, 135, 198, 270}) {
      if (rc || zc >= p.nz) break;
      q.zchunk = zc;
      Tiling t = make_tiling(&q, q.variant);
      t.keep = c.second.keep;
      if (t.zchunk != c.second.zchunk) timed.emplace_back(time_one(t), t);
    }
  }
  // the fixed rule's choice (timed first) stays unless another candidate is
  // more than 3% faster, so near-ties (timing noise) do not move the choice
  Tiling best = fixed;
  if (!rc) {
    const float base_ms = timed.front().first;
    float best_ms = base_ms;
    for (const auto &c : timed)
      if (c.first < best_ms) {
        best_ms = c.first;
        best = c.second;
      }
    if (best_ms > 0.97f * base_ms) best = fixed;
  }
  w->p.src[0] = src_x;
  w->fwd = best;
  w->cpml_fused = w->cpml && variant_fuses_cpml(w->fwd.variant);
  // Adjoint contexts: the adjoint step (two z queues, the forward field and
  // the imaging accumulator on top of the forward step's streams) is timed on
  // its own, on the zero fields with no residual (wave_adjoint clears every
  // buffer it reads before use): every 2.5D shape at its automatic z-chunk,
  // then the z-chunk list for the two fastest, the default kept unless
  // another is more than 3% faster.  All compute the same bits.
  if (!rc && p.adjoint) {
    const Layout &L = w->L;
    float *mu1 = reinterpret_cast<float *>(w->ws + L.mua);
    float *mu2 = reinterpret_cast<float *>(w->ws + L.mub);
    float *img = reinterpret_cast<float *>(w->ws + L.img);
    float *seg = reinterpret_cast<float *>(w->ws + L.seg);
    auto time_adj = [&](const Tiling &t) {
      StepArgs b = base_args(w, t);
      b.sx = -1;
      b.img = img;
      b.cur = mu1;
      b.prev = mu2;
      b.out = mu2;
      b.fwd = seg;
      if (w->fused_rec) b.box = w->box;
      int r = 0;
      for (int i = 0; i < 4 && !r; ++i) {
        if (i == 1) r = hip_rc(hipEventRecord(e0, w->stream));
        if (!r) r = hip_rc(launch_step(WAVE_F32, t.variant, true, b, w->stream));
      }
      if (!r) r = hip_rc(hipEventRecord(e1, w->stream));
      if (!r) r = hip_rc(hipEventSynchronize(e1));
      float ms = 0.f;
      if (!r) r = hip_rc(hipEventElapsedTime(&ms, e0, e1));
      if (r) rc = r;
      return r ? -1.f : ms;
    };
    const Tiling dflt = w->adj;
    std::vector<std::pair<float, Tiling>> ta{{time_adj(dflt), dflt}};
    for (int v = 0; v < variant_count() && !rc; ++v) {
      const Variant info = variant_info(v);
      if (info.family != 0 || p.nx % info.vec || v == dflt.variant) continue;
      wave_params q = p;
      q.variant = v;
      q.zchunk = 0;
      const Tiling t = make_tiling(&q, v);
      ta.emplace_back(time_adj(t), t);
    }
    std::vector<std::pair<float, Tiling>> top(ta.begin(), ta.end());
    std::sort(top.begin(), top.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    if (top.size() > 2) top.resize(2);
    for (const auto &c : top) {
      wave_params q = p;
      q.variant = c.second.variant;
      for (int zc : {9, 18, 27, 36, 45, 72, 99}) {
        if (rc || zc >= p.nz) break;
        q.zchunk = zc;
        const Tiling t = make_tiling(&q, q.variant);
        if (t.zchunk != c.second.zchunk) ta.emplace_back(time_adj(t), t);
      }
    }
    if (!rc) {
      const float base_ms = ta.front().first;
      float best_ms = base_ms;
      for (const auto &c : ta)
        if (c.first > 0.f && c.first < best_ms) {
          best_ms = c.first;
          w->adj = c.second;
        }
      if (best_ms > 0.97f * base_ms) w->adj = dflt;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!rc) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache.push_back(TuneEntry{p.nx, p.ny, p.nz, p.storage, p.cache_hint, p.model_bits == 16, w->cpml,
                                     p.adjoint != 0, best, w->adj});
  }
  return rc;
}

// CPML profiles along each axis (FP64 on the host): depth xi into a layer of
// W nodes, d = d0 xi^2 with d0 = -3 v_max ln(R) / (2 W h), alpha = pi f0 (1 - xi),
// b = exp(-(d + alpha) dt), a = d (b - 1) / (d + alpha) (0 where d = 0).
int setup_cpml(wave_ctx *w, float vmax) {
  const wave_params &p = w->p;
  const int W = p.cpml_width;
  const int n[3] = {p.nx, p.ny, p.nz};
  const double h[3] = {p.dx, p.dy, p.dz};
  const double pi = 3.14159265358979323846;
  std::vector<float> tab(2 * static_cast<size_t>(p.nx + p.ny + p.nz));
  float *dst_a = tab.data(), *dst_b = tab.data() + (p.nx + p.ny + p.nz);
  float *base_a = reinterpret_cast<float *>(w->ws + w->L.cpml_ab);
  float *base_b = base_a + (p.nx + p.ny + p.nz);
  CpmlArgs &c = w->cp;
  size_t off = 0;
  for (int ax = 0; ax < 3; ++ax) {
    const double d0 = -3.0 * vmax * std::log(p.cpml_reflection) / (2.0 * W * h[ax]);
    for (int i = 0; i < n[ax]; ++i) {
      const double xi = std::max(std::max(W - i, i - (n[ax] - 1 - W)), 0) / static_cast<double>(W);
      const double d = d0 * xi * xi, alpha = pi * p.cpml_f0 * (1.0 - xi);
      const double b = std::exp(-(d + alpha) * p.dt);
      dst_a[off + i] = static_cast<float>(d > 0.0 ? d * (b - 1.0) / (d + alpha) : 0.0);
      dst_b[off + i] = static_cast<float>(b);
    }
    c.ca[ax] = base_a + off;
    c.cb[ax] = base_b + off;
    off += n[ax];
    for (int m = 0; m < 4; ++m) c.d1w[ax][m] = static_cast<float>(kD1[m] / h[ax]);
    for (int m = 0; m < 5; ++m) c.d2w[ax][m] = static_cast<float>(kC[m] / (h[ax] * h[ax]));
    c.psi[ax] = reinterpret_cast<float *>(w->ws + w->L.cpml_slab[ax]);
    c.zeta[ax] = c.psi[ax] + slab_bytes(w, ax) / 8;
  }
  c.W = W;
  c.nx = p.nx;
  c.ny = p.ny;
  c.nz = p.nz;
  w->cpml = true;
  int rc = hip_rc(hipMemcpyAsync(base_a, tab.data(), 4 * tab.size(), hipMemcpyHostToDevice, w->stream));
  if (!rc) rc = hip_rc(hipStreamSynchronize(w->stream));
  return rc;
}

int create_ctx(const wave_params *p, const float *vel_dev, void *ws_dev, size_t ws_bytes, void *hip_stream,
               wave_t *out, int static_dev);

}  // namespace

extern "C" {

void wave_params_init(wave_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->dx = p->dy = p->dz = 1.0;
  p->dt = 1.0;
  p->sponge_alpha = 0.015;
  p->cpml_reflection = 1e-3;
  p->storage = WAVE_F32;
  p->src[0] = -1;
  p->tune = 1;
}

int wave_stable_dt(const wave_params *p, double vmax, double *dt_max) {
  if (!p || !dt_max || !(vmax > 0.0) || !std::isfinite(vmax)) return WAVE_EINVAL;
  if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->dz)) return WAVE_EINVAL;
  // leapfrog u+ = 2u - u- + (v dt)^2 L u is stable iff (v dt)^2 lambda <= 4 for
  // every eigenvalue magnitude lambda of -L; the largest is the stencil's
  // symbol at the Nyquist wavenumber, 2048/315 per axis, times sum_a h_a^-2
  const double peak = 2048.0 / 315.0;
  const double s = peak * (1.0 / (p->dx * p->dx) + 1.0 / (p->dy * p->dy) + 1.0 / (p->dz * p->dz));
  *dt_max = 2.0 / (vmax * std::sqrt(s));
  return WAVE_OK;
}

int wave_workspace_bytes(const wave_params *p, size_t *bytes) {
  if (!bytes) return WAVE_EINVAL;
  Layout L;
  const int rc = plan(p, &L);
  if (rc) return rc;
  *bytes = L.total;
  return WAVE_OK;
}

int wave_create(const wave_params *p, const float *vel_dev, void *ws_dev, size_t ws_bytes, void *hip_stream,
                wave_t *out) {
  return create_ctx(p, vel_dev, ws_dev, ws_bytes, hip_stream, out, -1);
}

}  // extern "C"

namespace {

int create_ctx(const wave_params *p, const float *vel_dev, void *ws_dev, size_t ws_bytes, void *hip_stream,
               wave_t *out, int static_dev) {
  if (!out || !vel_dev || !ws_dev) return WAVE_EINVAL;
  *out = nullptr;
  Layout L;
  int rc = plan(p, &L);
  if (rc) return rc;
  if (reinterpret_cast<uintptr_t>(ws_dev) % 256) return WAVE_EINVAL;
  if (ws_bytes < L.total) return WAVE_ENOSPC;

  wave_ctx *w = new (std::nothrow) wave_ctx();
  if (!w) return WAVE_EINVAL;
  w->static_dev = static_dev;
  w->p = *p;
  w->rec.assign(p->rec, p->rec + 3 * static_cast<size_t>(p->nrec));
  w->p.rec = nullptr;  // never keep the caller's pointer
  w->stream = static_cast<hipStream_t>(hip_stream);
  w->ws = static_cast<char *>(ws_dev);
  w->L = L;
  w->st = reinterpret_cast<StepState *>(w->ws + L.st);
  w->gx = reinterpret_cast<float *>(w->ws + L.gx);
  w->gy = reinterpret_cast<float *>(w->ws + L.gy);
  w->gz = reinterpret_cast<float *>(w->ws + L.gz);
  w->rz = reinterpret_cast<int32_t *>(w->ws + L.rz);
  w->rec_lin = reinterpret_cast<int64_t *>(w->ws + L.rec_lin);
  w->rec_node = reinterpret_cast<int64_t *>(w->ws + L.rec_node);
  w->rec_off = reinterpret_cast<int32_t *>(w->ws + L.rec_off);
  w->rec_ord = reinterpret_cast<int32_t *>(w->ws + L.rec_ord);
  w->grec = reinterpret_cast<float *>(w->ws + L.grec);
  w->m = reinterpret_cast<float *>(w->ws + L.m);
  w->fa = w->ws + L.fa;
  w->fb = w->ws + L.fb;
  w->fv = p->storage == WAVE_F32 ? nullptr : w->ws + L.fv;
  if (p->time_block == 2) {
    w->fc = w->ws + L.fc;
    w->fd = w->ws + L.fd;
  }
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  w->N = static_cast<size_t>(nx) * ny * nz;
  w->Np = static_cast<size_t>(nx) * ny * (static_cast<size_t>(nz) + kPadZ);

  // FP64 host tables
  const double ix2 = 1.0 / (p->dx * p->dx), iy2 = 1.0 / (p->dy * p->dy), iz2 = 1.0 / (p->dz * p->dz);
  w->c.k0a[0] = static_cast<float>(kC[0] * ix2);
  w->c.k0a[1] = static_cast<float>(kC[0] * iy2);
  w->c.k0a[2] = static_cast<float>(kC[0] * iz2);
  w->c.k0 = static_cast<float>(kC[0] * (ix2 + iy2 + iz2));
  for (int m = 1; m <= 4; ++m) {
    w->c.kx[m - 1] = static_cast<float>(kC[m] * ix2);
    w->c.ky[m - 1] = static_cast<float>(kC[m] * iy2);
    w->c.kz[m - 1] = static_cast<float>(kC[m] * iz2);
  }
  w->src_scale = static_cast<float>(p->dt * p->dt / (p->dx * p->dy * p->dz));
  const std::vector<float> gx = sponge_table(nx, p->sponge_width, p->sponge_alpha);
  const std::vector<float> gy = sponge_table(ny, p->sponge_width, p->sponge_alpha);
  std::vector<float> gz = sponge_table(nz, p->sponge_width, p->sponge_alpha);
  std::vector<int64_t> lin(p->nrec);
  for (int r = 0; r < p->nrec; ++r) {
    const int x = w->rec[3 * r], y = w->rec[3 * r + 1], z = w->rec[3 * r + 2];
    lin[r] = x + static_cast<int64_t>(nx) * (y + static_cast<int64_t>(ny) * z);
  }
  // receivers grouped by node, each group in receiver order: the adjoint
  // sums a node's residuals in that fixed order (duplicates included)
  std::vector<int32_t> ord(p->nrec), off;
  std::vector<int64_t> node;
  std::vector<float> grec;
  for (int r = 0; r < p->nrec; ++r) ord[r] = r;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return lin[a] < lin[b]; });
  for (int j = 0; j < p->nrec; ++j) {
    const int r = ord[j];
    if (node.empty() || node.back() != lin[r]) {
      const int x = w->rec[3 * r], y = w->rec[3 * r + 1], z = w->rec[3 * r + 2];
      node.push_back(lin[r]);
      off.push_back(j);
      grec.push_back(static_cast<float>(static_cast<double>(gx[x]) * gy[y] * gz[z]));
    }
  }
  off.push_back(p->nrec);
  w->nrec_nodes = static_cast<int>(node.size());
  w->fused_rec = detect_box(w->rec, p->nrec, &w->box);
  if (!w->fused_rec) w->box = RecBox{};
  // receiver-box plane index of every z-plane (-1: no receivers there); the
  // padding planes have sponge factor 0 (they stay zero) and no receivers
  std::vector<int32_t> rz(nz + kPadZ, -1);
  if (w->fused_rec)
    for (int l = 0; l < w->box.cnz; ++l) rz[w->box.z0 + l * w->box.sz] = l;

  // tiling: the forward step and (for adjoint contexts) the adjoint step
  // each get a shape; variant 0 picks the measured-best ones
  w->fwd = make_tiling(p, (p->variant > 0 && p->time_block == 0) ? p->variant : auto_variant(p));
  w->fwd.keep = p->cache_hint == 1;
  if (p->time_block == 2) w->pair = make_tiling(p, kPairVariant);
  if (p->adjoint) w->adj = make_tiling(p, p->variant > 0 ? p->variant : kAdjointVariant);

  StepState init{};
  init.vmin_bits = 0x7f800000u;
  init.vmax_bits = 0u;
  StepState back{};
  rc = hip_rc(hipMemcpyAsync(w->st, &init, sizeof(init), hipMemcpyHostToDevice, w->stream));
  if (!rc) rc = hip_rc(hipMemcpyAsync(w->gx, gx.data(), 4 * gx.size(), hipMemcpyHostToDevice, w->stream));
  if (!rc) rc = hip_rc(hipMemcpyAsync(w->gy, gy.data(), 4 * gy.size(), hipMemcpyHostToDevice, w->stream));
  gz.resize(nz + kPadZ, 0.f);
  if (!rc) rc = hip_rc(hipMemcpyAsync(w->gz, gz.data(), 4 * gz.size(), hipMemcpyHostToDevice, w->stream));
  if (!rc) rc = hip_rc(hipMemcpyAsync(w->rz, rz.data(), 4 * rz.size(), hipMemcpyHostToDevice, w->stream));
  if (!rc && p->nrec > 0) {
    rc = hip_rc(hipMemcpyAsync(w->rec_lin, lin.data(), 8 * lin.size(), hipMemcpyHostToDevice, w->stream));
    if (!rc) rc = hip_rc(hipMemcpyAsync(w->rec_node, node.data(), 8 * node.size(), hipMemcpyHostToDevice, w->stream));
    if (!rc) rc = hip_rc(hipMemcpyAsync(w->rec_off, off.data(), 4 * off.size(), hipMemcpyHostToDevice, w->stream));
    if (!rc) rc = hip_rc(hipMemcpyAsync(w->rec_ord, ord.data(), 4 * ord.size(), hipMemcpyHostToDevice, w->stream));
    if (!rc) rc = hip_rc(hipMemcpyAsync(w->grec, grec.data(), 4 * grec.size(), hipMemcpyHostToDevice, w->stream));
  }
  w->m16 = p->model_bits == 16;
  // float32 m is written by the range pass itself; 16-bit codes need the
  // range first (encoded below, once it is known on the host)
  if (!rc) rc = hip_rc(launch_init_m(vel_dev, w->m16 ? nullptr : w->m, w->N, static_cast<float>(p->dt), w->st,
                                     w->stream));
  if (!rc && !w->m16) rc = hip_rc(launch_fill_zero(w->m + w->N, 4 * (w->Np - w->N), w->stream));
  if (!rc) rc = hip_rc(hipMemcpyAsync(&back, w->st, sizeof(back), hipMemcpyDeviceToHost, w->stream));
  if (!rc) rc = hip_rc(hipStreamSynchronize(w->stream));
  if (!rc && (back.flags & 2u)) rc = WAVE_EINVAL;  // non-finite or non-positive velocity
  if (!rc) {
    float vmax;
    std::memcpy(&vmax, &back.vmax_bits, 4);
    const double Mmax = static_cast<double>(vmax) * p->dt * static_cast<double>(vmax) * p->dt;
    double dt_max = 0.0;
    if (wave_stable_dt(p, vmax, &dt_max) != WAVE_OK || p->dt > dt_max * (1.0 + 1e-12)) rc = WAVE_EUNSTABLE;
    // 16-bit scale bound: |M L A| <= Mmax (|k0| + sum_{a,m} 2 |c_m| / h_a^2) max|A|
    double kabs = 0.0;
    for (int m = 1; m <= 4; ++m) kabs += 2.0 * std::fabs(kC[m]) * (ix2 + iy2 + iz2);
    const double k0 = kC[0] * (ix2 + iy2 + iz2);
    w->gamma = static_cast<float>(Mmax * (std::fabs(k0) + kabs));
    if (!rc && w->m16) {  // codes of m = (v dt)^2 over [m_lo, m_hi] of this grid
      float vmin;
      std::memcpy(&vmin, &back.vmin_bits, 4);
      const float tlo = vmin * static_cast<float>(p->dt), thi = vmax * static_cast<float>(p->dt);
      w->m_lo = tlo * tlo;  // the float32 m of the extreme nodes, as the float32 path computes it
      w->m_step = (thi * thi - w->m_lo) / 65535.f;
      uint16_t *codes = reinterpret_cast<uint16_t *>(w->m);
      rc = hip_rc(launch_encode_m16(vel_dev, codes, w->N, static_cast<float>(p->dt), w->m_lo, w->m_step, w->stream));
      if (!rc) rc = hip_rc(launch_fill_zero(codes + w->N, 2 * (w->Np - w->N), w->stream));
    }
    if (!rc && p->cpml_width > 0) rc = setup_cpml(w, vmax);
    w->cpml_fused = w->cpml && variant_fuses_cpml(w->fwd.variant);
  }
  if (!rc && p->tune && p->variant == 0 && p->zchunk == 0 && p->time_block == 0) {
    rc = do_reset(w);  // zero fields (and CPML memory) for the timing runs
    if (!rc) rc = tune_forward(w);
  }
  if (!rc) rc = do_reset(w);
  if (rc) {
    delete w;
    return rc;
  }
  *out = w;
  return WAVE_OK;
}

}  // namespace

// A context in a device's static scratch array (the library's own memory):
// at most one per device at a time.
namespace {
std::mutex g_static_mu;
constexpr int kMaxStaticDevices = 64;
bool g_static_live[kMaxStaticDevices] = {};
}  // namespace

int wave::create_static_ctx(const wave_params *p, const float *vel_dev, void *scratch, size_t scratch_bytes,
                            void *hip_stream, wave_t *out, int device) {
  if (!p || !out || device < 0 || device >= kMaxStaticDevices) return WAVE_EINVAL;
  *out = nullptr;
  // no graph capture (instantiation allocates) and no tuning (its events)
  if (p->graph_steps != 0) return WAVE_EINVAL;
  wave_params q = *p;
  q.tune = 0;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_live[device]) return WAVE_ESTATE;
    g_static_live[device] = true;
  }
  const int rc = create_ctx(&q, vel_dev, scratch, scratch_bytes, hip_stream, out, device);
  if (rc) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_live[device] = false;
  }
  return rc;
}

extern "C" {

int wave_reset(wave_t w) {
  if (!w) return WAVE_EINVAL;
  return do_reset(w);
}

int wave_step(wave_t w, int32_t nsteps, const float *wavelet_dev, float *traces_dev) {
  if (!w || nsteps < 0) return WAVE_EINVAL;
  if (nsteps == 0) return WAVE_OK;
  if (w->p.src[0] >= 0 && !wavelet_dev) return WAVE_EINVAL;
  if (w->p.nrec > 0 && !traces_dev) return WAVE_EINVAL;
  return do_step(w, nsteps, wavelet_dev, traces_dev);
}

int wave_run(wave_t w, int32_t nt, const float *wavelet_dev, float *traces_dev) {
  if (!w || nt < 0) return WAVE_EINVAL;
  if (nt > 0 && w->p.src[0] >= 0 && !wavelet_dev) return WAVE_EINVAL;
  if (nt > 0 && w->p.nrec > 0 && !traces_dev) return WAVE_EINVAL;
  const int rc = do_reset(w);
  if (rc) return rc;
  return nt > 0 ? do_step(w, nt, wavelet_dev, traces_dev) : WAVE_OK;
}

int wave_adjoint(wave_t w, int32_t nt, const float *wavelet_dev, const float *resid_dev, float *grad_vel_dev) {
  if (!w) return WAVE_EINVAL;
  if (!w->p.adjoint) return WAVE_ESTATE;
  if (nt < 1 || nt > w->p.nt_max || !grad_vel_dev) return WAVE_EINVAL;
  if (w->p.src[0] >= 0 && !wavelet_dev) return WAVE_EINVAL;
  if (w->p.nrec > 0 && !resid_dev) return WAVE_EINVAL;
  const Layout &L = w->L;
  const int K = L.K;
  const size_t fb = 4 * w->N;  // bytes per float32 field
  float *ckpt = reinterpret_cast<float *>(w->ws + L.ckpt);
  float *seg = reinterpret_cast<float *>(w->ws + L.seg);
  float *mu1 = reinterpret_cast<float *>(w->ws + L.mua);  // mu^{k+1}
  float *mu2 = reinterpret_cast<float *>(w->ws + L.mub);  // mu^{k+2}
  float *img = reinterpret_cast<float *>(w->ws + L.img);
  auto slot = [&](int s) { return seg + static_cast<size_t>(s) * w->Np; };
  const int nseg = (nt + K - 1) / K;
  w->drop_graphs();

  // 1) forward run storing (A^{jK}, A^{jK-1}) for j = 1..nseg-1
  int rc = do_reset(w);
  for (int j = 1; j < nseg && !rc; ++j) {
    rc = enqueue_steps(w, K, wavelet_dev, nullptr, false);
    if (rc) break;
    w->n += K;
    float *ck = ckpt + 2 * static_cast<size_t>(j - 1) * w->N;
    rc = hip_rc(hipMemcpyAsync(ck, w->field(w->n), fb, hipMemcpyDeviceToDevice, w->stream));
    if (!rc) rc = hip_rc(hipMemcpyAsync(ck + w->N, w->field(w->n + 3), fb, hipMemcpyDeviceToDevice, w->stream));
  }
  // padded fields start zero (their padding planes stay zero)
  const size_t fbp = 4 * w->Np;
  if (!rc) rc = hip_rc(launch_fill_zero(mu1, fbp, w->stream));
  if (!rc) rc = hip_rc(launch_fill_zero(mu2, fbp, w->stream));
  if (!rc) rc = hip_rc(launch_fill_zero(img, fbp, w->stream));
  if (!rc) rc = hip_rc(launch_fill_zero(seg, fbp * (K + 2), w->stream));

  // 2) segments from last to first: recompute A^{jK+1..}, then adjoint steps
  for (int j = nseg - 1; j >= 0 && !rc; --j) {
    const int k_lo = j * K + 1, k_hi = std::min((j + 1) * K, nt);
    if (j == 0) {
      rc = hip_rc(launch_fill_zero(slot(0), fb, w->stream));
      if (!rc) rc = hip_rc(launch_fill_zero(slot(1), fb, w->stream));
    } else {
      const float *ck = ckpt + 2 * static_cast<size_t>(j - 1) * w->N;
      rc = hip_rc(hipMemcpyAsync(slot(1), ck, fb, hipMemcpyDeviceToDevice, w->stream));
      if (!rc) rc = hip_rc(hipMemcpyAsync(slot(0), ck + w->N, fb, hipMemcpyDeviceToDevice, w->stream));
    }
    if (!rc) rc = hip_rc(launch_set_n(w->st, j * K, w->stream));
    // slot s holds A^{jK - 1 + s}
    StepArgs a = base_args(w, w->fwd);
    a.wavelet = wavelet_dev;
    for (int k = 0; k < k_hi - j * K && !rc; ++k) {
      a.cur = slot(k + 1);
      a.prev = slot(k);
      a.out = slot(k + 2);
      a.k = k;
      rc = hip_rc(launch_step(WAVE_F32, w->fwd.variant, false, a, w->stream));
    }
    StepArgs b = base_args(w, w->adj);
    b.sx = -1;
    b.img = img;
    b.resid = resid_dev;
    if (w->fused_rec) b.box = w->box;
    for (int k = k_hi; k >= k_lo && !rc; --k) {
      b.cur = mu1;
      b.prev = mu2;
      b.out = mu2;  // mu^k overwrites mu^{k+2}
      b.fwd = slot(k - j * K + 1);
      b.resid_row = k - 1;
      rc = hip_rc(launch_step(WAVE_F32, w->adj.variant, true, b, w->stream));
      if (!rc && !w->fused_rec && w->p.nrec > 0)
        rc = hip_rc(launch_scatter(mu2, w->rec_node, w->rec_off, w->rec_ord, w->nrec_nodes, w->p.nrec, w->m, w->grec,
                                   resid_dev, k - 1, w->stream));
      std::swap(mu1, mu2);
    }
  }
  if (!rc) rc = hip_rc(launch_grad_final(img, w->m, static_cast<float>(w->p.dt), grad_vel_dev, w->N, w->stream));
  if (!rc) rc = do_reset(w);
  return rc;
}

int wave_read_field(wave_t w, int32_t which, float *out_dev) {
  if (!w || !out_dev || which < 0 || which > 2) return WAVE_EINVAL;
  const bool f32 = w->p.storage == WAVE_F32;
  if (which == 0)
    return hip_rc(launch_decode(w->p.storage, w->field(w->n), out_dev, w->N, w->st, 0, false, w->stream));
  if (which == 2) {
    if (f32) return WAVE_EINVAL;
    return hip_rc(launch_decode(w->p.storage, w->fv, out_dev, w->N, w->st, 0, true, w->stream));
  }
  if (f32)
    return hip_rc(launch_decode(w->p.storage, w->field(w->n + 3), out_dev, w->N, w->st, 3, false, w->stream));
  return hip_rc(launch_decode_prev(w->p.storage, w->field(w->n), w->fv, out_dev, w->gx, w->gy, w->gz, w->p.nx,
                                   w->p.ny, w->p.nz, w->st, w->stream));
}

int wave_write_field(wave_t w, int32_t which, const float *in_dev) {
  if (!w || !in_dev) return WAVE_EINVAL;
  if (w->p.storage == WAVE_F32) {
    if (which < 0 || which > 1) return WAVE_EINVAL;
    void *dst = w->field(which == 0 ? w->n : w->n + 3);
    return hip_rc(hipMemcpyAsync(dst, in_dev, 4 * w->N, hipMemcpyDeviceToDevice, w->stream));
  }
  if (which != 0 && which != 2) return WAVE_EINVAL;  // 16-bit storage keeps A^n and V^n
  return hip_rc(launch_encode_field(w->p.storage, in_dev, which == 0 ? w->field(w->n) : w->fv, w->N, w->st,
                                    which == 2, w->stream));
}

// Snapshot layout: 256-B header | step state | A fields 0 and 1 | V (16-bit)
// | CPML slabs, each section 256-B aligned; interiors only (the padding
// planes are zero in every context).
namespace {
struct StateHeader {
  uint64_t magic, bytes, field_bytes, slab_bytes;
  int32_t n, nx, ny, nz, storage, cpml_width, pad[2];
};
constexpr uint64_t kStateMagic = 0x31544154534556ull;  // "VESTAT1"

size_t state_bytes(const wave_ctx *w, size_t *field_bytes, size_t *slabs) {
  const size_t es = w->p.storage == WAVE_F32 ? 4 : 2;
  *field_bytes = es * w->N;
  *slabs = 0;
  if (w->cpml)
    for (int a = 0; a < 3; ++a) *slabs += slab_bytes(w, a);
  const int nfields = w->p.storage == WAVE_F32 ? 2 : 3;
  return 256 + 256 + nfields * align256(*field_bytes) + align256(*slabs);
}
}  // namespace

int wave_state_bytes(wave_t w, size_t *bytes) {
  if (!w || !bytes) return WAVE_EINVAL;
  size_t fb, sb;
  *bytes = state_bytes(w, &fb, &sb);
  return WAVE_OK;
}

int wave_save_state(wave_t w, void *dst_dev) {
  if (!w || !dst_dev) return WAVE_EINVAL;
  size_t fb, sb;
  const size_t total = state_bytes(w, &fb, &sb);
  StateHeader h{};
  h.magic = kStateMagic;
  h.bytes = total;
  h.field_bytes = fb;
  h.slab_bytes = sb;
  h.n = w->n;
  h.nx = w->p.nx;
  h.ny = w->p.ny;
  h.nz = w->p.nz;
  h.storage = w->p.storage;
  h.cpml_width = w->p.cpml_width;
  h.pad[0] = w->p.time_block;
  char *d = static_cast<char *>(dst_dev);
  int rc = hip_rc(hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, w->stream));
  if (!rc) rc = hip_rc(hipMemcpyAsync(d + 256, w->st, sizeof(StepState), hipMemcpyDeviceToDevice, w->stream));
  size_t off = 512;
  // the two stored levels: by buffer, or by role (A^n, A^{n-1}) when they
  // rotate through four buffers
  void *fields[3] = {w->fa, w->fb, w->fv};
  if (w->p.time_block == 2) {
    fields[0] = w->field(w->n);
    fields[1] = w->field(w->n + 3);
  }
  const int nfields = w->p.storage == WAVE_F32 ? 2 : 3;
  for (int k = 0; k < nfields && !rc; ++k, off += align256(fb))
    rc = hip_rc(hipMemcpyAsync(d + off, fields[k], fb, hipMemcpyDeviceToDevice, w->stream));
  for (int a = 0; a < 3 && w->cpml && !rc; ++a) {
    rc = hip_rc(hipMemcpyAsync(d + off, w->ws + w->L.cpml_slab[a], slab_bytes(w, a), hipMemcpyDeviceToDevice,
                               w->stream));
    off += slab_bytes(w, a);
  }
  if (!rc) rc = hip_rc(hipStreamSynchronize(w->stream));  // the header's host copy stays valid until here
  return rc;
}

int wave_load_state(wave_t w, const void *src_dev) {
  if (!w || !src_dev) return WAVE_EINVAL;
  size_t fb, sb;
  const size_t total = state_bytes(w, &fb, &sb);
  StateHeader h{};
  const char *src = static_cast<const char *>(src_dev);
  int rc = hip_rc(hipMemcpyAsync(&h, src, sizeof(h), hipMemcpyDeviceToHost, w->stream));
  if (!rc) rc = hip_rc(hipStreamSynchronize(w->stream));
  if (rc) return rc;
  if (h.magic != kStateMagic || h.bytes != total || h.field_bytes != fb || h.slab_bytes != sb || h.nx != w->p.nx ||
      h.ny != w->p.ny || h.nz != w->p.nz || h.storage != w->p.storage || h.cpml_width != w->p.cpml_width || h.n < 0 ||
      h.pad[0] != w->p.time_block)
    return WAVE_EINVAL;
  rc = hip_rc(hipMemcpyAsync(w->st, src + 256, sizeof(StepState), hipMemcpyDeviceToDevice, w->stream));
  size_t off = 512;
  void *fields[3] = {w->fa, w->fb, w->fv};
  if (w->p.time_block == 2) {
    fields[0] = w->field(h.n);
    fields[1] = w->field(h.n + 3);
  }
  const int nfields = w->p.storage == WAVE_F32 ? 2 : 3;
  for (int k = 0; k < nfields && !rc; ++k, off += align256(fb))
    rc = hip_rc(hipMemcpyAsync(fields[k], src + off, fb, hipMemcpyDeviceToDevice, w->stream));
  for (int a = 0; a < 3 && w->cpml && !rc; ++a) {
    rc = hip_rc(hipMemcpyAsync(w->ws + w->L.cpml_slab[a], src + off, slab_bytes(w, a), hipMemcpyDeviceToDevice,
                               w->stream));
    off += slab_bytes(w, a);
  }
  if (!rc) rc = hip_rc(hipStreamSynchronize(w->stream));
  if (!rc) w->n = h.n;
  return rc;
}

int wave_time_index(wave_t w, int32_t *n) {
  if (!w || !n) return WAVE_EINVAL;
  *n = w->n;
  return WAVE_OK;
}

int wave_sync_status(wave_t w, uint32_t *flags) {
  if (!w || !flags) return WAVE_EINVAL;
  int rc = hip_rc(launch_check_finite(w->p.storage, w->field(w->n), w->N, w->st, w->stream));
  StepState back{};
  if (!rc) rc = hip_rc(hipMemcpyAsync(&back, w->st, sizeof(back), hipMemcpyDeviceToHost, w->stream));
  if (!rc) rc = hip_rc(hipStreamSynchronize(w->stream));
  if (!rc) *flags = back.flags & WAVE_FLAG_NONFINITE;
  return rc;
}

int wave_destroy(wave_t w) {
  if (!w) return WAVE_EINVAL;
  int rc = WAVE_OK;
  const int dev = w->static_dev;
  if (dev >= 0) {
    // the next static context on this device reuses the same memory: let
    // this one's queued work finish first
    rc = hip_rc(hipStreamSynchronize(w->stream));
  }
  delete w;
  if (dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_live[dev] = false;
  }
  return rc;
}

int wave_variant_count(void) { return variant_count(); }

int wave_tiling(wave_t w, int32_t *out) {
  if (!w || !out) return WAVE_EINVAL;
  // variant 0 (automatic) runs its fallback shape: report the explicit
  // variant with that shape
  int v = w->p.time_block == 2 ? w->pair.variant : w->fwd.variant;
  for (int k = 1; v == 0 && k < variant_count(); ++k) {
    const Variant a = variant_info(0), b = variant_info(k);
    if (a.family == b.family && a.by == b.by && a.ry == b.ry && a.pd == b.pd && a.vec == b.vec) v = k;
  }
  out[0] = v;
  out[1] = w->p.time_block == 2 ? w->pair.zchunk : w->fwd.zchunk;
  out[2] = w->fwd.keep ? 1 : 0;
  return WAVE_OK;
}

int wave_variant_info(int32_t variant, int32_t *info) {
  if (!info || variant < 0 || variant >= variant_count()) return WAVE_EINVAL;
  const Variant v = variant_info(variant);
  info[0] = v.family;
  info[1] = v.by;
  info[2] = v.ry;
  info[3] = v.pd;
  info[4] = v.vec;
  return WAVE_OK;
}

const char *wave_status_string(int status) {
  switch (status) {
    case WAVE_OK: return "ok";
    case WAVE_EINVAL: return "invalid argument";
    case WAVE_EUNSTABLE: return "time step above the stability limit";
    case WAVE_ENOSPC: return "workspace too small";
    case WAVE_EHIP: return "HIP runtime error";
    case WAVE_ESTATE: return "call not valid for this context";
    default: return "unknown status";
  }
}

}  // extern "C"
