// Batched mixed-precision solves: many independent problems of different sizes
// solved together, each pass of the six-product FD solve of eq. 3D-Poisson and
// each FP64 residual launched once for the whole batch.
//
// A solve call builds, for every pass, one descriptor per solve (operands,
// geometry, epilogue, tile range in the launch's global tile numbering); the FP32
// pass kernel runs persistently over all tiles of all solves, and the residual
// kernel over all blocks of all solves with the same element degree k.  Solves
// that meet the tolerance drop out through a per-solve active flag, so later
// iterations only work on the rest.
//
// Split-BF16 batches (SEM_BF16X3): a solve whose every dimension reaches
// SPLIT_MIN_DIM runs the split-BF16 passes of the single solves (right-hand-side
// conversion, six DMA mode products, residual written as split BF16), one launch
// per pass, on one of NSIDE side streams; the side streams run concurrently with
// each other and with the persistent FP32 launches of the other solves on the
// batch stream, so a small pass need not fill the chip by itself.  These passes
// are 1.3-2.3x faster than the FP32 ones from n = 191 to 511 when run alone;
// with the concurrency the batch time is flat for thresholds of 48..96 (245-249
// ms for the 256-problem workload) and grows above (270 ms at 160, 343 at 256).
// Both paths refine in FP64 to the same tolerance.
//
// Tile shape: the FP32 kernel has 128 x 128, 96 x 128, 64 x 128 and 32 x 128 block tiles
// (factor rows x tensor rows).  Short contraction lengths waste most of a
// 128-row factor tile, so the shape is chosen per length bucket (16, 32, 64, 128,
// 256, 512 and above) by timing the candidates on the batch's own passes when the
// batch is created (an autotuner).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"
#include "plan_internal.h"
#include "tune.h"

namespace semfd {
namespace {

constexpr int NBUCKET = 6;
constexpr int SPLIT_MIN_DIM = 96;
// side streams of the split-BF16 solves (with the batch stream: the four hardware
// queues a process gets by default)
constexpr int NSIDE = 3;
constexpr int TUNE_REPS = 5;
constexpr int TILE_CANDIDATES[4] = {128, 96, 64, 32};
// pass variants: 0 = forward z from f (FP64 input), 1 = forward z from r,
// 2..5 = passes 1..4 (2 ... 4 = forward y, forward x + divide, backward z, backward y),
// 6 = backward x storing u (first iteration), 7 = backward x accumulating into u
constexpr int NVAR = 8;

int bucket_of(int L) {
  int b = 0;
  for (int cap = 16; b < NBUCKET - 1 && L > cap; cap *= 2) ++b;
  return b;
}

inline int pad8(int n) { return (n + 7) / 8 * 8; }

__global__ void zero_u64_n(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

struct Group {
  int var, tile_rows;
  int off, count;  // range in the descriptor array
  long tiles;
};

}  // namespace
}  // namespace semfd

using namespace semfd;

struct sem_batch {
  int count = 0;
  std::vector<sem_plan*> plans;
  std::vector<LpWork> lw;
  // entries whose plan already occurred earlier in the list (several right-hand
  // sides of one operator) get a workspace of their own
  std::vector<char> repeat;
  std::vector<void*> own_ws;
  std::vector<size_t> own_bytes;
  hipStream_t stream = nullptr;
  int cus = 1;
  char arch[64] = "unknown";  // device architecture name, part of the tuning-cache keys
  int tile_rows[NBUCKET] = {0, 0, 0, 0, 0, 0};
  LpDesc* d_desc = nullptr;
  ResDesc* d_rdesc = nullptr;
  int* d_active = nullptr;
  unsigned long long* d_norms = nullptr;
  std::vector<LpDesc> h_desc;
  std::vector<ResDesc> h_rdesc;
  std::vector<Group> groups;
  std::vector<Group> rgroups;  // residual groups: var = k
  hipStream_t side[NSIDE] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_start = nullptr;
  hipEvent_t ev_side[NSIDE] = {nullptr, nullptr, nullptr};
};

namespace semfd {
namespace {

// Geometry of pass s (0..5) of plan p: contracted axis, input/output pitches and
// rotated shapes, as in lp_fd.
struct PassGeo {
  int axis, dir, A, B, K, ldx, ldy;
};
PassGeo pass_geo(const sem_plan* p, int s) {
  const int nx = p->dims[0], ny = p->dims[1], nz = p->dims[2];
  switch (s) {
    case 0: return {2, 0, nx, ny, nz, pad8(nz), pad8(ny)};
    case 1: return {1, 0, nz, nx, ny, pad8(ny), pad8(nx)};
    case 2: return {0, 0, ny, nz, nx, pad8(nx), pad8(nz)};
    case 3: return {2, 1, nx, ny, nz, pad8(nz), pad8(ny)};
    case 4: return {1, 1, nz, nx, ny, pad8(ny), pad8(nx)};
    default: return {0, 1, ny, nz, nx, pad8(nx), nz};
  }
}

// Descriptor of variant v for solve i (f, u may be null while tuning).
LpDesc make_desc(sem_batch* b, int i, int v, const double* f, double* u) {
  sem_plan* p = b->plans[i];
  const LpWork& w = b->lw[i];
  const int s = v <= 1 ? 0 : (v >= 6 ? 5 : v - 1);
  const PassGeo g = pass_geo(p, s);
  LpDesc d;
  d.P = (long)g.A * g.B;
  d.K = g.K;
  d.L = g.K;
  d.A = g.A;
  d.B = g.B;
  d.ldx = g.ldx;
  d.ldy = g.ldy;
  d.f = p->lp_f32[g.axis][g.dir];
  d.ldf = p->lp_ld[g.axis];
  d.sid = i;
  // operands: r -> t0 -> t1 -> t0 -> t1 -> t0 -> u
  const void* in[6] = {w.r, w.t0, w.t1, w.t0, w.t1, w.t0};
  void* out[6] = {w.t0, w.t1, w.t0, w.t1, w.t0, (void*)u};
  d.x = in[s];
  d.y = out[s];
  if (v == 0) {
    d.x = f;
    d.ldx = p->dims[2];
  }
  if (s == 2) {
    d.epi.l0 = p->d_lam[0];
    d.epi.l1 = p->d_lam[1];
    d.epi.l2 = p->d_lam[2];
    d.epi.alpha = p->alpha;
    d.epi.b1 = 1.0;
    d.epi.b2 = 0.0;
  }
  if (s == 5) {
    d.epi.first = v == 6 ? 1 : 0;
    d.epi.norms = b->d_norms + 2 * i;
  }
  return d;
}

int tile_for(const sem_batch* b, int L) {
  const int t = b->tile_rows[bucket_of(L)];
  return t ? t : 128;
}

// Build all pass descriptors (grouped by variant and tile shape) and the residual
// descriptors (grouped by k) for one solve call.
// Solves with skip[i] set run outside the persistent launches and get no descriptor.
sem_status build_descs(sem_batch* b, const double* const* f, double* const* u, const std::vector<char>& skip) {
  b->h_desc.clear();
  b->groups.clear();
  for (int v = 0; v < NVAR; ++v)
    for (int tr : TILE_CANDIDATES) {
      Group g{v, tr, (int)b->h_desc.size(), 0, 0};
      for (int i = 0; i < b->count; ++i) {
        if (skip[i]) continue;
        LpDesc d = make_desc(b, i, v, f ? f[i] : nullptr, u ? u[i] : nullptr);
        if (tile_for(b, d.L) != tr) continue;
        d.tiles_l = (d.L + tr - 1) / tr;
        d.tile0 = g.tiles;
        g.tiles += (long)d.tiles_l * ((d.P + 127) / 128);
        b->h_desc.push_back(d);
        ++g.count;
      }
      if (g.count) b->groups.push_back(g);
    }
  b->h_rdesc.clear();
  b->rgroups.clear();
  for (int k = 1; k <= 8; ++k) {
    Group g{k, 0, (int)b->h_rdesc.size(), 0, 0};
    for (int i = 0; i < b->count; ++i) {
      sem_plan* p = b->plans[i];
      if (p->k != k || skip[i]) continue;
      ResidualArgs ra;
      ra.periodic = p->per_mask;
      ra.v = u ? u[i] : nullptr;
      ra.f = f ? f[i] : nullptr;
      ra.r = b->lw[i].r;
      ra.r_kind = 1;
      ra.ldr = b->lw[i].ldr;
      ra.cf = 1.0;
      ra.cd = p->alpha;
      ra.ch = 1.0;
      const double* hb[3] = {p->d_hb[0], p->d_hb[1], p->d_hb[2]};
      ResDesc rd;
      if (!residual_desc(ra, hb, k, p->dims, &rd)) return set_error(SEM_EINVAL, "sem_batch: residual descriptor");
      rd.sid = i;
      rd.block0 = g.tiles;
      g.tiles += (long)rd.gx * rd.gy * rd.gz;
      b->h_rdesc.push_back(rd);
      ++g.count;
    }
    if (g.count) b->rgroups.push_back(g);
  }
  hipError_t e = hipSuccess;
  if (!b->h_desc.empty())
    e = hipMemcpy(b->d_desc, b->h_desc.data(), b->h_desc.size() * sizeof(LpDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess && !b->h_rdesc.empty())
    e = hipMemcpy(b->d_rdesc, b->h_rdesc.data(), b->h_rdesc.size() * sizeof(ResDesc), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "sem_batch: descriptor upload");
  return SEM_OK;
}

hipError_t launch_group(sem_batch* b, const Group& g) {
  const int v = g.var;
  const int in_kind = v == 0 ? 0 : 1;
  const int out_kind = v >= 6 ? 0 : 1;
  const int epi = v >= 6 ? EPI_ACCUM : (v == 3 ? EPI_DIVIDE : EPI_STORE);
  const int grid = b->cus * lp_batch_blocks_per_cu(g.tile_rows);
  return launch_mode_f32_batch(in_kind, out_kind, epi, g.tile_rows, b->d_desc + g.off, g.count, g.tiles, b->d_active,
                               grid, b->stream);
}

hipError_t run_variant(sem_batch* b, int v) {
  for (const Group& g : b->groups)
    if (g.var == v) {
      hipError_t e = launch_group(b, g);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

// Time the candidate tile shapes on the batch's own forward-y passes, per bucket.
sem_status autotune(sem_batch* b) {
  // descriptors: a forward pass along every axis of every solve, FP32 in and out
  // inside the solve's own workspace (contents irrelevant for timing)
  std::vector<int> ones(b->count, 1);
  hipError_t e = hipMemcpy(b->d_active, ones.data(), ones.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "sem_batch: autotune");
  hipEvent_t t0, t1;
  if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess)
    return hip_fail(e, "sem_batch: autotune events");
  sem_status st = SEM_OK;
  for (int bk = 0; bk < NBUCKET && st == SEM_OK; ++bk) {
    std::vector<LpDesc> base;
    long work = 0;
    for (int i = 0; i < b->count; ++i)
      for (int s : {1, 2, 3}) {  // variants 2, 3, 4 = passes along y, x, z
        LpDesc d = make_desc(b, i, s + 1, nullptr, nullptr);
        if (bucket_of(d.L) != bk) continue;
        d.epi = EpiLP();
        base.push_back(d);
        work += d.P * (long)d.L;
      }
    if (base.empty()) continue;
    // the tuning cache holds the choice per device, length bucket and log2 of the
    // bucket's work (rows x length summed over its passes)
    char key[128];
    std::snprintf(key, sizeof(key), "%s|batch_f32|Lb%d|W%d", b->arch, bk, tune_bucket(work));
    int cached = 0;
    if (tune_lookup(key, &cached)) {
      b->tile_rows[bk] = cached;
      continue;
    }
    float best = INFINITY;
    int best_tr = 128;
    for (int tr : TILE_CANDIDATES) {
      std::vector<LpDesc> ds = base;
      long tiles = 0;
      for (LpDesc& d : ds) {
        d.tiles_l = (d.L + tr - 1) / tr;
        d.tile0 = tiles;
        tiles += (long)d.tiles_l * ((d.P + 127) / 128);
      }
      if ((e = hipMemcpy(b->d_desc, ds.data(), ds.size() * sizeof(LpDesc), hipMemcpyHostToDevice)) != hipSuccess) {
        st = hip_fail(e, "sem_batch: autotune upload");
        break;
      }
      const int grid = b->cus * lp_batch_blocks_per_cu(tr);
      // one warm-up launch, then the fastest of TUNE_REPS timed launches (the small
      // buckets run for microseconds, where single timings are noisy)
      float ms = INFINITY;
      e = launch_mode_f32_batch(1, 1, EPI_STORE, tr, b->d_desc, (int)ds.size(), tiles, b->d_active, grid, b->stream);
      for (int rep = 0; rep < TUNE_REPS && e == hipSuccess; ++rep) {
        float one = 0.f;
        e = hipEventRecord(t0, b->stream);
        if (e == hipSuccess)
          e = launch_mode_f32_batch(1, 1, EPI_STORE, tr, b->d_desc, (int)ds.size(), tiles, b->d_active, grid,
                                    b->stream);
        if (e == hipSuccess) e = hipEventRecord(t1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        if (e == hipSuccess) e = hipEventElapsedTime(&one, t0, t1);
        ms = std::min(ms, one);
      }
      if (e != hipSuccess) {
        st = hip_fail(e, "sem_batch: autotune run");
        break;
      }
      if (ms < best) {
        best = ms;
        best_tr = tr;
      }
    }
    b->tile_rows[bk] = best_tr;
    tune_store(key, best_tr);
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  return st;
}

// Low-precision factors of entry i's plan and the entry's workspace laid out for
// prec: the plan's own workspace, or for a repeated plan the entry's own one.
// Split-BF16 entries run the plan's own passes, whose launch shapes are tuned per
// plan; the FP32 entries run the batch's grouped launches (tuned by autotune).
sem_status prepare_entry(sem_batch* b, int i, sem_prec prec) {
  sem_plan* p = b->plans[i];
  if (!b->repeat[i]) return lp_prepare(p, prec, &b->lw[i], prec != SEM_F32);
  sem_status st = lp_factors(p, prec);
  if (st != SEM_OK) return st;
  const size_t need = workspace_need(p, prec);
  if (b->own_bytes[i] < need) {
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "sem_batch: workspace resize");
    (void)hipFree(b->own_ws[i]);
    b->own_ws[i] = nullptr;
    b->own_bytes[i] = 0;
    if ((e = hipMalloc(&b->own_ws[i], need)) != hipSuccess) {
      b->own_ws[i] = nullptr;
      return hip_fail(e, "sem_batch: workspace allocation");
    }
    b->own_bytes[i] = need;
  }
  return lp_layout(p, prec, b->own_ws[i], &b->lw[i]);
}

// One refinement iteration of solve i in split BF16 on `stream`: the FP64
// residual written as split BF16 (from the second iteration on), then the FD
// application that stores (first iteration) or accumulates the update into u and
// leaves max|delta|, max|u| in the solve's norm slots.
hipError_t split_iteration(sem_batch* b, int i, int it, const double* f, double* u, hipStream_t stream) {
  sem_plan* p = b->plans[i];
  const LpWork& w = b->lw[i];
  hipStream_t keep = p->stream;
  p->stream = stream;
  hipError_t e = hipSuccess;
  if (it > 0) {
    ResidualArgs ra;  // r = f - alpha u - H_3 u
    ra.periodic = p->per_mask;
    ra.v = u;
    ra.f = f;
    ra.r = w.r;
    ra.r_kind = w.rkind;
    ra.ldr = w.ldr;
    ra.rplane = w.rplane;
    ra.cf = 1.0;
    ra.cd = p->alpha;
    ra.ch = 1.0;
    const double* hb[3] = {p->d_hb[0], p->d_hb[1], p->d_hb[2]};
    e = launch_residual(ra, hb, p->k, p->dims, stream);
  }
  if (e == hipSuccess)
    e = lp_fd(p, w, Spectral{p->alpha, 1.0, 0.0}, it == 0 ? f : nullptr, u, it == 0 ? 1 : 0, b->d_norms + 2 * i);
  p->stream = keep;
  return e;
}

}  // namespace
}  // namespace semfd

extern "C" {

void sem_batch_destroy(sem_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (int s = 0; s < NSIDE; ++s) {
    if (b->side[s]) {
      (void)hipStreamSynchronize(b->side[s]);
      (void)hipStreamDestroy(b->side[s]);
    }
    if (b->ev_side[s]) (void)hipEventDestroy(b->ev_side[s]);
  }
  if (b->ev_start) (void)hipEventDestroy(b->ev_start);
  for (void* w : b->own_ws) (void)hipFree(w);
  (void)hipFree(b->d_desc);
  (void)hipFree(b->d_rdesc);
  (void)hipFree(b->d_active);
  (void)hipFree(b->d_norms);
  delete b;
}

sem_status sem_batch_create(int count, sem_plan* const* plans, sem_batch** out) {
  if (!out) return set_error(SEM_EINVAL, "sem_batch_create: null output");
  *out = nullptr;
  if (count < 1 || !plans) return set_error(SEM_EINVAL, "sem_batch_create: need count >= 1 plans");
  int dev = -1;
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return set_error(SEM_EINVAL, "sem_batch_create: null plan");
    if (plans[i]->k > 8) return set_error(SEM_EINVAL, "sem_batch_create: batched residual supports k <= 8");
    if (i == 0) dev = plans[i]->device;
    if (plans[i]->device != dev) return set_error(SEM_EINVAL, "sem_batch_create: plans on different devices");
  }
  sem_batch* b = new (std::nothrow) sem_batch;
  if (!b) return set_error(SEM_ENOMEM, "sem_batch_create: host allocation");
  b->count = count;
  b->plans.assign(plans, plans + count);
  b->lw.resize(count);
  b->repeat.assign(count, 0);
  b->own_ws.assign(count, nullptr);
  b->own_bytes.assign(count, 0);
  for (int i = 0; i < count; ++i)
    for (int j = 0; j < i && !b->repeat[i]; ++j) b->repeat[i] = plans[j] == plans[i];
  for (int i = 0; i < count; ++i) {
    sem_status st = prepare_entry(b, i, SEM_F32);
    if (st != SEM_OK) {
      sem_batch_destroy(b);
      return st;
    }
  }
  hipError_t e;
  int cus = 0;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) {
    sem_batch_destroy(b);
    return hip_fail(e, "sem_batch_create: device query");
  }
  b->cus = cus > 0 ? cus : 1;
  {
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) {
      sem_batch_destroy(b);
      return hip_fail(e, "sem_batch_create: device query");
    }
    std::snprintf(b->arch, sizeof(b->arch), "%s", prop.gcnArchName);
    for (char* c = b->arch; *c; ++c)
      if (*c == ':') *c = '_';
  }
  if ((e = hipMalloc(&b->d_desc, sizeof(LpDesc) * (size_t)std::max(NVAR * count, 3 * count))) != hipSuccess ||
      (e = hipMalloc(&b->d_rdesc, sizeof(ResDesc) * (size_t)count)) != hipSuccess ||
      (e = hipMalloc(&b->d_active, sizeof(int) * (size_t)count)) != hipSuccess ||
      (e = hipMalloc(&b->d_norms, 2 * sizeof(unsigned long long) * (size_t)count)) != hipSuccess) {
    sem_batch_destroy(b);
    return hip_fail(e, "sem_batch_create: device allocation");
  }
  for (int s = 0; s < NSIDE && e == hipSuccess; ++s) {
    e = hipStreamCreateWithFlags(&b->side[s], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_side[s], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_start, hipEventDisableTiming);
  if (e != hipSuccess) {
    sem_batch_destroy(b);
    return hip_fail(e, "sem_batch_create: side streams");
  }
  sem_status st = autotune(b);
  if (st != SEM_OK) {
    sem_batch_destroy(b);
    return st;
  }
  *out = b;
  return SEM_OK;
}

sem_status sem_batch_set_stream(sem_batch* b, void* s) {
  if (!b) return set_error(SEM_EINVAL, "sem_batch_set_stream: null handle");
  b->stream = (hipStream_t)s;
  return SEM_OK;
}

sem_status sem_batch_tile_rows(const sem_batch* b, int rows[6]) {
  if (!b || !rows) return set_error(SEM_EINVAL, "sem_batch_tile_rows: null argument");
  for (int k = 0; k < NBUCKET; ++k) rows[k] = b->tile_rows[k];
  return SEM_OK;
}

sem_status sem_batch_solve(sem_batch* b, sem_prec prec, double tol, int max_iter, const double* const* f,
                           double* const* u, int* iters) {
  if (!b || !f || !u || max_iter < 1 || !(tol >= 0.0) || !std::isfinite(tol))
    return set_error(SEM_EINVAL, "sem_batch_solve: invalid argument");
  for (int i = 0; i < b->count; ++i) {
    if (!f[i] || !u[i]) return set_error(SEM_EINVAL, "sem_batch_solve: null array");
    if (f[i] == u[i]) return set_error(SEM_EINVAL, "sem_batch_solve: u must not alias f");
    if (iters) iters[i] = 0;
  }
  if (prec == SEM_F64) {  // FP64 solves one after another on the batch stream
    for (int i = 0; i < b->count; ++i) {
      sem_plan* p = b->plans[i];
      hipStream_t keep = p->stream;
      p->stream = b->stream;
      sem_status st = sem_solve(p, f[i], u[i]);
      p->stream = keep;
      if (st != SEM_OK) return st;
      if (iters) iters[i] = 1;
    }
    return SEM_OK;
  }
  if (prec != SEM_F32 && prec != SEM_BF16X3)
    return set_error(SEM_EINVAL, "sem_batch_solve: batched solves run in SEM_F32, SEM_BF16X3 or SEM_F64");
  const int n = b->count;
  // which solves run in split BF16; every solve's workspace is (re)laid out for
  // this call, since a plan's workspace may have moved since the last one
  std::vector<char> split(n, 0);
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "sem_batch_solve: stream");
  for (int i = 0; i < n; ++i) {
    const int* d = b->plans[i]->dims;
    split[i] = prec == SEM_BF16X3 && std::min({d[0], d[1], d[2]}) >= SPLIT_MIN_DIM;
    sem_status st = prepare_entry(b, i, split[i] ? SEM_BF16X3 : SEM_F32);
    if (st != SEM_OK) return st;
  }
  sem_status st = build_descs(b, f, u, split);
  if (st != SEM_OK) return st;
  // split solves: largest first onto the least-loaded side stream (cost ~ N (nx + ny + nz))
  std::vector<int> order, lane(n, 0);
  for (int i = 0; i < n; ++i)
    if (split[i]) order.push_back(i);
  auto cost = [&](int i) {
    const int* d = b->plans[i]->dims;
    return (double)d[0] * d[1] * d[2] * (d[0] + d[1] + d[2]);
  };
  std::sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  double load[NSIDE] = {0.0, 0.0, 0.0};
  for (int i : order) {
    int s = 0;
    for (int t = 1; t < NSIDE; ++t)
      if (load[t] < load[s]) s = t;
    lane[i] = s;
    load[s] += cost(i);
  }
  // on an error after side-stream work was queued, wait for it before returning
  auto drain = [&]() {
    for (int s = 0; s < NSIDE; ++s) (void)hipStreamSynchronize(b->side[s]);
  };
  std::vector<int> active(n, 1), done_it(n, 0), dev_active(n, 0);
  std::vector<double> prev(n, INFINITY), prev2(n, INFINITY);
  std::vector<unsigned long long> hn(2 * n);
  sem_status result = SEM_OK;
  for (int it = 0; it < max_iter; ++it) {
    // the persistent launches see only the unconverged solves that they run
    for (int i = 0; i < n; ++i) dev_active[i] = active[i] && !split[i];
    if ((e = hipMemcpyAsync(b->d_active, dev_active.data(), n * sizeof(int), hipMemcpyHostToDevice, b->stream)) !=
        hipSuccess)
      return hip_fail(e, "sem_batch_solve: active flags");
    zero_u64_n<<<(2 * n + 255) / 256, 256, 0, b->stream>>>(b->d_norms, 2 * n);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "sem_batch_solve: norm reset");
    // split solves on the side streams, after the norm reset and concurrently with
    // the persistent launches below
    if (!order.empty()) {
      if ((e = hipEventRecord(b->ev_start, b->stream)) != hipSuccess) return hip_fail(e, "sem_batch_solve: event");
      for (int s = 0; s < NSIDE; ++s)
        if ((e = hipStreamWaitEvent(b->side[s], b->ev_start, 0)) != hipSuccess)
          return hip_fail(e, "sem_batch_solve: event");
      for (int i : order)
        if (active[i] && (e = split_iteration(b, i, it, f[i], u[i], b->side[lane[i]])) != hipSuccess) {
          drain();
          return hip_fail(e, "sem_batch_solve: split-BF16 solve");
        }
      for (int s = 0; s < NSIDE && e == hipSuccess; ++s) e = hipEventRecord(b->ev_side[s], b->side[s]);
      if (e != hipSuccess) {
        drain();
        return hip_fail(e, "sem_batch_solve: event");
      }
    }
    if (it > 0)
      for (const Group& g : b->rgroups)
        if ((e = launch_residual_batch(g.var, 1, b->d_rdesc + g.off, g.count, g.tiles, b->d_active, b->stream)) !=
            hipSuccess) {
          drain();
          return hip_fail(e, "sem_batch_solve: residual");
        }
    const int seq[6] = {it == 0 ? 0 : 1, 2, 3, 4, 5, it == 0 ? 6 : 7};
    for (int v : seq)
      if ((e = run_variant(b, v)) != hipSuccess) {
        drain();
        return hip_fail(e, "sem_batch_solve: mode products");
      }
    // the norm read-back waits for the side streams
    if (!order.empty())
      for (int s = 0; s < NSIDE && e == hipSuccess; ++s) e = hipStreamWaitEvent(b->stream, b->ev_side[s], 0);
    if (e != hipSuccess) {
      drain();
      return hip_fail(e, "sem_batch_solve: event");
    }
    if ((e = hipMemcpyAsync(hn.data(), b->d_norms, hn.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            b->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(b->stream)) != hipSuccess) {
      drain();
      return hip_fail(e, "sem_batch_solve: norm readback");
    }
    int left = 0;
    for (int i = 0; i < n; ++i) {
      if (!active[i]) continue;
      double dmax, umax;
      std::memcpy(&dmax, &hn[2 * i], 8);
      std::memcpy(&umax, &hn[2 * i + 1], 8);
      done_it[i] = it + 1;
      if (!std::isfinite(dmax) || !std::isfinite(umax)) {
        active[i] = 0;
        result = SEM_ENONFINITE;
        continue;
      }
      const double rel = umax > 0 ? dmax / umax : (dmax > 0 ? INFINITY : 0.0);
      if (refine_converged(rel, prev[i], prev2[i], tol)) {
        active[i] = 0;
        continue;
      }
      if (it >= 2 && rel > prev[i] && prev[i] > prev2[i]) {  // diverging at this precision
        active[i] = 0;
        if (result == SEM_OK) result = SEM_ENOCONV;
        continue;
      }
      prev2[i] = prev[i];
      prev[i] = rel;
      ++left;
    }
    if (!left) break;
  }
  if (iters)
    for (int i = 0; i < n; ++i) iters[i] = done_it[i];
  if (tol > 0)
    for (int i = 0; i < n; ++i)
      if (active[i] && result == SEM_OK) result = SEM_ENOCONV;
  if (result == SEM_ENONFINITE) return set_error(result, "sem_batch_solve: a solve produced a non-finite update");
  if (result == SEM_ENOCONV) return set_error(result, "sem_batch_solve: a solve did not meet the tolerance");
  return SEM_OK;
}

}  // extern "C"
