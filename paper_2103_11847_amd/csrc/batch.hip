// Batches of independent DC-LSQR / DC-GK solves (Algorithms 4-6 with the
// projected Tikhonov/GCV solve of Algorithm 5) of uneven size in shared
// launches.
//
// Planning runs the single-solve enqueue code once per instance with the
// context recording: every launch becomes a record (kernel, the instance's
// grid, argument bytes) tagged with its schedule point (phase, sub).  All
// instances pass the same sequence of phases, so the records of one kernel at
// one schedule point are merged into a single launch: its 1-D grid is the
// concatenation of the instances' grids, and a per-workgroup map gives each
// workgroup its instance and its (x, y, z) inside that instance's grid (see
// group_args).  The merged schedule is replayed in order on one stream, which
// keeps every instance's own launch order; it is captured into a HIP graph
// once.
#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "internal.h"

struct dctk_batch_s {
  dctk_ctx ctx;
  int count;
  std::vector<dctk_krylov> ws;
  dctk_solve_opts opts;
  struct Launch {
    const void* fn;
    dim3 grid;
    unsigned threads, shmem;
    std::vector<unsigned char> arg0;  // by-value argument (the only instance's, or a placeholder)
    size_t grp_off, bmap_off;         // offsets into dev (SIZE_MAX: null)
  };
  std::vector<Launch> launches;
  int single_launches;
  unsigned char* dev;  // argument arrays and workgroup maps of the merged launches
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace dctk {

static const size_t kNone = (size_t)-1;

static hipError_t replay(dctk_batch b, hipStream_t s) {
  for (auto& L : b->launches) {
    const void* grp = L.grp_off == kNone ? nullptr : (const void*)(b->dev + L.grp_off);
    const void* bmap = L.bmap_off == kNone ? nullptr : (const void*)(b->dev + L.bmap_off);
    void* kargs[3] = {L.arg0.data(), &grp, &bmap};
    hipError_t e = hipLaunchKernel(L.fn, L.grid, dim3(L.threads), kargs, L.shmem, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

static void batch_free(dctk_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->dev) (void)hipFree(b->dev);
  delete b;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace dctk

using namespace dctk;

extern "C" {

int dctk_batch_create(dctk_ctx ctx, int count, const dctk_krylov* ws, const void* const* C, void* const* X,
                      const dctk_solve_opts* opts, dctk_mlp mlp, double gate, int use_graph, dctk_batch* out) {
  if (!out) return DCTK_EINVAL;
  *out = nullptr;
  if (!ctx || !ws || !C || !X || !opts) return DCTK_EINVAL;
  if (count < 1 || count > DCTK_BATCH_MAX) return DCTK_EINVAL;
  if (ctx->rec) return DCTK_ESTATE;
  if (mlp && (opts->lambda >= 0.0 || opts->gcv_mode == 2 || opts->k_max < 8 || !(gate >= 1.0) || !std::isfinite(gate)))
    return DCTK_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (!ws[i] || !C[i] || !X[i]) return DCTK_EINVAL;
    if (ws[i]->kind != DCTK_KRYLOV_GKB || ws[i]->op->ctx->device != ctx->device) return DCTK_EINVAL;
    int r = check_solve_opts(opts, ws[i]);
    if (r) return r;
    // instances share no workspace and no operator (an operator's transform
    // scratch is written by its products, which run concurrently in a batch)
    for (int k = 0; k < i; ++k)
      if (ws[k] == ws[i] || ws[k]->op == ws[i]->op) return DCTK_EINVAL;
  }
  DCTK_HIP(ctx, hipSetDevice(ctx->device));

  // 1. record every instance's schedule
  std::vector<Recorder> recs(count);
  int single = 0;
  for (int i = 0; i < count; ++i) {
    ctx->rec = &recs[i];
    hipError_t e = mlp ? learned_enqueue(ctx, ws[i], mlp, C[i], X[i], opts, gate)
                       : lsqr_enqueue(ctx, ws[i], C[i], X[i], opts);
    ctx->rec = nullptr;
    if (e != hipSuccess) return hip_fail(ctx, e);
    single += (int)recs[i].recs.size();
  }

  // 2. merge: schedule point -> kernel -> (instance, record), in first-seen kernel order
  struct Member {
    int inst;
    const LaunchRec* r;
  };
  std::map<std::pair<int, int>, std::vector<std::pair<const void*, std::vector<Member>>>> points;
  for (int i = 0; i < count; ++i)
    for (const LaunchRec& r : recs[i].recs) {
      auto& kernels = points[{r.phase, r.sub}];
      auto it = std::find_if(kernels.begin(), kernels.end(), [&](const auto& kv) { return kv.first == r.fn; });
      if (it == kernels.end()) {
        kernels.push_back({r.fn, {}});
        it = kernels.end() - 1;
      }
      it->second.push_back(Member{i, &r});
    }

  dctk_batch b = new (std::nothrow) dctk_batch_s();
  if (!b) return DCTK_ENOMEM;
  b->ctx = ctx;
  b->count = count;
  b->ws.assign(ws, ws + count);
  b->opts = *opts;
  b->single_launches = single;
  b->dev = nullptr;
  b->graph = nullptr;
  b->exec = nullptr;

  // 3. lay out the argument arrays and workgroup maps of merged launches
  std::vector<unsigned char> host;
  for (auto& pt : points) {
    for (auto& kv : pt.second) {
      const std::vector<Member>& mem = kv.second;
      const LaunchRec& r0 = *mem[0].r;
      dctk_batch_s::Launch L;
      L.fn = mem.size() == 1 ? kv.first : r0.fn_group;
      L.threads = r0.threads;
      L.shmem = 0;
      L.arg0 = r0.args;
      L.grp_off = kNone;
      L.bmap_off = kNone;
      for (const Member& m : mem) L.shmem = std::max(L.shmem, m.r->shmem);
      if (mem.size() == 1) {
        L.grid = r0.grid;
      } else {
        const size_t asz = r0.args.size();
        size_t off = align_up(host.size(), 256);
        host.resize(off + asz * mem.size());
        for (size_t k = 0; k < mem.size(); ++k) memcpy(host.data() + off + k * asz, mem[k].r->args.data(), asz);
        L.grp_off = off;
        int64_t total = 0;
        for (const Member& m : mem) total += (int64_t)m.r->grid.x * m.r->grid.y * m.r->grid.z;
        if (total <= 0 || total > (int64_t)0x7fffffff) {
          delete b;
          return DCTK_EINVAL;
        }
        off = align_up(host.size(), 256);
        host.resize(off + sizeof(int4) * (size_t)total);
        int4* map = reinterpret_cast<int4*>(host.data() + off);
        int64_t w = 0;
        for (size_t k = 0; k < mem.size(); ++k) {
          const dim3 g = mem[k].r->grid;
          for (unsigned z = 0; z < g.z; ++z)
            for (unsigned y = 0; y < g.y; ++y)
              for (unsigned x = 0; x < g.x; ++x) map[w++] = make_int4((int)k, (int)x, (int)y, (int)z);
        }
        L.bmap_off = off;
        L.grid = dim3((unsigned)total);
      }
      b->launches.push_back(std::move(L));
    }
  }
  if (!host.empty()) {
    hipError_t e = hipMalloc((void**)&b->dev, host.size());
    if (e == hipSuccess) e = hipMemcpy(b->dev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      batch_free(b);
      return hip_fail(ctx, e);
    }
  }

  // 4. capture the schedule once (on a private stream: the null stream cannot be captured)
  if (use_graph) {
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t el = replay(b, cs);
      e = hipStreamEndCapture(cs, &b->graph);
      if (el != hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
      batch_free(b);
      return hip_fail(ctx, e);
    }
  }
  *out = b;
  return DCTK_OK;
}

int dctk_batch_run(dctk_ctx ctx, dctk_batch b) {
  if (!ctx || !b || b->ctx != ctx) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  if (b->exec) {
    DCTK_HIP(ctx, hipGraphLaunch(b->exec, ctx->stream));
  } else {
    DCTK_HIP(ctx, replay(b, ctx->stream));
  }
  for (dctk_krylov w : b->ws) {
    w->host_steps = b->opts.k_max;
    w->initialised = 1;
  }
  return DCTK_OK;
}

int dctk_batch_info(dctk_ctx ctx, dctk_batch b, dctk_solve_info* infos) {
  if (!ctx || !b || b->ctx != ctx || !infos) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  int first = DCTK_OK;
  for (int i = 0; i < b->count; ++i) {
    const int r = lsqr_info(ctx, b->ws[i], &b->opts, &infos[i]);
    if (r < 0) return r;
    if (first == DCTK_OK) first = r;
  }
  return first;
}

int dctk_batch_learned(dctk_ctx ctx, dctk_batch b, int* k_limit, int* accepted) {
  if (!ctx || !b || b->ctx != ctx) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  for (int i = 0; i < b->count; ++i) {
    KState* st = b->ws[i]->st;
    int kl = 0;
    double ok = 0.0;
    DCTK_HIP(ctx, hipMemcpyAsync(&kl, &st->k_limit, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    DCTK_HIP(ctx, hipMemcpyAsync(&ok, &st->gate_ok, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    DCTK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (k_limit) k_limit[i] = kl;
    if (accepted) accepted[i] = ok > 0.5 ? 1 : 0;
  }
  return DCTK_OK;
}

int dctk_batch_stats(dctk_batch b, int* merged_launches, int* single_launches) {
  if (!b) return DCTK_EINVAL;
  if (merged_launches) *merged_launches = (int)b->launches.size();
  if (single_launches) *single_launches = b->single_launches;
  return DCTK_OK;
}

int dctk_batch_destroy(dctk_batch b) {
  if (!b) return DCTK_EINVAL;
  (void)hipSetDevice(b->ctx->device);
  (void)hipStreamSynchronize(b->ctx->stream);
  batch_free(b);
  return DCTK_OK;
}

int dctk_batch_lsqr_tik_solve(dctk_ctx ctx, int count, const dctk_op* ops, const void* const* C, void* const* X,
                              const dctk_solve_opts* opts, dctk_solve_info* infos) {
  if (!ctx || !ops || !C || !X || !opts || !infos) return DCTK_EINVAL;
  if (count < 1 || count > DCTK_BATCH_MAX) return DCTK_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (!ops[i]) return DCTK_EINVAL;
    for (int k = 0; k < i; ++k)
      if (ops[k] == ops[i]) return DCTK_EINVAL;
  }
  std::vector<dctk_krylov> ws((size_t)count, nullptr);
  int r = DCTK_OK;
  for (int i = 0; i < count && r == DCTK_OK; ++i)
    r = dctk_krylov_create(ctx, ops[i], DCTK_KRYLOV_GKB, opts->k_max, DCTK_ORTHO_MGS, &ws[(size_t)i]);
  dctk_batch b = nullptr;
  if (r == DCTK_OK) r = dctk_batch_create(ctx, count, ws.data(), C, X, opts, nullptr, 1.0, 1, &b);
  if (r == DCTK_OK) r = dctk_batch_run(ctx, b);
  if (r == DCTK_OK) r = dctk_batch_info(ctx, b, infos);
  if (b) (void)dctk_batch_destroy(b);
  for (dctk_krylov w : ws)
    if (w) (void)dctk_krylov_destroy(w);
  return r;
}

}  // extern "C"
