// capi.hip -- the C entry points: argument checks, device set-up, the level
// loop of recursive spectral bisection (Alg. 1), and error reporting.
#include <dlfcn.h>

#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace rsb {
namespace {

thread_local std::string g_last_error;

// Named ranges for timeline tools (ROCTx), loaded at run time when
// RSB_ROCTX=1 so that the library carries no link dependency on them:
// rocprofv3 --marker-trace shows the call, each level and its phases.
struct Roctx {
  int (*push)(const char *) = nullptr;
  int (*pop)() = nullptr;
};
const Roctx &roctx() {
  static const Roctx r = [] {
    Roctx x;
    const char *e = std::getenv("RSB_ROCTX");
    if (!e || std::strcmp(e, "1") != 0) return x;
    void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
    if (!h) h = dlopen("/opt/rocm/lib/librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
    if (!h) return x;
    x.push = (int (*)(const char *))dlsym(h, "roctxRangePushA");
    x.pop = (int (*)())dlsym(h, "roctxRangePop");
    if (!x.push || !x.pop) x = Roctx{};
    return x;
  }();
  return r;
}
struct Range {
  bool on;
  explicit Range(const std::string &name) : on(roctx().push != nullptr) {
    if (on) roctx().push(name.c_str());
  }
  ~Range() {
    if (on) roctx().pop();
  }
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <typename F>
int guarded(F &&f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return RSB_ENOMEM;
  } catch (...) {
    g_last_error = "unexpected exception";
    return RSB_EINTERNAL;
  }
}

void check_opts(const rsb_opts *o) {
  if (!o) fail(RSB_EINVAL, "opts is NULL");
  if (o->struct_size != (int32_t)sizeof(rsb_opts))
    fail(RSB_EINVAL, "opts->struct_size mismatch (call rsb_opts_init)");
  if (o->graph < 0 || o->graph > 2) fail(RSB_EINVAL, "graph kind");
  if (o->method < 0 || o->method > 3) fail(RSB_EINVAL, "method");
  if (o->precision < 0 || o->precision > 1) fail(RSB_EINVAL, "precision");
  if (o->lanczos_m < 1 || o->lanczos_m > kMaxM) fail(RSB_EINVAL, "lanczos_m must be in [1, 250]");
  if (o->max_restarts < 0) fail(RSB_EINVAL, "negative max_restarts");
  if (!(o->tol > 0) || !(o->cg_tol > 0)) fail(RSB_EINVAL, "tolerances must be positive");
  if (o->inv_max_outer < 1 || o->cg_max_iter < 1) fail(RSB_EINVAL, "inverse iteration caps");
  if (o->cg_full_projection < 0 || o->cg_full_projection > kMaxFullProj)
    fail(RSB_EINVAL, "cg_full_projection must be in [0, 32]");
  if (o->autotune < 0 || o->autotune > 2) fail(RSB_EINVAL, "autotune");
  if (o->lanczos_keep < 0 || o->lanczos_keep > kMaxKeep ||
      (o->lanczos_keep > 0 && o->lanczos_keep >= o->lanczos_m))
    fail(RSB_EINVAL, "lanczos_keep must be 0 or in [1, min(16, lanczos_m - 1)]");
  if (o->method == RSB_BLOCK) {
    if (o->lanczos_m < 4 || o->lanczos_m > kBkMaxM || o->lanczos_m % 2)
      fail(RSB_EINVAL, "RSB_BLOCK: lanczos_m must be even and in [4, 48]");
    if (o->lanczos_keep % 2 || o->lanczos_keep > o->lanczos_m - 4)
      fail(RSB_EINVAL, "RSB_BLOCK: lanczos_keep must be even and at most lanczos_m - 4");
    if (o->gather_scatter) fail(RSB_EINVAL, "RSB_BLOCK does not take gather_scatter");
    if (o->second_solve) fail(RSB_EINVAL, "RSB_BLOCK gives the pair itself: no second_solve");
  }
  if (o->rows_per_thread != 0 && o->rows_per_thread != 2 && o->rows_per_thread != 4 &&
      o->rows_per_thread != 8)
    fail(RSB_EINVAL, "rows_per_thread must be 0, 2, 4 or 8");
  if (o->inv_precond != RSB_PRECOND_NONE && o->inv_precond != RSB_PRECOND_AMG)
    fail(RSB_EINVAL, "inv_precond must be RSB_PRECOND_NONE or RSB_PRECOND_AMG");
  if (o->amg_smooth < 0 || o->amg_smooth > 16) fail(RSB_EINVAL, "amg_smooth must be in [0, 16]");
  if (!(o->amg_sigma > 0.0 && o->amg_sigma < 2.0)) fail(RSB_EINVAL, "amg_sigma must be in (0, 2)");
  if (o->fiedler_sweep < 0 || o->fiedler_sweep > 64)
    fail(RSB_EINVAL, "fiedler_sweep must be in [0, 64]");
  if (o->fiedler_sweep > 0 && o->method != RSB_BLOCK &&
      (o->method == RSB_INVERSE_CG || o->lanczos_keep < 2))
    fail(RSB_EINVAL, "fiedler_sweep needs RSB_BLOCK, or Lanczos (RSB_LANCZOS or RSB_AUTO) with lanczos_keep >= 2");
  if (!(o->sweep_gap >= 0.0)) fail(RSB_EINVAL, "sweep_gap must be >= 0");
  if (o->warm_start != 0 && o->warm_start != 1) fail(RSB_EINVAL, "warm_start must be 0 or 1");
  if (o->reorder != 0 && o->reorder != 1) fail(RSB_EINVAL, "reorder must be 0 or 1");
  if (o->second_solve != 0 && o->second_solve != 1) fail(RSB_EINVAL, "second_solve must be 0 or 1");
  if (o->second_solve && o->fiedler_sweep < 1)
    fail(RSB_EINVAL, "second_solve needs fiedler_sweep > 0");
  if (o->lanczos_s != 1 && o->lanczos_s != 2) fail(RSB_EINVAL, "lanczos_s must be 1 or 2");
  if (o->pack_matrix < 0 || o->pack_matrix > 2) fail(RSB_EINVAL, "pack_matrix must be 0, 1 or 2");
  if (o->bfs_start != 0 && o->bfs_start != 1) fail(RSB_EINVAL, "bfs_start must be 0 or 1");
  if (o->gather_scatter != 0 && o->gather_scatter != 1)
    fail(RSB_EINVAL, "gather_scatter must be 0 or 1");
  if (o->gather_scatter && (o->graph != RSB_GRAPH_WEIGHTED || o->method == RSB_INVERSE_CG))
    fail(RSB_EINVAL, "gather_scatter needs graph RSB_GRAPH_WEIGHTED and Lanczos (RSB_LANCZOS or RSB_AUTO)");
  if (o->warm_start && o->method != RSB_BLOCK &&
      (o->method == RSB_INVERSE_CG || o->lanczos_keep < 2))
    fail(RSB_EINVAL, "warm_start needs RSB_BLOCK, or Lanczos (RSB_LANCZOS or RSB_AUTO) with lanczos_keep >= 2");
}

void setup_ctx(Ctx &ctx, const rsb_opts &o, bool private_stream = true) {
  int ndev = 0;
  RSB_HIP(hipGetDeviceCount(&ndev));
  if (o.device < 0 || o.device >= ndev) fail(RSB_EINVAL, "device ordinal out of range");
  RSB_HIP(hipSetDevice(o.device));
  ctx.device = o.device;
  ctx.stream = (hipStream_t)o.stream;
  if (!ctx.stream && private_stream) {
    // graph capture needs a real stream: use a private one for this call
    RSB_HIP(hipStreamCreateWithFlags(&ctx.stream, hipStreamNonBlocking));
    ctx.own_stream = true;
    // work the caller queued on the null stream must be visible to ours
    RSB_HIP(hipStreamSynchronize(nullptr));
  }
  ctx.limit = o.device_mem_limit;
  ctx.verbose = o.verbose;
  ctx.pack = o.pack_matrix;
  if (const char *env = std::getenv("RSB_LOG"))
    if (std::string(env) == "level") ctx.verbose = std::max(ctx.verbose, 1);
  if (const char *env = std::getenv("RSB_FAULT_INJECT")) {
    const std::string f(env);
    const size_t colon = f.find(':');
    if (colon != std::string::npos) {
      const int64_t at = std::atoll(f.c_str() + colon + 1);
      if (f.compare(0, colon, "alloc") == 0) ctx.fault.alloc_at = at;
      if (f.compare(0, colon, "launch") == 0) ctx.fault.launch_at = at;
      ctx.fault.stream = ctx.stream;
      fault_plan() = &ctx.fault;
    }
  }
  static std::once_flag once[64];
  if (o.device < 64)
    std::call_once(once[o.device], [&] {
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, o.device) == hipSuccess) {
        uint64_t thr = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
      }
    });
}

// Device copy of a caller array (or the caller's device pointer itself).
template <typename T>
struct InArr {
  DevBuf<T> own;
  const T *p = nullptr;
  void init(Ctx &ctx, const T *src, int64_t n, bool device) {
    if (device) {
      p = src;
      return;
    }
    own.alloc(ctx, std::max<int64_t>(n, 1));
    if (n > 0)
      RSB_HIP(hipMemcpyAsync(own.get(), src, n * sizeof(T), hipMemcpyHostToDevice, ctx.stream));
    p = own.get();
  }
};

template <typename T>
void copy_out(Ctx &ctx, T *dst, const T *dsrc, int64_t n, bool device) {
  if (n <= 0) return;
  RSB_HIP(hipMemcpyAsync(dst, dsrc, n * sizeof(T),
                         device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx.stream));
}

struct MeshIn {
  int64_t nelem;
  const int64_t *d_ids;
  int32_t nparts;
};

struct RunOut {
  int status = RSB_OK;
  int flip = 0;  // rsb_fiedler: the returned vector must be negated (sign rule)
  double lambda = 0.0, residual = 0.0;
};

// Tables of a single segment of a level (the per-subgraph reference mode).
struct OneSeg {
  DevBuf<SegDev> seg;
  DevBuf<BlkDev> blk;
  DevBuf<GrpDev> grp;
  int nblk = 0, ngrp = 0;
};

void one_segment_tables(const Level &L, int s, OneSeg &o, Ctx &ctx) {
  Level tmp;
  tmp.seg.push_back(L.seg[s]);
  tmp.nseg = 1;
  tmp.nrows = L.nrows;
  level_tables(tmp, L.rpt, ctx);
  o.seg = std::move(tmp.d_seg);
  o.blk = std::move(tmp.d_blk);
  o.grp = std::move(tmp.d_grp);
  o.nblk = tmp.nblk;
  o.ngrp = tmp.ngrp;
}

// Ritz buffers per segment: the kept count, or the pair of the block solver.
constexpr int kPairMinPerStep = 4;

int solve_keep(const rsb_opts &o) {
  return o.method == RSB_BLOCK ? std::max(o.lanczos_keep, 2) : o.lanczos_keep;
}

// Eigen-solve of one level: all segments batched, or one segment at a time.
// RSB_AUTO runs Lanczos and then, for every segment Lanczos left
// unconverged, inverse iteration from the random start (Sec. 7: the paper
// switched to inverse iteration where Lanczos did not converge).
int64_t solve_level(const Level &L, CompDev &C, SolveDev &S, const rsb_opts &o, void *work,
                    double *y64, double *y2, const double *warm, KernelProfile *prof,
                    int *amg_levels, int *fallbacks, Ctx &ctx) {
  const bool mixed = o.precision == RSB_MIXED;
  // two steps at a time only where every component this level solves has
  // more than kPairMinPerStep * lanczos_m elements: a cycle can exhaust the
  // Krylov space of a smaller graph (at most m + 1 elements, or fewer
  // distinct eigenvalues than m), and the block's single Gram-Schmidt pass
  // before its Cholesky QR can then miss the breakdown
  bool pairs = o.lanczos_s == 2 && o.method != RSB_BLOCK;
  if (pairs) {
    std::vector<SegState> hs(L.nseg);
    RSB_HIP(hipMemcpyAsync(hs.data(), S.st.get(), L.nseg * sizeof(SegState),
                           hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    for (const SegState &h : hs)
      if (h.solve && h.invsqrt_nc > 0.0 &&
          1.0 / (h.invsqrt_nc * h.invsqrt_nc) <= kPairMinPerStep * o.lanczos_m + 0.5)
        pairs = false;
  }
  auto run = [&](const LevelView &v, SolveDev &SS, bool graph, bool inverse) -> int64_t {
    if (o.method == RSB_BLOCK) {
      BlockParams bp{o.lanczos_m, o.lanczos_keep, o.max_restarts, o.tol,
                     o.seed,      warm,           o.fiedler_sweep, o.sweep_gap};
      return block_level(v, C, SS, bp, y64, y2, ctx);
    }
    if (inverse) {
      InverseParams ip{o.inv_max_outer, o.cg_max_iter, o.cg_tol,     o.tol,
                       o.seed,          o.inv_precond, o.amg_sigma,  o.amg_smooth,
                       amg_levels,      o.cg_full_projection};
      return inverse_level(v, C, SS, ip, work, y64, graph, ctx);
    }
    LanczosParams lp{o.lanczos_m, o.lanczos_keep, o.max_restarts, o.tol, graph ? 1 : 0,
                     o.seed,      prof,           v.nnz,          y2, warm,
                     pairs ? 1 : 0};
    return mixed ? lanczos_level<float>(v, C, SS, lp, work, y64, ctx)
                 : lanczos_level<double>(v, C, SS, lp, work, y64, ctx);
  };
  // segment s alone, with launches sized to it; its state goes back to S
  auto one = [&](int s, bool inverse) -> int64_t {
    OneSeg os;
    one_segment_tables(L, s, os, ctx);
    SolveDev S1;
    solve_alloc(S1, 1, os.nblk, os.ngrp, std::max(o.lanczos_m, 1), solve_keep(o), ctx);
    RSB_HIP(hipMemcpyAsync(S1.st.get(), S.st.get() + s, sizeof(SegState),
                           hipMemcpyDeviceToDevice, ctx.stream));
    LevelView v = view_of(L);
    v.nseg = 1;
    v.nblk = os.nblk;
    v.ngrp = os.ngrp;
    v.seg = os.seg.get();
    v.blk = os.blk.get();
    v.grp = os.grp.get();
    const double frac = (double)L.seg[s].npad / (double)std::max<int64_t>(L.nrows, 1);
    v.nnz = (int64_t)((double)L.nnz * frac);
    v.packed_nnz = (int64_t)((double)L.packed_nnz * frac);
    v.packed_slices = (int64_t)((double)L.packed_slices * frac);
    v.gs.only_seg = s;
    const int64_t steps = run(v, S1, false, inverse);
    RSB_HIP(hipMemcpyAsync(S.st.get() + s, S1.st.get(), sizeof(SegState),
                           hipMemcpyDeviceToDevice, ctx.stream));
    // the Ritz values of the last cycle (read by the sweep over the pair)
    if (!inverse)
      RSB_HIP(hipMemcpyAsync(S.tvals.get() + (int64_t)s * S.nkcap, S1.tvals.get(),
                             std::min(S.nkcap, S1.nkcap) * sizeof(double),
                             hipMemcpyDeviceToDevice, ctx.stream));
    int64_t c = 0, acc = 0;
    RSB_HIP(hipMemcpyAsync(&c, S1.counters.get(), sizeof(int64_t), hipMemcpyDeviceToHost,
                           ctx.stream));
    RSB_HIP(hipMemcpyAsync(&acc, S.counters.get(), sizeof(int64_t), hipMemcpyDeviceToHost,
                           ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    acc += c;
    RSB_HIP(hipMemcpyAsync(S.counters.get(), &acc, sizeof(int64_t), hipMemcpyHostToDevice,
                           ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return steps;
  };
  auto states = [&]() {
    std::vector<SegState> hs(L.nseg);
    RSB_HIP(hipMemcpyAsync(hs.data(), S.st.get(), L.nseg * sizeof(SegState),
                           hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return hs;
  };
  const bool inverse_only = o.method == RSB_INVERSE_CG;
  int64_t steps = 0;
  if (o.batched) {
    steps = run(view_of(L), S, o.use_hipgraph != 0, inverse_only);
  } else {
    // reference mode: every subgraph with its own launches sized to it
    const std::vector<SegState> hs = states();
    for (int s = 0; s < L.nseg; ++s) {
      if (!hs[s].solve) continue;
      steps += one(s, inverse_only);
      if (ctx.verbose >= 2 && (s % 64 == 63 || s + 1 == L.nseg))
        fprintf(stderr, "[rsb]   subgraph %d of %d solved\n", s + 1, L.nseg);
    }
  }
  if (o.method == RSB_AUTO) {
    const std::vector<SegState> hs = states();
    for (int s = 0; s < L.nseg; ++s) {
      if (!hs[s].solve || hs[s].converged) continue;
      if (fallbacks) ++*fallbacks;
      steps += one(s, true);
    }
  }
  return steps;
}

// The whole hot path for a batch of meshes: graph, then level by level
// components -> eigen-solve -> split -> compaction.  part: concatenated
// output (device).  If fiedler_y != nullptr, only the first level of a
// single mesh runs and its vector is written there (device, nelem values).
RunOut run_rsb(const std::vector<MeshIn> &meshes, int nv, const rsb_opts &o, Ctx &ctx,
               int32_t *d_part, rsb_stats *stats, double *fiedler_y) {
  RunOut out;
  const double t0 = now_ms();
  rsb_stats st{};
  // one range for the call and one for each phase in turn (ranges form a
  // stack: the previous phase is closed before the next one opens)
  Range call_range("rsb: partition");
  std::unique_ptr<Range> phase;
  auto phase_to = [&](const std::string &name) {
    phase.reset();
    phase.reset(new Range(name));
  };
  phase_to("rsb: dual graph");
  // 1. dual graphs
  std::vector<DevCsr> graphs(meshes.size());
  int64_t total = 0;
  for (size_t b = 0; b < meshes.size(); ++b) {
    build_dual_graph(meshes[b].d_ids, meshes[b].nelem, nv, o.graph, graphs[b], ctx);
    st.nnz += graphs[b].nnz;
    total += meshes[b].nelem;
  }
  if (total >= kMaxRows) fail(RSB_EINVAL, "too many elements (limit 2^28 per call)");
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  st.ms_graph = now_ms() - t0;
  // 2. level 0
  std::vector<const DevCsr *> gp;
  std::vector<int32_t> np;
  int64_t parts_total = 0;
  for (size_t b = 0; b < meshes.size(); ++b) {
    gp.push_back(&graphs[b]);
    np.push_back(fiedler_y ? 2 : meshes[b].nparts);
    parts_total += meshes[b].nparts;
  }
  const int rpt = o.rows_per_thread ? o.rows_per_thread : default_rpt(total);
  // start values by element: the BFS start of the first solve of each mesh
  // (taken in element order, before any reordering), then the parents'
  // second Ritz vectors of the warm start
  DevBuf<double> warm;
  if (o.warm_start || o.bfs_start) {
    warm.alloc(ctx, std::max<int64_t>(total, 1));
    fill_f64(warm.get(), total, std::nan(""), ctx);
  }
  if (o.bfs_start) {
    int64_t off = 0;
    for (size_t b = 0; b < meshes.size(); ++b) {
      if (np[b] >= 2) bfs_start_values(graphs[b], warm.get() + off, ctx);
      off += meshes[b].nelem;
    }
  }
  // locality order of each mesh's rows (not for rsb_fiedler, whose vector
  // is returned row by row)
  std::vector<DevBuf<int32_t>> perms;
  std::vector<const int32_t *> perm_ptr;
  if (o.reorder && !fiedler_y) {
    const double tr = now_ms();
    perms.resize(meshes.size());
    for (size_t b = 0; b < meshes.size(); ++b) {
      locality_order(graphs[b], perms[b], ctx);
      perm_ptr.push_back(perms[b].get());
    }
    st.ms_reorder = now_ms() - tr;
  }
  Level L0;
  level0_from_csr(L0, gp, np, rpt, ctx, perm_ptr.empty() ? nullptr : &perm_ptr);
  // gather-scatter operator: the vertex incidence of all meshes, once
  GsBase gsb;
  if (o.gather_scatter) {
    std::vector<const int64_t *> ids;
    std::vector<int64_t> ne;
    for (auto &m : meshes) {
      ids.push_back(m.d_ids);
      ne.push_back(m.nelem);
    }
    // element -> first-level row
    DevBuf<int32_t> rank(ctx, std::max<int64_t>(total, 1));
    fill_i32(rank.get(), total, 0, ctx);
    gs_rank_of_rows(L0.orig.get(), L0.nrows, rank.get(), ctx);
    gs_base_build(ids, ne, nv, rank.get(), gsb, ctx);
  }
  perms.clear();
  for (auto &g : graphs) {
    g.col.release();
    g.wgt.release();
    g.row_ptr.release();
  }
  if (d_part) fill_i32(d_part, total, -1, ctx);
  {  // meshes kept whole (one part)
    int64_t off = 0;
    for (size_t b = 0; b < meshes.size(); ++b) {
      if (np[b] < 2 && d_part) fill_i32(d_part + off, meshes[b].nelem, 0, ctx);
      off += meshes[b].nelem;
    }
  }
  // 3. work space sized for the largest level
  const int64_t cap_rows =
      round_up(total, kWave) + (int64_t)kWave * (parts_total + 2 * (int64_t)meshes.size());
  const size_t wlz = lanczos_workspace_bytes(cap_rows, o.lanczos_m, o.precision == RSB_MIXED,
                                             o.lanczos_keep);
  const size_t winv = inverse_workspace_bytes(cap_rows, o.cg_full_projection);
  const size_t wbytes = (o.method == RSB_INVERSE_CG) ? winv
                        : (o.method == RSB_AUTO) ? std::max(wlz, winv)
                                                 : wlz;
  DevBuf<char> work(ctx, wbytes);
  DevBuf<double> y64(ctx, cap_rows);
  DevBuf<double> y2;
  if (o.fiedler_sweep > 0 || o.warm_start) y2.alloc(ctx, cap_rows);
  DevBuf<uint8_t> side(ctx, cap_rows);
  KernelProfile prof;
  Level LA, LB;
  Level *L = &L0;
  Level *next = &LA;
  int level = 0;
  int worst = RSB_OK;
  while (L->nseg > 0) {
    const std::string lv = "rsb: level " + std::to_string(level);
    phase_to(lv + " components");
    const double ta = now_ms();
    const double prof_ms0 = prof.ms, prof_bytes0 = prof.bytes;
    SolveDev S;
    CompDev C;
    if (o.gather_scatter) gs_level_build(gsb, *L, total, L->gs, ctx);
    choose_tile(*L, o, work.get(), ctx);
    if (level == 0) {
      st.tile_rows = kBlock * L->rpt;
      st.packed_fraction = L->nnz > 0 ? (double)L->packed_nnz / (double)L->nnz : 0.0;
      st.matrix_bytes = matrix_bytes(view_of(*L));
      st.staged_fraction = L->nblk > 0 ? (double)L->staged_tiles / (double)L->nblk : 0.0;
    }
    if (level == 0 && o.profile && o.method != RSB_INVERSE_CG && !o.gather_scatter) {
      // the level-0 Laplacian SpMV on its own, in the Lanczos directions'
      // precision, with its algorithmic bytes: row pointers, the matrix as
      // read (32-bit words, or packed entries and their window bases), one
      // read of x and one write of y
      const bool f32 = o.precision == RSB_MIXED;
      const double sv = f32 ? 4.0 : 8.0, n = (double)L->nrows;
      st.spmv_alone_us = spmv_alone_us(view_of(*L), f32, 20, ctx);
      st.spmv_alone_bytes = 4.0 * (n + 1.0) + matrix_bytes(view_of(*L)) + 2.0 * sv * n;
      st.spmv_words_us = spmv_words_us(view_of(*L), f32, 20, ctx);
      st.spmv_words_bytes = 4.0 * (n + 1.0) + 4.0 * (double)L->nnz + 2.0 * sv * n;
    }
    solve_alloc(S, L->nseg, L->nblk, L->ngrp, std::max(o.lanczos_m, 1), solve_keep(o), ctx);
    components_and_targets(*L, C, S, ctx);
    phase_to(lv + " solve");
    int amg_levels = 0;
    const int64_t fp64_steps0 = ctx.fp64_level_steps;
    const bool read_warm = o.warm_start || (level == 0 && o.bfs_start);
    const int64_t steps = solve_level(*L, C, S, o, work.get(), y64.get(), y2.get(),
                                      read_warm ? warm.get() : nullptr,
                                      o.profile ? &prof : nullptr, &amg_levels, &st.fallbacks, ctx);
    if (o.warm_start) warm_update(*L, C, S, y2.get(), warm.get(), ctx);
    st.amg_levels = std::max(st.amg_levels, amg_levels);
    std::vector<SegState> hs(L->nseg);
    RSB_HIP(hipMemcpyAsync(hs.data(), S.st.get(), L->nseg * sizeof(SegState),
                           hipMemcpyDeviceToHost, ctx.stream));
    int64_t segsteps = 0;
    RSB_HIP(hipMemcpyAsync(&segsteps, S.counters.get(), sizeof(int64_t), hipMemcpyDeviceToHost,
                           ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    const double tb = now_ms();
    if (level == 0 && L->nseg >= 1 && hs[0].solve) {
      // the first bisection's Fiedler pair (of the first mesh)
      st.lambda2 = hs[0].rho;
      st.residual = hs[0].res;
    }
    st.ms_solve += tb - ta;
    st.level_steps += steps;
    st.segment_steps += segsteps;
    int disc = 0, notconv = 0, cyc = 0;
    for (auto &s : hs) {
      if (s.ncomp > 1) ++disc;
      if (s.solve && !s.converged) ++notconv;
      st.cycles += s.cycles;
      cyc = std::max(cyc, s.cycles);
    }
    // FP64 SpMV launches: all of them in FP64 mode; with FP32 directions,
    // steps 1-2 and the residual of every cycle, and every step of the
    // cycles continued with FP64 directions
    st.spmv_fp64 += (o.precision == RSB_MIXED && o.method != RSB_INVERSE_CG &&
                     o.method != RSB_BLOCK)
                        ? 3 * (int64_t)cyc + (ctx.fp64_level_steps - fp64_steps0)
                        : steps + cyc;
    st.disconnected += disc;
    st.not_converged += notconv;
    if (disc) worst = std::max(worst, RSB_WARN_DISCONNECTED);
    if (notconv && worst == RSB_OK) worst = RSB_WARN_NOT_CONVERGED;
    if (ctx.verbose >= 2)
      for (int i = 0; i < L->nseg; ++i)
        fprintf(stderr,
                "[rsb]   seg %d: n %d P %d ncomp %d solve %d conv %d cycles %d steps %lld "
                "res %.3e rho %.12g theta %.12g\n",
                i, L->seg[i].n, L->seg[i].P, hs[i].ncomp, hs[i].solve, hs[i].converged,
                hs[i].cycles, (long long)hs[i].steps, hs[i].res, hs[i].rho, hs[i].theta);
    double min_perp2 = 1e-12;
    // second_solve: the thick restart's own pair (second Ritz vector and
    // Ritz values), swept where the second solve's pair is not
    DevBuf<double> y2_thick;
    std::vector<double> tv_thick;
    if (o.second_solve) {
      // the pair from two solves: Lanczos again from another random start;
      // its vector becomes y2 and its Rayleigh quotient the second value of
      // the gap test, then the first solve's vector and state come back
      const int64_t nr = L->nrows;
      y2_thick.alloc(ctx, std::max<int64_t>(nr, 1));
      RSB_HIP(hipMemcpyAsync(y2_thick.get(), y2.get(), nr * sizeof(double),
                             hipMemcpyDeviceToDevice, ctx.stream));
      tv_thick.assign((size_t)L->nseg * S.nkcap, 0.0);
      RSB_HIP(hipMemcpyAsync(tv_thick.data(), S.tvals.get(), tv_thick.size() * sizeof(double),
                             hipMemcpyDeviceToHost, ctx.stream));
      DevBuf<double> y1(ctx, std::max<int64_t>(nr, 1));
      DevBuf<SegState> st1(ctx, L->nseg);
      RSB_HIP(hipMemcpyAsync(y1.get(), y64.get(), nr * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx.stream));
      RSB_HIP(hipMemcpyAsync(st1.get(), S.st.get(), L->nseg * sizeof(SegState),
                             hipMemcpyDeviceToDevice, ctx.stream));
      rsb_opts o2 = o;
      o2.seed = o.seed ^ 0x9E3779B97F4A7C15ull;
      o2.method = RSB_LANCZOS;
      int amg2 = 0;
      st.level_steps += solve_level(*L, C, S, o2, work.get(), y64.get(), nullptr, nullptr,
                                    o.profile ? &prof : nullptr, &amg2, nullptr, ctx);
      std::vector<SegState> h2(L->nseg);
      RSB_HIP(hipMemcpyAsync(h2.data(), S.st.get(), L->nseg * sizeof(SegState),
                             hipMemcpyDeviceToHost, ctx.stream));
      RSB_HIP(hipMemcpyAsync(y2.get(), y64.get(), nr * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx.stream));
      RSB_HIP(hipMemcpyAsync(y64.get(), y1.get(), nr * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx.stream));
      RSB_HIP(hipMemcpyAsync(S.st.get(), st1.get(), L->nseg * sizeof(SegState),
                             hipMemcpyDeviceToDevice, ctx.stream));
      RSB_HIP(hipStreamSynchronize(ctx.stream));
      std::vector<double> tv((size_t)L->nseg * S.nkcap, 0.0);
      for (int i = 0; i < L->nseg; ++i) {
        tv[(size_t)i * S.nkcap] = hs[i].rho;
        if (S.nkcap > 1) tv[(size_t)i * S.nkcap + 1] = h2[i].rho;
      }
      RSB_HIP(hipMemcpyAsync(S.tvals.get(), tv.data(), tv.size() * sizeof(double),
                             hipMemcpyHostToDevice, ctx.stream));
      RSB_HIP(hipStreamSynchronize(ctx.stream));
      min_perp2 = 0.01;
    }
    if (o.fiedler_sweep > 0) {
      std::vector<int32_t> on;
      fiedler_sweep(*L, C, S, y64.get(), y2.get(), o.fiedler_sweep, o.sweep_gap, &st.sweeps,
                    &st.sweep_moved, ctx, min_perp2, &on);
      if (o.second_solve && S.nkcap >= 2) {
        // segments the second solve's pair left unswept: the thick
        // restart's pair, with its gap and the usual perpendicular part
        std::vector<double> tv = tv_thick;
        bool any = false;
        for (int i = 0; i < L->nseg; ++i) {
          if (on[i]) tv[(size_t)i * S.nkcap + 1] = 1e300;
          else any = true;
        }
        if (any) {
          RSB_HIP(hipMemcpyAsync(S.tvals.get(), tv.data(), tv.size() * sizeof(double),
                                 hipMemcpyHostToDevice, ctx.stream));
          RSB_HIP(hipStreamSynchronize(ctx.stream));
          fiedler_sweep(*L, C, S, y64.get(), y2_thick.get(), o.fiedler_sweep, o.sweep_gap,
                        &st.sweeps, &st.sweep_moved, ctx);
        }
      }
    }
    if (fiedler_y) {
      const SegState &s = hs[0];
      RSB_HIP(hipMemcpyAsync(fiedler_y, y64.get(), meshes[0].nelem * sizeof(double),
                             hipMemcpyDeviceToDevice, ctx.stream));
      // the sign rule is applied by the split's sign pass
      split_level(*L, C, S, y64.get(), side.get(), ctx);
      SegState s2;
      RSB_HIP(hipMemcpyAsync(&s2, S.st.get(), sizeof(SegState), hipMemcpyDeviceToHost,
                             ctx.stream));
      RSB_HIP(hipStreamSynchronize(ctx.stream));
      out.lambda = s.solve ? s.rho : 0.0;
      out.residual = s.solve ? s.res : 0.0;
      out.flip = s2.flip;
      out.status = (s.ncomp > 1) ? RSB_WARN_DISCONNECTED
                                 : (s.solve && !s.converged ? RSB_WARN_NOT_CONVERGED : RSB_OK);
      st.lambda2 = out.lambda;
      st.residual = out.residual;
      st.levels = 1;
      st.kernel_ms = prof.ms;
      st.kernel_bytes = prof.bytes;
      st.kernel_launches = prof.launches;
      st.ms_total = now_ms() - t0;
      if (stats) {
        const int32_t sz = stats->struct_size;
        *stats = st;
        stats->struct_size = sz;
      }
      return out;
    }
    phase_to(lv + " split and compaction");
    split_level(*L, C, S, y64.get(), side.get(), ctx);
    compact_level(*L, side.get(), d_part, *next, rpt, ctx);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    st.ms_split += now_ms() - tb;
    if (ctx.verbose) {
      fprintf(stderr,
              "[rsb] level %d: %d segments, %lld rows, tile %d, %lld level-steps, max %d cycles, "
              "%.1f ms solve, %.1f ms split",
              level, L->nseg, (long long)L->nrows, kBlock * L->rpt, (long long)steps, cyc, tb - ta,
              now_ms() - tb);
      if (o.profile && prof.ms > prof_ms0)
        fprintf(stderr, "; projection kernel %.1f ms, %.0f GB/s", prof.ms - prof_ms0,
                (prof.bytes - prof_bytes0) / (prof.ms - prof_ms0) * 1e-6);
      fprintf(stderr, "\n");
    }
    ++level;
    // advance; level 0 stays alive for the metrics
    Level *done = L;
    L = next;
    next = (done == &L0) ? &LB : done;
    if (next != &L0) *next = Level();
  }
  st.levels = level;
  std::vector<int32_t> poff(meshes.size(), 0);
  {
    int32_t off = 0;
    for (size_t b = 0; b < meshes.size(); ++b) {
      poff[b] = off;
      off += meshes[b].nparts;
    }
  }
  phase_to("rsb: metrics");
  if (L0.nseg > 0) partition_metrics(L0, d_part, (int32_t)parts_total, poff, &st, ctx);
  RSB_HIP(hipStreamSynchronize(ctx.stream));
  st.kernel_ms = prof.ms;
  st.kernel_bytes = prof.bytes;
  st.kernel_launches = prof.launches;
  st.ms_total = now_ms() - t0;
  if (stats) {
    const int32_t sz = stats->struct_size;
    *stats = st;
    stats->struct_size = sz;
  }
  out.status = worst;
  return out;
}

__global__ void k_negate(double *y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = -y[i];
}

// Device-side validation of a caller CSR (device pointers): columns in
// range, weights in [0, 15], rows monotone.
__global__ void k_check_csr(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ w, int64_t n, int *__restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t a = rp[i], b = rp[i + 1];
  if (b < a || a < 0) {
    atomicOr(bad, 1);
    return;
  }
  for (int64_t p = a; p < b; ++p)
    if (col[p] < 0 || col[p] >= n || w[p] < 0 || w[p] > (int32_t)kWeightMask) {
      atomicOr(bad, 1);
      return;
    }
}

void check_mesh(int64_t nelem, int32_t nv, const int64_t *ids) {
  if (!ids) fail(RSB_EINVAL, "elem_vertex_ids is NULL");
  if (nelem < 1) fail(RSB_EINVAL, "nelem < 1");
  if (nv < 1) fail(RSB_EINVAL, "nv_per_elem < 1");
  if (nelem >= kMaxRows) fail(RSB_EINVAL, "nelem too large (limit 2^28)");
  if (nelem * nv >= ((int64_t)1 << 31)) fail(RSB_EINVAL, "nelem * nv too large");
}

void check_stats(rsb_stats *s) {
  if (s && s->struct_size != (int32_t)sizeof(rsb_stats))
    fail(RSB_EINVAL, "stats->struct_size must be sizeof(rsb_stats)");
}

}  // namespace
}  // namespace rsb

using namespace rsb;

namespace {

// Validated device copy of a caller CSR (row_ptr int64[n+1], col int32,
// weight int32 in [0, 15]).
void load_csr(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const int32_t *weight,
              const rsb_opts &o, Ctx &ctx, DevCsr &g) {
  if (n < 1 || n >= kMaxRows || !row_ptr || !col_idx || !weight) fail(RSB_EINVAL, "bad arguments");
  const bool dev = o.device_pointers != 0;
  int64_t nnz = 0;
  if (!dev) {
    nnz = row_ptr[n];
    if (row_ptr[0] != 0) fail(RSB_EINVAL, "row_ptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
      if (row_ptr[i + 1] < row_ptr[i]) fail(RSB_EINVAL, "row_ptr not monotone");
    for (int64_t p = 0; p < nnz; ++p) {
      if (col_idx[p] < 0 || col_idx[p] >= n) fail(RSB_EINVAL, "column out of range");
      if (weight[p] < 0 || weight[p] > (int32_t)kWeightMask)
        fail(RSB_EINVAL, "weight out of [0, 15]");
    }
  }
  setup_ctx(ctx, o);
  if (dev) {
    int64_t r0 = 0;
    RSB_HIP(hipMemcpyAsync(&nnz, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipMemcpyAsync(&r0, row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost, ctx.stream));
    DevBuf<int> bad(ctx, 1);
    RSB_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), ctx.stream));
    k_check_csr<<<(unsigned)((n + 255) / 256), 256, 0, ctx.stream>>>(row_ptr, col_idx, weight, n,
                                                                    bad.get());
    RSB_LAUNCHED();
    int hbad = 0;
    RSB_HIP(hipMemcpyAsync(&hbad, bad.get(), sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    if (hbad || r0 != 0) fail(RSB_EINVAL, "invalid CSR (row_ptr, column or weight)");
  }
  if (nnz < 0) fail(RSB_EINVAL, "row_ptr[n] < 0");
  g.n = n;
  g.nnz = nnz;
  g.row_ptr.alloc(ctx, n + 1);
  g.col.alloc(ctx, std::max<int64_t>(nnz, 1));
  g.wgt.alloc(ctx, std::max<int64_t>(nnz, 1));
  auto kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  RSB_HIP(hipMemcpyAsync(g.row_ptr.get(), row_ptr, (n + 1) * sizeof(int64_t), kind, ctx.stream));
  if (nnz > 0) {
    RSB_HIP(hipMemcpyAsync(g.col.get(), col_idx, nnz * sizeof(int32_t), kind, ctx.stream));
    RSB_HIP(hipMemcpyAsync(g.wgt.get(), weight, nnz * sizeof(int32_t), kind, ctx.stream));
  }
}

// AMG hierarchy of a whole CSR graph (one segment, every row taking part),
// for the test entry points.
struct CsrAmg {
  Level L;
  DevBuf<int32_t> root;
  DevBuf<SegState> st;
  AmgDev A;
};

void csr_amg_setup(const DevCsr &g, CsrAmg &t, Ctx &ctx) {
  std::vector<const DevCsr *> gs{&g};
  std::vector<int32_t> np{2};
  level0_from_csr(t.L, gs, np, default_rpt(g.n), ctx);
  // the single segment starts at row 0: rows below n are elements
  std::vector<int32_t> hroot(t.L.nrows);
  for (int64_t i = 0; i < t.L.nrows; ++i) hroot[i] = i < g.n ? 0 : -1;
  SegState hs{};
  hs.solve = 1;
  hs.strad = 0;
  hs.active = 1;
  t.root.alloc(ctx, t.L.nrows);
  t.st.alloc(ctx, 1);
  RSB_HIP(hipMemcpyAsync(t.root.get(), hroot.data(), t.L.nrows * sizeof(int32_t),
                         hipMemcpyHostToDevice, ctx.stream));
  RSB_HIP(hipMemcpyAsync(t.st.get(), &hs, sizeof(SegState), hipMemcpyHostToDevice, ctx.stream));
  amg_setup(view_of(t.L), t.root.get(), t.st.get(), t.A, ctx);
}

}  // namespace

extern "C" {

int rsb_opts_init(rsb_opts *o) {
  if (!o) return RSB_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(rsb_opts);
  o->graph = RSB_GRAPH_WEIGHTED;
  o->method = RSB_LANCZOS;
  o->precision = RSB_FP64;
  o->lanczos_m = 100;
  o->max_restarts = 50;
  o->tol = 1e-6;
  o->inv_max_outer = 50;
  o->cg_max_iter = 20000;
  o->cg_tol = 1e-8;
  o->cg_full_projection = 0;
  o->batched = 1;
  o->seed = 20261203ull;
  o->use_hipgraph = 1;
  o->autotune = 0;
  o->autotune_cache = nullptr;
  o->device = 0;
  o->device_pointers = 0;
  o->stream = nullptr;
  o->device_mem_limit = 0;
  o->verbose = 0;
  o->profile = 0;
  o->inv_precond = RSB_PRECOND_NONE;
  o->amg_smooth = 1;
  o->amg_sigma = 2.0 / 3.0;
  o->fiedler_sweep = 0;
  o->sweep_gap = 0.1;
  o->lanczos_s = 1;
  o->pack_matrix = 1;
  o->bfs_start = 0;
  return RSB_OK;
}

const char *rsb_strerror(int code) {
  switch (code) {
    case RSB_OK: return "success";
    case RSB_WARN_NOT_CONVERGED: return "eigen-solver hit its iteration caps (result valid)";
    case RSB_WARN_DISCONNECTED: return "a bisected graph was disconnected (result valid)";
    case RSB_EINVAL: return "invalid argument";
    case RSB_ENOMEM: return "out of device memory";
    case RSB_EDEVICE: return "HIP runtime error";
    case RSB_EBUFFER: return "output buffer too small";
    case RSB_EINTERNAL: return "internal error";
    default: return "unknown code";
  }
}

const char *rsb_last_error(void) { return g_last_error.c_str(); }

int rsb_dual_graph(int64_t nelem, int32_t nv, const int64_t *ids, const rsb_opts *opts,
                   int64_t *row_ptr, int32_t *col_idx, int32_t *weight, int64_t *nnz_inout) {
  return guarded([&]() -> int {
    check_opts(opts);
    check_mesh(nelem, nv, ids);
    if (!nnz_inout) fail(RSB_EINVAL, "nnz_inout is NULL");
    if (col_idx && (!row_ptr || !weight)) fail(RSB_EINVAL, "row_ptr/weight NULL");
    Ctx ctx;
    setup_ctx(ctx, *opts);
    const bool dev = opts->device_pointers != 0;
    InArr<int64_t> in;
    in.init(ctx, ids, nelem * nv, dev);
    DevCsr g;
    build_dual_graph(in.p, nelem, nv, opts->graph, g, ctx);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    if (!col_idx) {
      *nnz_inout = g.nnz;
      if (row_ptr) copy_out(ctx, row_ptr, g.row_ptr.get(), nelem + 1, dev);
      RSB_HIP(hipStreamSynchronize(ctx.stream));
      return RSB_OK;
    }
    if (*nnz_inout < g.nnz) {
      *nnz_inout = g.nnz;
      return RSB_EBUFFER;
    }
    copy_out(ctx, row_ptr, g.row_ptr.get(), nelem + 1, dev);
    copy_out(ctx, col_idx, g.col.get(), g.nnz, dev);
    copy_out(ctx, weight, g.wgt.get(), g.nnz, dev);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    *nnz_inout = g.nnz;
    return RSB_OK;
  });
}

int rsb_laplacian_apply(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                        const int32_t *weight, const double *x, double *y, const rsb_opts *opts) {
  return guarded([&]() -> int {
    check_opts(opts);
    if (!x || !y) fail(RSB_EINVAL, "bad arguments");
    Ctx ctx;
    DevCsr g;
    load_csr(n, row_ptr, col_idx, weight, *opts, ctx, g);
    const bool dev = opts->device_pointers != 0;
    InArr<double> xin;
    xin.init(ctx, x, n, dev);
    DevBuf<double> yd(ctx, n);
    laplacian_apply_csr(g, xin.p, yd.get(), ctx);
    copy_out(ctx, y, yd.get(), n, dev);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return RSB_OK;
  });
}

int rsb_gs_apply(int64_t nelem, int32_t nv, const int64_t *ids, const double *x, double *y,
                 const rsb_opts *opts) {
  return guarded([&]() -> int {
    check_opts(opts);
    check_mesh(nelem, nv, ids);
    if (!x || !y) fail(RSB_EINVAL, "bad arguments");
    Ctx ctx;
    setup_ctx(ctx, *opts);
    const bool dev = opts->device_pointers != 0;
    InArr<int64_t> in;
    in.init(ctx, ids, nelem * nv, dev);
    GsBase B;
    gs_base_build({in.p}, {nelem}, nv, nullptr, B, ctx);
    // one level holding the whole mesh as one subgraph, rows = elements
    Level L;
    L.nrows = round_up(nelem, kWave);
    L.nseg = 1;
    std::vector<int32_t> orig(L.nrows, -1);
    for (int64_t i = 0; i < nelem; ++i) orig[i] = (int32_t)i;
    L.orig.alloc(ctx, L.nrows);
    RSB_HIP(hipMemcpyAsync(L.orig.get(), orig.data(), L.nrows * sizeof(int32_t),
                           hipMemcpyHostToDevice, ctx.stream));
    SegDev sd{};
    sd.row0 = 0;
    sd.n = (int32_t)nelem;
    sd.npad = (int32_t)L.nrows;
    L.d_seg.alloc(ctx, 1);
    RSB_HIP(hipMemcpyAsync(L.d_seg.get(), &sd, sizeof(sd), hipMemcpyHostToDevice, ctx.stream));
    gs_level_build(B, L, nelem, L.gs, ctx);
    InArr<double> xin;
    xin.init(ctx, x, nelem, dev);
    DevBuf<double> xd(ctx, L.nrows), yd(ctx, L.nrows);
    RSB_HIP(hipMemsetAsync(xd.get(), 0, L.nrows * sizeof(double), ctx.stream));
    RSB_HIP(hipMemcpyAsync(xd.get(), xin.p, nelem * sizeof(double), hipMemcpyDeviceToDevice,
                           ctx.stream));
    gs_apply(view_of(L).gs, L.nrows, xd.get(), yd.get(), ctx);
    copy_out(ctx, y, yd.get(), nelem, dev);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return RSB_OK;
  });
}

int rsb_locality_order(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                       const int32_t *weight, int32_t *order, const rsb_opts *opts) {
  return guarded([&]() -> int {
    check_opts(opts);
    if (!order) fail(RSB_EINVAL, "bad arguments");
    Ctx ctx;
    DevCsr g;
    load_csr(n, row_ptr, col_idx, weight, *opts, ctx, g);
    DevBuf<int32_t> perm;
    locality_order(g, perm, ctx);
    copy_out(ctx, order, perm.get(), n, opts->device_pointers != 0);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return RSB_OK;
  });
}

int rsb_amg_level(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                  const int32_t *weight, int32_t level, const rsb_opts *opts, int32_t *nlevels,
                  int64_t *nrows, int64_t *nnz, int64_t *row_ptr_out, int64_t *col_out,
                  int64_t *weight_out, int64_t *gid_out, int64_t *agg_out) {
  return guarded([&]() -> int {
    check_opts(opts);
    if (!nlevels || !nrows || !nnz) fail(RSB_EINVAL, "nlevels/nrows/nnz is NULL");
    if (col_out && (!row_ptr_out || !weight_out || !gid_out || !agg_out))
      fail(RSB_EINVAL, "output arrays must all be given");
    Ctx ctx;
    DevCsr g;
    load_csr(n, row_ptr, col_idx, weight, *opts, ctx, g);
    CsrAmg t;
    csr_amg_setup(g, t, ctx);
    *nlevels = (int32_t)t.A.lv.size();
    if (level < 0 || level >= *nlevels) fail(RSB_EINVAL, "level out of range");
    const AmgLevelDev &Z = t.A.lv[level];
    // host copies of the level (coarse levels: sliced ELL with separate words)
    const int64_t rows = Z.n;
    std::vector<int32_t> seg(rows), agg(rows), gid(rows), len(rows);
    RSB_HIP(hipMemcpyAsync(seg.data(), Z.seg.get(), rows * 4, hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipMemcpyAsync(agg.data(), Z.agg.get(), rows * 4, hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipMemcpyAsync(gid.data(), Z.gid, rows * 4, hipMemcpyDeviceToHost, ctx.stream));
    RSB_HIP(hipMemcpyAsync(len.data(), Z.rowlen.get(), rows * 4, hipMemcpyDeviceToHost,
                           ctx.stream));
    const int64_t nch = rows / 64;
    std::vector<int64_t> cp(nch + 1);
    const int64_t words = level == 0 ? t.L.words : Z.words;
    std::vector<uint32_t> packed, w;
    std::vector<int32_t> col;
    RSB_HIP(hipMemcpyAsync(cp.data(), Z.mat.chunk_ptr, (nch + 1) * 8, hipMemcpyDeviceToHost,
                           ctx.stream));
    if (level == 0) {
      packed.resize(std::max<int64_t>(words, 1));
      RSB_HIP(hipMemcpyAsync(packed.data(), Z.mat.packed, words * 4, hipMemcpyDeviceToHost,
                             ctx.stream));
    } else {
      col.resize(std::max<int64_t>(words, 1));
      w.resize(std::max<int64_t>(words, 1));
      RSB_HIP(hipMemcpyAsync(col.data(), Z.mat.col, words * 4, hipMemcpyDeviceToHost, ctx.stream));
      RSB_HIP(hipMemcpyAsync(w.data(), Z.mat.wgt, words * 4, hipMemcpyDeviceToHost, ctx.stream));
    }
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    int64_t nr = 0, nz = 0;
    for (int64_t i = 0; i < rows; ++i)
      if (seg[i] >= 0) {
        if (i != nr) fail(RSB_EINTERNAL, "AMG level rows not contiguous");
        ++nr;
        nz += len[i];
      }
    *nrows = nr;
    *nnz = nz;
    if (!col_out) return RSB_OK;
    int64_t k = 0;
    for (int64_t i = 0; i < nr; ++i) {
      row_ptr_out[i] = k;
      const int64_t base = cp[i >> 6] + (i & 63), width = (cp[(i >> 6) + 1] - cp[i >> 6]) >> 6;
      for (int64_t q = 0; q < width; ++q) {
        const int64_t at = base + q * 64;
        const int64_t c = level == 0 ? (int64_t)colw_col(packed[at]) : col[at];
        const int64_t wt = level == 0 ? (int64_t)colw_wt(packed[at]) : (int64_t)w[at];
        if (wt == 0) continue;
        col_out[k] = c;
        weight_out[k] = wt;
        ++k;
      }
      gid_out[i] = gid[i];
      agg_out[i] = agg[i];
    }
    row_ptr_out[nr] = k;
    if (k != nz) fail(RSB_EINTERNAL, "AMG level row lengths disagree with slots");
    return RSB_OK;
  });
}

int rsb_amg_vcycle(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                   const int32_t *weight, const double *f, double *u, const rsb_opts *opts) {
  return guarded([&]() -> int {
    check_opts(opts);
    if (!f || !u) fail(RSB_EINVAL, "bad arguments");
    Ctx ctx;
    DevCsr g;
    load_csr(n, row_ptr, col_idx, weight, *opts, ctx, g);
    CsrAmg t;
    t.A.sigma = opts->amg_sigma;
    t.A.nsmooth = opts->amg_smooth;
    csr_amg_setup(g, t, ctx);
    const bool dev = opts->device_pointers != 0;
    InArr<double> fin;
    fin.init(ctx, f, n, dev);
    DevBuf<double> fl(ctx, t.L.nrows);
    RSB_HIP(hipMemsetAsync(fl.get(), 0, fl.bytes(), ctx.stream));
    RSB_HIP(hipMemcpyAsync(fl.get(), fin.p, n * sizeof(double), hipMemcpyDeviceToDevice,
                           ctx.stream));
    const double *res = amg_vcycle(t.A, fl.get(), nullptr, ctx.stream);
    if (res != amg_result(t.A)) fail(RSB_EINTERNAL, "V-cycle result buffer");
    copy_out(ctx, u, res, n, dev);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return RSB_OK;
  });
}

int rsb_split(int64_t n, const double *y, const int64_t *gid, int64_t n_low, uint8_t *side,
              const rsb_opts *opts) {
  return guarded([&]() -> int {
    check_opts(opts);
    if (n < 1 || n >= kMaxRows || !y || !gid || !side) fail(RSB_EINVAL, "bad arguments");
    if (n_low < 0 || n_low > n) fail(RSB_EINVAL, "n_low out of [0, n]");
    const bool dev = opts->device_pointers != 0;
    if (!dev) {
      for (int64_t i = 0; i < n; ++i)
        if (std::isnan(y[i])) fail(RSB_EINVAL, "NaN in y");
    }
    Ctx ctx;
    setup_ctx(ctx, *opts);
    InArr<double> yin;
    yin.init(ctx, y, n, dev);
    InArr<int64_t> gin;
    gin.init(ctx, gid, n, dev);
    DevBuf<uint8_t> sd(ctx, n);
    split_vector(yin.p, gin.p, n, n_low, sd.get(), ctx);
    copy_out(ctx, side, sd.get(), n, dev);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return RSB_OK;
  });
}

int rsb_fiedler(int64_t nelem, int32_t nv, const int64_t *ids, const rsb_opts *opts,
                double *fiedler_out, double *lambda2_out, rsb_stats *stats_out) {
  return guarded([&]() -> int {
    check_opts(opts);
    check_mesh(nelem, nv, ids);
    check_stats(stats_out);
    if (nelem < 2) fail(RSB_EINVAL, "nelem < 2");
    if (!fiedler_out || !lambda2_out) fail(RSB_EINVAL, "output pointer NULL");
    Ctx ctx;
    setup_ctx(ctx, *opts);
    const bool dev = opts->device_pointers != 0;
    InArr<int64_t> in;
    in.init(ctx, ids, nelem * nv, dev);
    std::vector<MeshIn> meshes{{nelem, in.p, 2}};
    DevBuf<double> yd(ctx, nelem);
    RunOut r = run_rsb(meshes, nv, *opts, ctx, nullptr, stats_out, yd.get());
    if (r.flip) {
      k_negate<<<(unsigned)((nelem + 255) / 256), 256, 0, ctx.stream>>>(yd.get(), nelem);
      RSB_LAUNCHED();
    }
    copy_out(ctx, fiedler_out, yd.get(), nelem, dev);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    *lambda2_out = r.lambda;
    return r.status;
  });
}

int rsb_partition(int64_t nelem, int32_t nv, const int64_t *ids, int32_t nparts,
                  const rsb_opts *opts, int32_t *part_out, rsb_stats *stats_out) {
  return guarded([&]() -> int {
    check_opts(opts);
    check_mesh(nelem, nv, ids);
    check_stats(stats_out);
    if (nparts < 1 || nparts > nelem) fail(RSB_EINVAL, "nparts must be in [1, nelem]");
    if (!part_out) fail(RSB_EINVAL, "part_out is NULL");
    Ctx ctx;
    setup_ctx(ctx, *opts);
    const bool dev = opts->device_pointers != 0;
    InArr<int64_t> in;
    in.init(ctx, ids, nelem * nv, dev);
    DevBuf<int32_t> own;
    int32_t *dpart = part_out;
    if (!dev) {
      own.alloc(ctx, nelem);
      dpart = own.get();
    }
    std::vector<MeshIn> meshes{{nelem, in.p, nparts}};
    RunOut r = run_rsb(meshes, nv, *opts, ctx, dpart, stats_out, nullptr);
    if (!dev) copy_out(ctx, part_out, (const int32_t *)dpart, nelem, false);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return r.status;
  });
}

int rsb_partition_noalloc(int64_t nelem, int32_t nv, const int64_t *ids, int32_t nparts,
                          const rsb_opts *opts, int32_t *part_out, rsb_stats *stats_out) {
  return guarded([&]() -> int {
    check_opts(opts);
    check_mesh(nelem, nv, ids);
    check_stats(stats_out);
    if (nparts < 1 || nparts > nelem) fail(RSB_EINVAL, "nparts must be in [1, nelem]");
    if (!part_out) fail(RSB_EINVAL, "part_out is NULL");
    if (nelem > RSB_NOALLOC_MAX_ELEMS || nparts > RSB_NOALLOC_MAX_PARTS)
      fail(RSB_EINVAL, "rsb_partition_noalloc takes at most " +
                           std::to_string(RSB_NOALLOC_MAX_ELEMS) + " elements and " +
                           std::to_string(RSB_NOALLOC_MAX_PARTS) + " parts (got " +
                           std::to_string(nelem) + " and " + std::to_string(nparts) + ")");
    // graph replay, profiling events and tile trials allocate: all off
    rsb_opts o = *opts;
    o.use_hipgraph = 0;
    o.profile = 0;
    o.autotune = 0;
    NoallocRegion &reg = noalloc_region(o.device);
    std::lock_guard<std::mutex> lock(reg.mu);
    Ctx ctx;
    setup_ctx(ctx, o, false);
    // (the last MiB is never handed out: a streaming kernel's unconditional
    // reads just past its buffer stay inside the array)
    reg.arena.reset(reg.ptr, reg.bytes - ((size_t)1 << 20));
    ctx.arena = &reg.arena;
    // whatever happens, the call's work on the region ends before the next
    // call may use it
    struct Drain {
      hipStream_t s;
      ~Drain() { (void)hipStreamSynchronize(s); }
    } drain{ctx.stream};
    const bool dev = o.device_pointers != 0;
    InArr<int64_t> in;
    in.init(ctx, ids, nelem * nv, dev);
    DevBuf<int32_t> own;
    int32_t *dpart = part_out;
    if (!dev) {
      own.alloc(ctx, nelem);
      dpart = own.get();
    }
    std::vector<MeshIn> meshes{{nelem, in.p, nparts}};
    RunOut r = run_rsb(meshes, nv, o, ctx, dpart, stats_out, nullptr);
    if (!dev) copy_out(ctx, part_out, (const int32_t *)dpart, nelem, false);
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return r.status;
  });
}

int rsb_hbm_probe(int32_t kind, int64_t bytes, int32_t reps, const rsb_opts *opts,
                  double *gbs_out) {
  return guarded([&]() -> int {
    check_opts(opts);
    if (kind < 0 || kind > 2 || bytes < 4096 || reps < 1 || !gbs_out)
      fail(RSB_EINVAL, "rsb_hbm_probe: kind 0, 1 or 2, bytes >= 4096, reps >= 1, gbs_out "
                       "non-NULL");
    Ctx ctx;
    setup_ctx(ctx, *opts);
    *gbs_out = hbm_probe_gbs(kind, bytes, reps, opts->device, ctx);
    return RSB_OK;
  });
}

int rsb_partition_batch(int32_t nmesh, const int64_t *nelem, int32_t nv,
                        const int64_t *const *ids, const int32_t *nparts, const rsb_opts *opts,
                        int32_t *const *part_out, rsb_stats *stats_out) {
  return guarded([&]() -> int {
    check_opts(opts);
    check_stats(stats_out);
    if (nmesh < 1 || !nelem || !ids || !nparts || !part_out) fail(RSB_EINVAL, "bad arguments");
    int64_t total = 0;
    for (int b = 0; b < nmesh; ++b) {
      check_mesh(nelem[b], nv, ids[b]);
      if (nparts[b] < 1 || nparts[b] > nelem[b]) fail(RSB_EINVAL, "nparts out of range");
      if (!part_out[b]) fail(RSB_EINVAL, "part_out entry NULL");
      total += nelem[b];
    }
    if (total >= kMaxRows) fail(RSB_EINVAL, "too many elements (limit 2^28 per call)");
    Ctx ctx;
    setup_ctx(ctx, *opts);
    const bool dev = opts->device_pointers != 0;
    std::vector<InArr<int64_t>> in(nmesh);
    std::vector<MeshIn> meshes;
    for (int b = 0; b < nmesh; ++b) {
      in[b].init(ctx, ids[b], nelem[b] * nv, dev);
      meshes.push_back({nelem[b], in[b].p, nparts[b]});
    }
    DevBuf<int32_t> dpart(ctx, total);
    RunOut r = run_rsb(meshes, nv, *opts, ctx, dpart.get(), stats_out, nullptr);
    int64_t off = 0;
    for (int b = 0; b < nmesh; ++b) {
      copy_out(ctx, part_out[b], (const int32_t *)dpart.get() + off, nelem[b], dev);
      off += nelem[b];
    }
    RSB_HIP(hipStreamSynchronize(ctx.stream));
    return r.status;
  });
}

}  // extern "C"
