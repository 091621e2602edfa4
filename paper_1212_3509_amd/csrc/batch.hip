// Batched full-format apply: many magnetization states on uneven grids.
//
// Every state has its own grid and factor tables (same quadrature rule).
// The 23 products per node of each state (see build_chunk in api.hip) are
// cut into tiles (64 columns x 16*RB rows of one job; on axes of at most
// kThinN cells, vector-ALU tiles of 256 thin_cols columns, launched apart
// before the stage's matrix-core tiles, one workgroup each); the tiles of one
// stage, over all states, form one list that a single persistent launch
// works off through a counter (each workgroup draws the next item; the tiles
// write disjoint outputs, so results are bitwise reproducible).  Items are
// sorted by decreasing cost, so the draw is a longest-first greedy schedule.  Nodes are
// processed in chunks sized to the workspace limit; the launch sequence can
// be captured once as a HIP graph and replayed.
//
// The row-block shape RB of each item comes from a tuning table keyed by
// (precision, axis length, outputs per job): by default the smallest RB that
// covers the axis in one row group, or the measured best after
// demag_batch_tune, which times the candidates on the device and can persist
// them as JSON.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

struct demag_batch {
  demag_prec prec;
  int count = 0;
  int M = 0;
  int kc = 0, nchunks = 0;
  int nmax = 0;
  int grid = 0;                                   // persistent workgroups per launch
  std::vector<demag_factors *> factors;
  std::vector<int64_t> off;                       // cell offsets, count + 1
  void *gens = nullptr;                           // all states' axis tables, FP32 or FP64
  std::vector<int64_t> gen_base;                  // [state][axis] element offsets into gens
  void *ws = nullptr;
  size_t ws_bytes = 0;
  // per chunk, per stage (z, y, x): device item lists
  struct Launch {
    demag::BatchItem *d_items = nullptr;
    int nitems = 0;
    demag::BatchItem *d_thin = nullptr;           // thin-axis items, one workgroup each
    int nthin = 0;
  };
  std::vector<std::vector<Launch>> launches;
  demag::MPJob *d_jobs = nullptr;
  demag::MPTerm *d_terms = nullptr;
  demag::MPGeom *d_geoms = nullptr;
  int *d_counters = nullptr;                      // one item counter per launch
  std::map<std::pair<int, int>, int> rb_choice;   // (n, nout) -> RB
  double flops = 0;                               // algorithmic FLOPs of one apply
  hipEvent_t used = nullptr;                      // recorded after each apply's work
  // captured graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *g_m = nullptr;
  void *g_phi = nullptr, *g_h = nullptr;
  hipStream_t g_stream = nullptr;
};

namespace demag {

namespace {

enum Buf { B_M = 0, B_Y1 = 1, B_Y2 = 2, B_PHI = 3, B_H = 4 };

int ceil_div(int a, int b) { return (a + b - 1) / b; }

demag_status build(demag_ctx *ctx, demag_batch *b) {
  const int M = b->M;
  const size_t esize = (b->prec == DEMAG_FP64) ? 8 : 4;
  const int64_t Ntot = b->off.back();
  // node chunk size: 12 intermediates per node per cell
  const size_t per_node = size_t(12) * Ntot * esize;
  int kc = M;
  while (kc > 1 && per_node * kc > ctx->ws_limit) kc = (kc + 1) / 2;
  if (per_node > ctx->ws_limit) {
    set_error("batch: workspace limit below one node of intermediates");
    return DEMAG_E_NOMEM;
  }
  b->kc = kc;
  b->nchunks = ceil_div(M, kc);
  std::vector<MPJob> jobs;
  std::vector<MPTerm> terms;
  std::vector<MPGeom> geoms;
  b->launches.assign(b->nchunks, std::vector<demag_batch::Launch>(3));
  std::vector<std::vector<std::vector<BatchItem>>> items(b->nchunks, std::vector<std::vector<BatchItem>>(3));
  std::vector<std::vector<std::vector<double>>> costs(b->nchunks, std::vector<std::vector<double>>(3));
  std::vector<std::vector<std::vector<BatchItem>>> thin(b->nchunks, std::vector<std::vector<BatchItem>>(3));
  b->flops = 0;
  for (int s = 0; s < b->count; ++s) {
    const demag_factors *f = b->factors[s];
    const int nx = f->n[0], ny = f->n[1], nz = f->n[2];
    const int64_t N = int64_t(nx) * ny * nz, P = int64_t(nx) * ny;
    const int64_t mo = 3 * b->off[s], po = b->off[s], ho = 3 * b->off[s];
    const int64_t wo = 6 * int64_t(kc) * b->off[s];   // state slice of Y1 and Y2
    const int gz = int(geoms.size());
    geoms.push_back(MPGeom{nz, int(P), int(P), 2 * nz - 1, P, 0, 0, 1, P});
    geoms.push_back(MPGeom{ny, nz * nx, nx, 2 * ny - 1, nx, P, P, ny, 1});
    geoms.push_back(MPGeom{nx, nz * ny, ny, 2 * nx - 1, ny, P, P, nx, 1});
    const int axis_of_stage[3] = {2, 1, 0};
    for (int c = 0; c < b->nchunks; ++c) {
      const int k0 = c * kc, kcc = std::min(kc, M - k0);
      auto y1 = [&](int kl, int sl) { return wo + (int64_t(kl) * 6 + sl) * N; };
      auto gen = [&](int stage, int type, int k) {
        return b->gen_base[size_t(s) * 3 + axis_of_stage[stage]] + int64_t(type * M + k) * (2 * f->n[axis_of_stage[stage]] - 1);
      };
      auto term = [&](int stage, int buf, int64_t off, int t0, int t1, int k) {
        MPTerm t{};
        t.in_buf = buf;
        t.in_off = off;
        t.gen[0] = t0 * M + k;
        t.gen[1] = t1 * M + k;
        t.gen_off[0] = gen(stage, t0, k);
        t.gen_off[1] = gen(stage, t1, k);
        return t;
      };
      auto add = [&](int stage, int nout, std::vector<MPTerm> ts, int ob0, int64_t oo0, double s0, int ob1,
                     int64_t oo1) {
        MPJob j{};
        j.term0 = int32_t(terms.size());
        j.nterms = int32_t(ts.size());
        j.out_buf[0] = ob0;
        j.out_off[0] = oo0;
        j.scale[0] = s0;
        j.out_buf[1] = ob1;
        j.out_off[1] = oo1;
        j.scale[1] = 1.0;
        for (auto &t : ts) terms.push_back(t);
        const int jid = int(jobs.size());
        jobs.push_back(j);
        const MPGeom &g = geoms[gz + stage];
        b->flops += 2.0 * g.n * double(g.n) * g.C * j.nterms * nout;
        if (g.n <= kThinN) {
          // thin axis: vector-ALU tiles of 256 thin_cols columns, own launch
          const int cols = 256 * thin_cols(thin_nmax(g.n), int(esize));
          for (int ct = 0; ct < ceil_div(g.C, cols); ++ct)
            thin[c][stage].push_back(BatchItem{jid, gz + stage, ct, 0, 0, int8_t(nout)});
          return;
        }
        int rb = default_rb(g.n);
        auto it = b->rb_choice.find({g.n, nout});
        if (it != b->rb_choice.end()) rb = it->second;
        const int rgs = ceil_div(g.n, 16 * rb), cts = ceil_div(g.C, 64);
        const double cost = double(j.nterms) * nout * (16.0 * rb) * g.n;
        for (int rg = 0; rg < rgs; ++rg)
          for (int ct = 0; ct < cts; ++ct) {
            items[c][stage].push_back(BatchItem{jid, gz + stage, ct, int16_t(rg), int8_t(rb), int8_t(nout)});
            costs[c][stage].push_back(cost);
          }
      };
      for (int kl = 0; kl < kcc; ++kl) {
        const int k = k0 + kl;
        // stage 1 (z): Y1 slots 0..5
        add(0, 2, {term(0, B_M, mo + 2 * N, F_X, F_P, k)}, B_Y1, y1(kl, 0), 1.0, B_Y1, y1(kl, 1));
        add(0, 2, {term(0, B_M, mo + 0, F_E, F_Q, k)}, B_Y1, y1(kl, 2), 1.0, B_Y1, y1(kl, 3));
        add(0, 2, {term(0, B_M, mo + N, F_E, F_Q, k)}, B_Y1, y1(kl, 4), 1.0, B_Y1, y1(kl, 5));
        // stage 2 (y): Y2 slots 0..5
        add(1, 2, {term(1, B_Y1, y1(kl, 0), F_E, F_Q, k), term(1, B_Y1, y1(kl, 4), F_X, F_P, k)}, B_Y2, y1(kl, 0),
            1.0, B_Y2, y1(kl, 1));
        add(1, 2, {term(1, B_Y1, y1(kl, 2), F_E, F_Q, k)}, B_Y2, y1(kl, 2), 1.0, B_Y2, y1(kl, 3));
        add(1, 1, {term(1, B_Y1, y1(kl, 1), F_E, F_E, k), term(1, B_Y1, y1(kl, 5), F_X, F_X, k)}, B_Y2, y1(kl, 4),
            1.0, B_Y2, y1(kl, 4));
        add(1, 1, {term(1, B_Y1, y1(kl, 3), F_E, F_E, k)}, B_Y2, y1(kl, 5), 1.0, B_Y2, y1(kl, 5));
      }
      // stage 3 (x): accumulate over the chunk's nodes
      std::vector<MPTerm> t3a, t3y, t3z;
      for (int kl = 0; kl < kcc; ++kl) {
        const int k = k0 + kl;
        t3a.push_back(term(2, B_Y2, y1(kl, 0), F_E, F_Q, k));
        t3a.push_back(term(2, B_Y2, y1(kl, 2), F_X, F_P, k));
        t3y.push_back(term(2, B_Y2, y1(kl, 1), F_E, F_E, k));
        t3y.push_back(term(2, B_Y2, y1(kl, 3), F_X, F_X, k));
        t3z.push_back(term(2, B_Y2, y1(kl, 4), F_E, F_E, k));
        t3z.push_back(term(2, B_Y2, y1(kl, 5), F_X, F_X, k));
      }
      add(2, 2, t3a, B_PHI, po, f->L, B_H, ho);
      add(2, 1, t3y, B_H, ho + N, 1.0, B_H, ho + N);
      add(2, 1, t3z, B_H, ho + 2 * N, 1.0, B_H, ho + 2 * N);
    }
  }
  // upload tables and cost-sorted item lists
  DEMAG_TRY_HIP(hipMalloc(&b->d_jobs, sizeof(MPJob) * jobs.size()));
  DEMAG_TRY_HIP(hipMemcpy(b->d_jobs, jobs.data(), sizeof(MPJob) * jobs.size(), hipMemcpyHostToDevice));
  DEMAG_TRY_HIP(hipMalloc(&b->d_terms, sizeof(MPTerm) * terms.size()));
  DEMAG_TRY_HIP(hipMemcpy(b->d_terms, terms.data(), sizeof(MPTerm) * terms.size(), hipMemcpyHostToDevice));
  DEMAG_TRY_HIP(hipMalloc(&b->d_geoms, sizeof(MPGeom) * geoms.size()));
  DEMAG_TRY_HIP(hipMemcpy(b->d_geoms, geoms.data(), sizeof(MPGeom) * geoms.size(), hipMemcpyHostToDevice));
  for (int c = 0; c < b->nchunks; ++c)
    for (int st = 0; st < 3; ++st) {
      auto &v = items[c][st];
      auto &w = costs[c][st];
      std::vector<size_t> idx(v.size());
      for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
      std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t bb) { return w[a] > w[bb]; });
      std::vector<BatchItem> sorted(v.size());
      for (size_t i = 0; i < idx.size(); ++i) sorted[i] = v[idx[i]];
      auto &L = b->launches[c][st];
      L.nitems = int(sorted.size());
      DEMAG_TRY_HIP(hipMalloc(&L.d_items, sizeof(BatchItem) * std::max<size_t>(1, sorted.size())));
      DEMAG_TRY_HIP(hipMemcpy(L.d_items, sorted.data(), sizeof(BatchItem) * sorted.size(), hipMemcpyHostToDevice));
      const auto &tv = thin[c][st];
      L.nthin = int(tv.size());
      if (L.nthin > 0) {
        DEMAG_TRY_HIP(hipMalloc(&L.d_thin, sizeof(BatchItem) * tv.size()));
        DEMAG_TRY_HIP(hipMemcpy(L.d_thin, tv.data(), sizeof(BatchItem) * tv.size(), hipMemcpyHostToDevice));
      }
    }
  DEMAG_TRY_HIP(hipMalloc(&b->d_counters, sizeof(int) * size_t(b->nchunks) * 3));
  b->ws_bytes = size_t(12) * kc * Ntot * esize;
  hipError_t e = hipMalloc(&b->ws, b->ws_bytes);
  if (e != hipSuccess) {
    b->ws = nullptr;
    set_error("batch: workspace allocation failed");
    return DEMAG_E_NOMEM;
  }
  return DEMAG_OK;
}

void release_tables(demag_batch *b) {
  for (auto &v : b->launches)
    for (auto &L : v) {
      if (L.d_items) (void)hipFree(L.d_items);
      if (L.d_thin) (void)hipFree(L.d_thin);
    }
  b->launches.clear();
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_terms) (void)hipFree(b->d_terms);
  if (b->d_geoms) (void)hipFree(b->d_geoms);
  if (b->d_counters) (void)hipFree(b->d_counters);
  b->d_counters = nullptr;
  if (b->ws) (void)hipFree(b->ws);
  b->d_jobs = nullptr;
  b->d_terms = nullptr;
  b->d_geoms = nullptr;
  b->ws = nullptr;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

demag_status enqueue(demag_ctx *ctx, demag_batch *b, const void *m, void *phi, void *h) {
  char *ws = static_cast<char *>(b->ws);
  const size_t esize = (b->prec == DEMAG_FP64) ? 8 : 4;
  void *y1 = ws;
  void *y2 = ws + size_t(6) * b->kc * b->off.back() * esize;
  void *bufs[6] = {const_cast<void *>(m), y1, y2, phi, h, nullptr};
  demag_status s = launch_reset_counters(ctx, b->d_counters, b->nchunks * 3);
  if (s != DEMAG_OK) return s;
  for (int c = 0; c < b->nchunks; ++c)
    for (int st = 0; st < 3; ++st) {
      const auto &L = b->launches[c][st];
      const int beta = (st == 2 && c > 0) ? 1 : 0;
      s = launch_thin_items(ctx, b->prec, L.d_thin, L.nthin, b->d_jobs, b->d_terms, b->d_geoms, bufs, b->gens, beta);
      if (s != DEMAG_OK) return s;
      s = launch_items(ctx, b->prec, L.d_items, L.nitems, b->grid, b->d_jobs, b->d_terms, b->d_geoms, bufs, b->gens,
                       b->nmax, beta, b->d_counters + c * 3 + st);
      if (s != DEMAG_OK) return s;
    }
  return DEMAG_OK;
}

std::string tune_key(demag_prec p, int n, int nout) {
  std::ostringstream o;
  o << (p == DEMAG_FP64 ? "fp64" : "fp32") << "/n" << n << "/nout" << nout;
  return o.str();
}

}  // namespace
}  // namespace demag

using namespace demag;

extern "C" {

demag_status demag_batch_create(demag_ctx *ctx, int32_t count, const demag_grid *grids, const demag_quad *quad,
                                demag_prec prec, demag_batch **out) {
  DEMAG_REQUIRE(ctx && grids && quad && out, "demag_batch_create: NULL argument");
  DEMAG_REQUIRE(count >= 1 && count <= 65536, "demag_batch_create: count must be in [1, 65536]");
  DEMAG_REQUIRE(prec == DEMAG_FP64 || prec == DEMAG_FP32, "demag_batch_create: FP64 or FP32 only");
  for (int s = 0; s < count; ++s)
    for (int d = 0; d < 3; ++d)
      DEMAG_REQUIRE(grids[s].n[d] >= 1 && grids[s].n[d] <= 1024, "demag_batch_create: 1 <= n <= 1024 per axis");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  auto b = std::make_unique<demag_batch>();
  b->prec = prec;
  b->count = count;
  b->off.assign(count + 1, 0);
  size_t gen_total = 0;
  for (int s = 0; s < count; ++s) {
    demag_factors *f = nullptr;
    demag_status st = demag_assemble_factors(ctx, &grids[s], quad, &f);
    if (st != DEMAG_OK) {
      for (auto *g : b->factors) demag_factors_free(g);
      return st;
    }
    b->factors.push_back(f);
    b->off[s + 1] = b->off[s] + int64_t(f->n[0]) * f->n[1] * f->n[2];
    for (int d = 0; d < 3; ++d) {
      b->gen_base.push_back(int64_t(gen_total));
      gen_total += axis_table_len(f, d);
      b->nmax = std::max(b->nmax, f->n[d]);
    }
  }
  b->M = b->factors[0]->M;
  const size_t esize = (prec == DEMAG_FP64) ? 8 : 4;
  DEMAG_TRY_HIP(hipMalloc(&b->gens, gen_total * esize));
  for (int s = 0; s < count; ++s)
    for (int d = 0; d < 3; ++d) {
      const demag_factors *f = b->factors[s];
      const void *src = (prec == DEMAG_FP64) ? static_cast<const void *>(f->f64[d]) : static_cast<const void *>(f->f32[d]);
      DEMAG_TRY_HIP(hipMemcpyAsync(static_cast<char *>(b->gens) + b->gen_base[size_t(s) * 3 + d] * esize, src,
                                   axis_table_len(f, d) * esize, hipMemcpyDeviceToDevice, ctx->stream));
    }
  // persistent grid: as many workgroups as fit on the chip at once
  int dev_cus = 0;
  DEMAG_TRY_HIP(hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  const int per_cu = items_blocks_per_cu(prec == DEMAG_FP64, items_lds_bytes(b->nmax, prec == DEMAG_FP64));
  b->grid = std::max(1, dev_cus * std::max(1, per_cu));
  demag_status st = build(ctx, b.get());
  if (st == DEMAG_OK) {
    // the table copies above are asynchronous: demag_batch_free waits for them
    if (hipEventCreateWithFlags(&b->used, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(b->used, ctx->stream) != hipSuccess) {
      (void)hipStreamSynchronize(ctx->stream);
      set_error("demag_batch_create: event record failed");
      st = DEMAG_E_HIP;
    }
  }
  if (st != DEMAG_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    if (b->used) (void)hipEventDestroy(b->used);
    release_tables(b.get());
    for (auto *g : b->factors) demag_factors_free(g);
    return st;
  }
  *out = b.release();
  return DEMAG_OK;
}

demag_status demag_batch_free(demag_batch *b) {
  if (!b) return DEMAG_OK;
  // wait for the last work that reads the batch's tables: the set-up's
  // copies or the last apply (the tuner synchronizes its own work)
  if (b->used) {
    (void)hipEventSynchronize(b->used);
    (void)hipEventDestroy(b->used);
  }
  release_tables(b);
  if (b->gens) (void)hipFree(b->gens);
  for (auto *f : b->factors) demag_factors_free(f);
  delete b;
  return DEMAG_OK;
}

demag_status demag_batch_offsets(const demag_batch *b, int64_t *cell_offsets) {
  DEMAG_REQUIRE(b && cell_offsets, "demag_batch_offsets: NULL argument");
  std::memcpy(cell_offsets, b->off.data(), sizeof(int64_t) * (b->count + 1));
  return DEMAG_OK;
}

demag_status demag_batch_info(const demag_batch *b, int32_t *node_chunk, int32_t *persistent_groups,
                              double *flops_per_apply) {
  DEMAG_REQUIRE(b, "demag_batch_info: NULL argument");
  if (node_chunk) *node_chunk = b->kc;
  if (persistent_groups) *persistent_groups = b->grid;
  if (flops_per_apply) *flops_per_apply = b->flops;
  return DEMAG_OK;
}

namespace {
demag_status batch_apply(demag_ctx *ctx, demag_batch *b, const void *m, void *phi, void *h, int32_t use_graph) {
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  {
    const demag_status cs = check_finite(ctx, m, size_t(3) * size_t(b->off.back()), b->prec == DEMAG_FP64,
                                         "demag_batch_apply");
    if (cs != DEMAG_OK) return cs;
  }
  hipEvent_t ev = nullptr;
  if (!use_graph) {
    demag_status st = prof_begin(ctx, &ev);
    if (st != DEMAG_OK) return st;
    st = enqueue(ctx, b, m, phi, h);
    if (st != DEMAG_OK) return st;
    if (ev) return prof_end(ctx, ev, std::string(b->prec == DEMAG_FP64 ? "fp64" : "fp32") + "/batch", b->flops, 0.0);
    return DEMAG_OK;
  }
  if (!b->exec || b->g_m != m || b->g_phi != phi || b->g_h != h || b->g_stream != ctx->stream) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    hipStream_t cs = nullptr;
    DEMAG_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    ctx->stream = cs;
    DEMAG_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    demag_status st = enqueue(ctx, b, m, phi, h);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    ctx->stream = saved;
    ctx->profiling = prof;
    (void)hipStreamDestroy(cs);
    if (st != DEMAG_OK) return st;
    DEMAG_TRY_HIP(e);
    b->graph = g;
    DEMAG_TRY_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->g_m = m;
    b->g_phi = phi;
    b->g_h = h;
    b->g_stream = ctx->stream;
  }
  demag_status st = prof_begin(ctx, &ev);
  if (st != DEMAG_OK) return st;
  DEMAG_TRY_HIP(hipGraphLaunch(b->exec, ctx->stream));
  if (ev) return prof_end(ctx, ev, std::string(b->prec == DEMAG_FP64 ? "fp64" : "fp32") + "/batch_graph", b->flops, 0.0);
  return DEMAG_OK;
}
}  // namespace

demag_status demag_batch_apply(demag_ctx *ctx, demag_batch *b, const void *m, void *phi, void *h, int32_t use_graph) {
  DEMAG_REQUIRE(ctx && b && m && phi && h, "demag_batch_apply: NULL argument");
  const demag_status st = batch_apply(ctx, b, m, phi, h, use_graph);
  if (st != DEMAG_OK) return st;
  if (!b->used) DEMAG_TRY_HIP(hipEventCreateWithFlags(&b->used, hipEventDisableTiming));
  DEMAG_TRY_HIP(hipEventRecord(b->used, ctx->stream));
  return DEMAG_OK;
}

// Autotuner: the row-block shape RB of every item is default_rb(n) shifted
// by one of {-1, 0, +1} powers of two per axis-length bucket (n <= 32,
// n <= 96, larger).  Starting from no shift, each bucket's two alternatives
// are timed in place (the whole batch apply, `reps` repetitions after a
// warm-up, on scratch fields), keeping a shift when it is faster.  Timing
// the persistent launch itself matters: a stage launched alone for one
// state prefers small tiles for parallelism that the batch already has.
// The resulting table {"fp32/n96/nout2": 8, ...} is merged into the JSON
// object at path; when the file already holds every class of the batch, it
// is used without timing.
demag_status demag_batch_tune(demag_ctx *ctx, demag_batch *b, const char *path, int32_t reps) {
  DEMAG_REQUIRE(ctx && b, "demag_batch_tune: NULL argument");
  DEMAG_REQUIRE(reps >= 1 && reps <= 100, "demag_batch_tune: reps must be in [1, 100]");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  std::map<std::string, int> cache;
  if (path) {
    std::ifstream in(path);
    std::string line, all;
    while (std::getline(in, line)) all += line;
    size_t pos = 0;
    while ((pos = all.find('"', pos)) != std::string::npos) {
      size_t end = all.find('"', pos + 1);
      if (end == std::string::npos) break;
      std::string key = all.substr(pos + 1, end - pos - 1);
      size_t colon = all.find(':', end);
      if (colon == std::string::npos) break;
      cache[key] = std::atoi(all.c_str() + colon + 1);
      pos = all.find_first_of(",}", colon);
      if (pos == std::string::npos) break;
    }
  }
  // axis lengths of the batch
  std::vector<int> lens;
  for (int s = 0; s < b->count; ++s)
    for (int d = 0; d < 3; ++d)
      if (std::find(lens.begin(), lens.end(), b->factors[s]->n[d]) == lens.end()) lens.push_back(b->factors[s]->n[d]);
  bool cached = true;
  for (int n : lens)
    for (int nout = 1; nout <= 2; ++nout) cached = cached && cache.count(tune_key(b->prec, n, nout));
  auto bucket = [](int n) { return n <= 32 ? 0 : n <= 96 ? 1 : 2; };
  auto shifted = [](int n, int sh) {
    int rb = default_rb(n);
    for (; sh > 0 && rb < 8; --sh) rb *= 2;
    for (; sh < 0 && rb > 1; ++sh) rb /= 2;
    return rb;
  };
  auto apply = [&](const int sh[3]) -> demag_status {
    b->rb_choice.clear();
    for (int n : lens)
      for (int nout = 1; nout <= 2; ++nout) b->rb_choice[{n, nout}] = shifted(n, sh[bucket(n)]);
    release_tables(b);
    return build(ctx, b);
  };
  if (cached) {
    b->rb_choice.clear();
    for (int n : lens)
      for (int nout = 1; nout <= 2; ++nout) b->rb_choice[{n, nout}] = cache[tune_key(b->prec, n, nout)];
    release_tables(b);
    return build(ctx, b);
  }
  // scratch fields (inputs zero: the work does not depend on the values)
  const size_t esize = (b->prec == DEMAG_FP64) ? 8 : 4;
  const size_t ncell = size_t(b->off.back());
  void *fields = nullptr;
  DEMAG_TRY_HIP(hipMalloc(&fields, 7 * ncell * esize));
  DEMAG_TRY_HIP(hipMemsetAsync(fields, 0, 7 * ncell * esize, ctx->stream));
  char *fb = static_cast<char *>(fields);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  demag_status st = DEMAG_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("demag_batch_tune: event creation failed");
    st = DEMAG_E_HIP;
  }
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  auto time_apply = [&](float &ms) -> demag_status {
    demag_status s2 = enqueue(ctx, b, fb, fb + 3 * ncell * esize, fb + 4 * ncell * esize);   // warm-up
    if (s2 != DEMAG_OK) return s2;
    DEMAG_TRY_HIP(hipEventRecord(e0, ctx->stream));
    for (int r = 0; r < reps && s2 == DEMAG_OK; ++r)
      s2 = enqueue(ctx, b, fb, fb + 3 * ncell * esize, fb + 4 * ncell * esize);
    if (s2 != DEMAG_OK) return s2;
    DEMAG_TRY_HIP(hipEventRecord(e1, ctx->stream));
    DEMAG_TRY_HIP(hipEventSynchronize(e1));
    DEMAG_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    return DEMAG_OK;
  };
  int best[3] = {0, 0, 0};
  float best_ms = 0;
  if (st == DEMAG_OK) st = apply(best);
  if (st == DEMAG_OK) st = time_apply(best_ms);
  for (int bk = 0; bk < 3 && st == DEMAG_OK; ++bk) {
    bool present = false;   // thin axes (vector-ALU tiles) have no row-block shape
    for (int n : lens) present |= (bucket(n) == bk && n > kThinN);
    if (!present) continue;
    for (int sh : {-1, 1}) {
      int trial[3] = {best[0], best[1], best[2]};
      trial[bk] = sh;
      float ms = 0;
      st = apply(trial);
      if (st == DEMAG_OK) st = time_apply(ms);
      if (st != DEMAG_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best[bk] = sh;
      }
    }
  }
  ctx->profiling = prof;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(fields);
  if (st != DEMAG_OK) return st;
  st = apply(best);
  if (st != DEMAG_OK) return st;
  for (int n : lens)
    for (int nout = 1; nout <= 2; ++nout) cache[tune_key(b->prec, n, nout)] = shifted(n, best[bucket(n)]);
  if (path) {
    std::ofstream outf(path);
    outf << "{";
    bool first = true;
    for (auto &kv : cache) {
      outf << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
      first = false;
    }
    outf << "}\n";
  }
  return DEMAG_OK;
}

}  // extern "C"
