// C-ABI entry points: contexts, factor assembly, full-format apply.
#include "internal.h"

#include <cmath>
#include <cstring>

namespace demag {

namespace {
thread_local std::string g_last_error;
}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

FullPlan::~FullPlan() {
  for (auto &stages : chunks)
    for (auto &sp : stages) {
      if (sp.d_jobs) (void)hipFree(sp.d_jobs);
      if (sp.d_terms) (void)hipFree(sp.d_terms);
    }
}

demag_status prof_begin(demag_ctx *ctx, hipEvent_t *ev) {
  *ev = nullptr;
  if (!ctx->profiling) return DEMAG_OK;
  if (ctx->prof_pool.size() < 2) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      DEMAG_TRY_HIP(hipEventCreate(&e));
      ctx->prof_pool.push_back(e);
    }
  }
  *ev = ctx->prof_pool.back();
  ctx->prof_pool.pop_back();
  DEMAG_TRY_HIP(hipEventRecord(*ev, ctx->stream));
  return DEMAG_OK;
}

demag_status prof_end(demag_ctx *ctx, hipEvent_t start, const std::string &label, double flops, double bytes) {
  if (!start) return DEMAG_OK;
  if (ctx->prof_pool.empty()) {
    hipEvent_t e;
    DEMAG_TRY_HIP(hipEventCreate(&e));
    ctx->prof_pool.push_back(e);
  }
  hipEvent_t stop = ctx->prof_pool.back();
  ctx->prof_pool.pop_back();
  DEMAG_TRY_HIP(hipEventRecord(stop, ctx->stream));
  ctx->prof_pending.push_back(ProfRecord{label, start, stop, flops, bytes});
  return DEMAG_OK;
}

namespace {

demag_status prof_drain(demag_ctx *ctx) {
  if (ctx->prof_pending.empty()) return DEMAG_OK;
  DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
  for (auto &r : ctx->prof_pending) {
    float ms = 0;
    DEMAG_TRY_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
    auto &t = ctx->prof_totals[r.label];
    t.ms += ms;
    t.flops += r.flops;
    t.bytes += r.bytes;
    t.launches += 1;
    ctx->prof_pool.push_back(r.start);
    ctx->prof_pool.push_back(r.stop);
  }
  ctx->prof_pending.clear();
  return DEMAG_OK;
}

constexpr double kPi = 3.141592653589793238462643383279502884;

// Nodes of the quadrature in the scaled domain (Sec. 3.3, Cor. kron_op,
// Thm. sinc_theo): t_k, tau_k = sinh t_k, alpha_k, and the per-axis factor
// weight w_k = (alpha_k / (2 pi^(3/2)))^(1/3).
demag_status make_nodes(const demag_quad *q, double hmin_scaled, demag_factors *f) {
  const int M = q->M;
  f->M = M;
  f->t.resize(M);
  f->tau.resize(M);
  f->alpha.resize(M);
  f->w.resize(M);
  const bool explicit_rule = q->t && q->alpha;
  DEMAG_REQUIRE(explicit_rule || (!q->t && !q->alpha), "quad: give both t and alpha or neither");
  double theta = 0.0;
  if (!explicit_rule) {
    if (q->step_rule == 0) {
      DEMAG_REQUIRE(q->c0 > 0 && std::isfinite(q->c0), "quad: c0 must be positive");
      DEMAG_REQUIRE(M >= 2, "quad: the c0 rule needs M >= 2 (theta = c0 ln M / M)");
      theta = q->c0 * std::log(double(M)) / M;
    } else if (q->step_rule == 1) {
      const double a = 2.0;
      const double b = 0.25 * (0.5 * hmin_scaled) * (0.5 * hmin_scaled);
      theta = std::log(2.0 * kPi * a * M / b) / (a * M);
    } else {
      DEMAG_REQUIRE(false, "quad: step_rule must be 0 or 1");
    }
  }
  for (int k = 0; k < M; ++k) {
    double t, alpha;
    if (explicit_rule) {
      t = q->t[k];
      alpha = q->alpha[k];
      DEMAG_REQUIRE(std::isfinite(t) && t > 0 && std::isfinite(alpha), "quad: explicit nodes need finite t_k > 0");
    } else {
      t = theta * (k + 1);
      const double sh = std::sinh(t);
      alpha = 2.0 * theta * std::cosh(t) * sh * sh;
    }
    f->t[k] = t;
    f->tau[k] = std::sinh(t);
    f->alpha[k] = alpha;
    f->w[k] = std::cbrt(alpha / (2.0 * std::pow(kPi, 1.5)));
  }
  return DEMAG_OK;
}

template <class V>
demag_status upload(const std::vector<V> &host, V **dev) {
  if (host.empty()) {
    *dev = nullptr;
    return DEMAG_OK;
  }
  DEMAG_TRY_HIP(hipMalloc(dev, sizeof(V) * host.size()));
  DEMAG_TRY_HIP(hipMemcpy(*dev, host.data(), sizeof(V) * host.size(), hipMemcpyHostToDevice));
  return DEMAG_OK;
}

enum Buf { B_M = 0, B_Y1 = 1, B_Y2 = 2, B_PHI = 3, B_H = 4 };

// Stage plans of one node chunk [k0, k0 + kc) of demag_apply_full.
//
// Mode order z, y, x.  Stage 1 (along z) forms, per node, the six products
//   Y1: 0 (m_z, X)  1 (m_z, P)  2 (m_x, E)  3 (m_x, Q)  4 (m_y, E)  5 (m_y, Q)
// Stage 2 (along y, stored transposed [z][x][y]) forms six sums
//   Y2: 0 U_phi = E Y1_0 + X Y1_4     1 U_y = Q Y1_0 + P Y1_4
//       2 V_phi = E Y1_2              3 V_y = Q Y1_2
//       4 U_z   = E Y1_1 + X Y1_5     5 V_z = E Y1_3
// Stage 3 (along x, stored back as [z][y][x]) accumulates over nodes
//   phi = E U_phi + X V_phi,  h_x = Q U_phi + P V_phi,
//   h_y = E U_y + X V_y,      h_z = E U_z + X V_z.
// Each output's triple of factor types is then that of the potential kernel
// K^q (X along q, E elsewhere) or its derivative along the field axis p
// (X -> P = -X', E -> Q = -E').  6 + 9 + 8 = 23 products per node.
// xsplit > 1: the x stage's sums over the chunk's nodes are cut into xsplit
// jobs of consecutive terms each, which write unscaled partial sums to the
// (then dead) Y1 region, partial s of output o (phi, h_x, h_y, h_z) at
// (4 s + o) N; launch_reduce_partials forms the outputs from them.
void build_chunk(const demag_factors *f, int k0, int kc, double phi_scale,
                 std::vector<StagePlan> &stages, int xsplit) {
  const int nx = f->n[0], ny = f->n[1], nz = f->n[2];
  const int64_t N = int64_t(nx) * ny * nz;
  const int M = f->M;
  auto gen = [M](int type, int k) { return type * M + k; };
  auto y1 = [N](int kl, int s) { return (int64_t(kl) * 6 + s) * N; };
  auto y2 = y1;

  const int64_t P = int64_t(nx) * ny;   // one z-plane
  // along z: columns (y, x) contiguous; output [z][y][x]
  MPGeom gz{nz, int(P), int(P), 2 * nz - 1, P, 0, 0, 1, P};
  // along y: columns (z, x); input [z][y][x]; output stored transposed [z][x][y]
  MPGeom gy{ny, nz * nx, nx, 2 * ny - 1, nx, P, P, ny, 1};
  // along x: columns (z, y); input [z][x][y]; output back in [z][y][x]
  MPGeom gx{nx, nz * ny, ny, 2 * nx - 1, ny, P, P, nx, 1};

  auto add_job = [](StagePlan &sp, std::initializer_list<MPTerm> terms, int ob0, int64_t oo0, double s0,
                    int ob1, int64_t oo1, double s1) {
    MPJob j{};
    j.term0 = int32_t(sp.terms.size());
    j.nterms = int32_t(terms.size());
    j.out_buf[0] = ob0;
    j.out_off[0] = oo0;
    j.scale[0] = s0;
    j.out_buf[1] = ob1;
    j.out_off[1] = oo1;
    j.scale[1] = s1;
    for (const auto &t : terms) sp.terms.push_back(t);
    sp.jobs.push_back(j);
  };
  auto term = [](int buf, int64_t off, int g0, int g1) {
    MPTerm t{};
    t.in_buf = buf;
    t.in_off = off;
    t.gen[0] = g0;
    t.gen[1] = g1;
    return t;
  };
  // element offsets of the generators in the stage axis' table
  const bool dense = f->dense;   // dense tables hold one n x n matrix per generator
  auto finish = [dense](StagePlan &sp) {
    const int64_t stride = dense ? int64_t(sp.geom.n) * sp.geom.n : int64_t(sp.geom.genlen);
    for (auto &t : sp.terms)
      for (int o = 0; o < 2; ++o) t.gen_off[o] = int64_t(t.gen[o]) * stride;
    sp.rb = default_rb(sp.geom.n);
  };

  StagePlan s1;
  s1.geom = gz;
  s1.axis = 2;
  s1.nout = 2;
  for (int kl = 0; kl < kc; ++kl) {
    const int k = k0 + kl;
    add_job(s1, {term(B_M, 2 * N, gen(F_X, k), gen(F_P, k))}, B_Y1, y1(kl, 0), 1.0, B_Y1, y1(kl, 1), 1.0);
    add_job(s1, {term(B_M, 0, gen(F_E, k), gen(F_Q, k))}, B_Y1, y1(kl, 2), 1.0, B_Y1, y1(kl, 3), 1.0);
    add_job(s1, {term(B_M, N, gen(F_E, k), gen(F_Q, k))}, B_Y1, y1(kl, 4), 1.0, B_Y1, y1(kl, 5), 1.0);
  }
  StagePlan s2a, s2b;
  s2a.geom = gy;
  s2a.axis = 1;
  s2a.nout = 2;
  s2b.geom = gy;
  s2b.axis = 1;
  s2b.nout = 1;
  // the two-term jobs of all nodes first, then the one-term jobs: the
  // workgroups are dispatched in job order, so the launch ends on short work
  for (int kl = 0; kl < kc; ++kl) {
    const int k = k0 + kl;
    add_job(s2a, {term(B_Y1, y1(kl, 0), gen(F_E, k), gen(F_Q, k)), term(B_Y1, y1(kl, 4), gen(F_X, k), gen(F_P, k))},
            B_Y2, y2(kl, 0), 1.0, B_Y2, y2(kl, 1), 1.0);
    add_job(s2b, {term(B_Y1, y1(kl, 1), gen(F_E, k), 0), term(B_Y1, y1(kl, 5), gen(F_X, k), 0)}, B_Y2, y2(kl, 4),
            1.0, 0, 0, 0.0);
  }
  for (int kl = 0; kl < kc; ++kl) {
    const int k = k0 + kl;
    add_job(s2a, {term(B_Y1, y1(kl, 2), gen(F_E, k), gen(F_Q, k))}, B_Y2, y2(kl, 2), 1.0, B_Y2, y2(kl, 3), 1.0);
    add_job(s2b, {term(B_Y1, y1(kl, 3), gen(F_E, k), 0)}, B_Y2, y2(kl, 5), 1.0, 0, 0, 0.0);
  }
  StagePlan s3a, s3b;
  s3a.geom = gx;
  s3a.axis = 0;
  s3a.nout = 2;
  s3b.geom = gx;
  s3b.axis = 0;
  s3b.nout = 1;
  // terms [t0, t1) of the 2 kc terms of an x-stage sum: job s of ns, every
  // one non-empty (ns <= 2 kc), so each partial is written
  const int ns = std::min(xsplit, 2 * kc);
  auto part = [kc, ns](int s, int &t0, int &t1) {
    t0 = s * 2 * kc / ns;
    t1 = (s + 1) * 2 * kc / ns;
  };
  for (int kl = 0; kl < kc; ++kl) {
    const int k = k0 + kl;
    s3a.terms.push_back(term(B_Y2, y2(kl, 0), gen(F_E, k), gen(F_Q, k)));
    s3a.terms.push_back(term(B_Y2, y2(kl, 2), gen(F_X, k), gen(F_P, k)));
  }
  for (int sp = 0; sp < ns; ++sp) {
    int t0, t1;
    part(sp, t0, t1);
    MPJob j{};
    j.term0 = t0;
    j.nterms = t1 - t0;
    if (xsplit > 1) {
      j.out_buf[0] = B_Y1;
      j.out_off[0] = (int64_t(4) * sp + 0) * N;
      j.scale[0] = 1.0;
      j.out_buf[1] = B_Y1;
      j.out_off[1] = (int64_t(4) * sp + 1) * N;
      j.scale[1] = 1.0;
    } else {
      j.out_buf[0] = B_PHI;
      j.out_off[0] = 0;
      j.scale[0] = phi_scale;
      j.out_buf[1] = B_H;
      j.out_off[1] = 0;
      j.scale[1] = 1.0;
    }
    s3a.jobs.push_back(j);
  }
  for (int p = 1; p <= 2; ++p) {
    const int base = int(s3b.terms.size());
    const int su = (p == 1) ? 1 : 4, sv = (p == 1) ? 3 : 5;
    for (int kl = 0; kl < kc; ++kl) {
      const int k = k0 + kl;
      s3b.terms.push_back(term(B_Y2, y2(kl, su), gen(F_E, k), 0));
      s3b.terms.push_back(term(B_Y2, y2(kl, sv), gen(F_X, k), 0));
    }
    for (int sp = 0; sp < ns; ++sp) {
      int t0, t1;
      part(sp, t0, t1);
      MPJob j{};
      j.term0 = base + t0;
      j.nterms = t1 - t0;
      j.out_buf[0] = (xsplit > 1) ? B_Y1 : B_H;
      j.out_off[0] = (xsplit > 1) ? (int64_t(4) * sp + 1 + p) * N : p * N;
      j.scale[0] = 1.0;
      s3b.jobs.push_back(j);
    }
  }
  for (StagePlan *sp : {&s1, &s2a, &s2b, &s3a, &s3b}) finish(*sp);
  stages.clear();
  stages.push_back(std::move(s1));
  stages.push_back(std::move(s2a));
  stages.push_back(std::move(s2b));
  stages.push_back(std::move(s3a));
  stages.push_back(std::move(s3b));
}

}  // namespace

void build_chunk_plan(const demag_factors *f, int k0, int kc, double phi_scale, std::vector<StagePlan> &stages) {
  build_chunk(f, k0, kc, phi_scale, stages, 1);
}

namespace {

// Workspace of demag_apply_full for a chunk of kc nodes: 12 intermediate
// tensors per node plus 4 scratch outputs.
size_t full_ws_bytes(const demag_factors *f, demag_prec prec, int kc) {
  const size_t esize = (prec == DEMAG_FP64) ? 8 : 4;
  const size_t N = size_t(f->n[0]) * f->n[1] * f->n[2];
  return (size_t(12) * kc + 4) * N * esize;
}

// Plan whose node chunks fit `limit` bytes of workspace.
demag_status get_plan(demag_ctx *ctx, demag_factors *f, demag_prec prec, size_t limit, FullPlan **out) {
  (void)ctx;
  int kc = f->M;
  if (limit < full_ws_bytes(f, prec, 1)) {
    set_error("workspace too small for one node (" + std::to_string(full_ws_bytes(f, prec, 1)) + " bytes needed)");
    return DEMAG_E_NOMEM;
  }
  while (kc > 1 && full_ws_bytes(f, prec, kc) > limit) kc = (kc + 1) / 2;
  // FP32 and bfloat16 splits: the x stage's sums over nodes run as kXSplit
  // jobs of partial sums, reduced in FP64 by one elementwise kernel, when the
  // chunk's Y1 region holds the 4 kXSplit partial outputs.  This gives the
  // stage more workgroups (it otherwise has one or two jobs) and cuts each
  // FP32 accumulation chain over the chunk's 2 kc terms of n products to a
  // quarter, which keeps the FP32 potential within 1e-6 of FP64 at 128^3.
  // FP64 keeps one job per sum (measured: the split saves 1.6 % at 128^3,
  // and the single chain keeps the batched FP64 apply bit-identical).
  constexpr int kXSplit = 4;
  const bool bf = (prec == DEMAG_BF16X2 || prec == DEMAG_BF16X3);
  const int xsplit = (prec != DEMAG_FP64 && 6 * kc >= 4 * kXSplit) ? kXSplit : 1;
  const int key_prec = (prec == DEMAG_FP64) ? 0 : bf ? 2 : 1;
  auto key = std::make_pair(key_prec, kc);
  auto it = f->plans.find(key);
  if (it != f->plans.end()) {
    *out = it->second.get();
    return DEMAG_OK;
  }
  auto plan = std::make_unique<FullPlan>();
  plan->kc = kc;
  plan->xsplit = xsplit;
  plan->nchunks = (f->M + kc - 1) / kc;
  plan->ws_elems = full_ws_bytes(f, prec, kc) / ((prec == DEMAG_FP64) ? 8 : 4);
  plan->chunks.resize(plan->nchunks);
  for (int c = 0; c < plan->nchunks; ++c) {
    const int k0 = c * kc;
    const int kcc = std::min(kc, f->M - k0);
    build_chunk(f, k0, kcc, f->L, plan->chunks[c], xsplit);
    for (auto &sp : plan->chunks[c]) {
      demag_status st = upload(sp.jobs, &sp.d_jobs);
      if (st != DEMAG_OK) return st;
      st = upload(sp.terms, &sp.d_terms);
      if (st != DEMAG_OK) return st;
    }
  }
  *out = plan.get();
  f->plans[key] = std::move(plan);
  return DEMAG_OK;
}

}  // namespace

// Grow the context workspace to at least `bytes` (stream-ordered reuse).
demag_status ensure_workspace(demag_ctx *ctx, size_t bytes) {
  if (ctx->ws_bytes >= bytes) return DEMAG_OK;
  if (ctx->ws) {
    DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    DEMAG_TRY_HIP(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  hipError_t e = hipMalloc(&ctx->ws, bytes);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    set_error(std::string("workspace allocation failed: ") + hipGetErrorString(e));
    return DEMAG_E_NOMEM;
  }
  ctx->ws_bytes = bytes;
  return DEMAG_OK;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

demag_status note_use(demag_ctx *ctx, const demag_factors *fc) {
  auto *f = const_cast<demag_factors *>(fc);
  if (!f->used) DEMAG_TRY_HIP(hipEventCreateWithFlags(&f->used, hipEventDisableTiming));
  DEMAG_TRY_HIP(hipEventRecord(f->used, ctx->stream));
  return DEMAG_OK;
}

namespace {
__global__ void k_clear_flag(int *flag) { *flag = 0; }

template <class T>
__global__ void k_check_finite(const T *__restrict__ x, size_t count, int *__restrict__ flag) {
  int bad = 0;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += size_t(gridDim.x) * blockDim.x)
    if (!isfinite(x[i])) bad = 1;
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}
}  // namespace

demag_status check_finite(demag_ctx *ctx, const void *x, size_t count, bool dbl, const char *what, int *dflag) {
  if (!ctx->check_inputs || count == 0) return DEMAG_OK;
  if (!dflag) {
    if (!ctx->d_flag) DEMAG_TRY_HIP(hipMalloc(&ctx->d_flag, sizeof(int)));
    dflag = ctx->d_flag;
  }
  k_clear_flag<<<1, 1, 0, ctx->stream>>>(dflag);
  const unsigned blocks = unsigned(std::min<size_t>((count + 255) / 256, 4096));
  if (dbl)
    k_check_finite<double><<<blocks, 256, 0, ctx->stream>>>(static_cast<const double *>(x), count, dflag);
  else
    k_check_finite<float><<<blocks, 256, 0, ctx->stream>>>(static_cast<const float *>(x), count, dflag);
  DEMAG_TRY_HIP(hipGetLastError());
  int flag = 0;
  DEMAG_TRY_HIP(hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
  if (flag) {
    set_error(std::string(what) + ": input holds NaN or infinite values");
    return DEMAG_E_INVAL;
  }
  return DEMAG_OK;
}

}  // namespace demag

using namespace demag;

extern "C" {

const char *demag_last_error(void) { return g_last_error.c_str(); }

demag_status demag_create(int device, void *hip_stream, demag_ctx **out) {
  DEMAG_REQUIRE(out, "demag_create: out is NULL");
  int count = 0;
  DEMAG_TRY_HIP(hipGetDeviceCount(&count));
  DEMAG_REQUIRE(device >= 0 && device < count, "demag_create: no such device");
  DEMAG_TRY_HIP(hipSetDevice(device));
  auto *ctx = new (std::nothrow) demag_ctx;
  if (!ctx) {
    set_error("demag_create: out of host memory");
    return DEMAG_E_NOMEM;
  }
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  // the allocation-free entry point's static scratch: its device address,
  // looked up once per device with the device current
  (void)scratch_init(device);
  *out = ctx;
  return DEMAG_OK;
}

demag_status demag_destroy(demag_ctx *ctx) {
  if (!ctx) return DEMAG_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->d_flag) (void)hipFree(ctx->d_flag);
  if (ctx->order_ev) (void)hipEventDestroy(ctx->order_ev);
  for (auto &r : ctx->prof_pending) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
  delete ctx;
  return DEMAG_OK;
}

demag_status demag_prepare_structured(demag_ctx *ctx, demag_factors *f) {
  DEMAG_REQUIRE(ctx && f, "demag_prepare_structured: NULL argument");
  DEMAG_REQUIRE(!f->dense, "demag_prepare_structured: needs a uniform grid (Toeplitz factors)");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  demag_status st = prepare_spectra(ctx, f);
  return st == DEMAG_OK ? note_use(ctx, f) : st;
}

demag_status demag_apply_columns(demag_ctx *ctx, demag_factors *f, demag_prec prec, const int32_t R[3],
                                 const float *const in[3], float *const out[3]) {
  DEMAG_REQUIRE(ctx && f && R && in && out, "demag_apply_columns: NULL argument");
  if (prec == DEMAG_BF16X2 || prec == DEMAG_BF16X3) {
    set_error("demag_apply_columns: the transforms' butterflies are no matrix-core contractions; no bfloat16 "
              "split (use DEMAG_FP32 or DEMAG_FP64)");
    return DEMAG_E_UNSUPPORTED;
  }
  DEMAG_REQUIRE(prec == DEMAG_FP64 || prec == DEMAG_FP32, "demag_apply_columns: unknown precision");
  DEMAG_REQUIRE(!f->dense, "demag_apply_columns: needs a uniform grid (Toeplitz factors)");
  for (int d = 0; d < 3; ++d) {
    DEMAG_REQUIRE(R[d] >= 0 && R[d] <= 65536, "demag_apply_columns: R out of range");
    DEMAG_REQUIRE(R[d] == 0 || (in[d] && out[d]), "demag_apply_columns: NULL column buffer");
    DEMAG_REQUIRE(fft_length(f->n[d]) <= 8192, "demag_apply_columns: n <= 4096 per axis");
  }
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  demag_status st = prepare_spectra(ctx, f);
  for (int d = 0; d < 3 && st == DEMAG_OK; ++d)
    st = check_finite(ctx, in[d], size_t(3) * R[d] * f->n[d], false, "demag_apply_columns");
  if (st == DEMAG_OK) st = launch_columns(ctx, f, prec, R, in, out, nullptr, 0);
  return st == DEMAG_OK ? note_use(ctx, f) : st;
}

namespace {
// Column numbering of the structured results (see demag.h).
inline int32_t col_index(int q, int s, int k, int l, int M, int R) { return ((q * 2 + s) * M + k) * R + l; }
inline int slot_of(int o, int d) { return (o == d + 1) ? 1 : 0; }
}  // namespace

demag_status demag_apply_cp(demag_ctx *ctx, demag_factors *f, demag_prec prec, int32_t r, const float *const U[3],
                            float *const out[3], int32_t *table) {
  DEMAG_REQUIRE(ctx && f && U && out, "demag_apply_cp: NULL argument");
  DEMAG_REQUIRE(r >= 1, "demag_apply_cp: rank must be >= 1");
  const int32_t R[3] = {r, r, r};
  demag_status st = demag_apply_columns(ctx, f, prec, R, U, out);
  if (st != DEMAG_OK || !table) return st;
  const int M = f->M;
  for (int o = 0; o < 4; ++o)
    for (int q = 0; q < 3; ++q)
      for (int k = 0; k < M; ++k)
        for (int l = 0; l < r; ++l) {
          int32_t *t = table + ((size_t(o) * 3 * M * r) + (size_t(q) * M + k) * r + l) * 3;
          for (int d = 0; d < 3; ++d) t[d] = col_index(q, slot_of(o, d), k, l, M, r);
        }
  return DEMAG_OK;
}

namespace {
void block_table(int M, const int32_t R[3], int32_t *table) {
  for (int o = 0; o < 4; ++o)
    for (int q = 0; q < 3; ++q)
      for (int k = 0; k < M; ++k) {
        int32_t *t = table + ((size_t(o) * 3 * M) + size_t(q) * M + k) * 3;
        for (int d = 0; d < 3; ++d) t[d] = col_index(q, slot_of(o, d), k, 0, M, R[d]);
      }
}
}  // namespace

demag_status demag_apply_tucker(demag_ctx *ctx, demag_factors *f, demag_prec prec, const int32_t r[3],
                                const float *const U[3], float *const out[3], int32_t *table) {
  DEMAG_REQUIRE(ctx && f && r && U && out, "demag_apply_tucker: NULL argument");
  DEMAG_REQUIRE(r[0] >= 1 && r[1] >= 1 && r[2] >= 1, "demag_apply_tucker: ranks must be >= 1");
  demag_status st = demag_apply_columns(ctx, f, prec, r, U, out);
  if (st == DEMAG_OK && table) block_table(f->M, r, table);
  return st;
}

demag_status demag_apply_tt(demag_ctx *ctx, demag_factors *f, demag_prec prec, int32_t r1, int32_t r2,
                            const float *G1, const float *G2, const float *G3, float *const out[3], int32_t *table) {
  DEMAG_REQUIRE(ctx && f && G1 && G2 && G3 && out, "demag_apply_tt: NULL argument");
  DEMAG_REQUIRE(r1 >= 1 && r2 >= 1, "demag_apply_tt: ranks must be >= 1");
  const int32_t R[3] = {r1, r1 * r2, r2};
  const float *const in[3] = {G1, G2, G3};
  demag_status st = demag_apply_columns(ctx, f, prec, R, in, out);
  if (st == DEMAG_OK && table) block_table(f->M, R, table);
  return st;
}

demag_status demag_bf16_split(demag_ctx *ctx, const float *x, uint16_t *parts, size_t count, int32_t nparts) {
  DEMAG_REQUIRE(ctx && (count == 0 || (x && parts)), "demag_bf16_split: NULL argument");
  DEMAG_REQUIRE(nparts >= 1 && nparts <= 3, "demag_bf16_split: nparts must be 1, 2 or 3");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  return launch_split(ctx, x, parts, count, nparts);
}

demag_status demag_profile_enable(demag_ctx *ctx, int32_t enable) {
  DEMAG_REQUIRE(ctx, "demag_profile_enable: ctx is NULL");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  demag_status st = prof_drain(ctx);
  if (st != DEMAG_OK) return st;
  if (enable) ctx->prof_totals.clear();
  ctx->profiling = enable != 0;
  return DEMAG_OK;
}

demag_status demag_profile_read(demag_ctx *ctx, int32_t max, char *labels, double *total_ms, int64_t *launches,
                                double *flops, double *bytes, int32_t *count) {
  DEMAG_REQUIRE(ctx && count && max >= 0, "demag_profile_read: NULL argument");
  DEMAG_REQUIRE(max == 0 || (labels && total_ms && launches && flops && bytes),
                "demag_profile_read: NULL output array");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  demag_status st = prof_drain(ctx);
  if (st != DEMAG_OK) return st;
  int i = 0;
  for (const auto &kv : ctx->prof_totals) {
    if (i >= max) break;
    std::strncpy(labels + 48 * i, kv.first.c_str(), 47);
    labels[48 * i + 47] = 0;
    total_ms[i] = kv.second.ms;
    launches[i] = kv.second.launches;
    flops[i] = kv.second.flops;
    bytes[i] = kv.second.bytes;
    ++i;
  }
  *count = i;
  return DEMAG_OK;
}

demag_status demag_set_stream(demag_ctx *ctx, void *hip_stream) {
  DEMAG_REQUIRE(ctx, "demag_set_stream: ctx is NULL");
  hipStream_t next = static_cast<hipStream_t>(hip_stream);
  if (next == ctx->stream) return DEMAG_OK;
  // later work on the new stream must not overtake work still queued on the
  // old one (it shares the context's workspace)
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  if (!ctx->order_ev) DEMAG_TRY_HIP(hipEventCreateWithFlags(&ctx->order_ev, hipEventDisableTiming));
  DEMAG_TRY_HIP(hipEventRecord(ctx->order_ev, ctx->stream));
  DEMAG_TRY_HIP(hipStreamWaitEvent(next, ctx->order_ev, 0));
  ctx->stream = next;
  return DEMAG_OK;
}

demag_status demag_set_input_check(demag_ctx *ctx, int32_t enable) {
  DEMAG_REQUIRE(ctx, "demag_set_input_check: ctx is NULL");
  ctx->check_inputs = enable != 0;
  return DEMAG_OK;
}

demag_status demag_set_workspace_limit(demag_ctx *ctx, size_t bytes) {
  DEMAG_REQUIRE(ctx, "demag_set_workspace_limit: ctx is NULL");
  ctx->ws_limit = bytes;
  return DEMAG_OK;
}

demag_status demag_set_tiles(demag_ctx *ctx, int32_t rows, int32_t cols) {
  DEMAG_REQUIRE(ctx, "demag_set_tiles: ctx is NULL");
  DEMAG_REQUIRE(rows == 0 || rows == 1 || rows == 2 || rows == 4 || rows == 8,
                "demag_set_tiles: rows must be 0, 1, 2, 4 or 8");
  DEMAG_REQUIRE(cols == 0 || cols == 1 || cols == 2, "demag_set_tiles: cols must be 0, 1 or 2");
  ctx->tile_rows = rows;
  ctx->tile_cols = cols;
  return DEMAG_OK;
}

demag_status demag_assemble_factors(demag_ctx *ctx, const demag_grid *grid, const demag_quad *quad,
                                    demag_factors **out) {
  DEMAG_REQUIRE(ctx && grid && quad && out, "demag_assemble_factors: NULL argument");
  for (int d = 0; d < 3; ++d) {
    DEMAG_REQUIRE(grid->n[d] >= 1 && grid->n[d] <= 4096, "grid: n must be in [1, 4096]");
    DEMAG_REQUIRE(grid->h[d] > 0 && std::isfinite(grid->h[d]), "grid: h must be positive");
  }
  DEMAG_REQUIRE(quad->M >= 1 && quad->M <= 256, "quad: M must be in [1, 256]");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  auto f = std::make_unique<demag_factors>();
  double L = 0.0;
  for (int d = 0; d < 3; ++d) {
    f->n[d] = grid->n[d];
    f->h[d] = grid->h[d];
    L = std::max(L, grid->n[d] * grid->h[d]);
  }
  f->L = L;
  double hmin = 1e300;
  for (int d = 0; d < 3; ++d) {
    f->hs[d] = grid->h[d] / L;
    hmin = std::min(hmin, f->hs[d]);
  }
  demag_status st = make_nodes(quad, hmin, f.get());
  if (st != DEMAG_OK) return st;
  for (int d = 0; d < 3; ++d) {
    const size_t cnt = axis_table_len(f.get(), d);
    hipError_t e1 = hipMalloc(&f->f64[d], cnt * sizeof(double));
    hipError_t e2 = hipMalloc(&f->f32[d], cnt * sizeof(float));
    hipError_t e3 = hipMalloc(&f->bf[d], 3 * cnt * sizeof(uint16_t));
    hipError_t e4 = hipSuccess;
    if (f->n[d] <= 1024)
      e4 = hipMalloc(&f->bfw[d], size_t(F_NTYPES) * f->M * window_entries(f->n[d]) * 3 * 16);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
      set_error("factor tables: device allocation failed");
      demag_factors_free(f.release());
      return DEMAG_E_NOMEM;
    }
  }
  st = launch_assemble(ctx, f.get());
  if (st == DEMAG_OK) st = launch_build_windows(ctx, f.get());
  if (st == DEMAG_OK) st = note_use(ctx, f.get());
  if (st != DEMAG_OK) {
    demag_factors_free(f.release());
    return st;
  }
  *out = f.release();
  return DEMAG_OK;
}

demag_status demag_assemble_factors_grid(demag_ctx *ctx, const int32_t n[3], const double *const edges[3],
                                         const demag_quad *quad, demag_factors **out) {
  DEMAG_REQUIRE(ctx && n && edges && quad && out, "demag_assemble_factors_grid: NULL argument");
  DEMAG_REQUIRE(quad->M >= 1 && quad->M <= 256, "quad: M must be in [1, 256]");
  double L = 0.0;
  for (int d = 0; d < 3; ++d) {
    DEMAG_REQUIRE(n[d] >= 1 && n[d] <= 1024 && edges[d], "grid: n must be in [1, 1024] with n + 1 edges");
    for (int i = 0; i < n[d]; ++i)
      DEMAG_REQUIRE(std::isfinite(edges[d][i]) && std::isfinite(edges[d][i + 1]) && edges[d][i + 1] > edges[d][i],
                    "grid: edges must increase strictly");
    L = std::max(L, edges[d][n[d]] - edges[d][0]);
  }
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  auto f = std::make_unique<demag_factors>();
  f->L = L;
  f->dense = true;
  // the scaled edges live in the handle: the assembly copies them to the
  // device asynchronously
  std::vector<double> *scaled = f->edges;
  double hmin = 1e300;
  for (int d = 0; d < 3; ++d) {
    f->n[d] = n[d];
    scaled[d].resize(size_t(n[d]) + 1);
    for (int i = 0; i <= n[d]; ++i) scaled[d][i] = (edges[d][i] - edges[d][0]) / L;
    double hm = 1e300;
    for (int i = 0; i < n[d]; ++i) hm = std::min(hm, scaled[d][i + 1] - scaled[d][i]);
    f->hs[d] = hm;            // smallest scaled cell of the axis
    f->h[d] = hm * L;
    hmin = std::min(hmin, hm);
  }
  demag_status st = make_nodes(quad, hmin, f.get());
  if (st != DEMAG_OK) return st;
  for (int d = 0; d < 3; ++d) {
    const size_t cnt = size_t(F_NTYPES) * f->M * size_t(n[d]) * n[d];
    if (hipMalloc(&f->f64[d], cnt * sizeof(double)) != hipSuccess ||
        hipMalloc(&f->f32[d], cnt * sizeof(float)) != hipSuccess ||
        hipMalloc(&f->bf[d], 3 * cnt * sizeof(uint16_t)) != hipSuccess) {
      set_error("dense factor tables: device allocation failed");
      demag_factors_free(f.release());
      return DEMAG_E_NOMEM;
    }
  }
  st = launch_assemble_dense(ctx, f.get(), scaled);
  if (st == DEMAG_OK) st = note_use(ctx, f.get());
  if (st != DEMAG_OK) {
    demag_factors_free(f.release());
    return st;
  }
  *out = f.release();
  return DEMAG_OK;
}

demag_status demag_factors_free(demag_factors *f) {
  if (!f) return DEMAG_OK;
  // the last enqueued work that reads the factors must be done
  if (f->used) {
    (void)hipEventSynchronize(f->used);
    (void)hipEventDestroy(f->used);
  }
  for (int d = 0; d < 3; ++d) {
    if (f->f64[d]) (void)hipFree(f->f64[d]);
    if (f->f32[d]) (void)hipFree(f->f32[d]);
    if (f->bf[d]) (void)hipFree(f->bf[d]);
    if (f->bfw[d]) (void)hipFree(f->bfw[d]);
    if (f->spec[d]) (void)hipFree(f->spec[d]);
    if (f->spec32[d]) (void)hipFree(f->spec32[d]);
    if (f->twiddle[d]) (void)hipFree(f->twiddle[d]);
  }
  if (f->k3) (void)hipFree(f->k3);
  delete f;
  return DEMAG_OK;
}

demag_status demag_factors_count(const demag_factors *f, int32_t *M) {
  DEMAG_REQUIRE(f && M, "demag_factors_count: NULL argument");
  *M = f->M;
  return DEMAG_OK;
}

demag_status demag_factors_length_scale(const demag_factors *f, double *L) {
  DEMAG_REQUIRE(f && L, "demag_factors_length_scale: NULL argument");
  *L = f->L;
  return DEMAG_OK;
}

demag_status demag_factors_nodes(const demag_factors *f, double *t, double *tau, double *alpha) {
  DEMAG_REQUIRE(f, "demag_factors_nodes: f is NULL");
  if (t) std::memcpy(t, f->t.data(), sizeof(double) * f->M);
  if (tau) std::memcpy(tau, f->tau.data(), sizeof(double) * f->M);
  if (alpha) std::memcpy(alpha, f->alpha.data(), sizeof(double) * f->M);
  return DEMAG_OK;
}

demag_status demag_factors_download(demag_ctx *ctx, const demag_factors *f, int32_t d, double *dst) {
  DEMAG_REQUIRE(ctx && f && dst, "demag_factors_download: NULL argument");
  DEMAG_REQUIRE(d >= 0 && d < 3, "demag_factors_download: axis must be 0, 1 or 2");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  DEMAG_TRY_HIP(hipMemcpyAsync(dst, f->f64[d], axis_table_len(f, d) * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
  DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
  return DEMAG_OK;
}

}  // extern "C"

namespace {
// demag_apply_full on the context workspace (ws == NULL, grown to the plan's
// need under the context's limit) or on a caller workspace of ws_bytes.
demag_status apply_full_impl(demag_ctx *ctx, const demag_factors *fc, demag_prec prec, const void *m, void *phi,
                             void *h, void *ws_user, size_t ws_user_bytes, const char *where) {
  DEMAG_REQUIRE(ctx && fc && m, std::string(where) + ": NULL argument");
  DEMAG_REQUIRE(phi || h, std::string(where) + ": phi and h are both NULL");
  DEMAG_REQUIRE(prec == DEMAG_FP64 || prec == DEMAG_FP32 || prec == DEMAG_BF16X2 || prec == DEMAG_BF16X3,
                std::string(where) + ": unknown precision");
  DEMAG_REQUIRE(aligned16(m) && aligned16(phi) && aligned16(h) && aligned16(ws_user),
                std::string(where) + ": buffers must be 16-byte aligned");
  for (int d = 0; d < 3; ++d)
    DEMAG_REQUIRE(fc->n[d] <= 1024, std::string(where) + ": full format supports n <= 1024 per axis");
  auto *f = const_cast<demag_factors *>(fc);
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  const int64_t N = int64_t(f->n[0]) * f->n[1] * f->n[2];
  const size_t esize = (prec == DEMAG_FP64) ? 8 : 4;
  demag_status st = check_finite(ctx, m, size_t(3) * N, prec == DEMAG_FP64, where);
  if (st != DEMAG_OK) return st;
  FullPlan *plan = nullptr;
  st = get_plan(ctx, f, prec, ws_user ? ws_user_bytes : ctx->ws_limit, &plan);
  if (st != DEMAG_OK) return st;
  char *ws = static_cast<char *>(ws_user);
  if (!ws) {
    st = ensure_workspace(ctx, plan->ws_elems * esize);
    if (st != DEMAG_OK) return st;
    ws = static_cast<char *>(ctx->ws);
  }
  char *y1 = ws;
  char *y2 = y1 + size_t(6) * plan->kc * N * esize;
  char *scratch = y2 + size_t(6) * plan->kc * N * esize;
  void *bufs[6] = {const_cast<void *>(m), y1, y2, phi ? phi : scratch, h ? h : scratch + N * esize, nullptr};
  for (int c = 0; c < plan->nchunks; ++c) {
    const auto &stages = plan->chunks[c];
    for (size_t s = 0; s < stages.size(); ++s) {
      // later chunks accumulate into the outputs (partial sums never do)
      const int beta = (s >= 3 && c > 0 && plan->xsplit == 1) ? 1 : 0;
      st = launch_left_stage(ctx, f, prec, stages[s], bufs, beta);
      if (st != DEMAG_OK) return st;
    }
    if (plan->xsplit > 1) {
      // one x-stage job per partial sum of this chunk (fewer than xsplit
      // when the chunk has fewer than 2 xsplit terms)
      const int ns = int(stages[3].jobs.size());
      st = launch_reduce_partials(ctx, prec, y1, ns, N, bufs[3], bufs[4], f->L, c > 0);
      if (st != DEMAG_OK) return st;
    }
  }
  return note_use(ctx, f);
}
}  // namespace

extern "C" {

demag_status demag_apply_full(demag_ctx *ctx, const demag_factors *f, demag_prec prec, const void *m, void *phi,
                              void *h) {
  return apply_full_impl(ctx, f, prec, m, phi, h, nullptr, 0, "demag_apply_full");
}

demag_status demag_apply_full_workspace_size(const demag_factors *f, demag_prec prec, size_t *one_chunk,
                                             size_t *minimum) {
  DEMAG_REQUIRE(f, "demag_apply_full_workspace_size: f is NULL");
  DEMAG_REQUIRE(prec == DEMAG_FP64 || prec == DEMAG_FP32 || prec == DEMAG_BF16X2 || prec == DEMAG_BF16X3,
                "demag_apply_full_workspace_size: unknown precision");
  if (one_chunk) *one_chunk = full_ws_bytes(f, prec, f->M);
  if (minimum) *minimum = full_ws_bytes(f, prec, 1);
  return DEMAG_OK;
}

demag_status demag_apply_full_ws(demag_ctx *ctx, const demag_factors *f, demag_prec prec, const void *m, void *phi,
                                 void *h, void *workspace, size_t workspace_bytes) {
  DEMAG_REQUIRE(workspace, "demag_apply_full_ws: workspace is NULL");
  return apply_full_impl(ctx, f, prec, m, phi, h, workspace, workspace_bytes, "demag_apply_full_ws");
}

demag_status demag_apply_fft(demag_ctx *ctx, demag_factors *f, const double *m, double *phi, double *h) {
  DEMAG_REQUIRE(ctx && f && m && phi && h, "demag_apply_fft: NULL argument");
  DEMAG_REQUIRE(!f->dense, "demag_apply_fft: needs a uniform grid (Toeplitz factors)");
  for (int d = 0; d < 3; ++d)
    DEMAG_REQUIRE(f->n[d] <= 1024, "demag_apply_fft: n <= 1024 per axis");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  demag_status st = prepare_fft3d(ctx, f);
  if (st != DEMAG_OK) return st;
  const size_t N = size_t(f->n[0]) * f->n[1] * f->n[2];
  st = check_finite(ctx, m, 3 * N, true, "demag_apply_fft");
  if (st != DEMAG_OK) return st;
  st = ensure_workspace(ctx, fft3d_workspace_bytes(f));
  if (st != DEMAG_OK) return st;
  st = launch_fft3d(ctx, f, m, phi, h, ctx->ws);
  return st == DEMAG_OK ? note_use(ctx, f) : st;
}

}  // extern "C"
