// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "demag.h"

namespace demag {

void set_error(const std::string &msg);

#define DEMAG_TRY_HIP(expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::demag::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));       \
      return DEMAG_E_HIP;                                                          \
    }                                                                              \
  } while (0)

#define DEMAG_REQUIRE(cond, msg)                                                   \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      ::demag::set_error(msg);                                                     \
      return DEMAG_E_INVAL;                                                        \
    }                                                                              \
  } while (0)

// Factor types per axis, in table order.
enum FactorType { F_E = 0, F_X = 1, F_P = 2, F_Q = 3, F_NTYPES = 4 };

// One term of a left Toeplitz product: input tensor (buffer id + element
// offset) times the Toeplitz matrix of a generator for each output o, given
// both as an index (type * M + k, used by the bfloat16 window tables) and as
// an element offset into the launch's generator table.
struct MPTerm {
  int32_t in_buf;
  int32_t gen[2];
  int32_t pad_;
  int64_t in_off;
  int64_t gen_off[2];
};

// One job: NOUT outputs accumulated over terms [term0, term0 + nterms).
struct MPJob {
  int32_t term0;
  int32_t nterms;
  int32_t out_buf[2];
  int64_t out_off[2];
  double scale[2];
};

// Geometry of one stage: out[i][c] = sum_terms sum_j T[i][j] in[j][c] with
// i, j < n and c < C.  The column index splits as c = co * C1 + ci; the input
// element of (j, c) is at co * in_S1 + ci + j * kstride, the output element
// of (i, c) at co * out_S1 + ci * out_cs + i * out_is.
struct MPGeom {
  int n;
  int C;
  int C1;
  int genlen;          // 2n - 1
  int64_t kstride;
  int64_t in_S1;
  int64_t out_S1;
  int64_t out_cs;
  int64_t out_is;
};

struct Bufs {
  void *p[6];
};

// A tile of the persistent batched launch.  rb = 0: a thin-axis tile
// (n <= kThinN) of 256 thin_cols(...) consecutive columns, ct counting those.
struct BatchItem {
  int32_t job;
  int32_t geom;
  int32_t ct;
  int16_t rg;
  int8_t rb;
  int8_t nout;
};

// Axes of at most kThinN cells take the vector-ALU tile: rows padded to
// thin_nmax(n), thin_cols(...) columns per lane.
constexpr int kThinN = 16;
__host__ __device__ constexpr int thin_nmax(int n) { return n <= 4 ? 4 : n <= 8 ? 8 : 16; }
__host__ __device__ constexpr int thin_cols(int nmax, int esize) { return nmax >= (esize == 8 ? 8 : 16) ? 1 : (esize == 8 ? 8 : 16) / nmax; }

// A stage launch: jobs with the same NOUT and geometry.
struct StagePlan {
  MPGeom geom;
  int axis;           // axis whose generators are used
  int nout;
  int rb = 8;         // row blocks of 16 per wave
  std::vector<MPJob> jobs;
  std::vector<MPTerm> terms;
  MPJob *d_jobs = nullptr;
  MPTerm *d_terms = nullptr;
};

// Plan of demag_apply_full for one node chunk size.
struct FullPlan {
  int kc = 0;                    // nodes per chunk
  int xsplit = 1;                // partial-sum jobs per x-stage sum
  int nchunks = 0;
  std::vector<std::vector<StagePlan>> chunks;   // per chunk: stage launches in order
  size_t ws_elems = 0;           // elements of workspace per chunk
  ~FullPlan();
};

} // namespace demag

namespace demag {
// Optional per-launch timing: an event pair around each kernel launch on the
// context's stream, accumulated by kernel label when read.
struct ProfRecord {
  std::string label;
  hipEvent_t start, stop;
  double flops, bytes;
};
struct ProfTotals {
  double ms = 0, flops = 0, bytes = 0;
  int64_t launches = 0;
};
}  // namespace demag

struct demag_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t order_ev = nullptr;   // orders a new stream after the previous one
  bool check_inputs = false;       // reject non-finite inputs before launching
  int *d_flag = nullptr;           // device flag of the finiteness check
  void *ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_limit = size_t(16) << 30;
  int tile_rows = 0;        // row blocks per full-format tile (0: by grid size)
  int tile_cols = 0;        // column blocks per bfloat16 tile (0: automatic)
  bool profiling = false;
  std::vector<demag::ProfRecord> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  std::map<std::string, demag::ProfTotals> prof_totals;
};

struct demag_factors {
  int n[3];
  double h[3];          // physical cell sizes
  double hs[3];         // scaled cell sizes (longest grid edge = 1)
  double L;             // length scale: physical = scaled * L
  int M;
  std::vector<double> t, tau, alpha, w;
  double *f64[3] = {nullptr, nullptr, nullptr};   // [4][M][2n-1] per axis
  float *f32[3] = {nullptr, nullptr, nullptr};
  uint16_t *bf[3] = {nullptr, nullptr, nullptr};  // [3 parts][4][M][2n-1] bf16 bits
  void *bfw[3] = {nullptr, nullptr, nullptr};      // [4][M][2n+151][3 parts] 16-byte windows (n <= 1024)
  bool spec_ready = false;
  double *spec[3] = {nullptr, nullptr, nullptr};   // [4][M][L/2+1] real or imaginary parts (structured path)
  float *spec32[3] = {nullptr, nullptr, nullptr};  // FP32 copies (structured path, FP32 transforms)
  void *twiddle[3] = {nullptr, nullptr, nullptr};  // double2 [L/2]
  double *k3 = nullptr;    // 3D kernel spectra, octant [Lz/2+1][Ly/2+1][pitch][10] (FFT apply)
  bool dense = false;      // non-uniform grid: f64[d] holds dense factors [4][M][n][n] (FP64 only)
  std::vector<double> edges[3];   // non-uniform grid: scaled cell edges (source of an async copy)
  hipEvent_t used = nullptr;      // recorded after the last enqueued work that reads the factors
  std::map<std::pair<int, int>, std::unique_ptr<demag::FullPlan>> plans;  // (prec class, kc)
};

namespace demag {
// Record-start / record-stop helpers (no-ops unless profiling is on).
demag_status prof_begin(demag_ctx *ctx, hipEvent_t *ev);
demag_status prof_end(demag_ctx *ctx, hipEvent_t start, const std::string &label, double flops, double bytes);
size_t axis_table_len(const demag_factors *f, int d);  // 4 * M * (2n_d - 1), dense: 4 * M * n_d^2
demag_status launch_assemble(demag_ctx *ctx, demag_factors *f);
demag_status launch_left_stage(demag_ctx *ctx, const demag_factors *f, demag_prec prec,
                               const StagePlan &sp, void *const bufs[6], int beta);
int window_entries(int n);
int default_rb(int n);
int stage_rows(const StagePlan &sp, demag_prec prec);
size_t items_lds_bytes(int nmax, bool fp64);
int items_blocks_per_cu(bool fp64, size_t lds);
void build_chunk_plan(const demag_factors *f, int k0, int kc, double phi_scale, std::vector<StagePlan> &stages);
demag_status launch_items(demag_ctx *ctx, demag_prec prec, const BatchItem *items, int nitems, int grid,
                          const MPJob *jobs, const MPTerm *terms, const MPGeom *geoms, void *const bufp[6],
                          const void *gens, int nmax, int beta, int *counter);
demag_status launch_thin_items(demag_ctx *ctx, demag_prec prec, const BatchItem *items, int nitems, const MPJob *jobs,
                               const MPTerm *terms, const MPGeom *geoms, void *const bufp[6], const void *gens,
                               int beta);
demag_status launch_reset_counters(demag_ctx *ctx, int *counters, int count);
demag_status launch_build_windows(demag_ctx *ctx, demag_factors *f);
// non-uniform grids: dense factors from the scaled cell edges (host, n_d + 1 per axis)
demag_status launch_assemble_dense(demag_ctx *ctx, demag_factors *f, const std::vector<double> edges[3]);
template <class T>
demag_status launch_dense_stage(hipStream_t s, const StagePlan &sp, const T *mats, const Bufs &bufs, int beta);
// Outputs from the x stage's partial sums (FP64 for DEMAG_FP64, else FP32):
// phi = phi_scale sum_s partials[4 s], h_p = sum_s partials[4 s + 1 + p]
// (element blocks of N), added in FP64, added to the outputs when
// accumulate is set.
demag_status launch_reduce_partials(demag_ctx *ctx, demag_prec prec, const void *partials, int nsplit, int64_t N,
                                    void *phi, void *h, double phi_scale, bool accumulate);
demag_status launch_left_stage_bf16(demag_ctx *ctx, const demag_factors *f, demag_prec prec,
                                    const StagePlan &sp, void *const bufs[6], int beta);
demag_status launch_split(demag_ctx *ctx, const float *x, uint16_t *parts, size_t count, int nparts);
// Dense-factor stage (non-uniform grids) with bfloat16-split products: parts
// = [3][table] bfloat16 bits of the axis' dense tables, part_stride elements apart.
demag_status launch_dense_stage_bf16(hipStream_t s, const StagePlan &sp, demag_prec prec, const uint16_t *parts,
                                     size_t part_stride, void *const bufp[6], int beta);
int fft_length(int n);
demag_status prepare_spectra(demag_ctx *ctx, demag_factors *f);
demag_status ensure_workspace(demag_ctx *ctx, size_t bytes);
// Record on the context's stream that work reading f has been enqueued
// (demag_factors_free waits for it).
demag_status note_use(demag_ctx *ctx, const demag_factors *f);
// With the context's input check on: DEMAG_E_INVAL if any of the count
// values at x (device, FP64 if dbl else FP32) is NaN or infinite (synchronizes
// the stream); a no-op otherwise.
demag_status check_finite(demag_ctx *ctx, const void *x, size_t count, bool dbl, const char *what,
                          int *flag = nullptr);
demag_status prepare_fft3d(demag_ctx *ctx, demag_factors *f);
size_t fft3d_workspace_bytes(const demag_factors *f);
demag_status launch_fft3d(demag_ctx *ctx, const demag_factors *f, const double *m, double *phi, double *h,
                          void *ws);
// Structured apply of column sets; the column spectra go to ws (ws_bytes,
// at least columns_workspace_bytes) or, with ws NULL, to the context workspace.
size_t columns_workspace_bytes(const demag_factors *f, const int32_t R[3]);
demag_status launch_columns(demag_ctx *ctx, const demag_factors *f, demag_prec prec, const int32_t R[3],
                            const float *const in[3], float *const out[3], void *ws, size_t ws_bytes);
// Device address of the static scratch array on `device` (set up by
// demag_create); NULL if its set-up failed.
demag_status scratch_init(int device);
} // namespace demag
