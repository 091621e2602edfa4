// Mode products with dense (non-Toeplitz) factor matrices: the full-format
// apply on non-uniform tensor-product grids (the collocation and Lemma
// sinc_mumag hold for any partition; only the Toeplitz structure is lost).
//
// out[i][c] = sum_terms sum_j A_term[i][j] in[j][c] in FP64 or FP32 on the
// matrix cores (v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4, the FP32 tables
// rounded once from the FP64 ones), with the same jobs, terms and stage geometry
// as the Toeplitz path; A_term is the n x n matrix of one factor type and
// node, at element offset gen_off in the axis' dense table [4][M][n][n].
// Tile: 64 rows x (16 NW CB) columns per workgroup (NW waves, each owning
// CB blocks of 16 columns and 4 row blocks); per chunk of KC K values the A
// tiles of the NOUT outputs and the input tile go through LDS, the next
// chunk's tiles loaded into registers while the current one is multiplied.
// LDS row strides: A rows of KC + 1 values.  8-byte LDS reads are served
// 16 lanes at a time, and the 16 lanes of one K value read 16 rows: an odd
// stride puts them in distinct banks (SQ_LDS_BANK_CONFLICT reads 0; an even
// stride of KC + 2 cost about 4 conflict cycles per read).  Input rows of
// NC + 16 values.
#include <type_traits>

#include "internal.h"

namespace demag {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// The 16x16x4 products of each type: accumulator type, the instruction, and
// the block row (or, with swapped operands, column) that register r of lane
// l holds: (l >> 4) + 4 r in FP64, 4 (l >> 4) + r in FP32.
template <class T> struct DMfma;
template <> struct DMfma<double> {
  using acc_t = d4;
  __device__ static inline acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int idx(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct DMfma<float> {
  using acc_t = f4;
  __device__ static inline acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int idx(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Workgroup shape: NW waves, each owning CB blocks of 16 columns and all 64
// rows (4 row blocks), so one A value read from LDS feeds CB products; KC K
// values per chunk; MINW waves per SIMD bound the registers.
template <class T, int NOUT, bool TRANS, int NW, int CB, int KC, int MINW>
__global__ __launch_bounds__(64 * NW, MINW) void k_dense_left(const MPJob *__restrict__ jobs,
                                                             const MPTerm *__restrict__ terms, Bufs bufs,
                                                             const T *__restrict__ mats, MPGeom g,
                                                             int col_tiles, int beta) {
  using MF = DMfma<T>;
  using acc_t = typename MF::acc_t;
  constexpr int NT = 64 * NW, NC = 16 * NW * CB;
  constexpr int kBr = KC * NC / NT;           // input tile values per thread
  constexpr int kAr = 64 * KC / NT;           // A tile values per thread and output
  constexpr int kBrows = NT / NC;             // K rows one pass of the threads stages
  static_assert(kBrows >= 1 && KC % kBrows == 0 && (64 * KC) % NT == 0, "tile shape");
  __shared__ T As[NOUT][64][KC + 1];
  __shared__ T Bs[KC][NC + 16];
  const MPJob job = jobs[blockIdx.y];
  if (job.nterms <= 0) return;
  const int ct = blockIdx.x % col_tiles, rg = blockIdx.x / col_tiles;
  const int n = g.n;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4;
  const int row0 = rg * 64;
  // input staging: this thread's column of the tile (columns past C read C - 1)
  const int cB = tid % NC, kB = tid / NC;
  const int cs = ct * NC + cB;
  const int cl = cs < g.C ? cs : g.C - 1;
  const size_t cin = size_t(cl / g.C1) * g.in_S1 + size_t(cl % g.C1);
  acc_t acc[NOUT][4][CB];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[o][rb][cb] = acc_t{0, 0, 0, 0};
  // (term, K chunk) pairs in one loop; the next pair's tiles are loaded into
  // registers while the current one is multiplied
  const int nch = (n + KC - 1) / KC;
  const int nq = job.nterms * nch;
  T bv[kBr], av[NOUT][kAr];
  auto load = [&](int q) {
    const int t = q / nch, j0 = (q - t * nch) * KC;
    const MPTerm &tm = terms[job.term0 + t];
    const T *in = static_cast<const T *>(bufs.p[tm.in_buf]) + tm.in_off + cin;
#pragma unroll
    for (int r = 0; r < kBr; ++r) {
      const int j = j0 + kB + kBrows * r;
      bv[r] = j < n ? in[size_t(j) * g.kstride] : T(0);
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      const T *A = mats + tm.gen_off[o];
#pragma unroll
      for (int r = 0; r < kAr; ++r) {
        const int e = tid + NT * r;
        const int i = row0 + e / KC, j = j0 + e % KC;
        av[o][r] = (i < n && j < n) ? A[size_t(i) * n + j] : T(0);
      }
    }
  };
  load(0);
  const int wc0 = wave * 16 * CB;   // this wave's first column in the tile
  for (int q = 0; q < nq; ++q) {
#pragma unroll
    for (int r = 0; r < kBr; ++r) Bs[kB + kBrows * r][cB] = bv[r];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
      for (int r = 0; r < kAr; ++r) {
        const int e = tid + NT * r;
        As[o][e / KC][e % KC] = av[o][r];
      }
    __syncthreads();
    if (q + 1 < nq) load(q + 1);
#pragma unroll
    for (int k4 = 0; k4 < KC / 4; ++k4) {
      T b[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) b[cb] = Bs[4 * k4 + kq][wc0 + 16 * cb + (lane & 15)];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
          const T a = As[o][16 * rb + (lane & 15)][4 * k4 + kq];
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            acc[o][rb][cb] = TRANS ? MF::step(b[cb], a, acc[o][rb][cb]) : MF::step(a, b[cb], acc[o][rb][cb]);
        }
    }
    __syncthreads();
  }
  if (TRANS) {
    // operands swapped: register r of lane l holds column MF::idx(l, r) of
    // the block and output row l % 16, so 16 lanes store contiguous values
    // of a row-contiguous output
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int cc = ct * NC + wc0 + 16 * cb + MF::idx(lane, r);
        if (cc >= g.C) continue;
        const size_t ocol = size_t(cc / g.C1) * g.out_S1 + size_t(cc % g.C1) * g.out_cs;
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
          T *out = static_cast<T *>(bufs.p[job.out_buf[o]]) + job.out_off[o] + ocol;
          const T scale = T(job.scale[o]);
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) {
            const int i = row0 + 16 * rb + (lane & 15);
            if (i < n) {
              const size_t idx = size_t(i) * g.out_is;
              T v = scale * acc[o][rb][cb][r];
              if (beta) v += out[idx];
              out[idx] = v;
            }
          }
        }
      }
    return;
  }
  // register r of lane l holds row MF::idx(l, r) of the 16 x 16 block, column l % 16
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int cc = ct * NC + wc0 + 16 * cb + (lane & 15);
    if (cc >= g.C) continue;
    const size_t ocol = size_t(cc / g.C1) * g.out_S1 + size_t(cc % g.C1) * g.out_cs;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      T *out = static_cast<T *>(bufs.p[job.out_buf[o]]) + job.out_off[o] + ocol;
      const T scale = T(job.scale[o]);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = row0 + 16 * rb + MF::idx(lane, r);
          if (i < n) {
            const size_t idx = size_t(i) * g.out_is;
            T v = scale * acc[o][rb][cb][r];
            if (beta) v += out[idx];
            out[idx] = v;
          }
        }
    }
  }
}

template <class T, int NW, int CB, int KC, int MINW>
void launch_dense_shape(hipStream_t s, const StagePlan &sp, const T *mats, const Bufs &bufs, int beta) {
  const MPGeom &g = sp.geom;
  constexpr int NC = 16 * NW * CB;
  const int col_tiles = (g.C + NC - 1) / NC;
  const int row_groups = (g.n + 63) / 64;
  dim3 grid(unsigned(col_tiles * row_groups), unsigned(sp.jobs.size()));
  // rows contiguous in the output (x and y stages): transposed blocks
  const bool tr = g.out_is == 1;
  if (sp.nout == 2) {
    if (tr)
      k_dense_left<T, 2, true, NW, CB, KC, MINW><<<grid, 64 * NW, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, mats, g,
                                                                          col_tiles, beta);
    else
      k_dense_left<T, 2, false, NW, CB, KC, MINW><<<grid, 64 * NW, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, mats, g,
                                                                           col_tiles, beta);
  } else {
    if (tr)
      k_dense_left<T, 1, true, NW, CB, KC, MINW><<<grid, 64 * NW, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, mats, g,
                                                                          col_tiles, beta);
    else
      k_dense_left<T, 1, false, NW, CB, KC, MINW><<<grid, 64 * NW, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, mats, g,
                                                                           col_tiles, beta);
  }
}

}  // namespace

template <class T>
demag_status launch_dense_stage(hipStream_t s, const StagePlan &sp, const T *mats, const Bufs &bufs, int beta) {
  // Shapes measured per stage at n = 128, M = 40: the x stages (input columns
  // strided, K contiguous) run best with 8 waves x 16 columns and 32-K chunks,
  // the y stages with 4 waves x 16 columns, 16-K chunks and three workgroups
  // per CU, the z stage with 4 waves x 32 columns and 16-K chunks.
  // FP32 accumulators take half the registers: twice the column blocks
  if constexpr (std::is_same_v<T, float>) {
    if (sp.axis == 0) launch_dense_shape<T, 8, 2, 32, 1>(s, sp, mats, bufs, beta);
    else if (sp.axis == 1) launch_dense_shape<T, 4, 2, 16, 2>(s, sp, mats, bufs, beta);
    else launch_dense_shape<T, 4, 4, 16, 2>(s, sp, mats, bufs, beta);
  } else {
    if (sp.axis == 0) launch_dense_shape<T, 8, 1, 32, 1>(s, sp, mats, bufs, beta);
    else if (sp.axis == 1) launch_dense_shape<T, 4, 1, 16, 3>(s, sp, mats, bufs, beta);
    else launch_dense_shape<T, 4, 2, 16, 2>(s, sp, mats, bufs, beta);
  }
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

template demag_status launch_dense_stage<double>(hipStream_t, const StagePlan &, const double *, const Bufs &, int);
template demag_status launch_dense_stage<float>(hipStream_t, const StagePlan &, const float *, const Bufs &, int);

}  // namespace demag
