// Mode products with dense (non-Toeplitz) factor matrices: the full-format
// apply on non-uniform tensor-product grids (the collocation and Lemma
// sinc_mumag hold for any partition; only the Toeplitz structure is lost).
//
// out[i][c] = sum_terms sum_j A_term[i][j] in[j][c] in FP64 on the matrix
// cores (v_mfma_f64_16x16x4), with the same jobs, terms and stage geometry
// as the Toeplitz path; A_term is the n x n matrix of one factor type and
// node, at element offset gen_off in the axis' dense table [4][M][n][n].
// Tile: 64 rows x 64 columns per workgroup (4 waves x 16 columns, 4 row
// blocks each); per chunk of 32 K values the A tiles of the NOUT outputs and
// the input tile go through LDS, the next chunk's tiles loaded into registers
// while the current one is multiplied.
#include "internal.h"

namespace demag {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int NOUT, bool TRANS>
__global__ __launch_bounds__(256) void k_dense_left(const MPJob *__restrict__ jobs, const MPTerm *__restrict__ terms,
                                                    Bufs bufs, const double *__restrict__ mats, MPGeom g,
                                                    int col_tiles, int beta) {
  constexpr int KC = 32;               // K values per chunk
  constexpr int kBr = KC * 64 / 256;   // input tile values per thread
  constexpr int kAr = 64 * KC / 256;   // A tile values per thread and output
  __shared__ double As[NOUT][64][KC + 1];
  __shared__ double Bs[KC][65];
  const MPJob job = jobs[blockIdx.y];
  if (job.nterms <= 0) return;
  const int ct = blockIdx.x % col_tiles, rg = blockIdx.x / col_tiles;
  const int n = g.n;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4;
  const int row0 = rg * 64;
  // input staging: this thread's column of the tile (columns past C read C - 1)
  const int cB = tid & 63;
  const int cs = ct * 64 + cB;
  const int cl = cs < g.C ? cs : g.C - 1;
  const size_t cin = size_t(cl / g.C1) * g.in_S1 + size_t(cl % g.C1);
  d4 acc[NOUT][4];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[o][rb] = d4{0, 0, 0, 0};
  // (term, K chunk) pairs in one loop; the next pair's tiles are loaded into
  // registers while the current one is multiplied
  const int nch = (n + KC - 1) / KC;
  const int nq = job.nterms * nch;
  double bv[kBr], av[NOUT][kAr];
  auto load = [&](int q) {
    const int t = q / nch, j0 = (q - t * nch) * KC;
    const MPTerm &tm = terms[job.term0 + t];
    const double *in = static_cast<const double *>(bufs.p[tm.in_buf]) + tm.in_off + cin;
#pragma unroll
    for (int r = 0; r < kBr; ++r) {
      const int j = j0 + (tid >> 6) + 4 * r;
      bv[r] = j < n ? in[size_t(j) * g.kstride] : 0.0;
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      const double *A = mats + tm.gen_off[o];
#pragma unroll
      for (int r = 0; r < kAr; ++r) {
        const int e = tid + 256 * r;
        const int i = row0 + e / KC, j = j0 + e % KC;
        av[o][r] = (i < n && j < n) ? A[size_t(i) * n + j] : 0.0;
      }
    }
  };
  load(0);
  for (int q = 0; q < nq; ++q) {
#pragma unroll
    for (int r = 0; r < kBr; ++r) Bs[(tid >> 6) + 4 * r][cB] = bv[r];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
      for (int r = 0; r < kAr; ++r) {
        const int e = tid + 256 * r;
        As[o][e / KC][e % KC] = av[o][r];
      }
    __syncthreads();
    if (q + 1 < nq) load(q + 1);
#pragma unroll
    for (int k4 = 0; k4 < KC / 4; ++k4) {
      const double b = Bs[4 * k4 + kq][wave * 16 + (lane & 15)];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
          acc[o][rb] = TRANS ? __builtin_amdgcn_mfma_f64_16x16x4f64(b, As[o][16 * rb + (lane & 15)][4 * k4 + kq],
                                                                     acc[o][rb], 0, 0, 0)
                             : __builtin_amdgcn_mfma_f64_16x16x4f64(As[o][16 * rb + (lane & 15)][4 * k4 + kq], b,
                                                                     acc[o][rb], 0, 0, 0);
    }
    __syncthreads();
  }
  if (TRANS) {
    // operands swapped: register r of lane l holds column (l >> 4) + 4 r of
    // the block and output row l % 16, so 16 lanes store 128 contiguous bytes
    // of a row-contiguous output
    const int cbase = ct * 64 + wave * 16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cc = cbase + (lane >> 4) + 4 * r;
      if (cc >= g.C) continue;
      const size_t ocol = size_t(cc / g.C1) * g.out_S1 + size_t(cc % g.C1) * g.out_cs;
#pragma unroll
      for (int o = 0; o < NOUT; ++o) {
        double *out = static_cast<double *>(bufs.p[job.out_buf[o]]) + job.out_off[o] + ocol;
        const double scale = job.scale[o];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          const int i = row0 + 16 * rb + (lane & 15);
          if (i < n) {
            const size_t idx = size_t(i) * g.out_is;
            double v = scale * acc[o][rb][r];
            if (beta) v += out[idx];
            out[idx] = v;
          }
        }
      }
    }
    return;
  }
  // register r of lane l holds row (l >> 4) + 4 r of the 16 x 16 block, column l % 16
  const int cc = ct * 64 + wave * 16 + (lane & 15);
  if (cc >= g.C) return;
  const size_t ocol = size_t(cc / g.C1) * g.out_S1 + size_t(cc % g.C1) * g.out_cs;
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    double *out = static_cast<double *>(bufs.p[job.out_buf[o]]) + job.out_off[o] + ocol;
    const double scale = job.scale[o];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + 16 * rb + (lane >> 4) + 4 * r;
        if (i < n) {
          const size_t idx = size_t(i) * g.out_is;
          double v = scale * acc[o][rb][r];
          if (beta) v += out[idx];
          out[idx] = v;
        }
      }
  }
}

}  // namespace

demag_status launch_dense_stage(hipStream_t s, const StagePlan &sp, const double *mats, const Bufs &bufs, int beta) {
  const MPGeom &g = sp.geom;
  const int col_tiles = (g.C + 63) / 64;
  const int row_groups = (g.n + 63) / 64;
  dim3 grid(unsigned(col_tiles * row_groups), unsigned(sp.jobs.size()));
  // rows contiguous in the output (x and y stages): transposed blocks
  const bool tr = g.out_is == 1;
  if (sp.nout == 2) {
    if (tr) k_dense_left<2, true><<<grid, 256, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, mats, g, col_tiles, beta);
    else k_dense_left<2, false><<<grid, 256, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, mats, g, col_tiles, beta);
  } else {
    if (tr) k_dense_left<1, true><<<grid, 256, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, mats, g, col_tiles, beta);
    else k_dense_left<1, false><<<grid, 256, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, mats, g, col_tiles, beta);
  }
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

}  // namespace demag
