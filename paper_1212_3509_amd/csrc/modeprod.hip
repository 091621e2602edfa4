// Left Toeplitz mode products on the matrix cores (FP64 and FP32).
//
// One launch computes, for every job and batch b,
//   out_o[b][i][c] = scale_o * sum_terms sum_j T_{gen(o,term)}[i][j] * in_term[b][j][c]
// (or stored transposed as out_o[b][c][i]), with the Toeplitz matrices
// T[i][j] = g[i - j + n - 1] generated from their length 2n-1 generators
// (Sec. 4.2) and never materialised.  This is the j-mode product of
// Eq. (modemul) along the axis whose index is j, batched over the other axes.
//
// Tiling (wave64, CDNA4): a workgroup of 4 waves covers 64 columns; each wave
// owns 16 columns and 16*RB rows as RB blocks of the 16x16x4 MFMA, for NOUT
// outputs that share the input fragment.  The B operand (input) is read
// straight from global memory, 16 consecutive columns per row, one value per
// lane per K-step; the A operand (Toeplitz) comes from the generator staged
// in LDS (one ds_read per fragment).  Loads of the next 8 K-steps are issued
// before the current 8 are multiplied.
#include "internal.h"

namespace demag {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <class T> struct Mfma;
template <> struct Mfma<double> {
  using acc_t = d4;
  __device__ static inline acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // v_mfma_f64_16x16x4: register r of lane l holds row (l >> 4) + 4 r.
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  using acc_t = f4;
  __device__ static inline acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // v_mfma_f32_16x16x4: register r of lane l holds row 4 (l >> 4) + r.
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

struct Bufs {
  void *p[6];
};

constexpr int kUnroll = 8;  // K-steps (of 4) prefetched ahead

template <class T, int RB, int NOUT, bool TR>
__global__ __launch_bounds__(256) void k_left(const MPJob *__restrict__ jobs,
                                              const MPTerm *__restrict__ terms, Bufs bufs,
                                              const T *__restrict__ gens, MPGeom g, int col_tiles,
                                              int beta) {
  extern __shared__ unsigned char smem_raw[];
  T *sg = reinterpret_cast<T *>(smem_raw);
  using Mf = Mfma<T>;
  using acc_t = typename Mf::acc_t;
  const int n = g.n;
  const int glds = 2 * n + 16 * RB + 32;
  const MPJob job = jobs[blockIdx.z];
  const int b = blockIdx.y;
  const int ct = blockIdx.x % col_tiles;
  const int rg = blockIdx.x / col_tiles;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  const int c = ct * 64 + wave * 16 + (lane & 15);
  const bool cvalid = c < g.C;
  const int row0 = rg * 16 * RB;
  // LDS index of T[row0 + (lane & 15)][kq] for j0 = 0; add 16 rb - j0.
  const int ibase = row0 + (lane & 15) - kq + n - 1 + 16;

  acc_t acc[NOUT][RB];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[o][rb] = acc_t{0, 0, 0, 0};

  for (int t = 0; t < job.nterms; ++t) {
    const MPTerm tm = terms[job.term0 + t];
    __syncthreads();
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      const T *gsrc = gens + size_t(tm.gen[o]) * g.genlen;
      for (int idx = threadIdx.x; idx < glds; idx += 256) {
        const int s = idx - 16;
        sg[o * glds + idx] = (s >= 0 && s < g.genlen) ? gsrc[s] : T(0);
      }
    }
    __syncthreads();
    const T *in = static_cast<const T *>(bufs.p[tm.in_buf]) + tm.in_off + size_t(b) * g.in_bstride +
                  (cvalid ? c : 0);
    T nxt[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int j = 4 * u + kq;
      nxt[u] = (cvalid && j < n) ? in[size_t(j) * g.kstride] : T(0);
    }
    for (int j0 = 0; j0 < n; j0 += 4 * kUnroll) {
      T cur[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) cur[u] = nxt[u];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int j = j0 + 4 * (kUnroll + u) + kq;
        nxt[u] = (cvalid && j < n) ? in[size_t(j) * g.kstride] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int jj = j0 + 4 * u;
        if (jj < n) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const int idx = ibase + 16 * rb - jj;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) acc[o][rb] = Mf::step(sg[o * glds + idx], cur[u], acc[o][rb]);
          }
        }
      }
    }
  }

  if (!cvalid) return;
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    T *out = static_cast<T *>(bufs.p[job.out_buf[o]]) + job.out_off[o] + size_t(b) * g.out_bstride;
    const T scale = T(job.scale[o]);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + 16 * rb + Mf::row(lane, r);
        if (i < n) {
          const size_t idx = TR ? size_t(c) * n + i : size_t(i) * g.C + c;
          T v = scale * acc[o][rb][r];
          if (beta) v += out[idx];
          out[idx] = v;
        }
      }
  }
}

template <class T, int RB, int NOUT>
demag_status launch_rb(hipStream_t s, const StagePlan &sp, const T *gens, const Bufs &bufs, int beta) {
  const MPGeom &g = sp.geom;
  const int col_tiles = (g.C + 63) / 64;
  const int row_groups = (g.n + 16 * RB - 1) / (16 * RB);
  dim3 grid(col_tiles * row_groups, g.B, unsigned(sp.jobs.size()));
  const size_t lds = size_t(NOUT) * (2 * g.n + 16 * RB + 32) * sizeof(T);
  if (g.transposed)
    k_left<T, RB, NOUT, true><<<grid, 256, lds, s>>>(sp.d_jobs, sp.d_terms, bufs, gens, g, col_tiles, beta);
  else
    k_left<T, RB, NOUT, false><<<grid, 256, lds, s>>>(sp.d_jobs, sp.d_terms, bufs, gens, g, col_tiles, beta);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

template <class T, int NOUT>
demag_status launch_nout(hipStream_t s, const StagePlan &sp, const T *gens, const Bufs &bufs, int beta) {
  const int n = sp.geom.n;
  if (n <= 16) return launch_rb<T, 1, NOUT>(s, sp, gens, bufs, beta);
  if (n <= 32) return launch_rb<T, 2, NOUT>(s, sp, gens, bufs, beta);
  if (n <= 64) return launch_rb<T, 4, NOUT>(s, sp, gens, bufs, beta);
  return launch_rb<T, 8, NOUT>(s, sp, gens, bufs, beta);
}

template <class T>
demag_status launch_typed(hipStream_t s, const StagePlan &sp, const T *gens, const Bufs &bufs, int beta) {
  if (sp.nout == 1) return launch_nout<T, 1>(s, sp, gens, bufs, beta);
  return launch_nout<T, 2>(s, sp, gens, bufs, beta);
}

}  // namespace

demag_status launch_left_stage(demag_ctx *ctx, const demag_factors *f, demag_prec prec,
                               const StagePlan &sp, void *const bufp[6], int beta) {
  if (sp.jobs.empty()) return DEMAG_OK;
  Bufs bufs;
  for (int i = 0; i < 6; ++i) bufs.p[i] = bufp[i];
  hipEvent_t ev = nullptr;
  demag_status st = prof_begin(ctx, &ev);
  if (st != DEMAG_OK) return st;
  const char *pname = "?";
  size_t esize = 4;
  if (prec == DEMAG_FP64) {
    st = launch_typed<double>(ctx->stream, sp, f->f64[sp.axis], bufs, beta);
    pname = "fp64";
    esize = 8;
  } else if (prec == DEMAG_FP32) {
    st = launch_typed<float>(ctx->stream, sp, f->f32[sp.axis], bufs, beta);
    pname = "fp32";
  } else {
    st = launch_left_stage_bf16(ctx, f, prec, sp, bufp, beta);
    pname = (prec == DEMAG_BF16X3) ? "bf16x3" : "bf16x2";
  }
  if (st != DEMAG_OK) return st;
  if (ev) {
    // Algorithmic work of the launch: each term of each job is a dense
    // n x n Toeplitz times n x (C B) product per output; compulsory traffic
    // reads each term's input once and writes (and, when accumulating,
    // reads) each output once.
    const MPGeom &g = sp.geom;
    const double slab = double(g.n) * g.C * g.B;
    double flops = 0, bytes = 0;
    // split precisions count every bfloat16 product they issue
    const double mult = (prec == DEMAG_BF16X3) ? 6.0 : (prec == DEMAG_BF16X2) ? 3.0 : 1.0;
    for (const auto &j : sp.jobs) {
      flops += mult * 2.0 * g.n * slab * j.nterms * sp.nout;
      bytes += slab * esize * (j.nterms + sp.nout * (beta ? 2 : 1));
    }
    const char axis = "xyz"[sp.axis];
    std::string label = std::string(pname) + "/" + axis + "/nout" + char('0' + sp.nout);
    st = prof_end(ctx, ev, label, flops, bytes);
  }
  return st;
}

}  // namespace demag
