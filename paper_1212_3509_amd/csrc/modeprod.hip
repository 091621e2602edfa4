// Left Toeplitz mode products on the matrix cores (FP64 and FP32).
//
// One launch computes, for every job,
//   out_o[i][c] = scale_o * sum_terms sum_j T_{gen(o,term)}[i][j] * in_term[j][c]
// with the Toeplitz matrices T[i][j] = g[i - j + n - 1] generated from their
// length-(2n-1) generators (Sec. 4.2) and never materialised.  This is the
// j-mode product of Eq. (modemul) along the axis whose index is j; the other
// two axes are flattened into the column index c = (co, ci), ci < C1, whose
// input and output addresses are co * S1 + ci * (inner stride) (MPGeom).
//
// Tiling (wave64, CDNA4): a workgroup of 4 waves covers 64 columns; each wave
// owns 16 columns and 16*RB rows as RB blocks of the 16x16x4 MFMA, for NOUT
// outputs that share the input fragment.  The B operand (input) is read
// straight from global memory, 16 consecutive columns per row, one value per
// lane per K-step; the A operand (Toeplitz) comes from the generator staged
// in LDS (one ds_read per fragment).
//
// Pipelining: the (term, K-chunk) pairs of a job form one loop; the loads of
// chunk q + 1 (which may belong to the next term) are in flight while chunk q
// is multiplied, and the next term's generators are fetched into registers a
// whole term ahead and written to the second of two LDS buffers, so a term
// boundary costs one barrier.  Every global load is unconditional (rows past
// n and columns past C read clamped, in-bounds addresses whose values are
// zeroed or never stored), so the compiler can count outstanding loads and
// wait only for the oldest ones.
//
// The same tile routine serves the batched path, where one persistent launch
// walks a list of (job, geometry, tile) items of many grids.
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

constexpr int kChunkSteps = 8;  // K-steps (of 4) per chunk
constexpr int kGenPer = 4;  // generator values per thread fetched a term ahead

__host__ __device__ inline size_t tile_lds_elems(int n, int RB, int NOUT) {
  return 2 * size_t(NOUT) * (2 * n + 16 * RB + 32);  // two generator buffers
}

// Generator value e of a term's staged block: output o = e / glds, generator
// index s = e % glds - 32 (zero outside [0, genlen)).  g0, g1: the term's
// generators of outputs 0 and 1.  Returns an in-bounds address for every e
// and sets ok when the value is a real generator entry.
template <class T, int NOUT>
__device__ __forceinline__ const T *gen_addr(const T *g0, const T *g1, int e, int glds, int gtot, int genlen,
                                             bool &ok) {
  const bool second = NOUT > 1 && e >= glds;
  const int s = e - (second ? glds : 0) - 32;
  ok = e < gtot && s >= 0 && s < genlen;
  const int sc = s < 0 ? 0 : (s >= genlen ? genlen - 1 : s);
  return (second ? g1 : g0) + sc;
}

// One 64-column x 16*RB-row tile of one job.  sg: LDS, tile_lds_elems(n, RB, NOUT).
// TRANS: multiply with the operands swapped, which yields the transposed
// 16x16 block (same fragments: the A and B layouts of the instruction are
// mirror images), so a lane's results run along the output rows i; chosen
// when rows are contiguous in memory (out_is == 1), giving 128-byte stores.
template <class T, int RB, int NOUT, bool TRANS, bool WHOLE = false>
__device__ __forceinline__ void left_tile(const MPJob &job, const MPTerm *__restrict__ terms, const Bufs &bufs,
                                          const T *__restrict__ gens, const MPGeom &g, int ct, int rg, int beta,
                                          T *sg) {
  using Mf = Mfma<T>;
  using acc_t = typename Mf::acc_t;
  // K-steps per chunk: FP32 on ragged axes takes chunks of 16 rows, which
  // halves the zero rows of a term's last chunk
  constexpr int kUnroll = (!WHOLE && sizeof(T) == 4) ? 4 : kChunkSteps;
  const int n = g.n;
  const int nterms = job.nterms;
  if (nterms <= 0) return;
  const int glds = 2 * n + 16 * RB + 32;
  const int gtot = NOUT * glds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  const int c = ct * 64 + wave * 16 + (lane & 15);
  const bool cvalid = c < g.C;
  // columns past C read column C - 1 and are never stored
  const int cl = cvalid ? c : g.C - 1;
  const int co = cl / g.C1, ci = cl % g.C1;
  const size_t cin = size_t(co) * g.in_S1 + ci;
  // WHOLE (n a multiple of 4 kChunkSteps): every chunk lies inside the n rows,
  // so its loads need no clamping and its inputs no masking; row j0 + 4 u +
  // kq is a uniform row pointer plus this lane's offset kq kstride + cin
  const size_t clane = size_t(kq) * g.kstride + cin;
  const int row0 = rg * 16 * RB;
  // LDS index of T[row0 + (lane & 15)][kq] for j0 = 0; add 16 rb - j0.
  // With 32 leading zeros and glds = 2n + 16 RB + 32 every index stays in
  // [1, glds): i < n + 16 RB - 1 and j < n + 31 (zero-input steps included).
  const int ibase = row0 + (lane & 15) - kq + n - 1 + 32;
  const int nch = (n + 4 * kUnroll - 1) / (4 * kUnroll);
  const int nq = nterms * nch;
  auto term_in = [&](int t) -> const T * {
    const MPTerm &tm = terms[job.term0 + t];
    return static_cast<const T *>(bufs.p[tm.in_buf]) + tm.in_off + cin;
  };

  acc_t acc[NOUT][RB];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[o][rb] = acc_t{0, 0, 0, 0};

  // the previous tile of a persistent workgroup may still read the buffers
  __syncthreads();
  auto gen0 = [&](int t) { return gens + terms[job.term0 + t].gen_off[0]; };
  auto gen1 = [&](int t) { return gens + terms[job.term0 + t].gen_off[NOUT > 1 ? 1 : 0]; };
  T greg[kGenPer];
  {
    const T *g0 = gen0(0), *g1 = gen1(0);
#pragma unroll
    for (int r = 0; r < kGenPer; ++r) {
      bool ok;
      greg[r] = *gen_addr<T, NOUT>(g0, g1, threadIdx.x + 256 * r, glds, gtot, g.genlen, ok);
    }
  }
  T nxt[kUnroll];
  auto load_chunk = [&](int t1, int j1) {
    if (WHOLE) {
      const MPTerm &tm = terms[job.term0 + t1];
      const T *base = static_cast<const T *>(bufs.p[tm.in_buf]) + tm.in_off;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) nxt[u] = (base + int64_t(j1 + 4 * u) * g.kstride)[clane];
    } else {
      const T *in1 = term_in(t1);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int j = min(j1 + 4 * u + kq, n - 1);
        nxt[u] = in1[size_t(j) * g.kstride];
      }
    }
  };
  load_chunk(0, 0);

  int t = 0, j0 = 0;
  for (int q = 0; q < nq; ++q) {
    if (j0 == 0) {
      // term t starts: its generators (fetched a term ahead) go to buffer t & 1,
      // last read during term t - 2, which every wave finished before the
      // barrier of term t - 1
      T *buf = sg + (t & 1) * gtot;
      const T *g0 = gen0(t), *g1 = gen1(t);
#pragma unroll
      for (int r = 0; r < kGenPer; ++r) {
        const int e = threadIdx.x + 256 * r;
        bool ok;
        gen_addr<T, NOUT>(g0, g1, e, glds, gtot, g.genlen, ok);
        if (e < gtot) buf[e] = ok ? greg[r] : T(0);
      }
      for (int e0 = 256 * kGenPer; e0 < gtot; e0 += 256) {  // long generators: the rest now
        const int e = e0 + threadIdx.x;
        bool ok;
        const T v = *gen_addr<T, NOUT>(g0, g1, e, glds, gtot, g.genlen, ok);
        if (e < gtot) buf[e] = ok ? v : T(0);
      }
      const int tn = min(t + 1, nterms - 1);
      const T *n0 = gen0(tn), *n1 = gen1(tn);
#pragma unroll
      for (int r = 0; r < kGenPer; ++r) {
        bool ok;
        greg[r] = *gen_addr<T, NOUT>(n0, n1, threadIdx.x + 256 * r, glds, gtot, g.genlen, ok);
      }
      __syncthreads();
    }
    const T *sgen = sg + (t & 1) * gtot;
    T cur[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) cur[u] = nxt[u];
    {
      // chunk q + 1: the next chunk of this term, else the first of the next
      // term; the last chunk of the job re-reads its own rows
      int t1 = t, j1 = j0 + 4 * kUnroll;
      if (j1 >= n) {
        j1 = (t + 1 < nterms) ? 0 : j0;
        t1 = min(t + 1, nterms - 1);
      }
      load_chunk(t1, j1);
    }
    // keep the next chunk's loads ahead of this chunk's products
    __builtin_amdgcn_sched_barrier(0);
    // one output: the Toeplitz fragments of step u + 1 are read from LDS
    // into a second register set before step u's products are issued (with
    // two outputs the second set costs a wave per SIMD in FP32 and does not
    // fit in FP64)
    constexpr bool kABuf = WHOLE && NOUT == 1;
    if constexpr (kABuf) {
      T a[2][NOUT][RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int o = 0; o < NOUT; ++o) a[0][o][rb] = sgen[o * glds + ibase + 16 * rb - j0];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (u + 1 < kUnroll) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int o = 0; o < NOUT; ++o)
              a[(u + 1) & 1][o][rb] = sgen[o * glds + ibase + 16 * rb - (j0 + 4 * (u + 1))];
        }
        __builtin_amdgcn_sched_barrier(0);
        const T b = cur[u];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int o = 0; o < NOUT; ++o)
            acc[o][rb] = TRANS ? Mf::step(b, a[u & 1][o][rb], acc[o][rb]) : Mf::step(a[u & 1][o][rb], b, acc[o][rb]);
      }
    } else {
      // K-steps of the chunk; on a ragged axis the last chunk of a term
      // stops at the first step wholly past n (its inputs are all zero), and
      // row blocks wholly past n (never stored) are skipped: both conditions
      // are uniform, and skipping adds nothing but exact zeros
      const int live_u = WHOLE ? kUnroll : min(kUnroll, (n - j0 + 3) >> 2);
      const int live_rb = WHOLE ? RB : min(RB, (n - row0 + 15) >> 4);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (!WHOLE && u >= live_u) break;
        const int jj = j0 + 4 * u;
        const T b = (WHOLE || jj + kq < n) ? cur[u] : T(0);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (!WHOLE && rb >= live_rb) break;
          const int idx = ibase + 16 * rb - jj;
#pragma unroll
          for (int o = 0; o < NOUT; ++o)
            acc[o][rb] = TRANS ? Mf::step(b, sgen[o * glds + idx], acc[o][rb])
                               : Mf::step(sgen[o * glds + idx], b, acc[o][rb]);
        }
      }
    }
    j0 += 4 * kUnroll;
    if (j0 >= n) {
      j0 = 0;
      ++t;
    }
  }

  if (TRANS) {
    // register r of lane l: column cbase + row(l, r), output row 16 rb + l % 16
    const int cbase = ct * 64 + wave * 16;
    size_t ob[4];
    bool okc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cc = cbase + Mf::row(lane, r);
      okc[r] = cc < g.C;
      const int cco = okc[r] ? cc / g.C1 : 0, cci = okc[r] ? cc % g.C1 : 0;
      ob[r] = size_t(cco) * g.out_S1 + size_t(cci) * g.out_cs;
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      T *out = static_cast<T *>(bufs.p[job.out_buf[o]]) + job.out_off[o];
      const T scale = T(job.scale[o]);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int i = row0 + 16 * rb + (lane & 15);
        if (i < n) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (okc[r]) {
              const size_t idx = ob[r] + size_t(i) * g.out_is;
              T v = scale * acc[o][rb][r];
              if (beta) v += out[idx];
              out[idx] = v;
            }
        }
      }
    }
    return;
  }
  if (!cvalid) return;
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    T *out = static_cast<T *>(bufs.p[job.out_buf[o]]) + job.out_off[o] + size_t(co) * g.out_S1 + size_t(ci) * g.out_cs;
    const T scale = T(job.scale[o]);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + 16 * rb + Mf::row(lane, r);
        if (i < n) {
          const size_t idx = size_t(i) * g.out_is;
          T v = scale * acc[o][rb][r];
          if (beta) v += out[idx];
          out[idx] = v;
        }
      }
  }
}

// Thin axes (n <= kThinN): the products of one job on the vector ALU.  A
// workgroup covers 256 CPT consecutive columns, lane l taking columns
// (ct CPT + k) 256 + l, k < CPT; each lane holds the n inputs of its columns
// and issues a term's n CPT loads at once.  A 16-row MFMA block would leave
// most rows empty here, and a 64-column tile holds too little work to hide
// its load latency.  Rows are padded to NMAX: inputs past n are zero and
// rows past n are never stored.  Each output sums term by term with j
// ascending, the same in the single-state and the batched launch.
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class T, int NMAX, int NOUT>
__device__ __forceinline__ void thin_tile(const MPJob &job, const MPTerm *__restrict__ terms, const Bufs &bufs,
                                          const T *__restrict__ gens, const MPGeom &g, int ct, int beta) {
  constexpr int CPT = thin_cols(NMAX, sizeof(T));
  const int n = g.n;
  size_t cin[CPT], cout[CPT];
  bool ok[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = (ct * CPT + k) * 256 + int(threadIdx.x);
    ok[k] = c < g.C;
    const int cl = ok[k] ? c : g.C - 1;
    const int co = cl / g.C1, ci = cl % g.C1;
    cin[k] = size_t(co) * g.in_S1 + ci;
    cout[k] = size_t(co) * g.out_S1 + size_t(ci) * g.out_cs;
  }
  T acc[NOUT][NMAX][CPT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
#pragma unroll
      for (int k = 0; k < CPT; ++k) acc[o][i][k] = T(0);
  for (int t = 0; t < job.nterms; ++t) {
    const MPTerm &tm = terms[job.term0 + t];
    const T *in = static_cast<const T *>(bufs.p[tm.in_buf]) + tm.in_off;
    T x[NMAX][CPT];
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
#pragma unroll
      for (int k = 0; k < CPT; ++k) x[j][k] = T(0);
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
      if (j < n) {
#pragma unroll
        for (int k = 0; k < CPT; ++k) x[j][k] = in[cin[k] + size_t(j) * g.kstride];
      }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      // gv[d] = T[i][j] for i - j = d - (NMAX - 1): generator entry d + n - NMAX
      const T *gp = gens + tm.gen_off[o];
      T gv[2 * NMAX - 1];
#pragma unroll
      for (int d = 0; d < 2 * NMAX - 1; ++d) {
        const int e = d + n - NMAX;
        gv[d] = (e >= 0 && e < g.genlen) ? gp[e] : T(0);
      }
#pragma unroll
      for (int j = 0; j < NMAX; ++j)
        if (j < n) {
#pragma unroll
          for (int i = 0; i < NMAX; ++i)
#pragma unroll
            for (int k = 0; k < CPT; ++k) acc[o][i][k] = fma_t(gv[i - j + NMAX - 1], x[j][k], acc[o][i][k]);
        }
    }
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    T *out = static_cast<T *>(bufs.p[job.out_buf[o]]) + job.out_off[o];
    const T scale = T(job.scale[o]);
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
      if (i < n) {
#pragma unroll
        for (int k = 0; k < CPT; ++k)
          if (ok[k]) {
            const size_t idx = cout[k] + size_t(i) * g.out_is;
            T v = scale * acc[o][i][k];
            if (beta) v += out[idx];
            out[idx] = v;
          }
      }
  }
}

template <class T, int NOUT>
__device__ __forceinline__ void thin_dispatch(const MPJob &job, const MPTerm *__restrict__ terms, const Bufs &bufs,
                                              const T *__restrict__ gens, const MPGeom &g, int ct, int beta) {
  if (g.n <= 4) thin_tile<T, 4, NOUT>(job, terms, bufs, gens, g, ct, beta);
  else if (g.n <= 8) thin_tile<T, 8, NOUT>(job, terms, bufs, gens, g, ct, beta);
  else thin_tile<T, 16, NOUT>(job, terms, bufs, gens, g, ct, beta);
}

template <class T, int NMAX, int NOUT>
__global__ __launch_bounds__(256) void k_thin(const MPJob *__restrict__ jobs, const MPTerm *__restrict__ terms,
                                              Bufs bufs, const T *__restrict__ gens, MPGeom g, int beta) {
  thin_tile<T, NMAX, NOUT>(jobs[blockIdx.y], terms, bufs, gens, g, blockIdx.x, beta);
}

template <class T, int RB, int NOUT, int AXIS, bool WHOLE>
__global__ __launch_bounds__(256, 2) void k_left(const MPJob *__restrict__ jobs, const MPTerm *__restrict__ terms,
                                              Bufs bufs, const T *__restrict__ gens, MPGeom g, int col_tiles,
                                              int beta) {
  extern __shared__ unsigned char smem_raw[];
  const MPJob job = jobs[blockIdx.y];
  // the x and y stages write rows contiguously; the z stage writes columns
  left_tile<T, RB, NOUT, AXIS != 2, WHOLE>(job, terms, bufs, gens, g, blockIdx.x % col_tiles, blockIdx.x / col_tiles,
                                           beta, reinterpret_cast<T *>(smem_raw));
}

// Persistent variant: workgroups take items from a counter (one atomic add
// per item, so the cost-sorted list is spread greedily over the chip); each
// item names its job, geometry, tile and the (RB, NOUT) shape chosen for it.
// Items write disjoint output tiles, so the result does not depend on which
// workgroup takes which item.  The counter starts at 0 (k_reset_counters)
// and every workgroup leaves once it draws an index past the list.
template <class T>
__global__ __launch_bounds__(256, 2) void k_left_items(const BatchItem *__restrict__ items, int nitems,
                                                    const MPJob *__restrict__ jobs, const MPTerm *__restrict__ terms,
                                                    const MPGeom *__restrict__ geoms, Bufs bufs,
                                                    const T *__restrict__ gens, int beta, int *counter) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ int next_item;
  T *sg = reinterpret_cast<T *>(smem_raw);
  for (;;) {
    if (threadIdx.x == 0) next_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = next_item;
    __syncthreads();   // every thread has read next_item before it is drawn again
    if (it >= nitems) break;
    const BatchItem item = items[it];
    const MPJob job = jobs[item.job];
    const MPGeom g = geoms[item.geom];
    const int key = (item.rb * 4 + item.nout) * 2 + (g.out_is == 1 ? 1 : 0);
    switch (key) {
#define DEMAG_ITEM_CASE(R, N)                                                                  \
  case (R * 4 + N) * 2: left_tile<T, R, N, false>(job, terms, bufs, gens, g, item.ct, item.rg, beta, sg); break; \
  case (R * 4 + N) * 2 + 1: left_tile<T, R, N, true>(job, terms, bufs, gens, g, item.ct, item.rg, beta, sg); break;
      DEMAG_ITEM_CASE(1, 1)
      DEMAG_ITEM_CASE(1, 2)
      DEMAG_ITEM_CASE(2, 1)
      DEMAG_ITEM_CASE(2, 2)
      DEMAG_ITEM_CASE(4, 1)
      DEMAG_ITEM_CASE(4, 2)
      DEMAG_ITEM_CASE(8, 1)
      DEMAG_ITEM_CASE(8, 2)
#undef DEMAG_ITEM_CASE
      default: break;  // shapes are validated when the item list is built
    }
  }
}

// Thin-axis items of a batched stage (BatchItem.rb = 0), one workgroup per
// item.  Kept apart from k_left_items, whose register allocation the
// vector-ALU tile would change.
template <class T>
__global__ __launch_bounds__(256) void k_thin_items(const BatchItem *__restrict__ items,
                                                    const MPJob *__restrict__ jobs, const MPTerm *__restrict__ terms,
                                                    const MPGeom *__restrict__ geoms, Bufs bufs,
                                                    const T *__restrict__ gens, int beta) {
  const BatchItem item = items[blockIdx.x];
  const MPJob job = jobs[item.job];
  const MPGeom g = geoms[item.geom];
  if (item.nout == 1) thin_dispatch<T, 1>(job, terms, bufs, gens, g, item.ct, beta);
  else thin_dispatch<T, 2>(job, terms, bufs, gens, g, item.ct, beta);
}

template <class T, int RB, int NOUT, int AXIS>
demag_status launch_axis(hipStream_t s, const StagePlan &sp, const T *gens, const Bufs &bufs, int beta) {
  const MPGeom &g = sp.geom;
  const int col_tiles = (g.C + 63) / 64;
  const int row_groups = (g.n + 16 * RB - 1) / (16 * RB);
  dim3 grid(col_tiles * row_groups, unsigned(sp.jobs.size()));
  const size_t lds = tile_lds_elems(g.n, RB, NOUT) * sizeof(T);
  auto k = (g.n % (4 * kChunkSteps) == 0) ? &k_left<T, RB, NOUT, AXIS, true> : &k_left<T, RB, NOUT, AXIS, false>;
  if (lds > 65536)
    DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      int(lds)));
  k<<<grid, 256, lds, s>>>(sp.d_jobs, sp.d_terms, bufs, gens, g, col_tiles, beta);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

template <class T, int RB, int NOUT>
demag_status launch_rb(hipStream_t s, const StagePlan &sp, const T *gens, const Bufs &bufs, int beta) {
  // one template instance per stage axis, so kernel traces separate the stages
  if (sp.axis == 0) return launch_axis<T, RB, NOUT, 0>(s, sp, gens, bufs, beta);
  if (sp.axis == 1) return launch_axis<T, RB, NOUT, 1>(s, sp, gens, bufs, beta);
  return launch_axis<T, RB, NOUT, 2>(s, sp, gens, bufs, beta);
}

template <class T, int NOUT>
demag_status launch_nout(hipStream_t s, int rb, const StagePlan &sp, const T *gens, const Bufs &bufs, int beta) {
  switch (rb) {
    case 1: return launch_rb<T, 1, NOUT>(s, sp, gens, bufs, beta);
    case 2: return launch_rb<T, 2, NOUT>(s, sp, gens, bufs, beta);
    case 4: return launch_rb<T, 4, NOUT>(s, sp, gens, bufs, beta);
    default: return launch_rb<T, 8, NOUT>(s, sp, gens, bufs, beta);
  }
}

template <class T, int NMAX>
demag_status launch_thin_nmax(hipStream_t s, const StagePlan &sp, const T *gens, const Bufs &bufs, int beta) {
  const MPGeom &g = sp.geom;
  const int cols = 256 * thin_cols(NMAX, sizeof(T));
  dim3 grid(unsigned((g.C + cols - 1) / cols), unsigned(sp.jobs.size()));
  if (sp.nout == 1) k_thin<T, NMAX, 1><<<grid, 256, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, gens, g, beta);
  else k_thin<T, NMAX, 2><<<grid, 256, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, gens, g, beta);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

template <class T>
demag_status launch_typed(hipStream_t s, int rb, const StagePlan &sp, const T *gens, const Bufs &bufs, int beta) {
  if (sp.geom.n <= kThinN) {
    const int nmax = thin_nmax(sp.geom.n);
    if (nmax == 4) return launch_thin_nmax<T, 4>(s, sp, gens, bufs, beta);
    if (nmax == 8) return launch_thin_nmax<T, 8>(s, sp, gens, bufs, beta);
    return launch_thin_nmax<T, 16>(s, sp, gens, bufs, beta);
  }
  if (sp.nout == 1) return launch_nout<T, 1>(s, rb, sp, gens, bufs, beta);
  return launch_nout<T, 2>(s, rb, sp, gens, bufs, beta);
}

}  // namespace

int default_rb(int n) { return n <= 16 ? 1 : n <= 32 ? 2 : n <= 64 ? 4 : 8; }

// Row blocks per tile for a stage: the tallest tile that covers the axis,
// lowered while the launch would give fewer than two workgroups per CU
// (256 CUs), e.g. the x stage's single job of all nodes' terms.
int stage_rows(const StagePlan &sp, demag_prec) {
  const int64_t col_tiles = (sp.geom.C + 63) / 64;  // 64 columns per tile (bfloat16: one block per wave)
  int rb = sp.rb;
  while (rb > 1 && col_tiles * ((sp.geom.n + 16 * rb - 1) / (16 * rb)) * int64_t(sp.jobs.size()) < 512) rb /= 2;
  return rb;
}

size_t items_lds_bytes(int nmax, bool fp64) {
  return tile_lds_elems(nmax, 8, 2) * (fp64 ? 8 : 4);
}

int items_blocks_per_cu(bool fp64, size_t lds) {
  int n = 0;
  hipError_t e = fp64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_left_items<double>, 256, lds)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_left_items<float>, 256, lds);
  return (e == hipSuccess && n > 0) ? n : 1;
}

__global__ void k_reset_counters(int *c, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) c[i] = 0;
}

demag_status launch_reset_counters(demag_ctx *ctx, int *counters, int count) {
  if (count <= 0) return DEMAG_OK;
  k_reset_counters<<<(count + 255) / 256, 256, 0, ctx->stream>>>(counters, count);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

demag_status launch_items(demag_ctx *ctx, demag_prec prec, const BatchItem *items, int nitems, int grid,
                          const MPJob *jobs, const MPTerm *terms, const MPGeom *geoms, void *const bufp[6],
                          const void *gens, int nmax, int beta, int *counter) {
  if (nitems == 0) return DEMAG_OK;
  Bufs bufs;
  for (int i = 0; i < 6; ++i) bufs.p[i] = bufp[i];
  const size_t lds = items_lds_bytes(nmax, prec == DEMAG_FP64);
  if (prec == DEMAG_FP64) {
    if (lds > 65536)
      DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_left_items<double>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    k_left_items<double><<<grid, 256, lds, ctx->stream>>>(items, nitems, jobs, terms, geoms, bufs,
                                                           static_cast<const double *>(gens), beta, counter);
  } else {
    if (lds > 65536)
      DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_left_items<float>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    k_left_items<float><<<grid, 256, lds, ctx->stream>>>(items, nitems, jobs, terms, geoms, bufs,
                                                          static_cast<const float *>(gens), beta, counter);
  }
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

demag_status launch_thin_items(demag_ctx *ctx, demag_prec prec, const BatchItem *items, int nitems, const MPJob *jobs,
                               const MPTerm *terms, const MPGeom *geoms, void *const bufp[6], const void *gens,
                               int beta) {
  if (nitems == 0) return DEMAG_OK;
  Bufs bufs;
  for (int i = 0; i < 6; ++i) bufs.p[i] = bufp[i];
  if (prec == DEMAG_FP64)
    k_thin_items<double><<<nitems, 256, 0, ctx->stream>>>(items, jobs, terms, geoms, bufs,
                                                          static_cast<const double *>(gens), beta);
  else
    k_thin_items<float><<<nitems, 256, 0, ctx->stream>>>(items, jobs, terms, geoms, bufs,
                                                         static_cast<const float *>(gens), beta);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

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
  const int rb = ctx->tile_rows > 0 ? ctx->tile_rows : stage_rows(sp, prec);
  if (f->dense && (prec == DEMAG_BF16X2 || prec == DEMAG_BF16X3)) {
    st = launch_dense_stage_bf16(ctx->stream, sp, prec, f->bf[sp.axis], axis_table_len(f, sp.axis), bufp, beta);
    pname = (prec == DEMAG_BF16X3) ? "dense_bf16x3" : "dense_bf16x2";
  } else if (f->dense && prec == DEMAG_FP32) {
    st = launch_dense_stage<float>(ctx->stream, sp, f->f32[sp.axis], bufs, beta);
    pname = "dense32";
  } else if (f->dense) {
    st = launch_dense_stage<double>(ctx->stream, sp, f->f64[sp.axis], bufs, beta);
    pname = "dense64";
    esize = 8;
  } else if (prec == DEMAG_FP64) {
    st = launch_typed<double>(ctx->stream, rb, sp, f->f64[sp.axis], bufs, beta);
    pname = "fp64";
    esize = 8;
  } else if (prec == DEMAG_FP32) {
    st = launch_typed<float>(ctx->stream, rb, sp, f->f32[sp.axis], bufs, beta);
    pname = "fp32";
  } else {
    st = launch_left_stage_bf16(ctx, f, prec, sp, bufp, beta);
    pname = (prec == DEMAG_BF16X3) ? "bf16x3" : "bf16x2";
  }
  if (st != DEMAG_OK) return st;
  if (ev) {
    // Algorithmic work of the launch: each term of each job is a dense
    // n x n Toeplitz times n x C product per output; compulsory traffic
    // reads each term's input once and writes (and, when accumulating,
    // reads) each output once.  Split precisions count every bfloat16
    // product they issue.
    const MPGeom &g = sp.geom;
    const double slab = double(g.n) * g.C;
    const double mult = (prec == DEMAG_BF16X3) ? 6.0 : (prec == DEMAG_BF16X2) ? 3.0 : 1.0;
    double flops = 0, bytes = 0;
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
