// Left Toeplitz mode products with bfloat16-split operands on the matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Same contraction as the FP32/FP64 kernel (Eq. (modemul) with Toeplitz
// factors, Sec. 4.2), but every FP32 operand x is written as
// x ~ hi + lo (+ lo2) with hi = bf16(x), lo = bf16(x - hi), lo2 = bf16(x - hi - lo)
// (round to nearest even) and each product is formed from the split parts:
//   two parts:   hi*hi + hi*lo + lo*hi                           (3 MFMAs)
//   three parts: the above + hi*lo2 + lo2*hi + lo*lo              (6 MFMAs)
// Input tensors (the magnetization and the FP32 intermediates) are split in
// registers as they are loaded; the factors are split once at assembly.
//
// Operand layouts of the 16x16x32 instruction: lane l holds A[l % 16][8 (l/16) + e]
// and B[8 (l/16) + e][l % 16], e = 0..7.  For the Toeplitz A = T[i][j] =
// g[i - j + n - 1] the eight values of a lane are consecutive generator
// entries in decreasing order, so the factors are stored as "windows": entry s
// of a window table holds R[s..s+7] of the reversed generator R[u] = g[2n-2-u]
// (zero outside), and a fragment is one aligned 16-byte LDS read.
#include <type_traits>

#include "internal.h"

namespace demag {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

__device__ inline void split_value(float x, __bf16 &h, __bf16 &l, __bf16 &l2) {
  h = __bf16(x);
  const float r = x - float(h);
  l = __bf16(r);
  const float r2 = r - float(l);
  l2 = __bf16(r2);
}

union Frag {
  uint4 u;
  bf8 v;
  bf2 p[4];
};

// Two values at a time: one packed conversion per part (round to nearest
// even), the bf16 -> FP32 widening is a shift or a mask.
__device__ inline void split_pair(float x0, float x1, bf2 &h, bf2 &l, bf2 &l2) {
  const f2 x = {x0, x1};
  h = __builtin_convertvector(x, bf2);
  const f2 r = x - __builtin_convertvector(h, f2);
  l = __builtin_convertvector(r, bf2);
  const f2 r2 = r - __builtin_convertvector(l, f2);
  l2 = __builtin_convertvector(r2, bf2);
}

// Toeplitz fragment a times input fragment b; TRANS gives the transposed
// 16x16 block (the instruction's A and B layouts mirror each other, so the
// same registers serve), whose lanes run along the output rows.
template <bool TRANS>
__device__ __forceinline__ f4 mma(bf8 a, bf8 b, f4 c) {
  return TRANS ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a, c, 0, 0, 0)
               : __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int kStageRounds = 3;  // window entries a thread loads per staging round

// LDS slots per window entry: the NOUT x PARTS windows of one entry side by
// side, padded to an odd count so that 8 lanes reading consecutive entries
// hit 8 different 16-byte bank groups.
template <int NOUT, int PARTS>
constexpr int window_slots() {
  return (NOUT * PARTS) | 1;
}

template <int NOUT, int PARTS>
size_t window_lds_bytes(int n, int rb) {
  return size_t(window_slots<NOUT, PARTS>()) * (n + 16 * rb + 23) * sizeof(uint4);
}

// Tile: 4 waves x 16*CB columns, 16*RB rows.  The (term, K-step) pairs of a
// job form one loop whose next step's input loads are issued right after the
// current step's inputs are split, so they are in flight while it is
// multiplied.  WHOLE (n a multiple of 32): every K-step lies inside the n
// rows and loads from a uniform row pointer plus a per-lane 32-bit byte
// offset; otherwise rows are clamped to n - 1 and the values past n of the
// last step are zeroed.  A term's windows are staged in
// rounds of up to 3 x 256 entries whose loads are all issued before the
// first LDS store; fragments are read at compile-time offsets from one
// per-lane address per K-step.
template <int RB, int CB, int NOUT, int PARTS, bool TRANS, bool WHOLE>
__global__ __launch_bounds__(256, 2) void k_left_bf16(const MPJob *__restrict__ jobs,
                                                   const MPTerm *__restrict__ terms, Bufs bufs,
                                                   const uint4 *__restrict__ wtab, MPGeom g, int nw,
                                                   int col_tiles, int beta) {
  constexpr int SL = window_slots<NOUT, PARTS>();
  extern __shared__ uint4 wl[];
  const int n = g.n;
  const int cnt = n + 16 * RB + 23;
  const int tot = NOUT * cnt;
  const MPJob job = jobs[blockIdx.y];
  const int nterms = job.nterms;
  if (nterms <= 0) return;
  const int ct = blockIdx.x % col_tiles;
  const int rg = blockIdx.x / col_tiles;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  // K rows of lane group kq within a step: 8 kp .. 8 kp + 7 with kp = 0, 2,
  // 1, 3 for kq = 0..3 (the same K order for A and B).  With the plain
  // order the window reads of lane groups 0 and 2 (and 1 and 3) fall into
  // the same LDS banks; this order makes them conflict-free.
  const int kp = ((kq & 1) << 1) | (kq >> 1);
  const int row0 = rg * 16 * RB;
  const int s0min = n - row0 - 16 * RB;
  // local window entry of this lane for rb = RB - 1, j0 = 0; row block rb
  // at K-step j0 reads entry lbase + 16 (RB - 1 - rb) + j0, which lies in
  // [0, cnt) for every rb < RB and j0 < n
  const int lbase = 15 - (lane & 15) + 8 * kp;
  int64_t inoff[CB], outoff[CB];
  uint32_t inb[CB];
  bool cval[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int c = ct * (64 * CB) + wave * (16 * CB) + 16 * cb + (lane & 15);
    cval[cb] = c < g.C;
    const int cl = cval[cb] ? c : g.C - 1;  // past the end: read column C - 1, never stored
    const int co = cl / g.C1, ci = cl % g.C1;
    inoff[cb] = int64_t(co) * g.in_S1 + ci;
    outoff[cb] = int64_t(co) * g.out_S1 + int64_t(ci) * g.out_cs;
    // byte offset of (row 8 kp, this column); used only in whole K-steps,
    // where the row is < n and the offset lies inside the input (< 4 GiB for
    // n <= 1024 per axis)
    inb[cb] = uint32_t((int64_t(8 * kp) * g.kstride + inoff[cb]) * 4);
  }
  auto term_in = [&](int t) -> const float * {
    const MPTerm &tm = terms[job.term0 + t];
    return static_cast<const float *>(bufs.p[tm.in_buf]) + tm.in_off;
  };
  float raw[CB][8];
  auto load_step = [&](const float *in, int j) {
    if (WHOLE) {
      // rows j .. j + 31, all < n: uniform row pointers
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const char *rowp = reinterpret_cast<const char *>(in + (int64_t(j) + e) * g.kstride);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) raw[cb][e] = *reinterpret_cast<const float *>(rowp + inb[cb]);
      }
    } else {
      // rows clamped to n - 1 (the values past n are zeroed when split)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int e = 0; e < 8; ++e) raw[cb][e] = in[size_t(min(j + 8 * kp + e, n - 1)) * g.kstride + inoff[cb]];
    }
  };

  f4 acc[NOUT][RB][CB];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[o][rb][cb] = f4{0, 0, 0, 0};

  const int nks = (n + 31) / 32;
  const int nq = nterms * nks;
  load_step(term_in(0), 0);
  int t = 0, j0 = 0;
  for (int q = 0; q < nq; ++q) {
    if (j0 == 0) {
      const MPTerm &tm = terms[job.term0 + t];
      const int gen0 = tm.gen[0], gen1 = tm.gen[NOUT > 1 ? 1 : 0];
      __syncthreads();  // every wave is done with the previous term's windows
      for (int e0 = 0; e0 < tot; e0 += 256 * kStageRounds) {
        uint4 v[kStageRounds][PARTS];
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r) {
          const int e = min(e0 + 256 * r + int(threadIdx.x), tot - 1);
          const bool second = NOUT > 1 && e >= cnt;
          const uint4 *src = wtab + (size_t(second ? gen1 : gen0) * nw + (s0min + 128) + (e - (second ? cnt : 0))) * 3;
#pragma unroll
          for (int p = 0; p < PARTS; ++p) v[r][p] = src[p];
        }
        // threads past the end rewrite entry tot - 1 with the value they
        // loaded from it (no branch, so every load is issued before a store)
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r) {
          const int e = min(e0 + 256 * r + int(threadIdx.x), tot - 1);
          const bool second = NOUT > 1 && e >= cnt;
          const int o = second ? 1 : 0, el = e - (second ? cnt : 0);
#pragma unroll
          for (int p = 0; p < PARTS; ++p) wl[el * SL + o * PARTS + p] = v[r][p];
        }
      }
      __syncthreads();
    }
    Frag bh[CB], bl[CB], bl2[CB];
    if (!WHOLE && j0 + 32 > n) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (j0 + 8 * kp + e >= n) raw[cb][e] = 0.0f;
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        split_pair(raw[cb][2 * e], raw[cb][2 * e + 1], bh[cb].p[e], bl[cb].p[e], bl2[cb].p[e]);
    {
      // next K-step: of this term, else the first of the next term; the
      // last step of the job re-reads its own rows
      int t1 = t, j1 = j0 + 32;
      if (j1 >= n) {
        j1 = (t + 1 < nterms) ? 0 : j0;
        t1 = min(t + 1, nterms - 1);
      }
      load_step(term_in(t1), j1);
    }
    // keep the loads ahead of the products
    __builtin_amdgcn_sched_barrier(0);
    const uint4 *wp = wl + (lbase + j0) * SL;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
      for (int o = 0; o < NOUT; ++o) {
        const uint4 *w = wp + 16 * (RB - 1 - rb) * SL + o * PARTS;
        Frag ah, al, al2;
        ah.u = w[0];
        al.u = w[1];
        if (PARTS == 3) al2.u = w[2];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          f4 a = acc[o][rb][cb];
          a = mma<TRANS>(ah.v, bh[cb].v, a);
          a = mma<TRANS>(ah.v, bl[cb].v, a);
          a = mma<TRANS>(al.v, bh[cb].v, a);
          if (PARTS == 3) {
            a = mma<TRANS>(ah.v, bl2[cb].v, a);
            a = mma<TRANS>(al2.v, bh[cb].v, a);
            a = mma<TRANS>(al.v, bl[cb].v, a);
          }
          acc[o][rb][cb] = a;
        }
      }
    }
    j0 += 32;
    if (j0 >= n) {
      j0 = 0;
      ++t;
    }
  }

  // beta (accumulate into the output) and whole row groups are uniform:
  // one branch picks the epilogue.  With beta the old values of a row block
  // (or column) are all loaded before its stores.
  auto epilogue = [&](auto beta_c, auto whole_c) {
    constexpr bool BETA = decltype(beta_c)::value;
    constexpr bool WROWS = decltype(whole_c)::value;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      float *out = static_cast<float *>(bufs.p[job.out_buf[o]]) + job.out_off[o];
      const float scale = float(job.scale[o]);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        if (TRANS) {
          // register r of lane l: column cbase + 4 (l/16) + r, output row
          // 16 rb + l % 16; rows are contiguous in the output (out_is = 1)
          const int cbase = ct * (64 * CB) + wave * (16 * CB) + 16 * cb;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int cc = cbase + 4 * kq + r;
            if (cc >= g.C) continue;
            float *col = out + int64_t(cc / g.C1) * g.out_S1 + int64_t(cc % g.C1) * g.out_cs + row0 + (lane & 15);
            float old[RB];
            if (BETA) {
#pragma unroll
              for (int rb = 0; rb < RB; ++rb)
                old[rb] = (WROWS || row0 + 16 * rb + (lane & 15) < n) ? col[16 * rb] : 0.0f;
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              if (WROWS || row0 + 16 * rb + (lane & 15) < n) {
                float v = scale * acc[o][rb][cb][r];
                if (BETA) v += old[rb];
                col[16 * rb] = v;
              }
            }
          }
          continue;
        }
        if (!cval[cb]) continue;
        // 16x16 output block: register r of lane l is row 4 (l/16) + r
        const uint32_t ob = uint32_t((outoff[cb] + int64_t(4 * kq) * g.out_is) * 4);
        auto dst = [&](int rb, int r) -> float * {
          if (WROWS) {
            char *rowp = reinterpret_cast<char *>(out + (int64_t(row0) + 16 * rb + r) * g.out_is);
            return reinterpret_cast<float *>(rowp + ob);
          }
          return out + outoff[cb] + size_t(row0 + 16 * rb + 4 * kq + r) * g.out_is;
        };
        auto ok = [&](int rb, int r) { return WROWS || row0 + 16 * rb + 4 * kq + r < n; };
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          float old[4];
          if (BETA) {
#pragma unroll
            for (int r = 0; r < 4; ++r) old[r] = ok(rb, r) ? *dst(rb, r) : 0.0f;
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (ok(rb, r)) {
              float v = scale * acc[o][rb][cb][r];
              if (BETA) v += old[r];
              *dst(rb, r) = v;
            }
          }
        }
      }
    }
  };
  if (row0 + 16 * RB <= n) {
    if (beta)
      epilogue(std::true_type{}, std::true_type{});
    else
      epilogue(std::false_type{}, std::true_type{});
  } else {
    if (beta)
      epilogue(std::true_type{}, std::false_type{});
    else
      epilogue(std::false_type{}, std::false_type{});
  }
}

template <int RB, int CB, int NOUT, int PARTS>
demag_status launch_bf(hipStream_t s, const StagePlan &sp, const uint4 *wtab, int nw, const Bufs &bufs,
                       int beta) {
  const MPGeom &g = sp.geom;
  const int col_tiles = (g.C + 64 * CB - 1) / (64 * CB);
  const int row_groups = (g.n + 16 * RB - 1) / (16 * RB);
  dim3 grid(col_tiles * row_groups, unsigned(sp.jobs.size()));
  const size_t lds = window_lds_bytes<NOUT, PARTS>(g.n, RB);
  // rows contiguous in the output (x and y stages): transposed blocks
  const bool trans = g.out_is == 1, whole = g.n % 32 == 0;
  auto k = trans ? (whole ? &k_left_bf16<RB, CB, NOUT, PARTS, true, true> : &k_left_bf16<RB, CB, NOUT, PARTS, true, false>)
                 : (whole ? &k_left_bf16<RB, CB, NOUT, PARTS, false, true> : &k_left_bf16<RB, CB, NOUT, PARTS, false, false>);
  if (lds > 65536)
    DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      int(lds)));
  k<<<grid, 256, lds, s>>>(sp.d_jobs, sp.d_terms, bufs, wtab, g, nw, col_tiles, beta);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

template <int CB, int NOUT, int PARTS>
demag_status launch_bf_rb(hipStream_t s, int rb, const StagePlan &sp, const uint4 *wtab, int nw, const Bufs &bufs,
                          int beta) {
  switch (rb) {
    case 1: return launch_bf<1, CB, NOUT, PARTS>(s, sp, wtab, nw, bufs, beta);
    case 2: return launch_bf<2, CB, NOUT, PARTS>(s, sp, wtab, nw, bufs, beta);
    case 4: return launch_bf<4, CB, NOUT, PARTS>(s, sp, wtab, nw, bufs, beta);
    default: return launch_bf<8, CB, NOUT, PARTS>(s, sp, wtab, nw, bufs, beta);
  }
}

template <int NOUT, int PARTS>
demag_status launch_bf_n(hipStream_t s, int rb, int cb, const StagePlan &sp, const uint4 *wtab, int nw,
                         const Bufs &bufs, int beta) {
  if (cb == 2) return launch_bf_rb<2, NOUT, PARTS>(s, rb, sp, wtab, nw, bufs, beta);
  return launch_bf_rb<1, NOUT, PARTS>(s, rb, sp, wtab, nw, bufs, beta);
}

// Dense (non-Toeplitz) factors, non-uniform grids: out[i][c] = sum_terms
// sum_j A[i][j] in[j][c] with the n x n matrices A split at assembly into
// PARTS bfloat16 parts ([part][type * M + k][n][n]) and the inputs split in
// registers, the products formed from the parts as above.  Tile: 64 rows
// (4 blocks of 16) x 64 CB columns (4 waves of CB blocks of 16), K chunks of
// 32 (one 16x16x32 step): per chunk the A tiles of the NOUT outputs (64 x 32
// per part, a 16-byte row segment per thread) go through LDS, and each lane
// loads its input fragments (eight values down each of its CB columns)
// straight from memory into registers, as the Toeplitz kernel does, and
// splits them before the chunk's barrier; the next chunk's A segments and
// inputs are loaded while the current one is multiplied.  A lane's fragment
// of a row block is one 16-byte LDS read per part (rows padded to 40
// values).  Staging the inputs through LDS as well measured 1.5 % slower
// (more LDS and vector instructions around the same products).
template <int NOUT, int PARTS, bool TRANS, int CB>
__global__ __launch_bounds__(256, 2) void k_dense_bf16(const MPJob *__restrict__ jobs,
                                                       const MPTerm *__restrict__ terms, Bufs bufs,
                                                       const uint16_t *__restrict__ parts, size_t part_stride,
                                                       MPGeom g, int col_tiles, int beta) {
  constexpr int KC = 32, AS = 40, NC = 64 * CB;
  __shared__ uint4 As[NOUT][PARTS][64][AS / 8];
  const MPJob job = jobs[blockIdx.y];
  if (job.nterms <= 0) return;
  const int ct = blockIdx.x % col_tiles, rg = blockIdx.x / col_tiles;
  const int n = g.n;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4;
  const int row0 = rg * 64;
  // A staging: thread -> (row t / 4, 8 K values at (t % 4) * 8)
  const int ar = tid >> 2, ak = (tid & 3) * 8;
  // input fragments straight from memory: K rows 8 kq .. 8 kq + 7 of this
  // lane's columns (past C: column C - 1, never stored)
  size_t cin[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int cs = ct * NC + wave * 16 * CB + 16 * cb + (lane & 15);
    const int cl = cs < g.C ? cs : g.C - 1;
    cin[cb] = size_t(cl / g.C1) * g.in_S1 + size_t(cl % g.C1);
  }
  f4 acc[NOUT][4][CB];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[o][rb][cb] = f4{0, 0, 0, 0};
  const int nch = (n + KC - 1) / KC;
  const int nq = job.nterms * nch;
  uint4 av[NOUT][PARTS];
  float raw[CB][8];
  auto load = [&](int q) {
    const int t = q / nch, j0 = (q - t * nch) * KC;
    const MPTerm &tm = terms[job.term0 + t];
    const float *in = static_cast<const float *>(bufs.p[tm.in_buf]) + tm.in_off;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = j0 + 8 * kq + e;
        raw[cb][e] = j < n ? in[cin[cb] + size_t(j) * g.kstride] : 0.0f;
      }
    const int i = row0 + ar, j = j0 + ak;
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
      for (int p = 0; p < PARTS; ++p) {
        const uint16_t *A = parts + size_t(p) * part_stride + tm.gen_off[o] + size_t(i) * n + j;
        if (i < n && j + 8 <= n && (n & 7) == 0) {
          av[o][p] = *reinterpret_cast<const uint4 *>(A);
        } else {
          uint16_t e8[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) e8[e] = (i < n && j + e < n) ? A[e] : uint16_t(0);
          av[o][p] = make_uint4(uint32_t(e8[0]) | (uint32_t(e8[1]) << 16), uint32_t(e8[2]) | (uint32_t(e8[3]) << 16),
                                uint32_t(e8[4]) | (uint32_t(e8[5]) << 16), uint32_t(e8[6]) | (uint32_t(e8[7]) << 16));
        }
      }
  };
  load(0);
  for (int q = 0; q < nq; ++q) {
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
      for (int p = 0; p < PARTS; ++p) As[o][p][ar][ak / 8] = av[o][p];
    Frag bh[CB], bl[CB], bl2[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        split_pair(raw[cb][2 * e], raw[cb][2 * e + 1], bh[cb].p[e], bl[cb].p[e], bl2[cb].p[e]);
    __syncthreads();
    if (q + 1 < nq) load(q + 1);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int o = 0; o < NOUT; ++o) {
        Frag ah, al, al2;
        ah.u = As[o][0][16 * rb + (lane & 15)][kq];
        if (PARTS > 1) al.u = As[o][1][16 * rb + (lane & 15)][kq];
        if (PARTS > 2) al2.u = As[o][2][16 * rb + (lane & 15)][kq];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          f4 a = acc[o][rb][cb];
          a = mma<TRANS>(ah.v, bh[cb].v, a);
          a = mma<TRANS>(ah.v, bl[cb].v, a);
          a = mma<TRANS>(al.v, bh[cb].v, a);
          if (PARTS == 3) {
            a = mma<TRANS>(ah.v, bl2[cb].v, a);
            a = mma<TRANS>(al2.v, bh[cb].v, a);
            a = mma<TRANS>(al.v, bl[cb].v, a);
          }
          acc[o][rb][cb] = a;
        }
      }
    __syncthreads();
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    float *out = static_cast<float *>(bufs.p[job.out_buf[o]]) + job.out_off[o];
    const float scale = float(job.scale[o]);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // register r of lane l: block element (4 (l >> 4) + r, l % 16); with
          // swapped operands row and column trade places
          const int bi = TRANS ? (lane & 15) : 4 * kq + r;
          const int bj = TRANS ? 4 * kq + r : (lane & 15);
          const int i = row0 + 16 * rb + bi;
          const int c = ct * NC + wave * 16 * CB + 16 * cb + bj;
          if (i < n && c < g.C) {
            float *dst = out + size_t(c / g.C1) * g.out_S1 + size_t(c % g.C1) * g.out_cs + size_t(i) * g.out_is;
            float v = scale * acc[o][rb][cb][r];
            if (beta) v += *dst;
            *dst = v;
          }
        }
  }
}

__global__ void k_build_windows(const uint16_t *__restrict__ bf, uint4 *__restrict__ wtab, int n, int ngen,
                                int nw, size_t part_stride) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;  // window entry
  const int gidx = blockIdx.y;                          // generator (type * M + k)
  if (s >= nw || gidx >= ngen) return;
  const int L = 2 * n - 1;
  for (int p = 0; p < 3; ++p) {
    const uint16_t *gsrc = bf + p * part_stride + size_t(gidx) * L;
    uint16_t v[8];
    for (int e = 0; e < 8; ++e) {
      const int u = s - 128 + e;        // index into the reversed generator
      v[e] = (u >= 0 && u <= L - 1) ? gsrc[L - 1 - u] : uint16_t(0);
    }
    uint4 w;
    w.x = uint32_t(v[0]) | (uint32_t(v[1]) << 16);
    w.y = uint32_t(v[2]) | (uint32_t(v[3]) << 16);
    w.z = uint32_t(v[4]) | (uint32_t(v[5]) << 16);
    w.w = uint32_t(v[6]) | (uint32_t(v[7]) << 16);
    wtab[(size_t(gidx) * nw + s) * 3 + p] = w;
  }
}

__global__ void k_split(const float *__restrict__ x, uint16_t *__restrict__ parts, size_t count, int nparts) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  __bf16 h, l, l2;
  split_value(x[i], h, l, l2);
  parts[i] = __builtin_bit_cast(uint16_t, h);
  if (nparts > 1) parts[count + i] = __builtin_bit_cast(uint16_t, l);
  if (nparts > 2) parts[2 * count + i] = __builtin_bit_cast(uint16_t, l2);
}

}  // namespace

int window_entries(int n) { return 2 * n + 151; }

demag_status launch_build_windows(demag_ctx *ctx, demag_factors *f) {
  for (int d = 0; d < 3; ++d) {
    if (!f->bfw[d]) continue;
    const int n = f->n[d];
    const int nw = window_entries(n);
    dim3 grid((nw + 127) / 128, F_NTYPES * f->M);
    k_build_windows<<<grid, 128, 0, ctx->stream>>>(f->bf[d], reinterpret_cast<uint4 *>(f->bfw[d]), n,
                                                   F_NTYPES * f->M, nw, axis_table_len(f, d));
    DEMAG_TRY_HIP(hipGetLastError());
  }
  return DEMAG_OK;
}

demag_status launch_left_stage_bf16(demag_ctx *ctx, const demag_factors *f, demag_prec prec, const StagePlan &sp,
                                    void *const bufp[6], int beta) {
  Bufs bufs;
  for (int i = 0; i < 6; ++i) bufs.p[i] = bufp[i];
  const uint4 *wtab = reinterpret_cast<const uint4 *>(f->bfw[sp.axis]);
  const int nw = window_entries(f->n[sp.axis]);
  if (!wtab) {
    set_error("bfloat16 window table missing (axis longer than the full-format limit)");
    return DEMAG_E_UNSUPPORTED;
  }
  const int rb = ctx->tile_rows > 0 ? ctx->tile_rows : stage_rows(sp, prec);
  // two column blocks per wave halve the LDS reads per product but need
  // more registers; one block measured faster on every stage of a 128^3 apply
  const int cb = ctx->tile_cols > 0 ? ctx->tile_cols : 1;
  if (prec == DEMAG_BF16X3)
    return sp.nout == 1 ? launch_bf_n<1, 3>(ctx->stream, rb, cb, sp, wtab, nw, bufs, beta)
                        : launch_bf_n<2, 3>(ctx->stream, rb, cb, sp, wtab, nw, bufs, beta);
  return sp.nout == 1 ? launch_bf_n<1, 2>(ctx->stream, rb, cb, sp, wtab, nw, bufs, beta)
                      : launch_bf_n<2, 2>(ctx->stream, rb, cb, sp, wtab, nw, bufs, beta);
}

demag_status launch_dense_stage_bf16(hipStream_t s, const StagePlan &sp, demag_prec prec, const uint16_t *parts,
                                     size_t part_stride, void *const bufp[6], int beta) {
  Bufs bufs;
  for (int i = 0; i < 6; ++i) bufs.p[i] = bufp[i];
  const MPGeom &g = sp.geom;
  constexpr int kCB = 2;   // 16-column blocks per wave (each A fragment read feeds kCB product sets)
  const int col_tiles = (g.C + 64 * kCB - 1) / (64 * kCB);
  const int row_groups = (g.n + 63) / 64;
  dim3 grid(unsigned(col_tiles * row_groups), unsigned(sp.jobs.size()));
  const bool tr = g.out_is == 1;   // rows contiguous in the output (x and y stages)
  const bool p3 = prec == DEMAG_BF16X3;
#define DEMAG_DENSE_BF(NO, PA, TR) \
  k_dense_bf16<NO, PA, TR, kCB><<<grid, 256, 0, s>>>(sp.d_jobs, sp.d_terms, bufs, parts, part_stride, g, col_tiles, \
                                                     beta)
  if (sp.nout == 2) {
    if (p3) { if (tr) DEMAG_DENSE_BF(2, 3, true); else DEMAG_DENSE_BF(2, 3, false); }
    else { if (tr) DEMAG_DENSE_BF(2, 2, true); else DEMAG_DENSE_BF(2, 2, false); }
  } else {
    if (p3) { if (tr) DEMAG_DENSE_BF(1, 3, true); else DEMAG_DENSE_BF(1, 3, false); }
    else { if (tr) DEMAG_DENSE_BF(1, 2, true); else DEMAG_DENSE_BF(1, 2, false); }
  }
#undef DEMAG_DENSE_BF
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

namespace {

// Four consecutive elements per thread of the 4 N outputs (phi, h_x, h_y,
// h_z), each the sum of nsplit partials.
template <class T>
__global__ void k_reduce_partials(const T *__restrict__ partials, int nsplit, int64_t N, T *__restrict__ phi,
                                  T *__restrict__ h, double phi_scale, int accumulate) {
  const int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * 4;
  const int o = int(blockIdx.y);                       // 0: phi, 1..3: h_x, h_y, h_z
  if (i >= N) return;
  T *out = (o == 0) ? phi : h + int64_t(o - 1) * N;
  const double scale = (o == 0) ? phi_scale : 1.0;
  const int cnt = int(N - i < 4 ? N - i : 4);
  // the partial sums are added in FP64 and rounded once
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < nsplit; ++s) {
    const T *src = partials + (int64_t(4) * s + o) * N + i;
    if (std::is_same_v<T, float> && cnt == 4 && ((reinterpret_cast<uintptr_t>(src) & 15u) == 0)) {
      const float4 v = *reinterpret_cast<const float4 *>(src);
      acc[0] += double(v.x);
      acc[1] += double(v.y);
      acc[2] += double(v.z);
      acc[3] += double(v.w);
    } else {
      for (int e = 0; e < cnt; ++e) acc[e] += double(src[e]);
    }
  }
  for (int e = 0; e < cnt; ++e) {
    const double v = scale * acc[e];
    out[i + e] = T(accumulate ? double(out[i + e]) + v : v);
  }
}

}  // namespace

demag_status launch_reduce_partials(demag_ctx *ctx, demag_prec prec, const void *partials, int nsplit, int64_t N,
                                    void *phi, void *h, double phi_scale, bool accumulate) {
  if (N == 0) return DEMAG_OK;
  hipEvent_t ev = nullptr;
  demag_status st = prof_begin(ctx, &ev);
  if (st != DEMAG_OK) return st;
  const int64_t threads = (N + 3) / 4;
  dim3 grid(unsigned((threads + 255) / 256), 4);
  const bool f64 = prec == DEMAG_FP64;
  if (f64)
    k_reduce_partials<double><<<grid, 256, 0, ctx->stream>>>(static_cast<const double *>(partials), nsplit, N,
                                                             static_cast<double *>(phi), static_cast<double *>(h),
                                                             phi_scale, accumulate ? 1 : 0);
  else
    k_reduce_partials<float><<<grid, 256, 0, ctx->stream>>>(static_cast<const float *>(partials), nsplit, N,
                                                            static_cast<float *>(phi), static_cast<float *>(h),
                                                            phi_scale, accumulate ? 1 : 0);
  DEMAG_TRY_HIP(hipGetLastError());
  if (ev) {
    const double es = f64 ? 8.0 : 4.0;
    const double bytes = es * N * 4.0 * (nsplit + (accumulate ? 2 : 1));
    const char *name = f64 ? "fp64" : prec == DEMAG_BF16X3 ? "bf16x3" : prec == DEMAG_BF16X2 ? "bf16x2" : "fp32";
    st = prof_end(ctx, ev, std::string(name) + "/x/reduce", 0.0, bytes);
  }
  return st;
}

demag_status launch_split(demag_ctx *ctx, const float *x, uint16_t *parts, size_t count, int nparts) {
  if (count == 0) return DEMAG_OK;
  k_split<<<unsigned((count + 255) / 256), 256, 0, ctx->stream>>>(x, parts, count, nparts);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

}  // namespace demag
