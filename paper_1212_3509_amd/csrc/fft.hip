// Structured apply, path (b): Toeplitz products of factor columns through
// zero-padded FFTs (Sec. 4.1 convolution theorem, Lemmas DFT_cp/DFT_tucker,
// Sec. 4.2 Toeplitz form and Eq. (fft_pot)).
//
// For axis d with n cells, every factor generator g (offsets J = -(n-1)..n-1)
// is embedded in a circulant of length L = 2^p >= 2n - 1:
//   c[J mod L] = g_J,  zeros elsewhere,
// so that for an input column u (length n, zero padded to L) the first n
// entries of the circular convolution c * u are the Toeplitz product T(g) u.
// E and P generators are even in J, so their spectra are real; X and Q are
// odd, so their spectra are imaginary.  The spectra are formed once per
// factor set in FP64 (direct cosine/sine sums).
//
// Transforms run in FP64: the roundoff of an FFT convolution is of order
// eps log2(L) |G|_inf |u|, which for the wide (low-pass) E factors on rough
// columns is far above eps |T u| in FP32, and on this chip FP64 vector
// arithmetic runs at the rate of unpacked FP32.  Columns are read and written
// as FP32.
//
// A real transform of length L is computed through a complex transform of
// length N = L/2 on z[m] = x[2m] + i x[2m+1], with the usual even/odd
// unpacking by W_L^f.  The complex transform runs in LDS as Stockham passes
// of radix 16/8/4/2 (N/R butterflies per pass, 256 threads).  Twiddles come
// from two 64-entry tables in LDS, W_N^e = W_N^(e mod 64) W_N^(64 (e div 64)),
// so no pass waits on global memory.
//
// Two launches per axis: k_fft_fwd transforms every input column once and
// stores its unpacked spectrum U[0..N] in the workspace; k_fft_jobs gives
// each workgroup a few jobs of one column: it loads the column's frequency
// pairs (f, N - f) into registers (from L2: every job group of a column reads
// the same 64 KB), and per job multiplies by a kernel spectrum, transforms
// back and writes the n outputs.
#include "internal.h"

#include <cmath>

namespace demag {

namespace {

constexpr int kThreads = 256;

struct alignas(16) c32 {   // 16-byte aligned: one ds_read_b128 / ds_write_b128 per point
  double x, y;
};
__device__ inline c32 cadd(c32 a, c32 b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline c32 csub(c32 a, c32 b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline c32 cmul(c32 a, c32 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline c32 cconj(c32 a) { return {a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV> __device__ inline c32 mul_mi(c32 a) { return INV ? c32{-a.y, a.x} : c32{a.y, -a.x}; }

// In-register DFTs of size 2, 4, 8, 16 (forward: exp(-2 pi i jk/R); inverse: +).
template <bool INV> __device__ inline void dft2(c32 &a, c32 &b) {
  c32 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}
template <bool INV> __device__ inline void dft4(c32 &a0, c32 &a1, c32 &a2, c32 &a3) {
  c32 s0 = cadd(a0, a2), d0 = csub(a0, a2);
  c32 s1 = cadd(a1, a3), d1 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(s0, s1);
  a2 = csub(s0, s1);
  a1 = cadd(d0, d1);
  a3 = csub(d0, d1);
}
// Generic small DFT by the 2-factor Cooley-Tukey split R = R1 * R2 on arrays.
template <bool INV, int R> __device__ inline void dftR(c32 *v);
template <> __device__ inline void dftR<false, 2>(c32 *v) { dft2<false>(v[0], v[1]); }
template <> __device__ inline void dftR<true, 2>(c32 *v) { dft2<true>(v[0], v[1]); }
template <> __device__ inline void dftR<false, 4>(c32 *v) { dft4<false>(v[0], v[1], v[2], v[3]); }
template <> __device__ inline void dftR<true, 4>(c32 *v) { dft4<true>(v[0], v[1], v[2], v[3]); }

// cos and sin of 2 pi e / 16 for e = 0..15; constants of the small DFTs.
#define C1_16 0.92387953251128675613
#define C2_16 0.70710678118654752440
#define C3_16 0.38268343236508977173
__device__ constexpr double kC16[16] = {1.0, C1_16, C2_16, C3_16, 0.0, -C3_16, -C2_16, -C1_16,
                                         -1.0, -C1_16, -C2_16, -C3_16, 0.0, C3_16, C2_16, C1_16};
__device__ constexpr double kS16[16] = {0.0, C3_16, C2_16, C1_16, 1.0, C1_16, C2_16, C3_16,
                                         0.0, -C3_16, -C2_16, -C1_16, -1.0, -C1_16, -C2_16, -C3_16};
// exp(-+2 pi i num / den), den dividing 16
__device__ inline c32 twiddle_const(int num, int den, bool inv) {
  const int e = (num * (16 / den)) & 15;
  return inv ? c32{kC16[e], kS16[e]} : c32{kC16[e], -kS16[e]};
}

// R = 8 as 4 x 2 and R = 16 as 4 x 4: x[k1 + R1 k2] = sum_b W_R^{b k1} W_R2^{b k2} sum_a x[R2 a + b] W_R1^{a k1}
template <bool INV, int R1, int R2> __device__ inline void dft_split(c32 *v) {
  c32 t[R1 * R2];
#pragma unroll
  for (int b = 0; b < R2; ++b) {
    c32 col[R1];
#pragma unroll
    for (int a = 0; a < R1; ++a) col[a] = v[R2 * a + b];
    dftR<INV, R1>(col);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) t[b * R1 + k1] = (b * k1 == 0) ? col[k1] : cmul(col[k1], twiddle_const(b * k1, R1 * R2, INV));
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    c32 row[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) row[b] = t[b * R1 + k1];
    dftR<INV, R2>(row);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = row[k2];
  }
}
template <> __device__ inline void dftR<false, 8>(c32 *v) { dft_split<false, 4, 2>(v); }
template <> __device__ inline void dftR<true, 8>(c32 *v) { dft_split<true, 4, 2>(v); }
template <> __device__ inline void dftR<false, 16>(c32 *v) { dft_split<false, 4, 4>(v); }
template <> __device__ inline void dftR<true, 16>(c32 *v) { dft_split<true, 4, 4>(v); }

// One Stockham pass of radix R over N points in LDS (in place: all reads of
// the pass complete before any write).  Ns = length of the sub-transforms
// already formed.  tw[e] = W_N^e (forward sign), e < N.
// LDS slot of point i: one pad slot after every 16 points, so the strided
// accesses of the Stockham passes (stride R points) spread over the banks.
__device__ inline int pd(int i) { return i + (i >> 4); }
__host__ __device__ inline int padded_points(int N) { return N + N / 16 + 1; }

// W_N^e (forward sign) from the two LDS tables: lo[i] = W_N^i (i < 64),
// hi[i] = W_N^(64 i) (i < N/64).
__device__ inline c32 twid(int e, const c32 *lo, const c32 *hi) {
  const c32 a = lo[e & 63];
  return (e >> 6) ? cmul(a, hi[e >> 6]) : a;
}

template <bool INV, int R>
__device__ inline void stockham_pass(c32 *buf, int N, int Ns, const c32 *tlo, const c32 *thi) {
  const int nb = N / R;
  constexpr int kMaxB = 16 / R > 0 ? (4096 / R + kThreads - 1) / kThreads : 1;
  c32 v[kMaxB][R];
  int jj[kMaxB];
#pragma unroll
  for (int q = 0; q < kMaxB; ++q) {
    const int j = threadIdx.x + q * kThreads;
    jj[q] = j;
    if (j < nb) {
      const int k = j & (Ns - 1);
      const int step = N / (Ns * R);          // W_{Ns R}^{k r} = W_N^{k r step}
      // twiddles w^r, r = 1..R-1, of w = W_N^{k step}: one table lookup,
      // then products (a few ulp in FP64)
      c32 w = twid((k * step) & (N - 1), tlo, thi);
      if (INV) w = cconj(w);
      c32 wr = w;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        c32 x = buf[pd(j + r * nb)];
        if (r > 0) {
          x = cmul(x, wr);
          wr = cmul(wr, w);
        }
        v[q][r] = x;
      }
      dftR<INV, R>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kMaxB; ++q) {
    const int j = jj[q];
    if (j < nb) {
      const int k = j & (Ns - 1);
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pd(base + r * Ns)] = v[q][r];
    }
  }
  __syncthreads();
}

// Complex FFT of N (power of 2, N <= 4096) points in LDS.
template <bool INV>
__device__ void fft_lds(c32 *buf, int N, const c32 *tlo, const c32 *thi) {
  int Ns = 1;
  while (Ns < N) {
    const int left = N / Ns;
    if (left >= 16) {
      stockham_pass<INV, 16>(buf, N, Ns, tlo, thi);
      Ns *= 16;
    } else if (left == 8) {
      stockham_pass<INV, 8>(buf, N, Ns, tlo, thi);
      Ns *= 8;
    } else if (left == 4) {
      stockham_pass<INV, 4>(buf, N, Ns, tlo, thi);
      Ns *= 4;
    } else {
      stockham_pass<INV, 2>(buf, N, Ns, tlo, thi);
      Ns *= 2;
    }
  }
}

// W_L^f = exp(-2 pi i f / L) for the real-transform unpacking, with L = 2N:
// W_L^f = W_N^{f/2} for even f; for odd f that times W_L^1 (passed in).
__device__ inline c32 wl(int f, int N, const c32 *tlo, const c32 *thi, c32 w1) {
  c32 w = twid((f >> 1) & (N - 1), tlo, thi);
  if (f & 1) w = cmul(w, w1);
  return w;
}

// Fill the two twiddle tables (LDS, 64 + 64 entries) from the global table
// tw[e] = W_N^e; callers synchronize before use.
__device__ inline void load_twiddles(c32 *tlo, c32 *thi, int N, const double2 *__restrict__ tw) {
  const int t = threadIdx.x;
  if (t < 64) {
    const double2 a = tw[t & (N - 1)];
    tlo[t] = c32{a.x, a.y};
  } else if (t < 128) {
    const int i = t - 64;
    const double2 a = (64 * i < N) ? tw[64 * i] : make_double2(1.0, 0.0);
    thi[i] = c32{a.x, a.y};
  }
}

// ---------------------------------------------------------------- spectra
// FP64 spectra of the circulant embeddings (direct sums): for even
// generators  G[f] = g_0 + 2 sum_{J>=1} g_J cos(2 pi f J / L),
// for odd ones the imaginary part  -2 sum_{J>=1} g_J sin(2 pi f J / L).
__global__ void k_spectra(const double *__restrict__ gens, double *__restrict__ spec, int n, int L, int M) {
  extern __shared__ double sh[];
  double *ctab = sh;           // cos(2 pi e / L), e < L
  double *g = sh + L;          // g_J, J = 0..n-1
  const int gen = blockIdx.y;  // type * M + k
  const int type = gen / M;
  const bool odd = (type == F_X || type == F_Q);
  for (int e = threadIdx.x; e < L; e += blockDim.x) ctab[e] = cospi(2.0 * double(e) / double(L));
  const double *src = gens + size_t(gen) * (2 * n - 1) + (n - 1);
  for (int J = threadIdx.x; J < n; J += blockDim.x) g[J] = src[J];
  __syncthreads();
  const int nf = L / 2 + 1;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += gridDim.x * blockDim.x) {
    double acc = 0.0;
    if (odd) {
      // sin(2 pi e / L) = cos(2 pi (e - L/4) / L)
      for (int J = 1; J < n; ++J) acc += g[J] * ctab[(int)((int64_t(f) * J - L / 4) & (L - 1))];
      acc = -2.0 * acc;
    } else {
      for (int J = 1; J < n; ++J) acc += g[J] * ctab[(int)((int64_t(f) * J) & (L - 1))];
      acc = g[0] + 2.0 * acc;
    }
    spec[size_t(gen) * nf + f] = acc;
  }
}

__global__ void k_twiddles(double2 *__restrict__ tw, int N) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double s, c;
  sincospi(-2.0 * double(e) / double(N), &s, &c);
  tw[e] = make_double2(c, s);
}

// ---------------------------------------------------------------- jobs
// frequency pairs (f, N - f), f = 0..N/2, per thread at N = 4096: 2049 pairs
constexpr int kMaxPairs = (4096 / 2 + 1 + kThreads - 1) / kThreads;

// Forward real transform of every column: U[col][f], f = 0..N (N + 1 values).
__global__ __launch_bounds__(kThreads) void k_fft_fwd(const float *__restrict__ in, c32 *__restrict__ U,
                                                      const double2 *__restrict__ tw, int n, int L) {
  extern __shared__ c32 wk[];   // N points (padded), then the twiddle tables
  const int N = L / 2;
  c32 *tlo = wk + padded_points(N), *thi = tlo + 64;
  const int col = blockIdx.x;
  load_twiddles(tlo, thi, N, tw);
  const float *u = in + size_t(col) * n;
  for (int m = threadIdx.x; m < N; m += kThreads) {
    const int a = 2 * m, b = 2 * m + 1;
    wk[pd(m)] = c32{a < n ? double(u[a]) : 0.0, b < n ? double(u[b]) : 0.0};
  }
  __syncthreads();
  fft_lds<false>(wk, N, tlo, thi);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const c32 w1{cw, sw};         // W_L^1
  // X[f] = E + W_L^f O with E = (Z[f] + conj Z[N-f])/2, O = (Z[f] - conj Z[N-f])/(2i)
  c32 *Uc = U + size_t(col) * (N + 1);
  for (int f = threadIdx.x; f <= N; f += kThreads) {
    const c32 zf = wk[pd(f & (N - 1))];
    const c32 zcc = cconj(wk[pd((N - f) & (N - 1))]);
    const c32 D{0.5 * (zf.x - zcc.x), 0.5 * (zf.y - zcc.y)};
    Uc[f] = cadd(c32{0.5 * (zf.x + zcc.x), 0.5 * (zf.y + zcc.y)}, cmul(wl(f, N, tlo, thi, w1), c32{D.y, -D.x}));
  }
}

// Grid: x = input column (q * R + l), y = job group.  Jobs of a column are
// its (s, k) pairs, j = s * M + k, in contiguous groups of jobs_per_group.
__global__ __launch_bounds__(kThreads) void k_fft_jobs(const c32 *__restrict__ U, float *__restrict__ out,
                                                       const double *__restrict__ spec,
                                                       const double2 *__restrict__ tw, int n, int L, int M, int R,
                                                       int axis, int jobs_per_group) {
  extern __shared__ c32 wk[];   // N points (padded), then the twiddle tables
  const int N = L / 2;
  c32 *tlo = wk + padded_points(N), *thi = tlo + 64;
  const int col = blockIdx.x;   // q * R + l
  const int q = col / R, l = col % R;
  load_twiddles(tlo, thi, N, tw);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const c32 w1{cw, sw};         // W_L^1
  // U[f] and U[N - f] for this thread's pairs f = threadIdx.x + p * kThreads <= N/2
  const c32 *Uc = U + size_t(col) * (N + 1);
  c32 uf[kMaxPairs], uc[kMaxPairs];
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) {
    const int f = threadIdx.x + p * kThreads;
    if (f <= N / 2) {
      uf[p] = Uc[f];
      uc[p] = Uc[N - f];
    }
  }
  __syncthreads();

  const int njobs = 2 * M;
  const int j0 = blockIdx.y * jobs_per_group;
  const int j1 = min(njobs, j0 + jobs_per_group);
  const double inv_n = 1.0 / double(N);
  for (int j = j0; j < j1; ++j) {
    const int s = j / M, k = j % M;
    // factor type of (axis, component q, slot s): X/P along q, E/Q elsewhere
    const int type = (axis == q) ? (s ? F_P : F_X) : (s ? F_Q : F_E);
    const bool odd = (type == F_X || type == F_Q);
    const double *gs = spec + size_t(type * M + k) * (N + 1);
    // Y = U G (G real or imaginary); pack Z[f] = E[f] + i O[f] for f and N - f
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) {
      const int f = threadIdx.x + p * kThreads;
      if (f <= N / 2) {
        const int fc = N - f;
        const double gf = gs[f], gc = gs[fc];
        c32 yf = uf[p], yc = uc[p];
        yf = odd ? c32{-yf.y * gf, yf.x * gf} : c32{yf.x * gf, yf.y * gf};
        yc = odd ? c32{-yc.y * gc, yc.x * gc} : c32{yc.x * gc, yc.y * gc};
        // Z[f] from (Y[f], Y[N-f]); Z[N-f] from (Y[N-f], Y[f])
        {
          const c32 ycc = cconj(yc);
          const c32 E{0.5 * (yf.x + ycc.x), 0.5 * (yf.y + ycc.y)};
          const c32 Dm{0.5 * (yf.x - ycc.x), 0.5 * (yf.y - ycc.y)};
          const c32 O = cmul(Dm, cconj(wl(f, N, tlo, thi, w1)));
          wk[pd(f & (N - 1))] = c32{E.x - O.y, E.y + O.x};
        }
        if (fc != f && fc < N) {
          const c32 yfc = cconj(yf);
          const c32 E{0.5 * (yc.x + yfc.x), 0.5 * (yc.y + yfc.y)};
          const c32 Dm{0.5 * (yc.x - yfc.x), 0.5 * (yc.y - yfc.y)};
          const c32 O = cmul(Dm, cconj(wl(fc, N, tlo, thi, w1)));
          wk[pd(fc)] = c32{E.x - O.y, E.y + O.x};
        }
      }
    }
    __syncthreads();
    fft_lds<true>(wk, N, tlo, thi);
    float *y = out + ((size_t(q) * 2 + s) * M + k) * size_t(R) * n + size_t(l) * n;
    for (int m = threadIdx.x; m < N; m += kThreads) {
      const c32 z = wk[pd(m)];
      const int a = 2 * m, b = 2 * m + 1;
      if (a < n) y[a] = float(z.x * inv_n);
      if (b < n) y[b] = float(z.y * inv_n);
    }
    __syncthreads();
  }
}

}  // namespace

int fft_length(int n) {
  int L = 2;
  while (L < 2 * n - 1) L *= 2;
  return L;
}

demag_status prepare_spectra(demag_ctx *ctx, demag_factors *f) {
  if (f->spec_ready) return DEMAG_OK;
  for (int d = 0; d < 3; ++d) {
    const int n = f->n[d];
    const int L = fft_length(n);
    const int N = L / 2;
    DEMAG_REQUIRE(N <= 4096, "structured apply supports n <= 4096 per axis");
    const size_t nspec = size_t(F_NTYPES) * f->M * (N + 1);
    DEMAG_TRY_HIP(hipMalloc(&f->spec[d], nspec * sizeof(double)));
    DEMAG_TRY_HIP(hipMalloc(&f->twiddle[d], size_t(N) * sizeof(double2)));
    k_twiddles<<<(N + 255) / 256, 256, 0, ctx->stream>>>(reinterpret_cast<double2 *>(f->twiddle[d]), N);
    DEMAG_TRY_HIP(hipGetLastError());
    const size_t lds = sizeof(double) * (size_t(L) + n);
    DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_spectra),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    dim3 grid((N + 1 + 255) / 256, F_NTYPES * f->M);
    k_spectra<<<grid, 256, lds, ctx->stream>>>(f->f64[d], f->spec[d], n, L, f->M);
    DEMAG_TRY_HIP(hipGetLastError());
  }
  f->spec_ready = true;
  return DEMAG_OK;
}

demag_status launch_columns(demag_ctx *ctx, const demag_factors *f, int d, int R, const float *in, float *out) {
  const int n = f->n[d];
  const int L = fft_length(n);
  const int N = L / 2;
  const int ncols = 3 * R;
  if (ncols == 0) return DEMAG_OK;
  // column spectra in the workspace
  demag_status st = ensure_workspace(ctx, sizeof(double2) * size_t(ncols) * (N + 1));
  if (st != DEMAG_OK) return st;
  c32 *U = static_cast<c32 *>(ctx->ws);
  // job groups per column: enough workgroups to fill the chip (>= 4 per CU)
  int target = 1;
  const int njobs = 2 * f->M;
  while (ncols * target < 1024 && target < njobs) target *= 2;
  const int per = (njobs + target - 1) / target;
  const int groups = (njobs + per - 1) / per;   // every group owns >= 1 job
  const size_t lds = sizeof(double2) * (size_t(padded_points(N)) + 128);
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_fwd),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_jobs),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  const double2 *tw = reinterpret_cast<const double2 *>(f->twiddle[d]);
  hipEvent_t ev = nullptr;
  st = prof_begin(ctx, &ev);
  if (st != DEMAG_OK) return st;
  k_fft_fwd<<<ncols, kThreads, lds, ctx->stream>>>(in, U, tw, n, L);
  DEMAG_TRY_HIP(hipGetLastError());
  k_fft_jobs<<<dim3(ncols, groups), kThreads, lds, ctx->stream>>>(U, out, f->spec[d], tw, n, L, f->M, R, d, per);
  DEMAG_TRY_HIP(hipGetLastError());
  if (ev) {
    const double jobs = double(ncols) * njobs;
    // real FFT of length L ~ 2.5 L log2 L flops, forward once per column
    const double lg = std::log2(double(L));
    const double flops = (jobs + ncols) * 2.5 * L * lg;
    // compulsory traffic: input columns, spectra, output columns
    const double bytes = 4.0 * (double(ncols) * n + jobs * n) + 8.0 * double(F_NTYPES) * f->M * (N + 1);
    st = prof_end(ctx, ev, std::string("fft/") + "xyz"[d], flops, bytes);
  }
  return st;
}

}  // namespace demag
