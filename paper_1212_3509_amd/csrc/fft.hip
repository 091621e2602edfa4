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
// factor set in FP64 (forward real FFTs of the one-sided generators).
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
// of radix 16/8/4/2 (N/R butterflies per pass, 256 threads; 4096-point lines:
// radix 8 with 512 threads).  Twiddles come
// from two 64-entry tables in LDS, W_N^e = W_N^(e mod 64) W_N^(64 (e div 64)),
// so no pass waits on global memory.
//
// Two launches per apply, covering the three axes: k_fft_fwd transforms
// every input column once and stores its unpacked spectrum U[0..N] in the
// workspace; k_fft_jobs gives each workgroup a few jobs of one column: per
// job it reads the column's frequency pairs (f, N - f) and the kernel
// spectrum (from L2: every job group of a column reads the same 64 KB),
// multiplies, transforms back and writes the n outputs.
//
// FP32 transforms (DEMAG_FP32): the forward transforms stay FP64, the kernel
// spectra and the per-job inverse transforms are FP32.  An FP32 rounding of
// a spectrum element is relative to that element and survives the product
// unchanged, and an FP32 inverse transform's roundoff is relative to the
// norm of its own output (Parseval), so the columns keep the 1e-6 bar; an
// FP32 forward transform would not (its roundoff, relative to the input
// column's norm, is shaped by the kernel spectrum).  The packing of the
// half-length complex inverse transform is linear in the two spectrum
// values a job multiplies: with G the kernel spectrum,
//   Z[f] = G[f] A[f] + G[N-f] B[f]   (even kernels, G real),
//   Z[f] = i (g[f] A[f] - g[N-f] B[f])   (odd kernels, G = i g),
//   A[f] = U[f] (1 + i conj W_L^f) / 2,  B[f] = conj U[N-f] (1 - i conj W_L^f) / 2,
// so k_fft_fwd<true> stores A and B (FP32) per column, and k_fft_jobs32 keeps
// each thread's 16 pairs in registers across the workgroup's jobs, forms its
// 16 points of Z per job and runs the first radix-16 pass on them in
// registers (no LDS round for the packing).
#include "fft_core.h"
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace demag {

namespace {

using namespace fftc;

constexpr int kThreads = 256;
constexpr int kThreadsW = 512;  // the 4096-point job kernels with half the points per lane
constexpr int kPoints = 4096;   // largest transform (N = L / 2)

__host__ __device__ inline int padded_points(int N) { return N + N / 16 + 1; }

// Fill the two twiddle tables (LDS, 64 + 64 entries) from the global table
// tw[e] = W_N^e; callers synchronize before use.
__device__ inline void load_twiddles(cplx *tlo, cplx *thi, int N, const double2 *__restrict__ tw) {
  const int t = threadIdx.x;
  if (t < 64) {
    const double2 a = tw[t & (N - 1)];
    tlo[t] = cplx{a.x, a.y};
  } else if (t < 128) {
    const int i = t - 64;
    const double2 a = (64 * i < N) ? tw[64 * i] : make_double2(1.0, 0.0);
    thi[i] = cplx{a.x, a.y};
  }
}

__global__ void k_twiddles(double2 *__restrict__ tw, int N) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double s, c;
  sincospi(-2.0 * double(e) / double(N), &s, &c);
  tw[e] = make_double2(c, s);
}

// Pass-major FP32 twiddles of plan PM (see pm_offset): entry i of the pass of
// sub-transform length Ns and radix R = W_N^(k r N / (Ns R)) rounded from
// the FP64 table, r = 1 + (i - off) / Ns, k = (i - off) % Ns.
__global__ void k_pm_twiddles(const double2 *__restrict__ tw, float *__restrict__ out, int N, int PM) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (PM == 16 ? pm_twiddle_count(N) : pm8_twiddle_count(N))) return;
  int Ns, R;
  if (PM == 16) {
    Ns = i < pm_offset(16, 256) ? 16 : 256;
    R = Ns == 16 ? 16 : N / 256;
  } else {
    Ns = i < pm_offset(8, 64) ? 8 : i < pm_offset(8, 512) ? 64 : 512;
    R = 8;
  }
  const int loc = i - pm_offset(PM, Ns);
  const int r = 1 + loc / Ns, k = loc % Ns;
  const int e = int((int64_t(k) * r * (N / (Ns * R))) & (N - 1));
  out[2 * i] = float(tw[e].x);
  out[2 * i + 1] = float(tw[e].y);
}

__global__ void k_to_f32(const double *__restrict__ src, float *__restrict__ dst, size_t count, double scale) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = float(src[i] * scale);
}

// ---------------------------------------------------------------- jobs
// frequency pairs (f, N - f), f = 0..N/2, per thread at N = 4096: 2049 pairs
constexpr int kMaxPairs = (kPoints / 2 + 1 + kThreads - 1) / kThreads;

// The three axes of one structured apply run in the same two launches; a
// workgroup finds its axis from the first column / workgroup of each.
struct ColAxis {
  const float *in;
  float *out;
  const double *spec;
  const float *spec32;       // FP32 copies of the kernel spectra (FP32 transforms)
  const cplx32 *tw32;        // FP32 twiddles W_N^e, e < N (FP32 transforms)
  const cplx32 *twpm;        // the same in pass-major order (pm_twiddle_count(N) entries)
  const cplx32 *twpm8;       // pass-major for the radix-8 plan (pm8_twiddle_count(N) entries)
  const double2 *tw;
  size_t u_off;              // first spectrum of this axis in U (points)
  int n, L, R;
  int col0, wg0;             // first column, first jobs workgroup
  int per, groups;           // jobs per group, groups per column
};
struct ColAxes {
  ColAxis a[3];
  int M;
};
// The hardware places workgroup lin on XCD lin % 8; this gives the
// workgroups of one XCD consecutive work indices.
__device__ inline unsigned xcd_work_index(unsigned lin, unsigned total) {
  const unsigned x = lin & 7u, slot = lin >> 3;
  const unsigned per = total >> 3, rem = total & 7u;
  return x * per + min(x, rem) + slot;
}
__device__ inline int axis_of(const ColAxes &P, int idx, bool wg) {
  int d = 0;
  for (int e = 1; e < 3; ++e)
    if (idx >= (wg ? P.a[e].wg0 : P.a[e].col0)) d = e;
  return d;
}

// Unpacking of a forward real transform from its half-length complex
// transform Z (in LDS, layout slot<1>) at f and N - f together, f <= N / 2:
//   X[f] = E_f + W_L^f O_f,   conj X[N - f] = E_f - W_L^f O_f,
// E_f = (Z[f] + conj Z[N-f]) / 2, O_f = (Z[f] - conj Z[N-f]) / (2i), since
// E_(N-f) = conj E_f, O_(N-f) = conj O_f and W_L^(N-f) = -conj W_L^f.
// AB == false: U[f] = X[f] and U[N - f] into dst (N + 1 values).  AB == true:
// the FP32 packing factors A[g] = X[g] (1 + i conj W_L^g) / 2 and
// B[g] = conj X[N - g] (1 - i conj W_L^g) / 2 at g = f and g = N - f < N
// into dst (A) and dst + N (B), using i conj W_L^(N-f) = -i W_L^f.
template <bool AB>
__device__ inline void unpack_pair(const cplx *wk, int f, int N, const cplx *tlo, const cplx *thi, cplx w1,
                                   void *dst) {
  const cplx zf = wk[slot<1>(f & (N - 1))];
  const cplx zcc = cconj(wk[slot<1>((N - f) & (N - 1))]);
  const cplx E{0.5 * (zf.x + zcc.x), 0.5 * (zf.y + zcc.y)};
  const cplx D{0.5 * (zf.x - zcc.x), 0.5 * (zf.y - zcc.y)};
  const cplx W = wl(f, N, tlo, thi, w1);
  const cplx WO = cmul(W, cplx{D.y, -D.x});   // W_L^f O_f, O_f = D / i
  const cplx xf = cadd(E, WO);                // X[f]
  const cplx xcc = csub(E, WO);               // conj X[N - f]
  const int fc = N - f;
  if constexpr (!AB) {
    cplx *U = static_cast<cplx *>(dst);
    U[f] = xf;
    if (fc != f) U[fc] = cconj(xcc);
  } else {
    cplx32 *Ac = static_cast<cplx32 *>(dst);
    cplx32 *Bc = Ac + N;
    const cplx iw{W.y, W.x};                  // i conj W_L^f
    const cplx a = cmul(xf, cplx{1.0 + iw.x, iw.y});
    const cplx b = cmul(xcc, cplx{1.0 - iw.x, -iw.y});
    Ac[f] = cplx32{float(0.5 * a.x), float(0.5 * a.y)};
    Bc[f] = cplx32{float(0.5 * b.x), float(0.5 * b.y)};
    if (f > 0 && fc != f) {
      const cplx iwc{W.y, -W.x};              // i conj W_L^fc = -i W_L^f
      const cplx ac = cmul(cconj(xcc), cplx{1.0 + iwc.x, iwc.y});
      const cplx bc = cmul(cconj(xf), cplx{1.0 - iwc.x, -iwc.y});
      Ac[fc] = cplx32{float(0.5 * ac.x), float(0.5 * ac.y)};
      Bc[fc] = cplx32{float(0.5 * bc.x), float(0.5 * bc.y)};
    }
  }
}

// Forward real transform of every column (FP64).  AB == false: the unpacked
// spectrum U[col][f], f = 0..N (N + 1 values, FP64).  AB == true: the FP32
// packing factors A[col][f], B[col][f], f < N (2 N values per column, A first).
template <bool AB>
__global__ __launch_bounds__(kThreads) void k_fft_fwd(const ColAxes P, void *__restrict__ Uout, int lds_points) {
  extern __shared__ cplx wk[];   // N points (padded), then the twiddle tables
  const int d = axis_of(P, blockIdx.x, false);
  const ColAxis &A = P.a[d];
  const int n = A.n, L = A.L, N = L / 2;
  cplx *tlo = wk + lds_points, *thi = tlo + 64;
  const int col = blockIdx.x - A.col0;
  load_twiddles(tlo, thi, N, A.tw);
  const float *u = A.in + size_t(col) * n;
  // all loads of a thread in flight before the LDS stores
  constexpr int kE = kPoints / kThreads;
  cplx v[kE];
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int m = threadIdx.x + q * kThreads;
    const int a = 2 * m, b = 2 * m + 1;
    v[q] = cplx{m < N && a < n ? double(u[a]) : 0.0, m < N && b < n ? double(u[b]) : 0.0};
  }
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int m = threadIdx.x + q * kThreads;
    if (m < N) wk[slot<true>(m)] = v[q];
  }
  __syncthreads();
  fft_lines<false, kThreads, kPoints, true>(wk, N, padded_points(N), 1, tlo, thi);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const cplx w1{cw, sw};         // W_L^1
  void *dst = AB ? static_cast<void *>(static_cast<cplx32 *>(Uout) + A.u_off + size_t(col) * (2 * N))
                 : static_cast<void *>(static_cast<cplx *>(Uout) + A.u_off + size_t(col) * (N + 1));
  for (int f = threadIdx.x; f <= N / 2; f += kThreads) unpack_pair<AB>(wk, f, N, tlo, thi, w1, dst);
}

// Forward real transforms of 4096-point lines (L = 8192, n = 2049..4096) with
// 512 threads, as k_fft_fwd otherwise.  z[m] = x[2m] + i x[2m+1] vanishes for
// m >= 2048 (2m >= n), so the first radix-8 pass takes its four nonzero
// inputs straight from the column into registers; three radix-8 passes in
// LDS follow; unpack_pair forms the outputs.
template <bool AB>
__global__ __launch_bounds__(kThreadsW) void k_fft_fwd_w(const ColAxes P, void *__restrict__ Uout, int lds_points) {
  constexpr int N = 4096, per = N / 8;
  extern __shared__ cplx wk[];   // N points, then the twiddle tables
  const int d = axis_of(P, blockIdx.x, false);
  const ColAxis &A = P.a[d];
  const int n = A.n;
  cplx *tlo = wk + lds_points, *thi = tlo + 64;
  const int col = blockIdx.x - A.col0;
  load_twiddles(tlo, thi, N, A.tw);
  const float *u = A.in + size_t(col) * n;
  const int g = threadIdx.x;
  cplx v[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a = 2 * (g + per * r), b = a + 1;
    v[r] = cplx{a < n ? double(u[a]) : 0.0, b < n ? double(u[b]) : 0.0};
  }
#pragma unroll
  for (int r = 4; r < 8; ++r) v[r] = cplx{0.0, 0.0};
  dftR<false, 8>(v);
#pragma unroll
  for (int r = 0; r < 8; ++r) wk[slot<1>(8 * g + r)] = v[r];
  __syncthreads();
  pass<false, 8, kThreadsW, N, N, 8, ToLds, 1>(wk, 0, 1, tlo, thi);
  pass<false, 8, kThreadsW, N, N, 64, ToLds, 1>(wk, 0, 1, tlo, thi);
  pass<false, 8, kThreadsW, N, N, 512, ToLds, 1>(wk, 0, 1, tlo, thi);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const cplx w1{cw, sw};         // W_L^1
  void *dst = AB ? static_cast<void *>(static_cast<cplx32 *>(Uout) + A.u_off + size_t(col) * (2 * N))
                 : static_cast<void *>(static_cast<cplx *>(Uout) + A.u_off + size_t(col) * (N + 1));
  for (int f = g; f <= N / 2; f += kThreadsW) unpack_pair<AB>(wk, f, N, tlo, thi, w1, dst);
}

// FP64 spectra of the circulant embeddings, one workgroup per generator
// (type * M + k): with A the forward real transform of the one-sided
// generator a_J = g_J, J < n, zero-padded to L (A[f] = sum_J a_J W_L^(fJ)),
// an even generator's embedding has the real spectrum
//   G[f] = g_0 + 2 sum_{J>=1} g_J cos(2 pi f J / L) = 2 Re A[f] - g_0,
// an odd one's (g_0 = 0) the imaginary part
//   -2 sum_{J>=1} g_J sin(2 pi f J / L) = 2 Im A[f],   f = 0..L/2.
__global__ __launch_bounds__(kThreads) void k_spectra(const double *__restrict__ gens, double *__restrict__ spec,
                                                      int n, int L, int M, const double2 *__restrict__ tw,
                                                      int lds_points) {
  extern __shared__ cplx wk[];   // N points (padded), then the twiddle tables
  const int N = L / 2;
  cplx *tlo = wk + lds_points, *thi = tlo + 64;
  const int gen = blockIdx.x;
  const int type = gen / M;
  const bool odd = (type == F_X || type == F_Q);
  load_twiddles(tlo, thi, N, tw);
  const double *a = gens + size_t(gen) * (2 * n - 1) + (n - 1);
  for (int m = threadIdx.x; m < N; m += kThreads) {
    const int i0 = 2 * m, i1 = 2 * m + 1;
    wk[slot<true>(m)] = cplx{i0 < n ? a[i0] : 0.0, i1 < n ? a[i1] : 0.0};
  }
  __syncthreads();
  fft_lines<false, kThreads, kPoints, true>(wk, N, padded_points(N), 1, tlo, thi);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const cplx w1{cw, sw};         // W_L^1
  const double g0 = a[0];
  double *out = spec + size_t(gen) * (N + 1);
  for (int f = threadIdx.x; f <= N; f += kThreads) {
    // A[f] = E + W_L^f O, E = (Z[f] + conj Z[N-f])/2, O = (Z[f] - conj Z[N-f])/(2i)
    const cplx zf = wk[slot<true>(f & (N - 1))];
    const cplx zcc = cconj(wk[slot<true>((N - f) & (N - 1))]);
    const cplx D{0.5 * (zf.x - zcc.x), 0.5 * (zf.y - zcc.y)};
    const cplx X = cadd(cplx{0.5 * (zf.x + zcc.x), 0.5 * (zf.y + zcc.y)}, cmul(wl(f, N, tlo, thi, w1), cplx{D.y, -D.x}));
    out[f] = odd ? 2.0 * X.y : 2.0 * X.x - g0;
  }
}

// Output of the inverse transform: point m of z holds x[2m] + i x[2m+1].
struct OutSink {
  float *y;
  int n;
  double inv_n;
  __device__ void operator()(int, int m, cplx z) const {
    const int a = 2 * m, b = 2 * m + 1;
    if (a < n) y[a] = float(z.x * inv_n);
    if (b < n) y[b] = float(z.y * inv_n);
  }
};

// Workgroup = (axis, input column q * R + l, job group).  Jobs of a column
// are its (s, k) pairs, j = s * M + k, in contiguous groups of A.per.
// Per job the column spectrum is read again (from L2) rather than held in
// registers, which keeps two workgroups resident per CU.
__global__ __launch_bounds__(kThreads) void k_fft_jobs(const ColAxes P, const cplx *__restrict__ Uall,
                                                       int lds_points) {
  extern __shared__ cplx wk[];   // N points (padded), then the twiddle tables
  // work index, XCD-grouped: the job groups of one column run on one XCD, so
  // its spectrum U is fetched into that L2 once
  const int w = int(xcd_work_index(blockIdx.x, gridDim.x));
  const int axis = axis_of(P, w, true);
  const ColAxis &A = P.a[axis];
  const int n = A.n, L = A.L, N = L / 2, R = A.R, M = P.M;
  cplx *tlo = wk + lds_points, *thi = tlo + 64;
  const int local = w - A.wg0;
  const int col = local / A.groups, grp = local - col * A.groups;   // col = q * R + l
  const int q = col / R, l = col % R;
  load_twiddles(tlo, thi, N, A.tw);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const cplx w1{cw, sw};         // W_L^1
  const cplx *Uc = Uall + A.u_off + size_t(col) * (N + 1);
  const double *spec = A.spec;
  float *out = A.out;
  __syncthreads();

  const int njobs = 2 * M;
  const int j0 = grp * A.per;
  const int j1 = min(njobs, j0 + A.per);
  const double inv_n = 1.0 / double(N);
  for (int j = j0; j < j1; ++j) {
    const int s = j / M, k = j % M;
    // factor type of (axis, component q, slot s): X/P along q, E/Q elsewhere
    const int type = (axis == q) ? (s ? F_P : F_X) : (s ? F_Q : F_E);
    const bool odd = (type == F_X || type == F_Q);
    const double *gs = spec + size_t(type * M + k) * (N + 1);
    // this thread's pairs f = threadIdx.x + p * kThreads <= N/2, in batches
    // of kB pairs whose loads (U[f], U[N - f], G[f], G[N - f]) are in flight
    // together; Y = U G (G real or imaginary), packed as Z[f] = E[f] + i O[f]
    // for f and N - f
    constexpr int kB = 3;
#pragma unroll 1
    for (int p0 = 0; p0 < kMaxPairs; p0 += kB) {
      cplx uf[kB], uc[kB];
      double gf[kB], gc[kB];
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        const int f = threadIdx.x + (p0 + i) * kThreads;
        if (p0 + i < kMaxPairs && f <= N / 2) {
          uf[i] = Uc[f];
          uc[i] = Uc[N - f];
          gf[i] = gs[f];
          gc[i] = gs[N - f];
        }
      }
#pragma unroll
      for (int i = 0; i < kB; ++i) {
        const int f = threadIdx.x + (p0 + i) * kThreads;
        if (p0 + i >= kMaxPairs || f > N / 2) continue;
        const int fc = N - f;
        cplx yf = uf[i], yc = uc[i];
        yf = odd ? cplx{-yf.y * gf[i], yf.x * gf[i]} : cplx{yf.x * gf[i], yf.y * gf[i]};
        yc = odd ? cplx{-yc.y * gc[i], yc.x * gc[i]} : cplx{yc.x * gc[i], yc.y * gc[i]};
        // Z[f] from (Y[f], Y[N-f]); Z[N-f] from (Y[N-f], Y[f])
        {
          const cplx ycc = cconj(yc);
          const cplx E{0.5 * (yf.x + ycc.x), 0.5 * (yf.y + ycc.y)};
          const cplx Dm{0.5 * (yf.x - ycc.x), 0.5 * (yf.y - ycc.y)};
          const cplx O = cmul(Dm, cconj(wl(f, N, tlo, thi, w1)));
          wk[slot<true>(f & (N - 1))] = cplx{E.x - O.y, E.y + O.x};
        }
        if (fc != f && fc < N) {
          const cplx yfc = cconj(yf);
          const cplx E{0.5 * (yc.x + yfc.x), 0.5 * (yc.y + yfc.y)};
          const cplx Dm{0.5 * (yc.x - yfc.x), 0.5 * (yc.y - yfc.y)};
          const cplx O = cmul(Dm, cconj(wl(fc, N, tlo, thi, w1)));
          wk[slot<true>(fc)] = cplx{E.x - O.y, E.y + O.x};
        }
      }
    }
    __syncthreads();
    // inverse transform; the last pass writes the n outputs (x[2m], x[2m+1]
    // = Re, Im z[m] / N) straight from registers
    float *y = out + ((size_t(q) * 2 + s) * M + k) * size_t(R) * n + size_t(l) * n;
    fft_lines_to<true, kThreads, kPoints, OutSink, true>(wk, N, padded_points(N), 1, tlo, thi,
                                          OutSink{y, n, inv_n});
    __syncthreads();
  }
}

// FP64 jobs on 4096-point lines with 512 threads (as k_fft_jobs): each
// thread packs the pairs f = t + 512 p, then the inverse transform runs as
// four radix-8 passes, the last writing the outputs.  Half the points per
// lane of the radix-16 plan, so four waves per SIMD instead of two.
__global__ __launch_bounds__(kThreadsW, 2) void k_fft_jobs64w(const ColAxes P, const cplx *__restrict__ Uall,
                                                              int lds_points) {
  constexpr int N = 4096;
  constexpr int kPairs = (N / 2 + 1 + kThreadsW - 1) / kThreadsW;
  extern __shared__ cplx wk[];   // N points, then the twiddle tables
  const int w = int(xcd_work_index(blockIdx.x, gridDim.x));
  const int axis = axis_of(P, w, true);
  const ColAxis &A = P.a[axis];
  const int n = A.n, R = A.R, M = P.M;
  cplx *tlo = wk + lds_points, *thi = tlo + 64;
  const int local = w - A.wg0;
  const int col = local / A.groups, grp = local - col * A.groups;   // col = q * R + l
  const int q = col / R, l = col % R;
  load_twiddles(tlo, thi, N, A.tw);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const cplx w1{cw, sw};         // W_L^1
  const cplx *Uc = Uall + A.u_off + size_t(col) * (N + 1);
  __syncthreads();
  const int njobs = 2 * M;
  const int j0 = grp * A.per;
  const int j1 = min(njobs, j0 + A.per);
  const double inv_n = 1.0 / double(N);
  for (int j = j0; j < j1; ++j) {
    const int s = j / M, k = j % M;
    const int type = (axis == q) ? (s ? F_P : F_X) : (s ? F_Q : F_E);
    const bool odd = (type == F_X || type == F_Q);
    const double *gs = A.spec + size_t(type * M + k) * (N + 1);
    // pairs in batches of kB whose loads are in flight together
    constexpr int kB = 1;
#pragma unroll 1
    for (int p0 = 0; p0 < kPairs; p0 += kB) {
    cplx uf[kB], uc[kB];
    double gf[kB], gc[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int f = min(int(threadIdx.x) + (p0 + i) * kThreadsW, N / 2);
      uf[i] = Uc[f];
      uc[i] = Uc[N - f];
      gf[i] = gs[f];
      gc[i] = gs[N - f];
    }
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int f = threadIdx.x + (p0 + i) * kThreadsW;
      if (p0 + i >= kPairs || f > N / 2) continue;
      const int fc = N - f;
      cplx yf = uf[i], yc = uc[i];
      yf = odd ? cplx{-yf.y * gf[i], yf.x * gf[i]} : cplx{yf.x * gf[i], yf.y * gf[i]};
      yc = odd ? cplx{-yc.y * gc[i], yc.x * gc[i]} : cplx{yc.x * gc[i], yc.y * gc[i]};
      {
        const cplx ycc = cconj(yc);
        const cplx E{0.5 * (yf.x + ycc.x), 0.5 * (yf.y + ycc.y)};
        const cplx Dm{0.5 * (yf.x - ycc.x), 0.5 * (yf.y - ycc.y)};
        const cplx O = cmul(Dm, cconj(wl(f, N, tlo, thi, w1)));
        wk[slot<true>(f & (N - 1))] = cplx{E.x - O.y, E.y + O.x};
      }
      if (fc != f && fc < N) {
        const cplx yfc = cconj(yf);
        const cplx E{0.5 * (yc.x + yfc.x), 0.5 * (yc.y + yfc.y)};
        const cplx Dm{0.5 * (yc.x - yfc.x), 0.5 * (yc.y - yfc.y)};
        const cplx O = cmul(Dm, cconj(wl(fc, N, tlo, thi, w1)));
        wk[slot<true>(fc)] = cplx{E.x - O.y, E.y + O.x};
      }
    }
    }
    __syncthreads();
    float *y = A.out + ((size_t(q) * 2 + s) * M + k) * size_t(R) * n + size_t(l) * n;
    run_passes<true, kThreadsW, N, N, 1, OutSink, true, 8, 8, 8, 8>(wk, 0, 1, tlo, thi, OutSink{y, n, inv_n});
    __syncthreads();
  }
}

// Output of the FP32 inverse transform (as OutSink; the 1 / N is in the
// FP32 kernel spectra).
struct OutSink32 {
  float *y;
  int n;
  __device__ void operator()(int, int m, cplx32 z) const {
    const int a = 2 * m;
    if (a + 1 < n) {
      *reinterpret_cast<float2 *>(y + a) = make_float2(z.x, z.y);
    } else if (a < n) {
      y[a] = z.x;
    }
  }
};

// Passes of the inverse transform after the first (radix 16, done by the
// caller in registers), with the last pass writing the outputs.
// Twiddles: the pass-major table (tlo, pm_twiddle_count(N) entries).
template <int N>
__device__ inline void inverse_rest(cplx32 *wk, const cplx32 *tlo, const cplx32 *thi, const OutSink32 &sink) {
  if constexpr (N == 256) {
    pass<true, 16, kThreads, kPoints, N, 16, OutSink32, true, 16>(wk, 0, 1, tlo, thi, sink);
  } else {
    pass<true, 16, kThreads, kPoints, N, 16, ToLds, true, 16>(wk, 0, 1, tlo, thi);
    pass<true, N / 256, kThreads, kPoints, N, 256, OutSink32, true, 16>(wk, 0, 1, tlo, thi, sink);
  }
}

// FP32 jobs of one column on a line of N >= 256 points: thread g < N / 16
// owns the points f = g + (N / 16) r, r < 16, of the first pass.
template <int N>
__device__ inline void jobs32_line(const ColAxis &A, int axis, int M, int q, int l, int j0, int j1,
                                   const cplx32 *__restrict__ AB, cplx32 *wk, const cplx32 *tlo, const cplx32 *thi) {
  constexpr int per = N / 16;
  const int g = threadIdx.x;
  const bool act = g < per;
  const int n = A.n, R = A.R;
  cplx32 a[16], b[16];
  if (act) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      a[r] = AB[g + per * r];
      b[r] = AB[N + g + per * r];
    }
  }
  for (int j = j0; j < j1; ++j) {
    const int s = j / M, k = j % M;
    const int type = (axis == q) ? (s ? F_P : F_X) : (s ? F_Q : F_E);
    const bool odd = (type == F_X || type == F_Q);
    const float *gs = A.spec32 + size_t(type * M + k) * (N + 1);
    if (act) {
      float gf[16], gc[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        gf[r] = gs[g + per * r];
        gc[r] = gs[N - g - per * r];
      }
      cplx32 v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (odd) {
          // i (g_f A - g_c B)
          const float re = gf[r] * a[r].x - gc[r] * b[r].x, im = gf[r] * a[r].y - gc[r] * b[r].y;
          v[r] = cplx32{-im, re};
        } else {
          v[r] = cplx32{gf[r] * a[r].x + gc[r] * b[r].x, gf[r] * a[r].y + gc[r] * b[r].y};
        }
      }
      dftR<true, 16>(v);
#pragma unroll
      for (int r = 0; r < 16; ++r) wk[slot<true>(16 * g + r)] = v[r];
    }
    __syncthreads();
    float *y = A.out + ((size_t(q) * 2 + s) * M + k) * size_t(R) * n + size_t(l) * n;
    inverse_rest<N>(wk, tlo, thi, OutSink32{y, n});
    __syncthreads();
  }
}

// FP32 jobs: workgroup = (axis, input column q * R + l, job group), as
// k_fft_jobs, on the column's FP32 packing factors A, B.
__global__ __launch_bounds__(kThreads) void k_fft_jobs32(const ColAxes P, const cplx32 *__restrict__ ABall) {
  __shared__ cplx32 wk[kPoints];
  __shared__ cplx32 tlo[kPoints];   // FP32 twiddles: pass-major (N >= 256) or W_N^e, e < N
  const cplx32 *thi = nullptr;
  const int w = int(xcd_work_index(blockIdx.x, gridDim.x));
  const int axis = axis_of(P, w, true);
  const ColAxis &A = P.a[axis];
  const int N = A.L / 2, R = A.R, M = P.M;
  const int local = w - A.wg0;
  const int col = local / A.groups, grp = local - col * A.groups;   // col = q * R + l
  const int q = col / R, l = col % R;
  // lines of N >= 256 points: the pass-major twiddles; shorter ones: W_N^e, e < N
  if (N >= 256) {
    for (int e = threadIdx.x; e < pm_twiddle_count(N); e += kThreads) tlo[e] = A.twpm[e];
  } else {
    for (int e = threadIdx.x; e < N; e += kThreads) tlo[e] = A.tw32[e];
  }
  __syncthreads();
  const cplx32 *AB = ABall + A.u_off + size_t(col) * (2 * N);
  const int njobs = 2 * M;
  const int j0 = grp * A.per;
  const int j1 = min(njobs, j0 + A.per);
  switch (N) {
    case 4096: jobs32_line<4096>(A, axis, M, q, l, j0, j1, AB, wk, tlo, thi); return;
    case 2048: jobs32_line<2048>(A, axis, M, q, l, j0, j1, AB, wk, tlo, thi); return;
    case 1024: jobs32_line<1024>(A, axis, M, q, l, j0, j1, AB, wk, tlo, thi); return;
    case 512: jobs32_line<512>(A, axis, M, q, l, j0, j1, AB, wk, tlo, thi); return;
    case 256: jobs32_line<256>(A, axis, M, q, l, j0, j1, AB, wk, tlo, thi); return;
    default: break;
  }
  // short lines (N < 256): the packed points through LDS, then all passes
  for (int j = j0; j < j1; ++j) {
    const int s = j / M, k = j % M;
    const int type = (axis == q) ? (s ? F_P : F_X) : (s ? F_Q : F_E);
    const bool odd = (type == F_X || type == F_Q);
    const float *gs = A.spec32 + size_t(type * M + k) * (N + 1);
    for (int f = threadIdx.x; f < N; f += kThreads) {
      const cplx32 a = AB[f], b = AB[N + f];
      const float gf = gs[f], gc = gs[N - f];
      if (odd) {
        const float re = gf * a.x - gc * b.x, im = gf * a.y - gc * b.y;
        wk[slot<true>(f)] = cplx32{-im, re};
      } else {
        wk[slot<true>(f)] = cplx32{gf * a.x + gc * b.x, gf * a.y + gc * b.y};
      }
    }
    __syncthreads();
    float *y = A.out + ((size_t(q) * 2 + s) * M + k) * size_t(R) * A.n + size_t(l) * A.n;
    fft_lines_to<true, kThreads, kPoints, OutSink32, true, float>(wk, N, 0, 1, tlo, thi, OutSink32{y, A.n});
    __syncthreads();
  }
}

// FP32 jobs on 4096-point lines with 512 threads: thread g owns the points
// f = g + 512 r, r < 8, of the first pass (radix 8, in registers), then
// three radix-8 passes in LDS (layout slot<2>) with the radix-8 pass-major
// twiddles.  Half the points per lane of k_fft_jobs32 (8 pairs of packing
// factors held across jobs instead of 16), so four waves per SIMD instead
// of two.
__global__ __launch_bounds__(kThreadsW, 2) void k_fft_jobs32w(const ColAxes P, const cplx32 *__restrict__ ABall) {
  constexpr int N = 4096, per = N / 8;
  __shared__ cplx32 wk[N];
  __shared__ cplx32 tpm[N];
  const int w = int(xcd_work_index(blockIdx.x, gridDim.x));
  const int axis = axis_of(P, w, true);
  const ColAxis &A = P.a[axis];
  const int n = A.n, R = A.R, M = P.M;
  const int local = w - A.wg0;
  const int col = local / A.groups, grp = local - col * A.groups;   // col = q * R + l
  const int q = col / R, l = col % R;
  for (int e = threadIdx.x; e < pm8_twiddle_count(N); e += kThreadsW) tpm[e] = A.twpm8[e];
  __syncthreads();
  const cplx32 *AB = ABall + A.u_off + size_t(col) * (2 * N);
  const int g = threadIdx.x;
  cplx32 a[8], b[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    a[r] = AB[g + per * r];
    b[r] = AB[N + g + per * r];
  }
  const int njobs = 2 * M;
  const int j0 = grp * A.per;
  const int j1 = min(njobs, j0 + A.per);
  for (int j = j0; j < j1; ++j) {
    const int s = j / M, k = j % M;
    const int type = (axis == q) ? (s ? F_P : F_X) : (s ? F_Q : F_E);
    const bool odd = (type == F_X || type == F_Q);
    const float *gs = A.spec32 + size_t(type * M + k) * (N + 1);
    float gf[8], gc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      gf[r] = gs[g + per * r];
      gc[r] = gs[N - g - per * r];
    }
    cplx32 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (odd) {
        const float re = gf[r] * a[r].x - gc[r] * b[r].x, im = gf[r] * a[r].y - gc[r] * b[r].y;
        v[r] = cplx32{-im, re};
      } else {
        v[r] = cplx32{gf[r] * a[r].x + gc[r] * b[r].x, gf[r] * a[r].y + gc[r] * b[r].y};
      }
    }
    dftR<true, 8>(v);
#pragma unroll
    for (int r = 0; r < 8; ++r) wk[slot<2>(8 * g + r)] = v[r];
    __syncthreads();
    float *y = A.out + ((size_t(q) * 2 + s) * M + k) * size_t(R) * n + size_t(l) * n;
    pass<true, 8, kThreadsW, N, N, 8, ToLds, 2, 8>(wk, 0, 1, tpm, tpm);
    pass<true, 8, kThreadsW, N, N, 64, ToLds, 2, 8>(wk, 0, 1, tpm, tpm);
    pass<true, 8, kThreadsW, N, N, 512, OutSink32, 2, 8>(wk, 0, 1, tpm, tpm, OutSink32{y, n});
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
    const int lds_points = padded_points(N);
    const size_t lds = sizeof(double2) * (size_t(lds_points) + 128);
    DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_spectra),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    k_spectra<<<F_NTYPES * f->M, kThreads, lds, ctx->stream>>>(f->f64[d], f->spec[d], n, L, f->M,
                                                               reinterpret_cast<const double2 *>(f->twiddle[d]),
                                                               lds_points);
    DEMAG_TRY_HIP(hipGetLastError());
    // FP32 spectra, then the FP32 twiddles W_N^e (2 N floats, 8-byte aligned: nspec is even or padded)
    const size_t nspec_pad = nspec + (nspec & 1);
    const size_t npm = size_t(pm_twiddle_count(N)) + size_t(pm8_twiddle_count(N));
    DEMAG_TRY_HIP(hipMalloc(&f->spec32[d], (nspec_pad + 2 * size_t(N) + 2 * npm) * sizeof(float)));
    // the FP32 spectra carry the inverse transform's 1 / N (a power of two:
    // exact in the normal range)
    k_to_f32<<<unsigned((nspec + 255) / 256), 256, 0, ctx->stream>>>(f->spec[d], f->spec32[d], nspec,
                                                                      1.0 / double(N));
    k_to_f32<<<unsigned((2 * size_t(N) + 255) / 256), 256, 0, ctx->stream>>>(
        reinterpret_cast<const double *>(f->twiddle[d]), f->spec32[d] + nspec_pad, 2 * size_t(N), 1.0);
    if (pm_twiddle_count(N) > 0)
      k_pm_twiddles<<<unsigned((pm_twiddle_count(N) + 255) / 256), 256, 0, ctx->stream>>>(
          reinterpret_cast<const double2 *>(f->twiddle[d]), f->spec32[d] + nspec_pad + 2 * size_t(N), N, 16);
    if (pm8_twiddle_count(N) > 0)
      k_pm_twiddles<<<unsigned((pm8_twiddle_count(N) + 255) / 256), 256, 0, ctx->stream>>>(
          reinterpret_cast<const double2 *>(f->twiddle[d]),
          f->spec32[d] + nspec_pad + 2 * size_t(N) + 2 * size_t(pm_twiddle_count(N)), N, 8);
    DEMAG_TRY_HIP(hipGetLastError());
  }
  f->spec_ready = true;
  return DEMAG_OK;
}

size_t columns_workspace_bytes(const demag_factors *f, const int32_t R[3]) {
  size_t pts = 0;
  for (int d = 0; d < 3; ++d) pts += size_t(3) * R[d] * (fft_length(f->n[d]) / 2 + 1);
  return sizeof(double2) * pts;
}

demag_status launch_columns(demag_ctx *ctx, const demag_factors *f, demag_prec prec, const int32_t R[3],
                            const float *const in[3], float *const out[3], void *ws, size_t ws_bytes) {
  const bool f32 = (prec == DEMAG_FP32);
  ColAxes P{};
  P.M = f->M;
  const int njobs = 2 * f->M;
  int ncols_all = 0, maxN = 1;
  size_t u_points = 0;
  double flops = 0.0, bytes = 0.0;
  for (int d = 0; d < 3; ++d) ncols_all += 3 * R[d];
  if (ncols_all == 0) return DEMAG_OK;
  // job groups per column: enough workgroups to fill the chip (>= 4 per CU)
  int target = 1;
  while (ncols_all * target < 1024 && target < njobs) target *= 2;
  const int per = (njobs + target - 1) / target;
  const int groups = (njobs + per - 1) / per;   // every group owns >= 1 job
  int col0 = 0, wg0 = 0;
  for (int d = 0; d < 3; ++d) {
    ColAxis &A = P.a[d];
    const int ncols = 3 * R[d];
    A.in = in[d];
    A.out = out[d];
    A.spec = f->spec[d];
    A.spec32 = f->spec32[d];
    {
      // the FP32 twiddles follow the FP32 spectra (see prepare_spectra)
      const size_t nspec = size_t(F_NTYPES) * f->M * (fft_length(f->n[d]) / 2 + 1);
      A.tw32 = reinterpret_cast<const cplx32 *>(f->spec32[d] + nspec + (nspec & 1));
      A.twpm = A.tw32 + fft_length(f->n[d]) / 2;
      A.twpm8 = A.twpm + pm_twiddle_count(fft_length(f->n[d]) / 2);
    }
    A.tw = reinterpret_cast<const double2 *>(f->twiddle[d]);
    A.n = f->n[d];
    A.L = fft_length(f->n[d]);
    A.R = R[d];
    A.col0 = col0;
    A.wg0 = wg0;
    A.per = per;
    A.groups = groups;
    A.u_off = u_points;
    col0 += ncols;
    wg0 += ncols * groups;
    // FP64: U[0..N] per column (16-byte points); FP32: A, B (2 N 8-byte points)
    u_points += size_t(ncols) * (f32 ? A.L : A.L / 2 + 1);
    if (ncols > 0) maxN = std::max(maxN, A.L / 2);
    // real FFT of length L ~ 2.5 L log2 L flops, forward once per column
    const double jobs = double(ncols) * njobs, lg = std::log2(double(A.L));
    flops += (jobs + ncols) * 2.5 * A.L * lg;
    // compulsory traffic: input columns, spectra, output columns
    bytes += 4.0 * (double(ncols) * A.n + jobs * A.n) + (f32 ? 4.0 : 8.0) * double(F_NTYPES) * f->M * (A.L / 2 + 1);
  }
  // column spectra of all three axes in the workspace (the context's, or
  // the caller's when ws is given)
  demag_status st = DEMAG_OK;
  const size_t need = (f32 ? sizeof(cplx32) : sizeof(double2)) * u_points;
  if (ws) {
    if (ws_bytes < need) {
      set_error("structured apply: workspace too small");
      return DEMAG_E_INVAL;
    }
  } else {
    st = ensure_workspace(ctx, need);
    if (st != DEMAG_OK) return st;
    ws = ctx->ws;
  }
  const int lds_points = padded_points(maxN);
  const size_t lds = sizeof(double2) * (size_t(lds_points) + 128);
  hipEvent_t ev = nullptr;
  // 4096-point lines on every axis with columns: the 512-thread kernels
  bool w4096 = true;
  for (int d = 0; d < 3; ++d) w4096 = w4096 && (R[d] == 0 || P.a[d].L == 8192);
  if (f32) {
    DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_fwd<true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_fwd_w<true>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    st = prof_begin(ctx, &ev);
    if (st != DEMAG_OK) return st;
    if (w4096) k_fft_fwd_w<true><<<ncols_all, kThreadsW, lds, ctx->stream>>>(P, ws, lds_points);
    else k_fft_fwd<true><<<ncols_all, kThreads, lds, ctx->stream>>>(P, ws, lds_points);
    DEMAG_TRY_HIP(hipGetLastError());
    if (w4096) k_fft_jobs32w<<<wg0, kThreadsW, 0, ctx->stream>>>(P, static_cast<const cplx32 *>(ws));
    else k_fft_jobs32<<<wg0, kThreads, 0, ctx->stream>>>(P, static_cast<const cplx32 *>(ws));
    DEMAG_TRY_HIP(hipGetLastError());
    if (ev) st = prof_end(ctx, ev, "fft32/xyz", flops, bytes);
    return st;
  }
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_fwd<false>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_jobs),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_jobs64w),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_fwd_w<false>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  st = prof_begin(ctx, &ev);
  if (st != DEMAG_OK) return st;
  if (w4096) k_fft_fwd_w<false><<<ncols_all, kThreadsW, lds, ctx->stream>>>(P, ws, lds_points);
  else k_fft_fwd<false><<<ncols_all, kThreads, lds, ctx->stream>>>(P, ws, lds_points);
  DEMAG_TRY_HIP(hipGetLastError());
  if (w4096) k_fft_jobs64w<<<wg0, kThreadsW, lds, ctx->stream>>>(P, static_cast<const cplx *>(ws), lds_points);
  else k_fft_jobs<<<wg0, kThreads, lds, ctx->stream>>>(P, static_cast<const cplx *>(ws), lds_points);
  DEMAG_TRY_HIP(hipGetLastError());
  if (ev) st = prof_end(ctx, ev, "fft/xyz", flops, bytes);
  return st;
}

}  // namespace demag
