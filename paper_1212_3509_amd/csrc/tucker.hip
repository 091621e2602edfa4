// The scalar potential of a Tucker magnetization by structured DFTs
// (Sec. 4.2, Alg. scpot_fft_tucker) with the tolerance-controlled steps it
// names, the approximate summation of Tucker tensors, and TT rounding (App. C).
//
//   set-up         the CP kernels of Eq. (conv_pot) (per component q the
//                  X generator of every node on axis q and the E generators on
//                  the other axes, node weights folded in), compressed to
//                  Tucker with tol by HOOI (Alg. HOOI), and the DFTs of their
//                  factor rows (Lemma DFT_tucker);
//   per component  the DFTs of the magnetization's factor rows; the Hadamard
//                  product in Fourier space (App. B, Eq. (t_had2): the
//                  Kronecker product of the cores, and per mode the products of
//                  every kernel row spectrum with every magnetization row
//                  spectrum); the inverse DFT cut to the convolution window;
//                  the product recompressed with tol;
//   summation      the three products side by side, recompressed with tol.
//
// Every recompression is HOOI on a small dense core.  The factor rows of the
// tensor are orthonormalised by classical Gram-Schmidt with one
// reorthogonalisation (a row whose residual is below 1e-14 of its norm is
// dependent and dropped); the core is the tensor in those bases, and HOOI runs
// on the core: with orthonormal bases, the singular values and left singular
// subspaces of the tensor's unfoldings are those of the core's, mapped by the
// bases.  Singular values and vectors of a matrix: Gram-Schmidt of its rows
// (in chunks of 16384 points, then once more over the stacked coefficients),
// then one-sided Jacobi on the columns of the small coefficient matrix, which
// keeps every singular value to rounding relative to its own size (an
// eigen-decomposition of the Gram matrix would lose the small ones).  Rank rule
// per mode (HOOI): the smallest r whose discarded singular values have a norm
// of at most eps / sqrt(3) of all of them.
//
// TT rounding (3D, cores G1 [r1][n1], G2 [r1][r2][n2], G3 [r2][n3]): the outer
// cores are orthonormalised, their coefficients multiplied into the middle
// core, then two truncated SVDs from the left discard singular values of norm
// at most eps / sqrt(2) |A| each.
//
// DFTs: complex Stockham transforms in LDS of L = 2^k >= 2n - 1 points
// (n <= 4096), two real rows per transform.  All arithmetic is FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fft_core.h"
#include "internal.h"

namespace demag {
namespace {

using fftc::cplx;

constexpr int kOT = 512;              // Gram-Schmidt workgroup
constexpr int kOPer = 32;             // points per thread
constexpr int kOLen = kOT * kOPer;    // longest row (chunk) per workgroup
constexpr int kOMax = 512;            // rows per orthonormalisation
constexpr int kSvd = 128;             // rows of a small SVD (rank cap per mode)
constexpr int kST = 1024;             // Jacobi workgroup
constexpr int kGrp = 16;              // lanes per column pair (kST / kGrp >= kSvd / 2)
constexpr double kDrop = 1e-14;       // dependent-row threshold (relative)
constexpr int kMaxN = 4096;           // mode sizes (L <= 8192)

__device__ inline double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Element e of row j: base[j * rs + (e / seg) * ss + e % seg].  Covers
// contiguous rows (seg = row length) and every unfolding of a C-order
// 3-tensor without copies.
struct RowView {
  const double *base;
  int64_t rs;
  int64_t ss;
  int64_t seg;
};

// Orthonormal rows spanning the k rows of Y, by classical Gram-Schmidt with
// one reorthogonalisation, one workgroup per chunk of `chunk` points
// (points [c chunk, min(len, (c + 1) chunk)) for workgroup c).  Workgroup c
// writes its orthonormal rows to Q + c kmax chunk (row stride chunk) and the
// coefficients of row j on them to C[j ldc + c kmax + i] (i < kmax; zero
// beyond the rows kept so far), so that row j = sum_i C[j][c kmax + i] q_i
// on the chunk, up to dropped residuals.  A row whose residual norm is at most
// drop times its norm is dependent and adds no basis row.  kout[c] = number
// kept, kmax + 1 if an independent row found the basis full.  Thread t owns
// the points t + kOT e of the chunk: the basis rows it writes are the ones it
// reads back.
template <int PER, int GRP>
__global__ __launch_bounds__(kOT) void k_orth(RowView Y, int k, int len, int chunk, double *__restrict__ Q, int kmax,
                                              double *__restrict__ C, int ldc, int *__restrict__ kout, double drop) {
  __shared__ double part[kOT / 64][kOMax];
  __shared__ double coef[kOMax];
  __shared__ double acc[kOMax];
  __shared__ double red[kOT / 64];
  const int c = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int e0 = c * chunk, m = min(chunk, len - e0);
  double *Qc = Q + size_t(c) * kmax * chunk;
  auto block_sum = [&](double x) {
    x = wave_sum(x);
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kOT / 64; ++w) t += red[w];
    __syncthreads();
    return t;
  };
  int kept = 0;
  bool overflow = false;
  for (int j = 0; j < k; ++j) {
    double v[PER];
    double sq = 0.0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int x = tid + kOT * e;
      v[e] = 0.0;
      if (x < m) {
        const int64_t g = e0 + x;
        v[e] = Y.base[j * Y.rs + (g / Y.seg) * Y.ss + g % Y.seg];
      }
      sq += v[e] * v[e];
    }
    const double nrm0 = block_sum(sq);
    for (int i = tid; i < kept; i += kOT) acc[i] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      // dot products with the basis rows, GRP at a time so that their loads
      // and cross-lane reductions overlap
      for (int i0 = 0; i0 < kept; i0 += GRP) {
        double d[GRP];
#pragma unroll
        for (int u = 0; u < GRP; ++u) d[u] = 0.0;
#pragma unroll
        for (int u = 0; u < GRP; ++u) {
          if (i0 + u < kept) {
            const double *qi = Qc + size_t(i0 + u) * chunk;
#pragma unroll
            for (int e = 0; e < PER; ++e) {
              const int x = tid + kOT * e;
              if (x < m) d[u] += qi[x] * v[e];
            }
          }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
          for (int u = 0; u < GRP; ++u) d[u] += __shfl_xor(d[u], o);
        }
        if (lane == 0) {
#pragma unroll
          for (int u = 0; u < GRP; ++u)
            if (i0 + u < kept) part[wave][i0 + u] = d[u];
        }
      }
      __syncthreads();
      for (int i = tid; i < kept; i += kOT) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kOT / 64; ++w) s += part[w][i];
        coef[i] = s;
        acc[i] += s;
      }
      __syncthreads();
      // v -= sum_i coef_i q_i: short chunks load GRP basis rows at a time
      // (long chunks have no registers for that)
      if constexpr (PER >= 16) {
#pragma unroll 4
        for (int i = 0; i < kept; ++i) {
          const double cf = coef[i];
          const double *qi = Qc + size_t(i) * chunk;
#pragma unroll
          for (int e = 0; e < PER; ++e) {
            const int x = tid + kOT * e;
            if (x < m) v[e] -= cf * qi[x];
          }
        }
      } else {
        for (int i0 = 0; i0 < kept; i0 += GRP) {
          double qv[GRP][PER];
#pragma unroll
          for (int u = 0; u < GRP; ++u) {
            const double *qi = Qc + size_t(i0 + u) * chunk;
#pragma unroll
            for (int e = 0; e < PER; ++e) {
              const int x = tid + kOT * e;
              qv[u][e] = (i0 + u < kept && x < m) ? qi[x] : 0.0;
            }
          }
#pragma unroll
          for (int u = 0; u < GRP; ++u) {
            const double cf = i0 + u < kept ? coef[i0 + u] : 0.0;
#pragma unroll
            for (int e = 0; e < PER; ++e) v[e] -= cf * qv[u][e];
          }
        }
      }
    }
    sq = 0.0;
#pragma unroll
    for (int e = 0; e < PER; ++e) sq += v[e] * v[e];
    const double nrm = block_sum(sq);
    const bool indep = nrm > 0.0 && nrm > drop * drop * nrm0;
    if (indep && kept == kmax) overflow = true;
    const bool keep = indep && kept < kmax;
    double *Cj = C + size_t(j) * ldc + size_t(c) * kmax;
    for (int i = tid; i < kmax; i += kOT) Cj[i] = i < kept ? acc[i] : ((keep && i == kept) ? sqrt(nrm) : 0.0);
    if (keep) {
      const double inv = 1.0 / sqrt(nrm);
      double *qk = Qc + size_t(kept) * chunk;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int x = tid + kOT * e;
        if (x < m) qk[x] = v[e] * inv;
      }
      ++kept;
    }
  }
  if (tid == 0) kout[c] = overflow ? kmax + 1 : kept;
}

// Basis rows of the two-level Gram-Schmidt: Q[i][c chunk + x] =
// sum_(a < kout[c]) Q2[i][c kmax1 + a] Qs[c][a][x] for i < *rho (chunk c's
// basis rows past kout[c] were never written and are not read).
__global__ __launch_bounds__(256) void k_tsqr_rows(const double *__restrict__ Qs, int kmax1, int chunk, int len,
                                                   const int *__restrict__ kout, const double *__restrict__ Q2, int ld2,
                                                   const int *__restrict__ rho, int kmax, double *__restrict__ Q) {
  const int c = blockIdx.y, xl = blockIdx.x * 256 + threadIdx.x, i0 = blockIdx.z * 8;
  const int x = c * chunk + xl;
  const int nr = min(*rho, kmax);
  if (xl >= chunk || x >= len || i0 >= nr) return;
  const int ka = min(kout[c], kmax1);
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0;
  const double *qs = Qs + size_t(c) * kmax1 * chunk + xl;
  for (int a = 0; a < ka; ++a) {
    const double v = qs[size_t(a) * chunk];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u < nr) acc[u] += Q2[size_t(i0 + u) * ld2 + size_t(c) * kmax1 + a] * v;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u)
    if (i0 + u < nr) Q[size_t(i0 + u) * len + x] = acc[u];
}

// Singular values and left singular vectors of the m x c matrix C (row
// stride ldc, m, c <= kSvd) by one-sided Jacobi on its columns: pairs of
// columns (round-robin order) are rotated until every pair is orthogonal to
// 1e-15 of the product of their norms; then C J = U diag(sig).  One group of
// kGrp lanes per pair, so all disjoint pairs of a step run at once.  Outputs
// sig[0..c) descending and U[i ldu + k] = column k of U (zero for a zero
// singular value).
__device__ inline double group_sum(double x) {
#pragma unroll
  for (int o = kGrp / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kGrp);
  return x;
}
__global__ __launch_bounds__(kST) void k_svd_cols(const double *__restrict__ C, int ldc, int m, int c,
                                                  double *__restrict__ sig, double *__restrict__ U, int ldu) {
  extern __shared__ double col[];   // column k at col + k * LD
  __shared__ double gmax[kST / kGrp];
  __shared__ double nrm[kSvd];
  __shared__ int stop;
  const int tid = threadIdx.x, grp = tid / kGrp, gl = tid % kGrp;
  const int cp = c + (c & 1), LD = m + 1;
  for (int e = tid; e < cp * m; e += kST) {
    const int k = e / m, i = e - k * m;
    col[k * LD + i] = k < c ? C[size_t(i) * ldc + k] : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60 && cp >= 2; ++sweep) {
    double off = 0.0;
    for (int step = 0; step < cp - 1; ++step) {
      if (grp < cp / 2) {
        auto idx = [&](int t) { return t == 0 ? 0 : 1 + (t - 1 + step) % (cp - 1); };
        double *x = col + idx(grp) * LD, *y = col + idx(cp - 1 - grp) * LD;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = gl; i < m; i += kGrp) {
          a += x[i] * x[i];
          b += y[i] * y[i];
          g += x[i] * y[i];
        }
        a = group_sum(a);
        b = group_sum(b);
        g = group_sum(g);
        if (fabs(g) > 1e-300 && fabs(g) > 1e-15 * sqrt(a * b)) {
          off = fmax(off, fabs(g) / sqrt(a * b));
          const double zeta = (b - a) / (2.0 * g);
          const double t = fabs(zeta) > 1e150 ? 0.5 / zeta
                                               : (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int i = gl; i < m; i += kGrp) {
            const double xi = x[i], yi = y[i];
            x[i] = cs * xi - sn * yi;
            y[i] = sn * xi + cs * yi;
          }
        }
      }
      __syncthreads();
    }
    if (gl == 0) gmax[grp] = off;
    __syncthreads();
    if (tid == 0) {
      double mx = 0.0;
      for (int w = 0; w < kST / kGrp; ++w) mx = fmax(mx, gmax[w]);
      stop = !(mx > 1e-15);
    }
    __syncthreads();
    if (stop) break;
  }
  for (int k = grp; k < c; k += kST / kGrp) {
    double s = 0.0;
    for (int i = gl; i < m; i += kGrp) s += col[k * LD + i] * col[k * LD + i];
    s = group_sum(s);
    if (gl == 0) nrm[k] = sqrt(s);
  }
  __syncthreads();
  for (int k = tid; k < c; k += kST) {
    const double s = nrm[k];
    int rank = 0;
    for (int j = 0; j < c; ++j)
      if (nrm[j] > s || (nrm[j] == s && j < k)) ++rank;
    sig[rank] = s;
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int i = 0; i < m; ++i) U[size_t(i) * ldu + rank] = col[k * LD + i] * inv;
  }
}

// Y = X x_p A for X of dims (d0, d1, d2), C order: Y(.., j, ..) =
// sum_i A[j sa + i sb] X(.., i, ..), j < J; with acc set, added to Y.
__global__ __launch_bounds__(256) void k_mode_mul(const double *__restrict__ X, int d0, int d1, int d2, int p,
                                                  const double *__restrict__ A, int64_t sa, int64_t sb, int J,
                                                  double *__restrict__ Y, int acc) {
  const int e0 = p == 0 ? J : d0, e1 = p == 1 ? J : d1, e2 = p == 2 ? J : d2;
  const int64_t total = int64_t(e0) * e1 * e2;
  const int dp = p == 0 ? d0 : (p == 1 ? d1 : d2);
  const int64_t step = p == 0 ? int64_t(d1) * d2 : (p == 1 ? d2 : 1);
  for (int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; o < total; o += int64_t(gridDim.x) * blockDim.x) {
    const int c = int(o % e2), b = int((o / e2) % e1), a = int(o / (int64_t(e1) * e2));
    const int j = p == 0 ? a : (p == 1 ? b : c);
    const int64_t base = (int64_t(p == 0 ? 0 : a) * d1 + (p == 1 ? 0 : b)) * d2 + (p == 2 ? 0 : c);
    double s = 0.0;
    for (int i = 0; i < dp; ++i) s += A[j * sa + i * sb] * X[base + i * step];
    Y[o] = acc ? Y[o] + s : s;
  }
}

// E[(l0 k0 + i0)][(l1 k1 + i1)][(l2 k2 + i2)] = D[l0][l1][l2] K[i0][i1][i2]
// (Eq. (t_had2): D the magnetization core, ranks r; K the kernel core, ranks k).
__global__ __launch_bounds__(256) void k_kron3(const double *__restrict__ D, int r0, int r1, int r2,
                                               const double *__restrict__ K, int k0, int k1, int k2,
                                               double *__restrict__ E) {
  const int E1 = r1 * k1, E2 = r2 * k2;
  const int64_t total = int64_t(r0 * k0) * E1 * E2;
  for (int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; o < total; o += int64_t(gridDim.x) * blockDim.x) {
    const int c = int(o % E2), b = int((o / E2) % E1), a = int(o / (int64_t(E1) * E2));
    const double d = D[(int64_t(a / k0) * r1 + b / k1) * r2 + c / k2];
    const double kk = K[(int64_t(a % k0) * k1 + b % k1) * k2 + c % k2];
    E[o] = d * kk;
  }
}

// Core of a CP tensor in orthonormal bases: G[a][b][c] = sum_t C0[t][a]
// C1[t][b] C2[t][c] (C_p[t][i] = coefficient of term t's mode-p row on basis
// row i, row stride ld).
__global__ __launch_bounds__(256) void k_cp_core(const double *__restrict__ C0, const double *__restrict__ C1,
                                                 const double *__restrict__ C2, int ld, int T, int g0, int g1, int g2,
                                                 double *__restrict__ G) {
  const int64_t total = int64_t(g0) * g1 * g2;
  for (int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; o < total; o += int64_t(gridDim.x) * blockDim.x) {
    const int c = int(o % g2), b = int((o / g2) % g1), a = int(o / (int64_t(g1) * g2));
    double s = 0.0;
    for (int t = 0; t < T; ++t) s += C0[size_t(t) * ld + a] * C1[size_t(t) * ld + b] * C2[size_t(t) * ld + c];
    G[o] = s;
  }
}

// out[k ldo + x] = sum_i V[i ldv + k] Q[i ldq + x] for k < r, x < len, i < rho.
__global__ __launch_bounds__(256) void k_rows_combine(const double *__restrict__ V, int ldv, const double *__restrict__ Q,
                                                      int64_t ldq, int rho, int r, int len, double *__restrict__ out,
                                                      int64_t ldo) {
  constexpr int kB = 8;
  const int x = blockIdx.x * 256 + threadIdx.x, k0 = blockIdx.y * kB;
  if (x >= len) return;
  double a[kB];
#pragma unroll
  for (int u = 0; u < kB; ++u) a[u] = 0.0;
  for (int i = 0; i < rho; ++i) {
    const double q = Q[i * ldq + x];
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (k0 + u < r) a[u] += V[size_t(i) * ldv + k0 + u] * q;
  }
#pragma unroll
  for (int u = 0; u < kB; ++u)
    if (k0 + u < r) out[(k0 + u) * ldo + x] = a[u];
}

// Sum of squares: one partial per workgroup.
__global__ __launch_bounds__(256) void k_sumsq(const double *__restrict__ x, int64_t count, double *__restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < count; i += int64_t(gridDim.x) * 256) s += x[i] * x[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_zero(double *__restrict__ x, int64_t count) {
  for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < count; i += int64_t(gridDim.x) * 256) x[i] = 0.0;
}

// x = (1, 0, 0, ...): the basis of a set of rows that are all zero.
__global__ __launch_bounds__(256) void k_unit(double *__restrict__ x, int64_t count) {
  for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < count; i += int64_t(gridDim.x) * 256)
    x[i] = i == 0 ? 1.0 : 0.0;
}

// DFT (L points, zero-padded) of the nrows real rows (length len, stride ld):
// rows 2w and 2w + 1 go through one complex transform z = a + i b, then
// A_f = (z_f + conj z_{-f}) / 2, B_f = (z_f - conj z_{-f}) / (2i).  spec
// [nrows][L].
template <int KT, int KP>
__global__ __launch_bounds__(KT) void k_row_spectra(const double *__restrict__ rows, int64_t ld, int len, int nrows,
                                                    int L, cplx *__restrict__ spec) {
  extern __shared__ cplx lds[];
  cplx *buf = lds, *tlo = lds + fftc::cap(KP), *thi = tlo + 64;
  fftc::make_twiddles(tlo, thi, L);
  const int a = 2 * blockIdx.x, b = a + 1;
  const double *ra = rows + a * ld;
  const double *rb = b < nrows ? rows + b * ld : nullptr;
  for (int x = threadIdx.x; x < L; x += KT)
    buf[fftc::pd(x)] = cplx{x < len ? ra[x] : 0.0, (rb != nullptr && x < len) ? rb[x] : 0.0};
  __syncthreads();
  fftc::fft_lines<false, KT, KP>(buf, L, fftc::line_stride(L, 1), 1, tlo, thi);
  for (int f = threadIdx.x; f < L; f += KT) {
    const cplx zf = buf[fftc::pd(f)], zc = fftc::cconj(buf[fftc::pd((L - f) & (L - 1))]);
    spec[size_t(a) * L + f] = cplx{0.5 * (zf.x + zc.x), 0.5 * (zf.y + zc.y)};
    if (rb != nullptr) spec[size_t(b) * L + f] = cplx{0.5 * (zf.y - zc.y), -0.5 * (zf.x - zc.x)};
  }
}

// Factor rows of the Hadamard product in Fourier space, transformed back:
// row t = l rk + i (l < rm a magnetization row, i < rk a kernel row) is the
// window [n - 1, 2n - 1) of IDFT(SK[i] SM[l]) (the Toeplitz product of the
// kernel generator with the magnetization row).  Rows 2w and 2w + 1 share one
// inverse transform: IDFT(P + i P') = p + i p' for real p, p'.
template <int KT, int KP>
__global__ __launch_bounds__(KT) void k_conv_rows(const cplx *__restrict__ SK, int rk, const cplx *__restrict__ SM,
                                                  int rm, int L, int n, double *__restrict__ out, int64_t ldo) {
  extern __shared__ cplx lds[];
  cplx *buf = lds, *tlo = lds + fftc::cap(KP), *thi = tlo + 64;
  fftc::make_twiddles(tlo, thi, L);
  const int T = rk * rm;
  const int t1 = 2 * blockIdx.x, t2 = t1 + 1;
  const bool two = t2 < T;
  const cplx *k1 = SK + size_t(t1 % rk) * L, *m1 = SM + size_t(t1 / rk) * L;
  const cplx *k2 = two ? SK + size_t(t2 % rk) * L : nullptr, *m2 = two ? SM + size_t(t2 / rk) * L : nullptr;
  for (int f = threadIdx.x; f < L; f += KT) {
    cplx z = fftc::cmul(k1[f], m1[f]);
    if (two) {
      const cplx w = fftc::cmul(k2[f], m2[f]);
      z = cplx{z.x - w.y, z.y + w.x};
    }
    buf[fftc::pd(f)] = z;
  }
  __syncthreads();
  fftc::fft_lines<true, KT, KP>(buf, L, fftc::line_stride(L, 1), 1, tlo, thi);
  const double s = 1.0 / double(L);
  for (int j = threadIdx.x; j < n; j += KT) {
    const cplx z = buf[fftc::pd(j + n - 1)];
    out[t1 * ldo + j] = z.x * s;
    if (two) out[t2 * ldo + j] = z.y * s;
  }
}

// CP -> TT (ranks (R, R)): G2[a][b][j] = (a == b) lam_a U2[a][j].
__global__ __launch_bounds__(256) void k_cp_tt_mid(const double *__restrict__ lam, const double *__restrict__ U2, int R,
                                                   int n, double *__restrict__ G2) {
  const int64_t total = int64_t(R) * R * n;
  for (int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; o < total; o += int64_t(gridDim.x) * blockDim.x) {
    const int j = int(o % n), b = int((o / n) % R), a = int(o / (int64_t(n) * R));
    G2[o] = a == b ? lam[a] * U2[int64_t(a) * n + j] : 0.0;
  }
}

// Tucker -> TT middle core: G2[a][c][j] = sum_b core[a][b][c] U2[b][j].
__global__ __launch_bounds__(256) void k_tucker_tt_mid(const double *__restrict__ core, int r0, int r1, int r2,
                                                       const double *__restrict__ U2, int n, double *__restrict__ G2) {
  const int64_t total = int64_t(r0) * r2 * n;
  for (int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; o < total; o += int64_t(gridDim.x) * blockDim.x) {
    const int j = int(o % n), c = int((o / n) % r2), a = int(o / (int64_t(n) * r2));
    double s = 0.0;
    for (int b = 0; b < r1; ++b) s += core[(int64_t(a) * r1 + b) * r2 + c] * U2[int64_t(b) * n + j];
    G2[o] = s;
  }
}

// TT -> Tucker core in the fibres' basis: core[a][i][b] = C[(a r2 + b) ldc + i]
// (C: coefficients of fibre G2[a, b, :] on basis row i), i < rho.
__global__ __launch_bounds__(256) void k_tt_core(const double *__restrict__ C, int ldc, int r1, int r2, int rho,
                                                 double *__restrict__ core) {
  const int64_t total = int64_t(r1) * rho * r2;
  for (int64_t o = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; o < total; o += int64_t(gridDim.x) * blockDim.x) {
    const int b = int(o % r2), i = int((o / r2) % rho), a = int(o / (int64_t(r2) * rho));
    core[o] = C[(int64_t(a) * r2 + b) * ldc + i];
  }
}

// ------------------------------------------------------------------ host side

int dft_length(int n) {
  int L = 1;
  while (L < 2 * n - 1) L <<= 1;
  return L;
}

// Device buffers of one call, freed when it returns, after the stream has
// drained.
struct DevMem {
  hipStream_t stream;
  std::vector<void *> ptrs;
  bool failed = false;
  explicit DevMem(hipStream_t s) : stream(s) {}
  template <class T> T *get(size_t count) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
      failed = true;
      return nullptr;
    }
    ptrs.push_back(p);
    return static_cast<T *>(p);
  }
  ~DevMem() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(stream);
    for (void *p : ptrs) (void)hipFree(p);
  }
};

#define TK_ALLOC(var, T, count)                                   \
  T *var = mem.get<T>(count);                                     \
  do {                                                            \
    if (var == nullptr) {                                         \
      set_error("tucker: device allocation failed");              \
      return DEMAG_E_NOMEM;                                       \
    }                                                             \
  } while (0)

#define TK_LAUNCH()                                               \
  do {                                                            \
    hipError_t e_ = hipGetLastError();                            \
    if (e_ != hipSuccess) {                                       \
      set_error(std::string("tucker: launch: ") + hipGetErrorString(e_)); \
      return DEMAG_E_HIP;                                         \
    }                                                             \
  } while (0)

int grid_for(int64_t total) { return int(std::min<int64_t>((total + 255) / 256, 4096)); }

RowView contiguous(const double *base, int64_t ld, int64_t len) { return RowView{base, ld, 0, std::max<int64_t>(len, 1)}; }

// Rows of the mode-p unfolding of a C-order tensor of dims d (row count d[p]).
RowView unfolding(const double *T, const int d[3], int p) {
  const int64_t d12 = int64_t(d[1]) * d[2];
  if (p == 0) return RowView{T, d12, 0, std::max<int64_t>(d12, 1)};
  if (p == 1) return RowView{T, d[2], d12, std::max(d[2], 1)};
  return RowView{T, 1, d[2], 1};
}

// k_orth with the points per thread sized to the chunk: short chunks keep
// more basis rows' loads in flight.
void launch_orth(hipStream_t st, int grid, RowView Y, int k, int len, int chunk, double *Q, int kmax, double *C,
                 int ldc, int *kout) {
  if (chunk <= kOT * 4)
    k_orth<4, 16><<<grid, kOT, 0, st>>>(Y, k, len, chunk, Q, kmax, C, ldc, kout, kDrop);
  else
    k_orth<kOPer, 4><<<grid, kOT, 0, st>>>(Y, k, len, chunk, Q, kmax, C, ldc, kout, kDrop);
}

// Orthonormal basis of the k rows of Y (length len <= 16384 chunks): basis
// rows Q [kmax][len] (only with want_q), coefficients C [k][kmax], basis size
// *rho.  Short rows: Gram-Schmidt in one workgroup.  Longer rows: every chunk
// of the points in a workgroup of its own (bases Qs, coefficients C1 of the
// rows on them, stacked per row), then Gram-Schmidt of the stacked
// coefficient rows (bases Q2, coefficients C): row j = sum_i C[j][i] q_i with
// q_i = sum_(c, a) Q2[i][(c, a)] (chunk c's basis row a).  The chunk count
// balances the two levels (about sqrt(len / k) chunks).
demag_status orth_rows(demag_ctx *ctx, DevMem &mem, RowView Y, int k, int64_t len, int kmax, bool want_q, double **Q,
                       double **C, int *rho) {
  DEMAG_REQUIRE(k >= 1 && k <= kOMax && len >= 1 && kmax >= 1 && kmax <= kOMax,
                "tucker: orthonormalisation of " + std::to_string(k) + " rows exceeds its limits");
  int64_t nch = 1;
  if (len > 2048) nch = std::max<int64_t>(2, std::llround(std::sqrt(double(len) / std::min(k, kSvd))));
  int64_t chunk = (len + nch - 1) / nch;
  int kmax1 = int(std::min<int64_t>(k, chunk));
  while (nch > 1 && nch * kmax1 > kOLen) {
    nch = kOLen / kmax1;
    chunk = (len + nch - 1) / nch;
    kmax1 = int(std::min<int64_t>(k, chunk));
  }
  DEMAG_REQUIRE(chunk <= kOLen, "tucker: rows of " + std::to_string(len) + " points are too long");
  nch = (len + chunk - 1) / chunk;
  TK_ALLOC(c, double, size_t(k) * kmax);
  TK_ALLOC(ko, int, 1);
  double *q = nullptr;
  if (nch == 1) {
    TK_ALLOC(q1, double, size_t(kmax) * len);
    launch_orth(ctx->stream, 1, Y, k, int(len), int(len), q1, kmax, c, kmax, ko);
    TK_LAUNCH();
    q = q1;
  } else {
    const int ld1 = int(nch) * kmax1;
    TK_ALLOC(Qs, double, size_t(nch) * kmax1 * chunk);
    TK_ALLOC(C1, double, size_t(k) * ld1);
    TK_ALLOC(ko1, int, nch);
    launch_orth(ctx->stream, int(nch), Y, k, int(len), int(chunk), Qs, kmax1, C1, ld1, ko1);
    TK_LAUNCH();
    TK_ALLOC(Q2, double, size_t(kmax) * ld1);
    launch_orth(ctx->stream, 1, contiguous(C1, ld1, ld1), k, ld1, ld1, Q2, kmax, c, kmax, ko);
    TK_LAUNCH();
    if (want_q) {
      TK_ALLOC(qq, double, size_t(kmax) * len);
      dim3 g(unsigned((chunk + 255) / 256), unsigned(nch), unsigned((kmax + 7) / 8));
      k_tsqr_rows<<<g, 256, 0, ctx->stream>>>(Qs, kmax1, int(chunk), int(len), ko1, Q2, ld1, ko, kmax, qq);
      TK_LAUNCH();
      q = qq;
    }
  }
  int h = 0;
  DEMAG_TRY_HIP(hipMemcpyAsync(&h, ko, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
  if (h > kmax) {
    set_error("tucker: more than " + std::to_string(kmax) + " independent rows");
    return DEMAG_E_UNSUPPORTED;
  }
  if (h == 0) {
    // every row is zero (a zero tensor): one unit basis row, zero coefficients
    if (q != nullptr) {
      k_unit<<<grid_for(len), 256, 0, ctx->stream>>>(q, len);
      TK_LAUNCH();
    }
    h = 1;
  }
  *Q = q;
  *C = c;
  *rho = h;
  return DEMAG_OK;
}

// Singular values (host, descending) and left singular vectors U [m][kSvd]
// (device, column k = vector k) of the m rows of Y (length len): the rows'
// coefficients on an orthonormal basis, then one-sided Jacobi.
demag_status svd_rows(demag_ctx *ctx, DevMem &mem, RowView Y, int m, int64_t len, std::vector<double> &sig,
                      double **U) {
  DEMAG_REQUIRE(m >= 1 && m <= kSvd, "tucker: more than " + std::to_string(kSvd) + " rows in one mode");
  double *C = nullptr, *Q = nullptr;
  int kc = 0;
  demag_status st = orth_rows(ctx, mem, Y, m, len, m, false, &Q, &C, &kc);
  if (st != DEMAG_OK) return st;
  TK_ALLOC(sd, double, kSvd);
  TK_ALLOC(u, double, size_t(m) * kSvd);
  // a zero matrix (unit basis row, zero coefficients): no singular values,
  // and the first unit vector as its only left singular vector
  k_unit<<<grid_for(int64_t(m) * kSvd), 256, 0, ctx->stream>>>(u, int64_t(m) * kSvd);
  TK_LAUNCH();
  sig.assign(kc, 0.0);
  if (kc > 0) {
    const size_t lds = size_t(kc + (kc & 1)) * (m + 1) * sizeof(double);
    k_svd_cols<<<1, kST, lds, ctx->stream>>>(C, m, m, kc, sd, u, kSvd);
    TK_LAUNCH();
    DEMAG_TRY_HIP(hipMemcpyAsync(sig.data(), sd, kc * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
  }
  *U = u;
  return DEMAG_OK;
}

// Smallest r >= 1 whose tail sig[r:] has norm at most bound (the whole
// length if none).
int tail_rank(const std::vector<double> &sig, double bound) {
  const int n = int(sig.size());
  std::vector<double> tail(n + 1, 0.0);
  for (int i = n - 1; i >= 0; --i) tail[i] = tail[i + 1] + sig[i] * sig[i];
  for (int r = 1; r <= n; ++r)
    if (r == n || std::sqrt(tail[r]) <= bound) return r;
  return std::max(n, 1);
}
int tucker_rank(const std::vector<double> &sig, double eps) {
  double tot = 0.0;
  for (double s : sig) tot += s * s;
  if (tot == 0.0) return 1;
  return tail_rank(sig, eps / std::sqrt(3.0) * std::sqrt(tot));
}

demag_status mode_mul(demag_ctx *ctx, const double *X, const int d[3], int p, const double *A, int64_t sa, int64_t sb,
                      int J, double *Y, bool acc) {
  int64_t total = int64_t(J);
  for (int s = 0; s < 3; ++s)
    if (s != p) total *= d[s];
  if (total == 0) return DEMAG_OK;
  k_mode_mul<<<grid_for(total), 256, 0, ctx->stream>>>(X, d[0], d[1], d[2], p, A, sa, sb, J, Y, acc ? 1 : 0);
  TK_LAUNCH();
  return DEMAG_OK;
}

double sum_squares(demag_ctx *ctx, DevMem &mem, const double *x, int64_t count, demag_status *st) {
  const int g = std::max(1, std::min(grid_for(count), 256));
  double *part = mem.get<double>(g);
  if (part == nullptr) {
    *st = DEMAG_E_NOMEM;
    return 0.0;
  }
  k_sumsq<<<g, 256, 0, ctx->stream>>>(x, count, part);
  std::vector<double> h(g);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(h.data(), part, g * sizeof(double), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    *st = DEMAG_E_HIP;
    return 0.0;
  }
  double s = 0.0;
  for (double v : h) s += v;
  *st = DEMAG_OK;
  return s;
}

// HOOI (Alg. HOOI) on the dense core G of dims rho: truncated HOSVD, then
// sweeps until the squared core norm changes by at most 1e-13 relative (at
// most 20).  Outputs: ranks r, bases V[p] [rho_p][kSvd] (first r_p columns),
// core [r0][r1][r2].
struct Hooi {
  int r[3];
  double *V[3];
  double *core;
};
demag_status hooi_core(demag_ctx *ctx, DevMem &mem, const double *G, const int rho[3], double eps, Hooi &out) {
  std::vector<double> sig;
  for (int p = 0; p < 3; ++p) {
    const int64_t len = int64_t(rho[0]) * rho[1] * rho[2] / rho[p];
    demag_status st = svd_rows(ctx, mem, unfolding(G, rho, p), rho[p], len, sig, &out.V[p]);
    if (st != DEMAG_OK) return st;
    out.r[p] = std::min(tucker_rank(sig, eps), int(sig.size()));
    out.r[p] = std::max(out.r[p], 1);
  }
  const int64_t big = int64_t(rho[0]) * rho[1] * rho[2];
  TK_ALLOC(t1, double, big);
  TK_ALLOC(t2, double, big);
  TK_ALLOC(core, double, big);
  auto project = [&](int skip, int dims_out[3]) -> demag_status {
    // t2 = G x_s V_s^T for the modes s != skip (skip = -1: all three, into core)
    const double *src = G;
    int d[3] = {rho[0], rho[1], rho[2]};
    int done = 0, nmodes = skip < 0 ? 3 : 2;
    for (int s = 0; s < 3; ++s) {
      if (s == skip) continue;
      double *dst = (++done == nmodes) ? (skip < 0 ? core : t2) : (src == t1 ? t2 : t1);
      demag_status st = mode_mul(ctx, src, d, s, out.V[s], 1, kSvd, out.r[s], dst, false);
      if (st != DEMAG_OK) return st;
      d[s] = out.r[s];
      src = dst;
    }
    for (int s = 0; s < 3; ++s) dims_out[s] = d[s];
    return DEMAG_OK;
  };
  double prev = -1.0;
  for (int sweep = 0; sweep < 20; ++sweep) {
    for (int p = 0; p < 3; ++p) {
      int d[3];
      demag_status st = project(p, d);
      if (st != DEMAG_OK) return st;
      st = svd_rows(ctx, mem, unfolding(t2, d, p), d[p], int64_t(d[0]) * d[1] * d[2] / d[p], sig, &out.V[p]);
      if (st != DEMAG_OK) return st;
      out.r[p] = std::max(1, std::min(tucker_rank(sig, eps), int(sig.size())));
    }
    int d[3];
    demag_status st = project(-1, d);
    if (st != DEMAG_OK) return st;
    const double fit = sum_squares(ctx, mem, core, int64_t(d[0]) * d[1] * d[2], &st);
    if (st != DEMAG_OK) return st;
    if (prev >= 0.0 && std::fabs(fit - prev) <= 1e-13 * std::max(fit, 1e-300)) break;
    prev = fit;
  }
  out.core = core;
  return DEMAG_OK;
}

template <int KT, int KP>
size_t fft_lds() {
  return size_t(fftc::cap(KP) + 128) * sizeof(cplx);
}

demag_status set_fft_attrs(int device) {
  static std::mutex mu;
  static uint64_t done = 0;   // one bit per device
  std::lock_guard<std::mutex> lock(mu);
  if (device < 64 && ((done >> device) & 1u)) return DEMAG_OK;
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_row_spectra<256, 4096>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(fft_lds<256, 4096>())));
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_row_spectra<512, 8192>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(fft_lds<512, 8192>())));
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv_rows<256, 4096>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(fft_lds<256, 4096>())));
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv_rows<512, 8192>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(fft_lds<512, 8192>())));
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_svd_cols),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    int(size_t(kSvd) * (kSvd + 1) * sizeof(double))));
  if (device < 64) done |= uint64_t(1) << device;
  return DEMAG_OK;
}

demag_status row_spectra(demag_ctx *ctx, const double *rows, int64_t ld, int len, int nrows, int L, cplx *spec) {
  const int g = (nrows + 1) / 2;
  if (L <= 4096)
    k_row_spectra<256, 4096><<<g, 256, fft_lds<256, 4096>(), ctx->stream>>>(rows, ld, len, nrows, L, spec);
  else
    k_row_spectra<512, 8192><<<g, 512, fft_lds<512, 8192>(), ctx->stream>>>(rows, ld, len, nrows, L, spec);
  TK_LAUNCH();
  return DEMAG_OK;
}

demag_status conv_rows(demag_ctx *ctx, const cplx *SK, int rk, const cplx *SM, int rm, int L, int n, double *out) {
  const int g = (rk * rm + 1) / 2;
  if (L <= 4096)
    k_conv_rows<256, 4096><<<g, 256, fft_lds<256, 4096>(), ctx->stream>>>(SK, rk, SM, rm, L, n, out, n);
  else
    k_conv_rows<512, 8192><<<g, 512, fft_lds<512, 8192>(), ctx->stream>>>(SK, rk, SM, rm, L, n, out, n);
  TK_LAUNCH();
  return DEMAG_OK;
}

// A Tucker tensor on the device: core [r0][r1][r2], rows[p] [r_p][len_p].
struct DTucker {
  int r[3];
  const double *core;
  const double *rows[3];
};

// Approximate summation (and single-tensor recompression) of Tucker tensors
// with mode sizes n: the rows of every term side by side are
// orthonormalised per mode, the sum's core in those bases is accumulated term
// by term (core x_p C_p^T), and HOOI with eps runs on it.  Result: ranks
// r, core (device, from mem), rows[p] [r_p][n_p] (device, from mem).
struct TuckerOut {
  int r[3];
  double *core;
  double *rows[3];
};
demag_status recompress_sum(demag_ctx *ctx, DevMem &mem, const int n[3], const std::vector<DTucker> &terms, double eps,
                            TuckerOut &out) {
  double *Q[3], *Cf[3];
  int rho[3], tot[3];
  for (int p = 0; p < 3; ++p) {
    tot[p] = 0;
    for (const DTucker &t : terms) tot[p] += t.r[p];
    DEMAG_REQUIRE(tot[p] <= kOMax, "tucker: more than " + std::to_string(kOMax) + " factor rows in one mode");
    TK_ALLOC(all, double, size_t(tot[p]) * n[p]);
    int off = 0;
    for (const DTucker &t : terms) {
      DEMAG_TRY_HIP(hipMemcpyAsync(all + size_t(off) * n[p], t.rows[p], size_t(t.r[p]) * n[p] * sizeof(double),
                                   hipMemcpyDeviceToDevice, ctx->stream));
      off += t.r[p];
    }
    demag_status st = orth_rows(ctx, mem, contiguous(all, n[p], n[p]), tot[p], n[p], std::min(tot[p], kSvd), true,
                                &Q[p], &Cf[p], &rho[p]);
    if (st == DEMAG_E_UNSUPPORTED && tot[p] > kSvd) {
      set_error("tucker: the factor rows of one mode span more than " + std::to_string(kSvd) + " dimensions");
      return DEMAG_E_UNSUPPORTED;
    }
    if (st != DEMAG_OK) return st;
    rho[p] = std::max(rho[p], 1);
  }
  const int64_t gsize = int64_t(rho[0]) * rho[1] * rho[2];
  TK_ALLOC(G, double, gsize);
  k_zero<<<grid_for(gsize), 256, 0, ctx->stream>>>(G, gsize);
  TK_LAUNCH();
  // scratch for the partial mode products of one term
  int64_t big = 0;
  for (const DTucker &t : terms) {
    big = std::max(big, int64_t(rho[0]) * t.r[1] * t.r[2]);
    big = std::max(big, int64_t(rho[0]) * rho[1] * t.r[2]);
  }
  TK_ALLOC(s1, double, big);
  TK_ALLOC(s2, double, big);
  int off[3] = {0, 0, 0};
  for (const DTucker &t : terms) {
    int d[3] = {t.r[0], t.r[1], t.r[2]};
    // mode p: A[j][i] = coefficient of the term's row i on basis row j = Cf[p][(off + i) kmax + j]
    const int ldc[3] = {std::min(tot[0], kSvd), std::min(tot[1], kSvd), std::min(tot[2], kSvd)};
    demag_status st = mode_mul(ctx, t.core, d, 0, Cf[0] + size_t(off[0]) * ldc[0], 1, ldc[0], rho[0], s1, false);
    if (st != DEMAG_OK) return st;
    d[0] = rho[0];
    st = mode_mul(ctx, s1, d, 1, Cf[1] + size_t(off[1]) * ldc[1], 1, ldc[1], rho[1], s2, false);
    if (st != DEMAG_OK) return st;
    d[1] = rho[1];
    st = mode_mul(ctx, s2, d, 2, Cf[2] + size_t(off[2]) * ldc[2], 1, ldc[2], rho[2], G, true);
    if (st != DEMAG_OK) return st;
    for (int p = 0; p < 3; ++p) off[p] += t.r[p];
  }
  Hooi h;
  demag_status st = hooi_core(ctx, mem, G, rho, eps, h);
  if (st != DEMAG_OK) return st;
  for (int p = 0; p < 3; ++p) {
    out.r[p] = h.r[p];
    TK_ALLOC(rows, double, size_t(h.r[p]) * n[p]);
    dim3 g((n[p] + 255) / 256, (h.r[p] + 7) / 8);
    k_rows_combine<<<g, 256, 0, ctx->stream>>>(h.V[p], kSvd, Q[p], n[p], rho[p], h.r[p], n[p], rows, n[p]);
    TK_LAUNCH();
    out.rows[p] = rows;
  }
  out.core = h.core;
  return DEMAG_OK;
}

demag_status copy_out(demag_ctx *ctx, const TuckerOut &t, const int n[3], int32_t rmax, int32_t rout[3], double *core,
                      double *const rows[3]) {
  for (int p = 0; p < 3; ++p) rout[p] = t.r[p];
  for (int p = 0; p < 3; ++p)
    if (t.r[p] > rmax) {
      set_error("tucker: rank " + std::to_string(t.r[p]) + " exceeds rmax " + std::to_string(rmax));
      return DEMAG_E_UNSUPPORTED;
    }
  DEMAG_TRY_HIP(hipMemcpyAsync(core, t.core, size_t(t.r[0]) * t.r[1] * t.r[2] * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
  for (int p = 0; p < 3; ++p)
    DEMAG_TRY_HIP(hipMemcpyAsync(rows[p], t.rows[p], size_t(t.r[p]) * n[p] * sizeof(double), hipMemcpyDeviceToDevice,
                                 ctx->stream));
  DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
  return DEMAG_OK;
}

}  // namespace
}  // namespace demag

using namespace demag;

// Compressed kernels of one factor set (Alg. scpot_fft_tucker, set-up).
struct demag_ktucker {
  int n[3], L[3];
  int r[3][3];                 // [component][mode]
  double tol;
  double *core[3] = {nullptr, nullptr, nullptr};
  double *rows[3][3] = {};     // [component][mode] [r][2 n - 1]
  cplx *spec[3][3] = {};       // [component][mode] [r][L]
  int device = 0;
};

extern "C" demag_status demag_ktucker_free(demag_ktucker *kt) {
  if (kt == nullptr) return DEMAG_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(kt->device);
  for (int q = 0; q < 3; ++q) {
    (void)hipFree(kt->core[q]);
    for (int p = 0; p < 3; ++p) {
      (void)hipFree(kt->rows[q][p]);
      (void)hipFree(kt->spec[q][p]);
    }
  }
  (void)hipSetDevice(prev);
  delete kt;
  return DEMAG_OK;
}

extern "C" demag_status demag_ktucker_create(demag_ctx *ctx, const demag_factors *f, double tol, demag_ktucker **out) {
  DEMAG_REQUIRE(ctx != nullptr && f != nullptr && out != nullptr, "demag_ktucker_create: NULL argument");
  *out = nullptr;
  DEMAG_REQUIRE(!f->dense, "demag_ktucker_create: uniform grids only (Toeplitz factors)");
  DEMAG_REQUIRE(tol > 0.0 && tol < 1.0, "demag_ktucker_create: tol must lie in (0, 1)");
  DEMAG_REQUIRE(f->M >= 1 && f->M <= kOMax, "demag_ktucker_create: too many nodes");
  for (int p = 0; p < 3; ++p) {
    DEMAG_REQUIRE(f->n[p] >= 1 && f->n[p] <= kMaxN, "demag_ktucker_create: mode sizes 1..4096");
    DEMAG_REQUIRE(f->f64[p] != nullptr, "demag_ktucker_create: factor tables not assembled");
  }
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  demag_status st = set_fft_attrs(ctx->device);
  if (st != DEMAG_OK) return st;
  auto *kt = new demag_ktucker();
  kt->device = ctx->device;
  kt->tol = tol;
  for (int p = 0; p < 3; ++p) {
    kt->n[p] = f->n[p];
    kt->L[p] = dft_length(f->n[p]);
  }
  const int M = f->M;
  for (int q = 0; q < 3 && st == DEMAG_OK; ++q) {
    DevMem mem(ctx->stream);
    auto body = [&]() -> demag_status {
      double *Q[3], *Cf[3];
      int rho[3];
      for (int p = 0; p < 3; ++p) {
        const int len = 2 * f->n[p] - 1;
        const int type = p == q ? F_X : F_E;
        const double *D = f->f64[p] + size_t(type) * M * len;
        demag_status s = orth_rows(ctx, mem, contiguous(D, len, len), M, len, std::min(M, kSvd), true, &Q[p],
                                   &Cf[p], &rho[p]);
        if (s != DEMAG_OK) return s;
        rho[p] = std::max(rho[p], 1);
      }
      const int ld = std::min(M, kSvd);
      const int64_t gsize = int64_t(rho[0]) * rho[1] * rho[2];
      TK_ALLOC(G, double, gsize);
      k_cp_core<<<grid_for(gsize), 256, 0, ctx->stream>>>(Cf[0], Cf[1], Cf[2], ld, M, rho[0], rho[1], rho[2], G);
      TK_LAUNCH();
      Hooi h;
      demag_status s = hooi_core(ctx, mem, G, rho, tol, h);
      if (s != DEMAG_OK) return s;
      const size_t csize = size_t(h.r[0]) * h.r[1] * h.r[2];
      DEMAG_TRY_HIP(hipMalloc(&kt->core[q], csize * sizeof(double)));
      DEMAG_TRY_HIP(hipMemcpyAsync(kt->core[q], h.core, csize * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
      for (int p = 0; p < 3; ++p) {
        const int len = 2 * f->n[p] - 1;
        kt->r[q][p] = h.r[p];
        DEMAG_TRY_HIP(hipMalloc(&kt->rows[q][p], size_t(h.r[p]) * len * sizeof(double)));
        DEMAG_TRY_HIP(hipMalloc(&kt->spec[q][p], size_t(h.r[p]) * kt->L[p] * sizeof(cplx)));
        dim3 g((len + 255) / 256, (h.r[p] + 7) / 8);
        k_rows_combine<<<g, 256, 0, ctx->stream>>>(h.V[p], kSvd, Q[p], len, rho[p], h.r[p], len, kt->rows[q][p], len);
        TK_LAUNCH();
        s = row_spectra(ctx, kt->rows[q][p], len, len, h.r[p], kt->L[p], kt->spec[q][p]);
        if (s != DEMAG_OK) return s;
      }
      DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
      return DEMAG_OK;
    };
    st = body();
  }
  if (st != DEMAG_OK) {
    demag_ktucker_free(kt);
    return st;
  }
  note_use(ctx, f);
  *out = kt;
  return DEMAG_OK;
}

extern "C" demag_status demag_ktucker_ranks(const demag_ktucker *kt, int32_t q, int32_t r[3]) {
  DEMAG_REQUIRE(kt != nullptr && r != nullptr && q >= 0 && q < 3, "demag_ktucker_ranks: bad argument");
  for (int p = 0; p < 3; ++p) r[p] = kt->r[q][p];
  return DEMAG_OK;
}

extern "C" demag_status demag_ktucker_copy(demag_ctx *ctx, const demag_ktucker *kt, int32_t q, double *core,
                                           double *const rows[3]) {
  DEMAG_REQUIRE(ctx != nullptr && kt != nullptr && q >= 0 && q < 3 && core != nullptr && rows != nullptr,
                "demag_ktucker_copy: bad argument");
  for (int p = 0; p < 3; ++p) DEMAG_REQUIRE(rows[p] != nullptr, "demag_ktucker_copy: NULL row buffer");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  DEMAG_TRY_HIP(hipMemcpyAsync(core, kt->core[q], size_t(kt->r[q][0]) * kt->r[q][1] * kt->r[q][2] * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
  for (int p = 0; p < 3; ++p)
    DEMAG_TRY_HIP(hipMemcpyAsync(rows[p], kt->rows[q][p], size_t(kt->r[q][p]) * (2 * kt->n[p] - 1) * sizeof(double),
                                 hipMemcpyDeviceToDevice, ctx->stream));
  DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
  return DEMAG_OK;
}

namespace {
demag_status check_terms(const demag_tucker_in *t, int count, const char *what) {
  for (int i = 0; i < count; ++i) {
    DEMAG_REQUIRE(t[i].core != nullptr, std::string(what) + ": NULL core");
    for (int p = 0; p < 3; ++p) {
      DEMAG_REQUIRE(t[i].r[p] >= 1 && t[i].r[p] <= kSvd, std::string(what) + ": ranks 1..128");
      DEMAG_REQUIRE(t[i].rows[p] != nullptr, std::string(what) + ": NULL factor rows");
    }
  }
  return DEMAG_OK;
}
}  // namespace

extern "C" demag_status demag_potential_tucker(demag_ctx *ctx, const demag_ktucker *kt, const demag_tucker_in m[3],
                                               double tol, int32_t rmax, int32_t rout[3], double *core,
                                               double *const rows[3]) {
  DEMAG_REQUIRE(ctx != nullptr && kt != nullptr && m != nullptr && rout != nullptr && core != nullptr &&
                    rows != nullptr,
                "demag_potential_tucker: NULL argument");
  DEMAG_REQUIRE(tol > 0.0 && tol < 1.0, "demag_potential_tucker: tol must lie in (0, 1)");
  DEMAG_REQUIRE(rmax >= 1, "demag_potential_tucker: rmax >= 1");
  for (int p = 0; p < 3; ++p) DEMAG_REQUIRE(rows[p] != nullptr, "demag_potential_tucker: NULL output rows");
  demag_status st = check_terms(m, 3, "demag_potential_tucker");
  if (st != DEMAG_OK) return st;
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  st = set_fft_attrs(ctx->device);
  if (st != DEMAG_OK) return st;
  DevMem mem(ctx->stream);
  std::vector<DTucker> prods;
  for (int q = 0; q < 3; ++q) {
    const int *rk = kt->r[q], *rm = m[q].r;
    double *W[3];
    for (int p = 0; p < 3; ++p) {
      DEMAG_REQUIRE(int64_t(rk[p]) * rm[p] <= kOMax,
                    "demag_potential_tucker: kernel rank times magnetization rank above 512 in one mode");
      TK_ALLOC(SM, cplx, size_t(rm[p]) * kt->L[p]);
      st = row_spectra(ctx, m[q].rows[p], kt->n[p], kt->n[p], rm[p], kt->L[p], SM);
      if (st != DEMAG_OK) return st;
      TK_ALLOC(w, double, size_t(rk[p]) * rm[p] * kt->n[p]);
      st = conv_rows(ctx, kt->spec[q][p], rk[p], SM, rm[p], kt->L[p], kt->n[p], w);
      if (st != DEMAG_OK) return st;
      W[p] = w;
    }
    const int64_t esize = int64_t(rk[0]) * rm[0] * rk[1] * rm[1] * rk[2] * rm[2];
    TK_ALLOC(E, double, esize);
    k_kron3<<<grid_for(esize), 256, 0, ctx->stream>>>(m[q].core, rm[0], rm[1], rm[2], kt->core[q], rk[0], rk[1], rk[2],
                                                      E);
    TK_LAUNCH();
    DTucker prod{{rk[0] * rm[0], rk[1] * rm[1], rk[2] * rm[2]}, E, {W[0], W[1], W[2]}};
    TuckerOut t;
    st = recompress_sum(ctx, mem, kt->n, {prod}, tol, t);
    if (st != DEMAG_OK) return st;
    prods.push_back(DTucker{{t.r[0], t.r[1], t.r[2]}, t.core, {t.rows[0], t.rows[1], t.rows[2]}});
  }
  TuckerOut sum;
  st = recompress_sum(ctx, mem, kt->n, prods, tol, sum);
  if (st != DEMAG_OK) return st;
  return copy_out(ctx, sum, kt->n, rmax, rout, core, rows);
}

extern "C" demag_status demag_tucker_sum(demag_ctx *ctx, const int32_t n[3], int32_t nterms,
                                         const demag_tucker_in *terms, double tol, int32_t rmax, int32_t rout[3],
                                         double *core, double *const rows[3]) {
  DEMAG_REQUIRE(ctx != nullptr && n != nullptr && terms != nullptr && rout != nullptr && core != nullptr &&
                    rows != nullptr,
                "demag_tucker_sum: NULL argument");
  DEMAG_REQUIRE(nterms >= 1 && nterms <= kOMax, "demag_tucker_sum: 1..512 terms");
  DEMAG_REQUIRE(tol > 0.0 && tol < 1.0, "demag_tucker_sum: tol must lie in (0, 1)");
  DEMAG_REQUIRE(rmax >= 1, "demag_tucker_sum: rmax >= 1");
  for (int p = 0; p < 3; ++p) {
    DEMAG_REQUIRE(n[p] >= 1 && n[p] <= kOLen, "demag_tucker_sum: mode sizes 1..16384");
    DEMAG_REQUIRE(rows[p] != nullptr, "demag_tucker_sum: NULL output rows");
  }
  demag_status st = check_terms(terms, nterms, "demag_tucker_sum");
  if (st != DEMAG_OK) return st;
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  DevMem mem(ctx->stream);
  std::vector<DTucker> ts;
  for (int i = 0; i < nterms; ++i)
    ts.push_back(DTucker{{terms[i].r[0], terms[i].r[1], terms[i].r[2]}, terms[i].core,
                         {terms[i].rows[0], terms[i].rows[1], terms[i].rows[2]}});
  const int nn[3] = {n[0], n[1], n[2]};
  TuckerOut out;
  st = recompress_sum(ctx, mem, nn, ts, tol, out);
  if (st != DEMAG_OK) return st;
  return copy_out(ctx, out, nn, rmax, rout, core, rows);
}

extern "C" demag_status demag_tt_round(demag_ctx *ctx, const int32_t n[3], int32_t r1, int32_t r2, const double *G1,
                                       const double *G2, const double *G3, double tol, int32_t rmax, int32_t rout[2],
                                       double *G1o, double *G2o, double *G3o) {
  DEMAG_REQUIRE(ctx != nullptr && n != nullptr && G1 != nullptr && G2 != nullptr && G3 != nullptr && rout != nullptr &&
                    G1o != nullptr && G2o != nullptr && G3o != nullptr,
                "demag_tt_round: NULL argument");
  DEMAG_REQUIRE(r1 >= 1 && r1 <= kSvd && r2 >= 1 && r2 <= kSvd, "demag_tt_round: ranks 1..128");
  for (int p = 0; p < 3; ++p) DEMAG_REQUIRE(n[p] >= 1 && n[p] <= kOLen, "demag_tt_round: mode sizes 1..16384");
  DEMAG_REQUIRE(tol > 0.0 && tol < 1.0, "demag_tt_round: tol must lie in (0, 1)");
  DEMAG_REQUIRE(rmax >= 1, "demag_tt_round: rmax >= 1");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  demag_status st = set_fft_attrs(ctx->device);
  if (st != DEMAG_OK) return st;
  DevMem mem(ctx->stream);
  // outer cores orthonormalised: G1 rows = C1 Q1, G3 rows = C3 Q3
  double *Q1, *C1, *Q3, *C3;
  int k1, k3;
  st = orth_rows(ctx, mem, contiguous(G1, n[0], n[0]), r1, n[0], r1, true, &Q1, &C1, &k1);
  if (st != DEMAG_OK) return st;
  st = orth_rows(ctx, mem, contiguous(G3, n[2], n[2]), r2, n[2], r2, true, &Q3, &C3, &k3);
  if (st != DEMAG_OK) return st;
  k1 = std::max(k1, 1);
  k3 = std::max(k3, 1);
  // middle core M[a'][c'][j] = sum_{a,c} C1[a][a'] G2[a][c][j] C3[c][c']
  TK_ALLOC(T1, double, size_t(k1) * r2 * n[1]);
  TK_ALLOC(Mid, double, size_t(k1) * k3 * n[1]);
  int d[3] = {r1, r2, n[1]};
  st = mode_mul(ctx, G2, d, 0, C1, 1, r1, k1, T1, false);
  if (st != DEMAG_OK) return st;
  d[0] = k1;
  st = mode_mul(ctx, T1, d, 1, C3, 1, r2, k3, Mid, false);
  if (st != DEMAG_OK) return st;
  d[1] = k3;
  const double nrm = std::sqrt(sum_squares(ctx, mem, Mid, int64_t(k1) * k3 * n[1], &st));
  if (st != DEMAG_OK) return st;
  const double delta = tol / std::sqrt(2.0) * nrm;
  // first truncation: left singular vectors of the rows a' of M (length k3 n2)
  std::vector<double> sig;
  double *U = nullptr;
  st = svd_rows(ctx, mem, unfolding(Mid, d, 0), k1, int64_t(k3) * n[1], sig, &U);
  if (st != DEMAG_OK) return st;
  const int s1 = tail_rank(sig, delta);
  TK_ALLOC(M1, double, size_t(s1) * k3 * n[1]);
  st = mode_mul(ctx, Mid, d, 0, U, 1, kSvd, s1, M1, false);   // M1[k] = sum_a' U[a'][k] M[a']
  if (st != DEMAG_OK) return st;
  d[0] = s1;
  TK_ALLOC(H1, double, size_t(s1) * n[0]);
  {
    dim3 g((n[0] + 255) / 256, (s1 + 7) / 8);
    k_rows_combine<<<g, 256, 0, ctx->stream>>>(U, kSvd, Q1, n[0], k1, s1, n[0], H1, n[0]);
    TK_LAUNCH();
  }
  // second truncation: left singular vectors of the rows c' of M1 (mode 1)
  double *W = nullptr;
  st = svd_rows(ctx, mem, unfolding(M1, d, 1), k3, int64_t(s1) * n[1], sig, &W);
  if (st != DEMAG_OK) return st;
  const int s2 = tail_rank(sig, delta);
  TK_ALLOC(H2, double, size_t(s1) * s2 * n[1]);
  st = mode_mul(ctx, M1, d, 1, W, 1, kSvd, s2, H2, false);
  if (st != DEMAG_OK) return st;
  TK_ALLOC(H3, double, size_t(s2) * n[2]);
  {
    dim3 g((n[2] + 255) / 256, (s2 + 7) / 8);
    k_rows_combine<<<g, 256, 0, ctx->stream>>>(W, kSvd, Q3, n[2], k3, s2, n[2], H3, n[2]);
    TK_LAUNCH();
  }
  rout[0] = s1;
  rout[1] = s2;
  if (s1 > rmax || s2 > rmax) {
    DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
    set_error("demag_tt_round: rank above rmax");
    return DEMAG_E_UNSUPPORTED;
  }
  DEMAG_TRY_HIP(hipMemcpyAsync(G1o, H1, size_t(s1) * n[0] * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  DEMAG_TRY_HIP(
      hipMemcpyAsync(G2o, H2, size_t(s1) * s2 * n[1] * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  DEMAG_TRY_HIP(hipMemcpyAsync(G3o, H3, size_t(s2) * n[2] * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
  return DEMAG_OK;
}

extern "C" demag_status demag_cp_to_tt(demag_ctx *ctx, const int32_t n[3], int32_t R, const double *lam,
                                       const double *const U[3], double *G1, double *G2, double *G3) {
  DEMAG_REQUIRE(ctx != nullptr && n != nullptr && lam != nullptr && U != nullptr && G1 != nullptr && G2 != nullptr &&
                    G3 != nullptr,
                "demag_cp_to_tt: NULL argument");
  DEMAG_REQUIRE(R >= 1, "demag_cp_to_tt: R >= 1");
  for (int p = 0; p < 3; ++p) {
    DEMAG_REQUIRE(U[p] != nullptr, "demag_cp_to_tt: NULL factor rows");
    DEMAG_REQUIRE(n[p] >= 1, "demag_cp_to_tt: mode sizes >= 1");
  }
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  DEMAG_TRY_HIP(hipMemcpyAsync(G1, U[0], size_t(R) * n[0] * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  DEMAG_TRY_HIP(hipMemcpyAsync(G3, U[2], size_t(R) * n[2] * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  const int64_t total = int64_t(R) * R * n[1];
  k_cp_tt_mid<<<grid_for(total), 256, 0, ctx->stream>>>(lam, U[1], R, n[1], G2);
  TK_LAUNCH();
  return DEMAG_OK;
}

extern "C" demag_status demag_tucker_to_tt(demag_ctx *ctx, const int32_t n[3], const demag_tucker_in *t, double *G1,
                                           double *G2, double *G3) {
  DEMAG_REQUIRE(ctx != nullptr && n != nullptr && t != nullptr && G1 != nullptr && G2 != nullptr && G3 != nullptr,
                "demag_tucker_to_tt: NULL argument");
  demag_status st = check_terms(t, 1, "demag_tucker_to_tt");
  if (st != DEMAG_OK) return st;
  for (int p = 0; p < 3; ++p) DEMAG_REQUIRE(n[p] >= 1, "demag_tucker_to_tt: mode sizes >= 1");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  DEMAG_TRY_HIP(hipMemcpyAsync(G1, t->rows[0], size_t(t->r[0]) * n[0] * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
  DEMAG_TRY_HIP(hipMemcpyAsync(G3, t->rows[2], size_t(t->r[2]) * n[2] * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
  const int64_t total = int64_t(t->r[0]) * t->r[2] * n[1];
  k_tucker_tt_mid<<<grid_for(total), 256, 0, ctx->stream>>>(t->core, t->r[0], t->r[1], t->r[2], t->rows[1], n[1], G2);
  TK_LAUNCH();
  return DEMAG_OK;
}

extern "C" demag_status demag_tt_to_tucker(demag_ctx *ctx, const int32_t n[3], int32_t r1, int32_t r2,
                                           const double *G1, const double *G2, const double *G3, double tol,
                                           int32_t rmax, int32_t rout[3], double *core, double *const rows[3]) {
  DEMAG_REQUIRE(ctx != nullptr && n != nullptr && G1 != nullptr && G2 != nullptr && G3 != nullptr && rout != nullptr &&
                    core != nullptr && rows != nullptr,
                "demag_tt_to_tucker: NULL argument");
  DEMAG_REQUIRE(r1 >= 1 && r1 <= kSvd && r2 >= 1 && r2 <= kSvd && int64_t(r1) * r2 <= kOMax,
                "demag_tt_to_tucker: ranks 1..128 with r1 r2 <= 512");
  for (int p = 0; p < 3; ++p) {
    DEMAG_REQUIRE(n[p] >= 1 && n[p] <= kOLen, "demag_tt_to_tucker: mode sizes 1..16384");
    DEMAG_REQUIRE(rows[p] != nullptr, "demag_tt_to_tucker: NULL output rows");
  }
  DEMAG_REQUIRE(tol > 0.0 && tol < 1.0, "demag_tt_to_tucker: tol must lie in (0, 1)");
  DEMAG_REQUIRE(rmax >= 1, "demag_tt_to_tucker: rmax >= 1");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  DevMem mem(ctx->stream);
  // the middle mode: an orthonormal basis of the r1 r2 fibres G2[a, b, :]
  double *Q2 = nullptr, *C2 = nullptr;
  int rho = 0;
  const int kmax = std::min(r1 * r2, kSvd);
  demag_status st = orth_rows(ctx, mem, contiguous(G2, n[1], n[1]), r1 * r2, n[1], kmax, true, &Q2, &C2, &rho);
  if (st == DEMAG_E_UNSUPPORTED) {
    set_error("demag_tt_to_tucker: the middle core's fibres span more than 128 dimensions");
    return st;
  }
  if (st != DEMAG_OK) return st;
  TK_ALLOC(c0, double, size_t(r1) * rho * r2);
  k_tt_core<<<grid_for(int64_t(r1) * rho * r2), 256, 0, ctx->stream>>>(C2, kmax, r1, r2, rho, c0);
  TK_LAUNCH();
  const int nn[3] = {n[0], n[1], n[2]};
  DTucker term{{r1, rho, r2}, c0, {G1, Q2, G3}};
  TuckerOut out;
  st = recompress_sum(ctx, mem, nn, {term}, tol, out);
  if (st != DEMAG_OK) return st;
  return copy_out(ctx, out, nn, rmax, rout, core, rows);
}
