// Tolerance-controlled recompression of a CP tensor to Tucker form by HOOI
// (Sec. 2.2, Alg. HOOI; the remark after it: for a tensor given as a sum of
// terms every mode product is formed term by term).
//
// X = sum_t lam_t a_t^(1) o a_t^(2) o a_t^(3), with the factor columns taken
// from the structured apply's column sets through a term table.  For mode p
// (q < s the other two) HOOI needs the leading left singular vectors of the
// unfolding Y_(p) of X x_q U_q^T x_s U_s^T, an n_p x r_q r_s matrix equal to
//   A_p^T diag(lam) KR,  KR[t][(a, b)] = (A_q U_q^T)[t][a] (A_s U_s^T)[t][b].
// It is never formed.  A randomized range finder (test matrix G given by the
// caller) gives K = rmax + 8 candidate directions Yg = Y_(p) G, orthonormalised
// by block Gram-Schmidt with reorthogonalisation (dependent ones dropped); the small
// matrix B = Q Y_(p) (K x r_q r_s) then has the leading singular values and,
// through the eigenvectors of B B^T, the leading singular vectors of Y_(p).
// The rank follows the tolerance rule on those singular values (capped at
// rmax).  Initial factors: the same range finder on the unprojected
// unfoldings, with Khatri-Rao test vectors (Omega_q[j] kron Omega_s[j]).
//
// All arithmetic is FP64.  Symmetric eigenproblems (K <= 72) run as a
// parallel cyclic Jacobi iteration in one workgroup's LDS, Gram-Schmidt
// within blocks of 8 rows in one workgroup (mode sizes up to 8192); the long
// contractions are plain tiled kernels (this is a set-up computation, not on
// the apply's hot path).  The relative error is computed without the
// cancellation of |X|^2 - |core|^2: the residual splits into the orthogonal
// parts (I - P1) X, P1 (I - P2) X, P1 P2 (I - P3) X, each a CP tensor whose
// squared norm is a weighted sum of products of Gram matrices of its columns.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace demag {

namespace {

constexpr int kOversample = 8;
constexpr int kMaxRank = 64;
constexpr int kMaxK = kMaxRank + kOversample;   // 72

// Ab[t][i] = cols[table[t][p]][i] in FP64 (rows = factor columns of mode p).
__global__ void k_gather(const float *__restrict__ cols, const int32_t *__restrict__ table, int p, int T, int n,
                         double *__restrict__ Ab) {
  const int t = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T || i >= n) return;
  Ab[size_t(t) * n + i] = double(cols[size_t(table[3 * t + p]) * n + i]);
}

// C[a][b] = sum_i X[a][i] Y[b][i] for a < na, b < nb, i < len (rows of X and
// Y at strides ldx, ldy; C at stride ldc).  32 x 32 outputs per workgroup,
// 2 x 2 per thread, chunks of 32 points through LDS.
__global__ __launch_bounds__(256) void k_xty(const double *__restrict__ X, int ldx, const double *__restrict__ Y,
                                             int ldy, int na, int nb, int len, double *__restrict__ C, int ldc) {
  __shared__ double xs[32][33], ys[32][33];
  const int a0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int i0 = 0; i0 < len; i0 += 32) {
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
      const int r = e >> 5, c = e & 31;
      const int i = i0 + c;
      xs[r][c] = (a0 + r < na && i < len) ? X[size_t(a0 + r) * ldx + i] : 0.0;
      ys[r][c] = (b0 + r < nb && i < len) ? Y[size_t(b0 + r) * ldy + i] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < 32; ++c) {
      const double x0 = xs[2 * ty][c], x1 = xs[2 * ty + 1][c];
      const double y0 = ys[2 * tx][c], y1 = ys[2 * tx + 1][c];
      acc[0][0] += x0 * y0;
      acc[0][1] += x0 * y1;
      acc[1][0] += x1 * y0;
      acc[1][1] += x1 * y1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int a = a0 + 2 * ty + u, b = b0 + 2 * tx + v;
      if (a < na && b < nb) C[size_t(a) * ldc + b] = acc[u][v];
    }
}

// C[b][i] = sum_a z(a, b) X[a][i] (z(a, b) = Z[a * sza + b * szb]) for b < nb,
// i < len, a < na; with X0 non-NULL, C = X0 - that (residual columns).
__global__ __launch_bounds__(256) void k_ztx(const double *__restrict__ Z, int sza, int szb,
                                             const double *__restrict__ X, int ldx, int na, int nb, int len,
                                             double *__restrict__ C, int ldc, const double *__restrict__ X0,
                                             int ldx0) {
  constexpr int kB = 8;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int b0 = blockIdx.y * kB;
  double acc[kB];
#pragma unroll
  for (int u = 0; u < kB; ++u) acc[u] = 0.0;
  if (i < len) {
    for (int a = 0; a < na; ++a) {
      const double x = X[size_t(a) * ldx + i];
#pragma unroll
      for (int u = 0; u < kB; ++u)
        if (b0 + u < nb) acc[u] += Z[size_t(a) * sza + size_t(b0 + u) * szb] * x;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int b = b0 + u;
      if (b >= nb) continue;
      C[size_t(b) * ldc + i] = X0 ? X0[size_t(b) * ldx0 + i] - acc[u] : acc[u];
    }
  }
}

// Initial range finder: Z[t][j] = lam_t Pq[t][j] Ps[t][j] (Khatri-Rao test vectors).
__global__ void k_kr_diag(const double *__restrict__ lam, const double *__restrict__ Pq,
                          const double *__restrict__ Ps, int T, int K, double *__restrict__ Z) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T * K) return;
  const int t = e / K;
  Z[e] = lam[t] * Pq[e] * Ps[e];
}

// Sweep range finder: Z[t][j] = lam_t sum_a Pq[t][a] sum_b Ps[t][b] G[(a rs + b) K + j].
__global__ __launch_bounds__(128) void k_zg(const double *__restrict__ lam, const double *__restrict__ Pq,
                                            const double *__restrict__ Ps, int ld, int rq, int rs,
                                            const double *__restrict__ G, int K, double *__restrict__ Z) {
  __shared__ double pq[kMaxK], ps[kMaxK];
  const int t = blockIdx.x;
  for (int a = threadIdx.x; a < rq; a += blockDim.x) pq[a] = Pq[size_t(t) * ld + a];
  for (int b = threadIdx.x; b < rs; b += blockDim.x) ps[b] = Ps[size_t(t) * ld + b];
  __syncthreads();
  const int j = threadIdx.x;
  if (j >= K) return;
  double acc = 0.0;
  for (int a = 0; a < rq; ++a) {
    double inner = 0.0;
    const double *g = G + size_t(a) * rs * K + j;
    for (int b = 0; b < rs; ++b) inner += ps[b] * g[size_t(b) * K];
    acc += pq[a] * inner;
  }
  Z[size_t(t) * K + j] = lam[t] * acc;
}

// B[j][a rs + b] = sum_t V[j][t] lam_t Pq[t][a] Ps[t][b]  (j < nj, m = rq rs).
__global__ __launch_bounds__(256) void k_bmat(const double *__restrict__ V, int ldv, const double *__restrict__ lam,
                                              const double *__restrict__ Pq, const double *__restrict__ Ps,
                                              int ld, int rq, int rs, int T, double *__restrict__ B, int ldb) {
  const int j = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= rq * rs) return;
  const int a = e / rs, b = e - a * rs;
  double acc = 0.0;
  for (int t = 0; t < T; ++t) acc += V[size_t(j) * ldv + t] * lam[t] * Pq[size_t(t) * ld + a] * Ps[size_t(t) * ld + b];
  B[size_t(j) * ldb + e] = acc;
}

// Symmetric eigen-decomposition of W (K x K, K <= kMaxK) by the cyclic
// Jacobi method in one workgroup: per step the round-robin ordering gives K/2
// disjoint index pairs, each zeroed by a plane rotation J (A <- J^T A J,
// V <- V J); sweeps end when the off-diagonal part is below 1e-15 of the
// Frobenius norm.  Outputs: d[c] (descending) and E[j][c] = component j of
// eigenvector c.
__global__ __launch_bounds__(256) void k_jacobi(const double *__restrict__ W, int ldw, int K, double *__restrict__ d,
                                                double *__restrict__ E, int lde) {
  extern __shared__ double js[];
  const int Kp = K + (K & 1);
  const int LD = Kp + 1;
  double *a = js, *v = a + Kp * LD;
  double *cs = v + Kp * LD, *sn = cs + Kp / 2;
  double *red = sn + Kp / 2;   // 256 partial sums x 2
  int *pp = reinterpret_cast<int *>(red + 512), *qq = pp + Kp / 2;
  const int tid = threadIdx.x;
  for (int e = tid; e < Kp * Kp; e += 256) {
    const int i = e / Kp, j = e - i * Kp;
    a[i * LD + j] = (i < K && j < K) ? W[size_t(i) * ldw + j] : 0.0;
    v[i * LD + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < Kp * Kp; e += 256) {
      const int i = e / Kp, j = e - i * Kp;
      const double x = a[i * LD + j];
      tot += x * x;
      if (i != j) off += x * x;
    }
    red[tid] = off;
    red[256 + tid] = tot;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) {
        red[tid] += red[tid + h];
        red[256 + tid] += red[256 + tid + h];
      }
      __syncthreads();
    }
    const bool done = !(red[0] > 1e-30 * red[256]);
    __syncthreads();
    if (done || Kp < 2) break;
    for (int step = 0; step < Kp - 1; ++step) {
      if (tid < Kp / 2) {
        const int k = tid;
        auto idx = [&](int m) { return m == 0 ? 0 : 1 + (m - 1 + step) % (Kp - 1); };
        const int p = idx(k), q = idx(Kp - 1 - k);
        const double apq = a[p * LD + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-300) {
          const double th = (a[q * LD + q] - a[p * LD + p]) / (2.0 * apq);
          // t = the smaller root of t^2 + 2 th t - 1 = 0 (~ 1 / (2 th) for large th)
          const double t = fabs(th) > 1e150 ? 0.5 / th
                                            : (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs[k] = c;
        sn[k] = s;
        pp[k] = p;
        qq[k] = q;
      }
      __syncthreads();
      // rows p, q of every pair
      for (int e = tid; e < (Kp / 2) * Kp; e += 256) {
        const int k = e / Kp, j = e - k * Kp;
        const int p = pp[k], q = qq[k];
        const double c = cs[k], s = sn[k];
        const double ap = a[p * LD + j], aq = a[q * LD + j];
        a[p * LD + j] = c * ap - s * aq;
        a[q * LD + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of every pair, and of V
      for (int e = tid; e < (Kp / 2) * Kp; e += 256) {
        const int k = e / Kp, i = e - k * Kp;
        const int p = pp[k], q = qq[k];
        const double c = cs[k], s = sn[k];
        const double ap = a[i * LD + p], aq = a[i * LD + q];
        a[i * LD + p] = c * ap - s * aq;
        a[i * LD + q] = s * ap + c * aq;
        const double vp = v[i * LD + p], vq = v[i * LD + q];
        v[i * LD + p] = c * vp - s * vq;
        v[i * LD + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // descending order (ties by index)
  for (int i = tid; i < K; i += 256) {
    const double di = a[i * LD + i];
    int rank = 0;
    for (int j = 0; j < K; ++j) {
      const double dj = a[j * LD + j];
      if (dj > di || (dj == di && j < i)) ++rank;
    }
    d[rank] = di;
    for (int j = 0; j < K; ++j) E[size_t(j) * lde + rank] = v[j * LD + i];
  }
}

// Orthonormal rows Q (returned count *kout) spanning the k rows of Y
// (length n <= 8192): classical Gram-Schmidt with one reorthogonalisation
// per row; a row whose norm falls below drop times its reference norm (ref2:
// squared norms before earlier projections, else its own) is dependent and
// dropped.  One workgroup; thread tid owns the points
// x = tid + 256 e, so the rows it writes are the rows it reads back.
constexpr int kCgsPer = 32;
__device__ inline double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
__global__ __launch_bounds__(256) void k_cgs2(const double *__restrict__ Y, int k, int n, double *__restrict__ Q,
                                              int *__restrict__ kout, double drop, const double *__restrict__ ref2) {
  __shared__ double part[4][kMaxK + 1];
  __shared__ double coef[kMaxK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  auto block_sum = [&](double x) {
    x = wave_sum(x);
    if (lane == 0) part[wave][kMaxK] = x;
    __syncthreads();
    const double t = part[0][kMaxK] + part[1][kMaxK] + part[2][kMaxK] + part[3][kMaxK];
    __syncthreads();
    return t;
  };
  int kept = 0;
  for (int j = 0; j < k; ++j) {
    double v[kCgsPer];
    double sq = 0.0;
#pragma unroll
    for (int e = 0; e < kCgsPer; ++e) {
      const int x = tid + 256 * e;
      v[e] = x < n ? Y[size_t(j) * n + x] : 0.0;
      sq += v[e] * v[e];
    }
    const double own = block_sum(sq);
    const double nrm0 = ref2 ? ref2[j] : own;   // reference: the row before any projection
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < kept; ++i) {
        double d = 0.0;
#pragma unroll
        for (int e = 0; e < kCgsPer; ++e) {
          const int x = tid + 256 * e;
          if (x < n) d += Q[size_t(i) * n + x] * v[e];
        }
        d = wave_sum(d);
        if (lane == 0) part[wave][i] = d;
      }
      __syncthreads();
      if (tid < kept) coef[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
      __syncthreads();
      for (int i = 0; i < kept; ++i) {
        const double c = coef[i];
#pragma unroll
        for (int e = 0; e < kCgsPer; ++e) {
          const int x = tid + 256 * e;
          if (x < n) v[e] -= c * Q[size_t(i) * n + x];
        }
      }
    }
    sq = 0.0;
#pragma unroll
    for (int e = 0; e < kCgsPer; ++e) sq += v[e] * v[e];
    const double nrm = block_sum(sq);
    if (nrm > 0.0 && nrm > drop * drop * nrm0) {
      const double inv = 1.0 / sqrt(nrm);
#pragma unroll
      for (int e = 0; e < kCgsPer; ++e) {
        const int x = tid + 256 * e;
        if (x < n) Q[size_t(kept) * n + x] = v[e] * inv;
      }
      ++kept;
    }
  }
  if (tid == 0) *kout = kept;
}

// ref2[j] = |Y[j]|^2 (one workgroup per row).
__global__ __launch_bounds__(256) void k_rownorm2(const double *__restrict__ Y, int n, double *__restrict__ ref2) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double y = Y[size_t(j) * n + i];
    s += y * y;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) ref2[j] = red[0] + red[1] + red[2] + red[3];
}

size_t jacobi_lds(int K) {
  const int Kp = K + (K & 1);
  return sizeof(double) * (2 * size_t(Kp) * (Kp + 1) + Kp + 512) + sizeof(int) * Kp;
}

// E[j][c] /= sqrt(d[c]) for c < nc (columns of the kept eigenvectors).
__global__ void k_scale_cols(double *__restrict__ E, int lde, int K, int nc, const double *__restrict__ d) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * nc) return;
  const int j = e / nc, c = e - j * nc;
  E[size_t(j) * lde + c] /= sqrt(d[c]);
}

// core[(a r2 + b) r3 + c] = sum_t lam_t P1[t][a] P2[t][b] P3[t][c].
__global__ void k_core(const double *__restrict__ lam, const double *__restrict__ P1, const double *__restrict__ P2,
                       const double *__restrict__ P3, int ld, int r1, int r2, int r3, int T,
                       double *__restrict__ core) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r1 * r2 * r3) return;
  const int a = e / (r2 * r3), b = (e / r3) % r2, c = e % r3;
  double acc = 0.0;
  for (int t = 0; t < T; ++t) acc += lam[t] * P1[size_t(t) * ld + a] * P2[size_t(t) * ld + b] * P3[size_t(t) * ld + c];
  core[e] = acc;
}

// Partial sums of lam_t lam_u G0[t][u] G1[t][u] G2[t][u] over rows t of a block.
__global__ __launch_bounds__(256) void k_quadform(const double *__restrict__ lam, const double *__restrict__ G0,
                                                  const double *__restrict__ G1, const double *__restrict__ G2,
                                                  int T, double *__restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  const int t = blockIdx.x;
  for (int u = threadIdx.x; u < T; u += 256) {
    const size_t e = size_t(t) * T + u;
    acc += lam[u] * G0[e] * G1[e] * G2[e];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[t] = lam[t] * red[0];
}

inline void others(int p, int &q, int &s) {
  q = (p == 0) ? 1 : 0;
  s = (p == 2) ? 1 : 2;
}

unsigned blocks(size_t n, int per) { return unsigned((n + per - 1) / per); }

struct Rc {
  demag_ctx *ctx;
  hipStream_t st;
  int T, K;
  int n[3];
  const double *lam;
  double *Ab[3], *P[3], *Ut[3];
  double *Z, *Y, *Q1, *Q2, *V, *B, *W, *E, *d, *core, *grams[6], *R, *partial;
  int *icount;

  demag_status xty(const double *X, int ldx, const double *Yv, int ldy, int na, int nb, int len, double *C,
                   int ldc) {
    if (na <= 0 || nb <= 0) return DEMAG_OK;
    k_xty<<<dim3(blocks(na, 32), blocks(nb, 32)), 256, 0, st>>>(X, ldx, Yv, ldy, na, nb, len, C, ldc);
    DEMAG_TRY_HIP(hipGetLastError());
    return DEMAG_OK;
  }
  demag_status ztx(const double *Zv, int sza, int szb, const double *X, int ldx, int na, int nb, int len,
                   double *C, int ldc, const double *X0 = nullptr, int ldx0 = 0) {
    if (nb <= 0 || len <= 0) return DEMAG_OK;
    k_ztx<<<dim3(blocks(len, 256), blocks(nb, 8)), 256, 0, st>>>(Zv, sza, szb, X, ldx, na, nb, len, C, ldc, X0,
                                                               ldx0);
    DEMAG_TRY_HIP(hipGetLastError());
    return DEMAG_OK;
  }
  // eigenvalues (descending) to the host, eigenvectors in E [K][K]
  demag_status eig(const double *Wm, int k, std::vector<double> &dh) {
    const size_t lds = jacobi_lds(k);
    DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_jacobi),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    k_jacobi<<<1, 256, lds, st>>>(Wm, kMaxK, k, d, E, kMaxK);
    DEMAG_TRY_HIP(hipGetLastError());
    dh.assign(k, 0.0);
    DEMAG_TRY_HIP(hipMemcpyAsync(dh.data(), d, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    DEMAG_TRY_HIP(hipStreamSynchronize(st));
    return DEMAG_OK;
  }
  // rows of Yin (k x len) -> orthonormal rows Qout spanning them (count
  // kout): block Gram-Schmidt, blocks of 8 rows projected twice against the
  // rows kept so far (two tiled products each), then Gram-Schmidt within the
  // block in one workgroup; dependence is judged against each row's norm
  // before any projection
  demag_status orthonormalize(const double *Yin, int k, int len, double *Qout, int &kout) {
    constexpr int kBlk = 8;
    k_rownorm2<<<k, 256, 0, st>>>(Yin, len, d);
    DEMAG_TRY_HIP(hipGetLastError());
    double *Ta = Q1, *Tb = Q1 + size_t(kBlk) * len;
    int kept = 0;
    for (int b0 = 0; b0 < k; b0 += kBlk) {
      const int nb = std::min(kBlk, k - b0);
      const double *src = Yin + size_t(b0) * len;
      if (kept > 0) {
        for (int pass = 0; pass < 2; ++pass) {
          double *dst = pass == 0 ? Ta : Tb;
          demag_status s = xty(src, len, Qout, len, nb, kept, len, W, kMaxK);
          if (s != DEMAG_OK) return s;
          s = ztx(W, 1, kMaxK, Qout, len, kept, nb, len, dst, len, src, len);
          if (s != DEMAG_OK) return s;
          src = dst;
        }
      }
      k_cgs2<<<1, 256, 0, st>>>(src, nb, len, Qout + size_t(kept) * len, icount, 1e-13, d + b0);
      DEMAG_TRY_HIP(hipGetLastError());
      int h = 0;
      DEMAG_TRY_HIP(hipMemcpyAsync(&h, icount, sizeof(int), hipMemcpyDeviceToHost, st));
      DEMAG_TRY_HIP(hipStreamSynchronize(st));
      kept += h;
    }
    kout = kept;
    return DEMAG_OK;
  }
  demag_status quadform(const double *G0, const double *G1, const double *G2, double &out) {
    k_quadform<<<T, 256, 0, st>>>(lam, G0, G1, G2, T, partial);
    DEMAG_TRY_HIP(hipGetLastError());
    std::vector<double> h(T);
    DEMAG_TRY_HIP(hipMemcpyAsync(h.data(), partial, sizeof(double) * T, hipMemcpyDeviceToHost, st));
    DEMAG_TRY_HIP(hipStreamSynchronize(st));
    out = 0.0;
    for (double x : h) out += x;
    return DEMAG_OK;
  }
};

// Smallest r >= 1 whose discarded singular values have norm <= eps/sqrt(3) of all.
int rank_rule(const std::vector<double> &sig2, double eps) {
  double total = 0.0;
  for (double x : sig2) total += std::max(x, 0.0);
  if (!(total > 0.0)) return 1;
  const double bound2 = eps * eps / 3.0 * total;
  double tail = 0.0;
  int r = int(sig2.size());
  // tail(r) = sum_{i >= r} sig2[i]; smallest r >= 1 with tail(r) <= bound2
  for (int i = int(sig2.size()) - 1; i >= 1; --i) {
    tail += std::max(sig2[i], 0.0);
    if (tail <= bound2) r = i;
    else break;
  }
  return std::max(r, 1);
}

}  // namespace

extern "C" demag_status demag_recompress_cp(demag_ctx *ctx, const int32_t n[3], int32_t T, const float *const cols[3],
                                            const int32_t ncols[3], const int32_t *table, const double *lam,
                                            double eps, int32_t rmax, int32_t max_sweeps, const double *omega,
                                            const double *gmat, double *const U[3], double *core, int32_t ranks[3],
                                            double *rel_err, int32_t *sweeps) {
  DEMAG_REQUIRE(ctx && n && cols && ncols && table && lam && omega && gmat && U && core && ranks && rel_err,
                "demag_recompress_cp: NULL argument");
  DEMAG_REQUIRE(T >= 1 && T <= 16384, "demag_recompress_cp: 1 <= T <= 16384 terms");
  DEMAG_REQUIRE(rmax >= 1 && rmax <= kMaxRank, "demag_recompress_cp: 1 <= rmax <= 64");
  DEMAG_REQUIRE(eps > 0.0 && eps < 1.0, "demag_recompress_cp: 0 < eps < 1");
  DEMAG_REQUIRE(max_sweeps >= 1 && max_sweeps <= 100, "demag_recompress_cp: 1 <= max_sweeps <= 100");
  for (int p = 0; p < 3; ++p) {
    DEMAG_REQUIRE(n[p] >= 1 && n[p] <= 256 * kCgsPer && cols[p] && U[p] && ncols[p] >= 1,
                  "demag_recompress_cp: bad mode size, column set or factor buffer");
  }
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  // the term table is small: check its column indices on the host
  {
    std::vector<int32_t> tab(size_t(T) * 3);
    DEMAG_TRY_HIP(hipMemcpyAsync(tab.data(), table, sizeof(int32_t) * tab.size(), hipMemcpyDeviceToHost, st));
    DEMAG_TRY_HIP(hipStreamSynchronize(st));
    for (int t = 0; t < T; ++t)
      for (int p = 0; p < 3; ++p)
        DEMAG_REQUIRE(tab[size_t(t) * 3 + p] >= 0 && tab[size_t(t) * 3 + p] < ncols[p],
                      "demag_recompress_cp: table entry out of range");
  }
  const int K = rmax + kOversample;
  const int nmax = std::max(n[0], std::max(n[1], n[2]));
  // workspace (doubles)
  const size_t sz_ab = size_t(T) * (size_t(n[0]) + n[1] + n[2]);
  const size_t sz_p = 3 * size_t(T) * kMaxK;
  const size_t sz_ut = size_t(kMaxK) * (size_t(n[0]) + n[1] + n[2]);
  const size_t sz_z = size_t(T) * kMaxK;
  const size_t sz_y = 3 * size_t(kMaxK) * nmax;
  const size_t sz_v = size_t(kMaxK) * T;
  const size_t sz_b = size_t(kMaxK) * kMaxK * kMaxK;
  const size_t sz_w = 2 * size_t(kMaxK) * kMaxK + kMaxK;
  const size_t sz_core = size_t(kMaxK) * kMaxK * kMaxK;
  const size_t sz_g = 6 * size_t(T) * T;
  const size_t sz_r = size_t(T) * nmax;
  const size_t total = sz_ab + sz_p + sz_ut + sz_z + sz_y + sz_v + sz_b + sz_w + sz_core + sz_g + sz_r + T + 1;
  demag_status s = ensure_workspace(ctx, total * sizeof(double));
  if (s != DEMAG_OK) return s;
  Rc rc{};
  rc.ctx = ctx;
  rc.st = st;
  rc.T = T;
  rc.K = K;
  rc.lam = lam;
  double *w = static_cast<double *>(ctx->ws);
  for (int p = 0; p < 3; ++p) {
    rc.n[p] = n[p];
    rc.Ab[p] = w;
    w += size_t(T) * n[p];
  }
  for (int p = 0; p < 3; ++p) {
    rc.P[p] = w;
    w += size_t(T) * kMaxK;
  }
  for (int p = 0; p < 3; ++p) {
    rc.Ut[p] = w;
    w += size_t(kMaxK) * n[p];
  }
  rc.Z = w; w += sz_z;
  rc.Y = w; w += size_t(kMaxK) * nmax;
  rc.Q1 = w; w += size_t(kMaxK) * nmax;
  rc.Q2 = w; w += size_t(kMaxK) * nmax;
  rc.V = w; w += sz_v;
  rc.B = w; w += sz_b;
  rc.W = w; w += size_t(kMaxK) * kMaxK;
  rc.E = w; w += size_t(kMaxK) * kMaxK;
  rc.d = w; w += kMaxK;
  rc.core = w; w += sz_core;
  for (int g = 0; g < 6; ++g) {
    rc.grams[g] = w;
    w += size_t(T) * T;
  }
  rc.R = w; w += sz_r;
  rc.partial = w; w += T;
  rc.icount = reinterpret_cast<int *>(w);

  for (int p = 0; p < 3; ++p) {
    k_gather<<<dim3(blocks(n[p], 256), T), 256, 0, st>>>(cols[p], table, p, T, n[p], rc.Ab[p]);
    DEMAG_TRY_HIP(hipGetLastError());
  }
  int r[3];
  // initial factors: range finder on the unprojected unfoldings
  {
    const double *om[3];
    om[0] = omega;
    om[1] = om[0] + size_t(K) * n[0];
    om[2] = om[1] + size_t(K) * n[1];
    for (int p = 0; p < 3; ++p) {
      int q, sx;
      others(p, q, sx);
      if ((s = rc.xty(rc.Ab[q], n[q], om[q], n[q], T, K, n[q], rc.P[q], kMaxK)) != DEMAG_OK) return s;
      if ((s = rc.xty(rc.Ab[sx], n[sx], om[sx], n[sx], T, K, n[sx], rc.P[sx], kMaxK)) != DEMAG_OK) return s;
      // Z[t][j] = lam_t Pq[t][j] Ps[t][j] with row stride kMaxK -> pack at stride K
      k_kr_diag<<<blocks(size_t(T) * kMaxK, 256), 256, 0, st>>>(lam, rc.P[q], rc.P[sx], T, kMaxK, rc.Z);
      DEMAG_TRY_HIP(hipGetLastError());
      if ((s = rc.ztx(rc.Z, kMaxK, 1, rc.Ab[p], n[p], T, K, n[p], rc.Y, n[p])) != DEMAG_OK) return s;
      if ((s = rc.orthonormalize(rc.Y, K, n[p], rc.Ut[p], r[p])) != DEMAG_OK) return s;
      if (r[p] == 0) {
        set_error("demag_recompress_cp: the tensor is zero");
        return DEMAG_E_INVAL;
      }
    }
  }
  // HOOI sweeps
  double fit_old = -1.0, fit = 0.0;
  int done = 0;
  for (int sw = 1; sw <= max_sweeps; ++sw) {
    done = sw;
    for (int p = 0; p < 3; ++p) {
      int q, sx;
      others(p, q, sx);
      const int rq = r[q], rs = r[sx];
      if ((s = rc.xty(rc.Ab[q], n[q], rc.Ut[q], n[q], T, rq, n[q], rc.P[q], kMaxK)) != DEMAG_OK) return s;
      if ((s = rc.xty(rc.Ab[sx], n[sx], rc.Ut[sx], n[sx], T, rs, n[sx], rc.P[sx], kMaxK)) != DEMAG_OK) return s;
      k_zg<<<T, 128, 0, st>>>(lam, rc.P[q], rc.P[sx], kMaxK, rq, rs, gmat, K, rc.Z);
      DEMAG_TRY_HIP(hipGetLastError());
      if ((s = rc.ztx(rc.Z, K, 1, rc.Ab[p], n[p], T, K, n[p], rc.Y, n[p])) != DEMAG_OK) return s;
      int kq = 0;
      if ((s = rc.orthonormalize(rc.Y, K, n[p], rc.Q2, kq)) != DEMAG_OK) return s;
      if (kq == 0) {
        set_error("demag_recompress_cp: the projected tensor vanished");
        return DEMAG_E_INVAL;
      }
      // V[j][t] = Q[j] . a_t^(p);  B = V diag(lam) KR;  W = B B^T
      if ((s = rc.xty(rc.Q2, n[p], rc.Ab[p], n[p], kq, T, n[p], rc.V, T)) != DEMAG_OK) return s;
      const int m = rq * rs;
      k_bmat<<<dim3(blocks(m, 256), kq), 256, 0, st>>>(rc.V, T, lam, rc.P[q], rc.P[sx], kMaxK, rq, rs, T, rc.B, m);
      DEMAG_TRY_HIP(hipGetLastError());
      if ((s = rc.xty(rc.B, m, rc.B, m, kq, kq, m, rc.W, kMaxK)) != DEMAG_OK) return s;
      std::vector<double> sig2;
      if ((s = rc.eig(rc.W, kq, sig2)) != DEMAG_OK) return s;
      int rp = std::min(rank_rule(sig2, eps), int(rmax));
      rp = std::min(rp, kq);
      // U_p rows = leading left singular vectors: E[:, c]^T Q
      if ((s = rc.ztx(rc.E, kMaxK, 1, rc.Q2, n[p], kq, rp, n[p], rc.Ut[p], n[p])) != DEMAG_OK) return s;
      r[p] = rp;
    }
    // core and fit
    for (int p = 0; p < 3; ++p)
      if ((s = rc.xty(rc.Ab[p], n[p], rc.Ut[p], n[p], T, r[p], n[p], rc.P[p], kMaxK)) != DEMAG_OK) return s;
    const int ncore = r[0] * r[1] * r[2];
    k_core<<<blocks(ncore, 256), 256, 0, st>>>(lam, rc.P[0], rc.P[1], rc.P[2], kMaxK, r[0], r[1], r[2], T, rc.core);
    DEMAG_TRY_HIP(hipGetLastError());
    std::vector<double> ch(ncore);
    DEMAG_TRY_HIP(hipMemcpyAsync(ch.data(), rc.core, sizeof(double) * ncore, hipMemcpyDeviceToHost, st));
    DEMAG_TRY_HIP(hipStreamSynchronize(st));
    fit = 0.0;
    for (double x : ch) fit += x * x;
    if (fit_old >= 0.0 && std::fabs(fit - fit_old) <= 1e-13 * std::max(fit, 1e-300)) break;
    fit_old = fit;
  }
  // |X|^2 and the residual norm (core and P[p] are those of the final factors)
  double **G = rc.grams;
  for (int p = 0; p < 3; ++p)
    if ((s = rc.xty(rc.Ab[p], n[p], rc.Ab[p], n[p], T, T, n[p], G[p], T)) != DEMAG_OK) return s;
  double x2 = 0.0;
  if ((s = rc.quadform(G[0], G[1], G[2], x2)) != DEMAG_OK) return s;
  // projected-column Grams of modes 0 and 1 (coordinates P[p] = A_p U_p^T)
  for (int p = 0; p < 2; ++p)
    if ((s = rc.xty(rc.P[p], kMaxK, rc.P[p], kMaxK, T, T, r[p], G[3 + p], T)) != DEMAG_OK) return s;
  double res2 = 0.0;
  for (int p = 0; p < 3; ++p) {
    // residual columns R = A_p - P_p U_p and their Gram in G[5]
    if ((s = rc.ztx(rc.P[p], 1, kMaxK, rc.Ut[p], n[p], r[p], T, n[p], rc.R, n[p], rc.Ab[p], n[p])) != DEMAG_OK)
      return s;
    if ((s = rc.xty(rc.R, n[p], rc.R, n[p], T, T, n[p], G[5], T)) != DEMAG_OK) return s;
    const double *g0 = p == 0 ? G[5] : G[3];
    const double *g1 = p == 0 ? G[1] : (p == 1 ? G[5] : G[4]);
    const double *g2 = p == 2 ? G[5] : G[2];
    double part = 0.0;
    if ((s = rc.quadform(g0, g1, g2, part)) != DEMAG_OK) return s;
    res2 += part;
  }
  for (int p = 0; p < 3; ++p) {
    DEMAG_TRY_HIP(hipMemcpyAsync(U[p], rc.Ut[p], sizeof(double) * size_t(r[p]) * n[p], hipMemcpyDeviceToDevice, st));
    ranks[p] = r[p];
  }
  DEMAG_TRY_HIP(hipMemcpyAsync(core, rc.core, sizeof(double) * size_t(r[0]) * r[1] * r[2], hipMemcpyDeviceToDevice,
                               st));
  DEMAG_TRY_HIP(hipStreamSynchronize(st));
  *rel_err = x2 > 0.0 ? std::sqrt(std::max(res2, 0.0) / x2) : 0.0;
  if (sweeps) *sweeps = done;
  return DEMAG_OK;
}

}  // namespace demag
