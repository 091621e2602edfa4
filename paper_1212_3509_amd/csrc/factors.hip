// Factor assembly (FP64): the 1D cell integrals of the separable kernel.
//
// For node tau and axis cell size h, offset J = -(n-1)..n-1 and the interval
// [a, b] = [(J - 1/2) h, (J + 1/2) h] seen from the target midpoint
// (Sec. 4.2, below Eq. (conv_op)):
//   E(J)  = int_a^b exp(-tau^2 x^2) dx = sqrt(pi)/(2 tau) (erf(tau b) - erf(tau a))
//   X(J)  = int_a^b x exp(-tau^2 x^2) dx = (exp(-tau^2 a^2) - exp(-tau^2 b^2)) / (2 tau^2)
//   X'(J) = b exp(-tau^2 b^2) - a exp(-tau^2 a^2)        (d/ds of X over [s-h/2, s+h/2])
//   E'(J) = -2 tau^2 X(J)                                  (d/ds of E)
// (Eq. (sep_integrands) and the closed form Eq. (f_anal)).  E and X' are even
// in J, X is odd.  Cancellation is avoided by evaluating E for intervals far
// right of 0 as a difference of erfc, and X as -exp(-tau^2 a^2) expm1(-tau^2
// (b^2 - a^2)) / (2 tau^2) with b^2 - a^2 = 2 J h^2.
//
// Stored per axis as [type][k][J + n - 1] with the node weight folded in as
// w_k = (alpha_k / (2 pi^(3/2)))^(1/3) and the sign of h = -grad phi in the
// derivative types: E~ = w E, X~ = w X, P~ = -w X', Q~ = -w E' = 2 tau^2 w X.
#include "internal.h"

#include <cmath>

namespace demag {

namespace {

__global__ void k_assemble_axis(double *__restrict__ out, int n, int M, double h,
                                const double *__restrict__ tau, const double *__restrict__ w) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;  // 0..n-1
  const int k = blockIdx.y;
  if (J >= n || k >= M) return;
  const double t = tau[k];
  const double wk = w[k];
  const double t2 = t * t;
  const double a = (J - 0.5) * h;
  const double b = (J + 0.5) * h;
  const double sqrt_pi = 1.7724538509055160273;
  double E, X, Xp;
  if (J == 0) {
    E = sqrt_pi / t * erf(0.5 * t * h);
    X = 0.0;
  } else {
    const double ta = t * a, tb = t * b;
    const double diff = (ta > 0.5) ? (erfc(ta) - erfc(tb)) : (erf(tb) - erf(ta));
    E = sqrt_pi / (2.0 * t) * diff;
    X = -exp(-t2 * a * a) * expm1(-t2 * (2.0 * J * h * h)) / (2.0 * t2);
  }
  Xp = b * exp(-t2 * b * b) - a * exp(-t2 * a * a);
  const size_t L = 2 * size_t(n) - 1;
  const size_t plane = size_t(M) * L;
  double *row = out + size_t(k) * L;
  const size_t ip = size_t(J) + n - 1, im = size_t(n) - 1 - J;
  row[F_E * plane + ip] = wk * E;
  row[F_E * plane + im] = wk * E;
  row[F_X * plane + ip] = wk * X;
  row[F_X * plane + im] = -wk * X;
  row[F_P * plane + ip] = -wk * Xp;
  row[F_P * plane + im] = -wk * Xp;
  row[F_Q * plane + ip] = 2.0 * t2 * wk * X;
  row[F_Q * plane + im] = -2.0 * t2 * wk * X;
}

// Dense factors of a non-uniform axis: for target cell i (centre xi_i) and
// source cell j = [x_j, x_{j+1}] the integration interval in u = xi_i - y is
// [a, b] = [xi_i - x_{j+1}, xi_i - x_j]; E, X and X' as in the Toeplitz case
// (erfc differences for intervals away from 0 on either side; X through
// expm1 anchored at the endpoint nearer 0).  out[((type M + k) n + i) n + j].
__global__ void k_assemble_dense(double *__restrict__ out, const double *__restrict__ edges, int n, int M,
                                 const double *__restrict__ tau, const double *__restrict__ w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (e >= n * n || k >= M) return;
  const int i = e / n, j = e - i * n;
  const double t = tau[k], wk = w[k], t2 = t * t;
  const double xi = 0.5 * (edges[i] + edges[i + 1]);
  const double a = xi - edges[j + 1], b = xi - edges[j];
  const double sqrt_pi = 1.7724538509055160273;
  const double ta = t * a, tb = t * b;
  double diff;
  if (ta > 0.5) diff = erfc(ta) - erfc(tb);
  else if (tb < -0.5) diff = erfc(-tb) - erfc(-ta);
  else diff = erf(tb) - erf(ta);
  const double E = sqrt_pi / (2.0 * t) * diff;
  const double d2 = (b - a) * (b + a);   // b^2 - a^2
  const double X = (d2 >= 0.0) ? -exp(-t2 * a * a) * expm1(-t2 * d2) / (2.0 * t2)
                               : exp(-t2 * b * b) * expm1(t2 * d2) / (2.0 * t2);
  const double Xp = b * exp(-t2 * b * b) - a * exp(-t2 * a * a);
  const size_t nn = size_t(n) * n, plane = size_t(M) * nn;
  const size_t o = size_t(k) * nn + e;
  out[F_E * plane + o] = wk * E;
  out[F_X * plane + o] = wk * X;
  out[F_P * plane + o] = -wk * Xp;
  out[F_Q * plane + o] = 2.0 * t2 * wk * X;
}

// FP32 copy and bfloat16 split (round to nearest even by integer arithmetic)
// of the FP32 value: hi = bf16(x), lo = bf16(x - hi), lo2 = bf16(x - hi - lo).
__device__ inline uint16_t bf16_rne_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ inline float bf16_bits_to_float(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

__global__ void k_convert(const double *__restrict__ src, float *__restrict__ f32,
                          uint16_t *__restrict__ bf, size_t count) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float x = float(src[i]);
  f32[i] = x;
  uint16_t h = bf16_rne_bits(x);
  float r = x - bf16_bits_to_float(h);
  uint16_t l = bf16_rne_bits(r);
  float r2 = r - bf16_bits_to_float(l);
  uint16_t l2 = bf16_rne_bits(r2);
  bf[i] = h;
  bf[count + i] = l;
  bf[2 * count + i] = l2;
}

__global__ void k_to_float(const double *__restrict__ src, float *__restrict__ dst, size_t count) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = float(src[i]);
}

}  // namespace

size_t axis_table_len(const demag_factors *f, int d) {
  const size_t n = size_t(f->n[d]);
  return size_t(F_NTYPES) * f->M * (f->dense ? n * n : 2 * n - 1);
}

demag_status launch_assemble(demag_ctx *ctx, demag_factors *f) {
  double *d_tau = nullptr, *d_w = nullptr;
  DEMAG_TRY_HIP(hipMallocAsync(&d_tau, sizeof(double) * f->M, ctx->stream));
  DEMAG_TRY_HIP(hipMallocAsync(&d_w, sizeof(double) * f->M, ctx->stream));
  DEMAG_TRY_HIP(hipMemcpyAsync(d_tau, f->tau.data(), sizeof(double) * f->M, hipMemcpyHostToDevice, ctx->stream));
  DEMAG_TRY_HIP(hipMemcpyAsync(d_w, f->w.data(), sizeof(double) * f->M, hipMemcpyHostToDevice, ctx->stream));
  for (int d = 0; d < 3; ++d) {
    const int n = f->n[d];
    dim3 grid((n + 127) / 128, f->M);
    k_assemble_axis<<<grid, 128, 0, ctx->stream>>>(f->f64[d], n, f->M, f->hs[d], d_tau, d_w);
    DEMAG_TRY_HIP(hipGetLastError());
    const size_t cnt = axis_table_len(f, d);
    k_convert<<<unsigned((cnt + 255) / 256), 256, 0, ctx->stream>>>(f->f64[d], f->f32[d], f->bf[d], cnt);
    DEMAG_TRY_HIP(hipGetLastError());
  }
  // The host vectors are copied before these frees run (stream order).
  DEMAG_TRY_HIP(hipFreeAsync(d_tau, ctx->stream));
  DEMAG_TRY_HIP(hipFreeAsync(d_w, ctx->stream));
  return DEMAG_OK;
}

demag_status launch_assemble_dense(demag_ctx *ctx, demag_factors *f, const std::vector<double> edges[3]) {
  double *d_tau = nullptr, *d_w = nullptr, *d_edges = nullptr;
  const size_t ne = edges[0].size() + edges[1].size() + edges[2].size();
  DEMAG_TRY_HIP(hipMallocAsync(&d_tau, sizeof(double) * f->M, ctx->stream));
  DEMAG_TRY_HIP(hipMallocAsync(&d_w, sizeof(double) * f->M, ctx->stream));
  DEMAG_TRY_HIP(hipMallocAsync(&d_edges, sizeof(double) * ne, ctx->stream));
  DEMAG_TRY_HIP(hipMemcpyAsync(d_tau, f->tau.data(), sizeof(double) * f->M, hipMemcpyHostToDevice, ctx->stream));
  DEMAG_TRY_HIP(hipMemcpyAsync(d_w, f->w.data(), sizeof(double) * f->M, hipMemcpyHostToDevice, ctx->stream));
  size_t off = 0;
  for (int d = 0; d < 3; ++d) {
    DEMAG_TRY_HIP(hipMemcpyAsync(d_edges + off, edges[d].data(), sizeof(double) * edges[d].size(),
                                 hipMemcpyHostToDevice, ctx->stream));
    const int n = f->n[d];
    dim3 grid(unsigned((size_t(n) * n + 255) / 256), unsigned(f->M));
    k_assemble_dense<<<grid, 256, 0, ctx->stream>>>(f->f64[d], d_edges + off, n, f->M, d_tau, d_w);
    DEMAG_TRY_HIP(hipGetLastError());
    if (f->f32[d]) {   // FP32 copy for the FP32 apply, its bfloat16 parts for the split ones
      const size_t cnt = axis_table_len(f, d);
      k_to_float<<<unsigned((cnt + 255) / 256), 256, 0, ctx->stream>>>(f->f64[d], f->f32[d], cnt);
      DEMAG_TRY_HIP(hipGetLastError());
      if (f->bf[d]) {
        const demag_status st = launch_split(ctx, f->f32[d], f->bf[d], cnt, 3);
        if (st != DEMAG_OK) return st;
      }
    }
    off += edges[d].size();
  }
  // the host vectors are copied before these frees run (stream order); the
  // pageable copies above complete before they return
  DEMAG_TRY_HIP(hipFreeAsync(d_tau, ctx->stream));
  DEMAG_TRY_HIP(hipFreeAsync(d_w, ctx->stream));
  DEMAG_TRY_HIP(hipFreeAsync(d_edges, ctx->stream));
  return DEMAG_OK;
}

}  // namespace demag
