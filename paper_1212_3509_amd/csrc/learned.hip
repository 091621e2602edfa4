// Learned shortened quadrature: a small network proposes R' (16..32) nodes
// and weights for a grid and tolerance; an FP64 judge measures the kernel
// error of any rule against an accurate reference rule; a per-grid
// Levenberg-Marquardt fit in the network's output space gives the training
// targets and polishes the network's proposal; the full rule is the
// fallback.  (Not in the paper: built on its sinc rule, Cor. kron_op, and its
// separable kernels, Eqs. (sep_integrands), (f_anal).)
//
// Network: 6 -> 64 -> 64 -> 64 -> 65, GELU(x) = x Phi(x) on the hidden layers,
// FP32, parameters flat [W1 (64x6, row = output), b1, W2, b2, W3, b3, W4
// (65x64), b4].  Inputs per case: aspect ratios n_d/n_max, log2(1/h)/6 - 1,
// (log10 tol + 6.5)/2.5, (R' - 24)/8.  Outputs: y_0..31 node offsets,
// y_32..63 log-weight offsets, y_64 predicted log10 error.
//
// Rule from outputs (base: the sinc rule with R' nodes, c0 = 2.15):
//   theta = c0 ln(R')/R', t_k = k theta,
//   t'_k = t_k + 0.45 theta tanh(y_k),
//   alpha'_k = 2 theta cosh t'_k sinh^2 t'_k exp(tanh(y_{32+k}))
// (the weight follows its node: the trapezoid weight of the substituted
// integrand at the moved node, times a free factor).
// Judge: at S sampled offsets J_s with weights w_s, nine kernel values per rule
//   [K^x, K^y, K^z, F_xx, F_yy, F_zz, F_xy, F_xz, F_yz]
//   K^q  = W prod_d f_d with f = X along q, E elsewhere;
//   F_pq = the same for h_p <- m_q with axis p differentiated (X -> P = -X',
//          E -> Q = 2 tau^2 X), W = alpha / (2 pi^(3/2)),
// against K_ref from the sinc rule with the step of Thm. sinc_theo and 96
// nodes:  e_phi^2 = sum_s w_s sum_{c<3} dK_c^2 / sum_s w_s sum_{c<3} K_ref,c^2,
// e_h^2 the same over the field values with multiplicity m_c (2 for the
// off-diagonal F_pq, which stand for F_pq and F_qp), err^2 = e_phi^2 + e_h^2.
// With w_s the number of cell pairs each sampled offset stands for, these
// estimate the relative Frobenius-norm errors of the discrete potential and
// field operators; the certificate (k_cert_*) computes them exactly, over
// every offset of the grid.
// Fit: residuals r_(s,c) = sqrt(w_s m_c / D_c) (K - K_ref)_c(J_s) (|r| = err,
// D_c = the reference's weighted sum of squares of c's class);
// Levenberg-Marquardt steps (A + mu diag A) d = -J^T r, A = J^T J, in
// u_k = 0.45 tanh(y_k), v_k = tanh(y_{32+k}) (k < R'; t'_k = t_k + theta u_k,
// alpha'_k carries exp(v_k)), projected onto |u| <= 0.44, |v| <= 0.99 and
// kept when err drops (mu / 3), else mu * 4; the fitted outputs are
// y = atanh(u / 0.45), atanh(v).
// The Jacobian uses the closed-form tau-derivatives of the 1D factors:
//   dE/dtau = (X' - E)/tau,  dX/dtau = (b^2 e_b - a^2 e_a - 2X)/tau,
//   dX'/dtau = -2 tau (b^3 e_b - a^3 e_a),  e_a = exp(-tau^2 a^2),
// with tau = sinh t' and d ln alpha'/d t' = tanh t' + 2 coth t'.
// Training (distillation of the fits): Adam on
//   mean_b [ ln(1 + d^T H d) + lambda (y_64 - log10 err*)^2 ],  d = x(y) - x*,
// H = J^T J / err*^2 at each case's fitted x* (the Gauss-Newton estimate of
// err(x)^2 / err*^2 - 1), or on plain squared output errors against the
// fitted outputs (clipped to [-3, 3]) when no H is given.
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace demag {

namespace {

constexpr int kIn = 6, kH = 64, kOut = 65, kRmax = 32, kNcomp = 9;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH * kH, oW4 = oB3 + kH, oB4 = oW4 + kOut * kH, kParams = oB4 + kOut;
static_assert(kParams == 12993, "parameter count");
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kC0 = 2.15;

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ------------------------------------------------------------------ network
// One 64-thread workgroup per sample.  Z, A: [B][3][64] pre-activations and
// activations of the hidden layers (for the backward pass).
__global__ __launch_bounds__(64) void k_mlp_forward(const float *__restrict__ P, const float *__restrict__ X, int B,
                                                    float *__restrict__ Y, float *__restrict__ Z,
                                                    float *__restrict__ A) {
  __shared__ float a[kH];
  __shared__ float x[kIn];
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= B) return;
  if (j < kIn) x[j] = X[size_t(b) * kIn + j];
  __syncthreads();
  float z = P[oB1 + j];
  for (int i = 0; i < kIn; ++i) z += P[oW1 + j * kIn + i] * x[i];
  float act = gelu(z);
  if (Z) Z[(size_t(b) * 3 + 0) * kH + j] = z;
  if (A) A[(size_t(b) * 3 + 0) * kH + j] = act;
  a[j] = act;
  __syncthreads();
  for (int l = 1; l < 3; ++l) {
    const int oW = (l == 1) ? oW2 : oW3, oB = (l == 1) ? oB2 : oB3;
    z = P[oB + j];
    for (int i = 0; i < kH; ++i) z += P[oW + j * kH + i] * a[i];
    act = gelu(z);
    if (Z) Z[(size_t(b) * 3 + l) * kH + j] = z;
    if (A) A[(size_t(b) * 3 + l) * kH + j] = act;
    __syncthreads();
    a[j] = act;
    __syncthreads();
  }
  for (int o = j; o < kOut; o += kH) {
    float y = P[oB4 + o];
    for (int i = 0; i < kH; ++i) y += P[oW4 + o * kH + i] * a[i];
    Y[size_t(b) * kOut + o] = y;
  }
}

// Deltas of the hidden pre-activations, D: [B][3][64].
__global__ __launch_bounds__(64) void k_mlp_delta(const float *__restrict__ P, const float *__restrict__ Z,
                                                  const float *__restrict__ dY, int B, float *__restrict__ D) {
  __shared__ float d[kOut];
  const int b = blockIdx.x, i = threadIdx.x;
  if (b >= B) return;
  for (int o = i; o < kOut; o += kH) d[o] = dY[size_t(b) * kOut + o];
  __syncthreads();
  float s = 0.0f;
  for (int o = 0; o < kOut; ++o) s += P[oW4 + o * kH + i] * d[o];
  float di = s * gelu_grad(Z[(size_t(b) * 3 + 2) * kH + i]);
  D[(size_t(b) * 3 + 2) * kH + i] = di;
  __syncthreads();
  d[i] = di;
  __syncthreads();
  for (int l = 1; l >= 0; --l) {
    const int oW = (l == 1) ? oW3 : oW2;   // weights of layer l+1 (maps layer l to l+1)
    s = 0.0f;
    for (int o = 0; o < kH; ++o) s += P[oW + o * kH + i] * d[o];
    di = s * gelu_grad(Z[(size_t(b) * 3 + l) * kH + i]);
    D[(size_t(b) * 3 + l) * kH + i] = di;
    __syncthreads();
    d[i] = di;
    __syncthreads();
  }
}

// Parameter gradients, one thread per parameter, summed over samples in a
// fixed order (deterministic).
__global__ void k_mlp_grad(const float *__restrict__ X, const float *__restrict__ A, const float *__restrict__ D,
                           const float *__restrict__ dY, int B, float *__restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  // locate (layer, row j, column i or bias)
  int layer, j, i = -1, nin;
  if (p < oB1) { layer = 0; nin = kIn; j = (p - oW1) / kIn; i = (p - oW1) % kIn; }
  else if (p < oW2) { layer = 0; nin = kIn; j = p - oB1; }
  else if (p < oB2) { layer = 1; nin = kH; j = (p - oW2) / kH; i = (p - oW2) % kH; }
  else if (p < oW3) { layer = 1; nin = kH; j = p - oB2; }
  else if (p < oB3) { layer = 2; nin = kH; j = (p - oW3) / kH; i = (p - oW3) % kH; }
  else if (p < oW4) { layer = 2; nin = kH; j = p - oB3; }
  else if (p < oB4) { layer = 3; nin = kH; j = (p - oW4) / kH; i = (p - oW4) % kH; }
  else { layer = 3; nin = kH; j = p - oB4; }
  (void)nin;
  float s = 0.0f;
  for (int b = 0; b < B; ++b) {
    const float delta = (layer == 3) ? dY[size_t(b) * kOut + j] : D[(size_t(b) * 3 + layer) * kH + j];
    float in = 1.0f;
    if (i >= 0) in = (layer == 0) ? X[size_t(b) * kIn + i] : A[(size_t(b) * 3 + layer - 1) * kH + i];
    s += delta * in;
  }
  G[p] = s;
}

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ m,
                       float *__restrict__ v, int n, int step, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float g = G[p];
  const float mm = b1 * m[p] + (1.0f - b1) * g;
  const float vv = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / (1.0f - powf(b1, float(step)));
  const float vh = vv / (1.0f - powf(b2, float(step)));
  P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------------------ rules
// Rules from outputs (or the plain base rule when Y == NULL): t, alpha [B][KM].
__global__ void k_rules(const float *__restrict__ Y, const int *__restrict__ R, int B, int KM,
                        double *__restrict__ t, double *__restrict__ alpha) {
  const int b = blockIdx.x, k = threadIdx.x;
  if (b >= B || k >= KM) return;
  const int r = R[b];
  double tk = 0.0, ak = 0.0;
  if (k < r) {
    const double theta = kC0 * log(double(r)) / r;
    tk = (k + 1) * theta;
    const double sh = sinh(tk);
    ak = 2.0 * theta * cosh(tk) * sh * sh;
    if (Y) {
      tk += 0.45 * theta * tanh(double(Y[size_t(b) * kOut + k]));
      const double shp = sinh(tk);
      ak = 2.0 * theta * cosh(tk) * shp * shp * exp(tanh(double(Y[size_t(b) * kOut + kRmax + k])));
    }
  }
  t[size_t(b) * KM + k] = tk;
  alpha[size_t(b) * KM + k] = ak;
}

// Reference rules (sinc rule, step of Thm. sinc_theo, M nodes) per case.
__global__ void k_ref_rules(const double *__restrict__ hmin, int B, int M, double *__restrict__ t,
                            double *__restrict__ alpha) {
  const int b = blockIdx.x;
  for (int k = threadIdx.x; k < M && b < B; k += blockDim.x) {
    const double a = 2.0, bb = 0.25 * (0.5 * hmin[b]) * (0.5 * hmin[b]);
    const double theta = log(2.0 * kPi * a * M / bb) / (a * M);
    const double tk = (k + 1) * theta;
    const double sh = sinh(tk);
    t[size_t(b) * M + k] = tk;
    alpha[size_t(b) * M + k] = 2.0 * theta * cosh(tk) * sh * sh;
  }
}

// 1D factors at offset J (any sign) for node tau and cell size h, and their
// tau-derivatives.  f[0] = E, f[1] = X, f[2] = P = -X', f[3] = Q = 2 tau^2 X.
__device__ __forceinline__ void factors_1d(int J, double tau, double h, double f[4], double df[4]) {
  const int Ja = J < 0 ? -J : J;
  const double sg = J < 0 ? -1.0 : 1.0;
  const double a = (Ja - 0.5) * h, b = (Ja + 0.5) * h;
  const double t2 = tau * tau;
  const double ea = exp(-t2 * a * a), eb = exp(-t2 * b * b);
  double E, X;
  if (Ja == 0) {
    E = 1.7724538509055160273 / tau * erf(0.5 * tau * h);
    X = 0.0;
  } else {
    const double ta = tau * a, tb = tau * b;
    const double diff = (ta > 0.5) ? (erfc(ta) - erfc(tb)) : (erf(tb) - erf(ta));
    E = 1.7724538509055160273 / (2.0 * tau) * diff;
    X = -ea * expm1(-t2 * (2.0 * Ja * h * h)) / (2.0 * t2);
  }
  const double Xp = b * eb - a * ea;
  const double dE = (Xp - E) / tau;
  const double dX = (b * b * eb - a * a * ea - 2.0 * X) / tau;
  const double dXp = -2.0 * tau * (b * b * b * eb - a * a * a * ea);
  f[0] = E;
  f[1] = sg * X;
  f[2] = -Xp;
  f[3] = sg * 2.0 * t2 * X;
  df[0] = dE;
  df[1] = sg * dX;
  df[2] = -dXp;
  df[3] = sg * (4.0 * tau * X + 2.0 * t2 * dX);
}

// factor type along axis d (x, y, z) of component c; loops over c are
// unrolled so the types are compile-time constants and the factor arrays
// stay in registers
__host__ __device__ constexpr int ftype(int c, int d) {
  constexpr int T[kNcomp][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1},   // K^x, K^y, K^z
                                {2, 0, 0}, {0, 2, 0}, {0, 0, 2},   // F_xx, F_yy, F_zz
                                {3, 1, 0}, {3, 0, 1}, {0, 3, 1}};  // F_xy, F_xz, F_yz
  return T[c][d];
}

// Kernel values of each case's rule at its sentinels: K [B][S][9].
__global__ __launch_bounds__(128) void k_judge_values(const int *__restrict__ grids, const double *__restrict__ hmin,
                               const int *__restrict__ sent, int S, const double *__restrict__ t,
                               const double *__restrict__ alpha, const int *__restrict__ R, int KM, int B,
                               double *__restrict__ K) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * S) return;
  const int b = idx / S, s = idx % S;
  const double h = hmin[b];
  const int *J = sent + (size_t(b) * S + s) * 3;
  const int r = R ? R[b] : KM;
  double acc[kNcomp] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < r; ++k) {
    const double tk = t[size_t(b) * KM + k];
    const double tau = sinh(tk);
    const double W = alpha[size_t(b) * KM + k] / (2.0 * pow(kPi, 1.5));
    double f[3][4], df[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d) factors_1d(J[d], tau, h, f[d], df[d]);
#pragma unroll
    for (int c = 0; c < kNcomp; ++c) acc[c] += W * f[0][ftype(c, 0)] * f[1][ftype(c, 1)] * f[2][ftype(c, 2)];
  }
  for (int c = 0; c < kNcomp; ++c) K[(size_t(b) * S + s) * kNcomp + c] = acc[c];
}

// multiplicity of each kernel value in the operator's Frobenius norm
__host__ __device__ constexpr double kmult(int c) { return c >= 6 ? 2.0 : 1.0; }

// err per case (and e_phi, e_h in parts[B][2] if given) and the residual
// weights resid = w_s m_c / D_c (K - K_ref) per offset and value.
__global__ void k_judge_err(const double *__restrict__ K, const double *__restrict__ Kref,
                            const double *__restrict__ wts, int B, int S, double *__restrict__ err,
                            double *__restrict__ parts, double *__restrict__ resid) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double num[2] = {0.0, 0.0}, den[2] = {0.0, 0.0};
  for (int s = 0; s < S; ++s) {
    const double w = wts[size_t(b) * S + s];
    const double *k = K + (size_t(b) * S + s) * kNcomp;
    const double *r = Kref + (size_t(b) * S + s) * kNcomp;
    for (int c = 0; c < kNcomp; ++c) {
      const int cl = c < 3 ? 0 : 1;
      num[cl] += w * kmult(c) * (k[c] - r[c]) * (k[c] - r[c]);
      den[cl] += w * kmult(c) * r[c] * r[c];
    }
  }
  const double ep = sqrt(num[0] / den[0]), eh = sqrt(num[1] / den[1]);
  err[b] = sqrt(ep * ep + eh * eh);
  if (parts) {
    parts[2 * size_t(b)] = ep;
    parts[2 * size_t(b) + 1] = eh;
  }
  if (resid)
    for (int s = 0; s < S; ++s) {
      const double w = wts[size_t(b) * S + s];
      for (int c = 0; c < kNcomp; ++c) {
        const size_t i = (size_t(b) * S + s) * kNcomp + c;
        resid[i] = w * kmult(c) / den[c < 3 ? 0 : 1] * (K[i] - Kref[i]);
      }
    }
}

// d err / d t'_k and d err / d alpha'_k: [B][KM].
__global__ __launch_bounds__(128) void k_judge_grad(const int *__restrict__ grids, const double *__restrict__ hmin,
                             const int *__restrict__ sent, int S, const double *__restrict__ t,
                             const double *__restrict__ alpha, const int *__restrict__ R, int KM, int B,
                             const double *__restrict__ resid, const double *__restrict__ err,
                             double *__restrict__ dt, double *__restrict__ dalpha) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * KM) return;
  const int b = idx / KM, k = idx % KM;
  double gt = 0.0, ga = 0.0;
  if (k < R[b]) {
    const double h = hmin[b];
    const double tk = t[size_t(b) * KM + k];
    const double tau = sinh(tk), ch = cosh(tk);
    const double c = 1.0 / (2.0 * pow(kPi, 1.5));
    const double W = alpha[size_t(b) * KM + k] * c;
    for (int s = 0; s < S; ++s) {
      const int *J = sent + (size_t(b) * S + s) * 3;
      double f[3][4], df[3][4];
  #pragma unroll
    for (int d = 0; d < 3; ++d) factors_1d(J[d], tau, h, f[d], df[d]);
      const double *r = resid + (size_t(b) * S + s) * kNcomp;
#pragma unroll
      for (int q = 0; q < kNcomp; ++q) {
        const int t0 = ftype(q, 0), t1 = ftype(q, 1), t2 = ftype(q, 2);
        const double prod = f[0][t0] * f[1][t1] * f[2][t2];
        const double dprod = df[0][t0] * f[1][t1] * f[2][t2] + f[0][t0] * df[1][t1] * f[2][t2] +
                             f[0][t0] * f[1][t1] * df[2][t2];
        ga += r[q] * c * prod;
        gt += r[q] * W * ch * dprod;
      }
    }
    const double scale = 1.0 / err[b];
    gt *= scale;
    ga *= scale;
  }
  dt[idx] = gt;
  dalpha[idx] = ga;
}

// ------------------------------------------------------------------ certificate
// Weighted sums over the offsets J >= 0 of a grid of the squared kernel
// differences between a rule (M nodes) and the reference (96 nodes), and of
// the reference's squared kernels, for the potential values and the field
// values (with multiplicity), with the weights c_x(Jx) c_y(Jy) c_z(Jz),
// c_d(j) = (n_d - j) (1 if j == 0 else 2): the number of cell pairs an
// offset and its sign images stand for.  Per axis the offsets are given as
// sample positions with weights (every j below kCertExact with c_d(j); past
// it, blocks of cells represented by their midpoints with the blocks' summed
// weights), so grids up to kCertExact cells per axis are summed exactly.
constexpr int kCertExact = 512;

// Factor tables at the sample positions: T[type][k][i] = w_k^(1/3) f_type(pos_i)
// for the KT = M + 96 nodes (rule first).
__global__ void k_cert_factors(const int *__restrict__ pos, int np, const double *__restrict__ tau,
                               const double *__restrict__ wcr, int KT, double h, double *__restrict__ T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, k = blockIdx.y;
  if (i >= np) return;
  double f[4], df[4];
  factors_1d(pos[i], tau[k], h, f, df);
  for (int t = 0; t < 4; ++t) T[(size_t(t) * KT + k) * np + i] = wcr[k] * f[t];
}

// One workgroup per (y, z) sample pair at a time (grid-stride over pairs),
// threads over the x samples; the y-z factor products of the six (type_y,
// type_z) combinations the nine values need are staged in LDS per pair.
// partial[block][4] = the block's weighted sums (phi diff, phi ref, field
// diff, field ref).
__global__ __launch_bounds__(256) void k_cert_sums(const double *__restrict__ Tx, const double *__restrict__ Ty,
                                                   const double *__restrict__ Tz, const double *__restrict__ wx,
                                                   const double *__restrict__ wy, const double *__restrict__ wz,
                                                   int npx, int npy, int npz, int KT, int M,
                                                   double *__restrict__ partial) {
  extern __shared__ double yz[];   // [6][KT]
  __shared__ double red[4][256];
  const int tid = threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int pair = blockIdx.x; pair < npy * npz; pair += gridDim.x) {
    const int iy = pair % npy, iz = pair / npy;
    __syncthreads();
    for (int k = tid; k < KT; k += blockDim.x) {
      const double ey = Ty[(size_t(F_E) * KT + k) * npy + iy], xy = Ty[(size_t(F_X) * KT + k) * npy + iy];
      const double py = Ty[(size_t(F_P) * KT + k) * npy + iy], qy = Ty[(size_t(F_Q) * KT + k) * npy + iy];
      const double ez = Tz[(size_t(F_E) * KT + k) * npz + iz], xz = Tz[(size_t(F_X) * KT + k) * npz + iz];
      const double pz = Tz[(size_t(F_P) * KT + k) * npz + iz];
      yz[0 * KT + k] = ey * ez;   // K^x, F_xx
      yz[1 * KT + k] = xy * ez;   // K^y, F_xy
      yz[2 * KT + k] = ey * xz;   // K^z, F_xz
      yz[3 * KT + k] = py * ez;   // F_yy
      yz[4 * KT + k] = ey * pz;   // F_zz
      yz[5 * KT + k] = qy * xz;   // F_yz
    }
    __syncthreads();
    const double wyz = wy[iy] * wz[iz];
    for (int ix = tid; ix < npx; ix += blockDim.x) {
      double d[kNcomp], r[kNcomp];
#pragma unroll
      for (int c = 0; c < kNcomp; ++c) d[c] = r[c] = 0.0;
      for (int k = 0; k < KT; ++k) {
        const double e = Tx[(size_t(F_E) * KT + k) * npx + ix], x = Tx[(size_t(F_X) * KT + k) * npx + ix];
        const double p = Tx[(size_t(F_P) * KT + k) * npx + ix], q = Tx[(size_t(F_Q) * KT + k) * npx + ix];
        const double v[kNcomp] = {x * yz[k],          e * yz[KT + k],     e * yz[2 * KT + k],
                                  p * yz[k],          e * yz[3 * KT + k], e * yz[4 * KT + k],
                                  q * yz[KT + k],     q * yz[2 * KT + k], e * yz[5 * KT + k]};
        if (k < M) {
#pragma unroll
          for (int c = 0; c < kNcomp; ++c) d[c] += v[c];
        } else {
#pragma unroll
          for (int c = 0; c < kNcomp; ++c) {
            d[c] -= v[c];
            r[c] += v[c];
          }
        }
      }
      const double w = wx[ix] * wyz;
      acc[0] += w * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      acc[1] += w * (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      acc[2] += w * (d[3] * d[3] + d[4] * d[4] + d[5] * d[5] + 2.0 * (d[6] * d[6] + d[7] * d[7] + d[8] * d[8]));
      acc[3] += w * (r[3] * r[3] + r[4] * r[4] + r[5] * r[5] + 2.0 * (r[6] * r[6] + r[7] * r[7] + r[8] * r[8]));
    }
  }
  for (int i = 0; i < 4; ++i) red[i][tid] = acc[i];
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (tid < st)
      for (int i = 0; i < 4; ++i) red[i][tid] += red[i][tid + st];
    __syncthreads();
  }
  if (tid < 4) partial[size_t(blockIdx.x) * 4 + tid] = red[tid][0];
}

// Sum of the per-block partials in a fixed order: out[4].
__global__ __launch_bounds__(256) void k_cert_final(const double *__restrict__ partial, int nblk,
                                                    double *__restrict__ out) {
  __shared__ double red[4][256];
  const int tid = threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = tid; b < nblk; b += blockDim.x)
    for (int i = 0; i < 4; ++i) acc[i] += partial[size_t(b) * 4 + i];
  for (int i = 0; i < 4; ++i) red[i][tid] = acc[i];
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (tid < st)
      for (int i = 0; i < 4; ++i) red[i][tid] += red[i][tid + st];
    __syncthreads();
  }
  if (tid < 4) out[tid] = red[tid][0];
}

// Output gradients of the supervised loss and per-case loss values.
__global__ void k_target_grads(const float *__restrict__ Y, const float *__restrict__ T, const int *__restrict__ R,
                               int B, float lambda, float *__restrict__ dY, float *__restrict__ loss) {
  __shared__ float part[kOut];
  const int b = blockIdx.x, o = threadIdx.x;
  if (b >= B) return;
  const int r = R[b];
  float g = 0.0f, l = 0.0f;
  if (o < kOut) {
    const float y = Y[size_t(b) * kOut + o];
    if (o == 64) {
      const float d = y - T[size_t(b) * kOut + 64];
      g = 2.0f * lambda * d / B;
      l = lambda * d * d;
    } else if ((o % kRmax) < r) {
      const float d = y - fminf(3.0f, fmaxf(-3.0f, T[size_t(b) * kOut + o]));
      g = 2.0f * d / (2.0f * r * B);
      l = d * d / (2.0f * r);
    }
    dY[size_t(b) * kOut + o] = g;
    part[o] = l;
  }
  __syncthreads();
  if (o == 0) {
    float sum = 0.0f;
    for (int i = 0; i < kOut; ++i) sum += part[i];
    loss[b] = sum;
  }
}

// ------------------------------------------------------------------ fit
constexpr int kFitSB = 8;        // sentinels per pass: 8 x 32 nodes = 256 threads
constexpr int kNP = 2 * kRmax;   // fitted outputs y_k, y_{32+k}
constexpr int kMaxS = 256;

constexpr double kUMax = 0.44, kVMax = 0.99;

struct FitLds {
  double val[kFitSB][kNcomp][kRmax];  // node contributions to the kernel values
  double jt[kFitSB][kNcomp][kRmax];   // d r / d u_k (per node)
  double ja[kFitSB][kNcomp][kRmax];   // d r / d v_k
  double res[kFitSB * kNcomp];
  double A[kNP][kNP + 1];
  double g[kNP];
  double y[kNP], yc[kNP], d[kNP];
  double tp[kRmax], ap[kRmax], dty[kRmax], lat[kRmax], sa[kRmax];
  double isig[kMaxS][2];   // sqrt(w_s / D_phi), sqrt(w_s / D_h) per offset
  double dsum[2];
  double err2, err_cur, mu;
  int ok;
};

// scale of the residual of value c at offset s: sqrt(w_s m_c / D_class(c))
__device__ __forceinline__ double residual_scale(const FitLds &L, int s, int c) {
  return c < 3 ? L.isig[s][0] : (c >= 6 ? 1.4142135623730950488 * L.isig[s][1] : L.isig[s][1]);
}

// node parameters of x = (u, v) (threads k < R): t', alpha' and the
// derivatives the Jacobian needs
__device__ inline void fit_nodes(FitLds &L, const double *xv, int R) {
  const int k = threadIdx.x;
  if (k < R) {
    const double theta = kC0 * log(double(R)) / R;
    const double tp = (k + 1) * theta + theta * xv[k];
    const double sh = sinh(tp);
    L.tp[k] = tp;
    L.ap[k] = 2.0 * theta * cosh(tp) * sh * sh * exp(xv[kRmax + k]);
    L.dty[k] = theta;                        // d t' / d u
    L.lat[k] = tanh(tp) + 2.0 / tanh(tp);    // d ln alpha' / d t'
    L.sa[k] = 1.0;                           // d ln alpha' / d v
  }
}

// One pass over all sentinels: err^2 of the current node parameters into
// L.err2; with jac, also A = J^T J (rows of L.A) and g = J^T r (L.g).
__device__ void fit_pass(FitLds &L, int b, int S, int R, double h, const int *__restrict__ sent,
                         const double *__restrict__ Kref, bool jac) {
  const int tid = threadIdx.x;
  const int sl = tid >> 5, k = tid & 31;
  // J^T J: thread (p, qj) sums row p against columns qj + 4 cc, so the four
  // lanes of one p read four consecutive doubles (distinct LDS banks)
  const int p = tid >> 2, qj = tid & 3;
  const double cW = 1.0 / (2.0 * pow(kPi, 1.5));
  double acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = 0.0;
  double gacc = 0.0, e2 = 0.0;
  for (int s0 = 0; s0 < S; s0 += kFitSB) {
    const int s = s0 + sl;
    if (k < R && s < S) {
      const int *J = sent + (size_t(b) * S + s) * 3;
      const double tp = L.tp[k], tau = sinh(tp), ch = cosh(tp);
      const double W = L.ap[k] * cW;
      double f[3][4], df[3][4];
  #pragma unroll
    for (int d = 0; d < 3; ++d) factors_1d(J[d], tau, h, f[d], df[d]);
#pragma unroll
      for (int c = 0; c < kNcomp; ++c) {
        const double is = residual_scale(L, s, c);
        const int t0 = ftype(c, 0), t1 = ftype(c, 1), t2 = ftype(c, 2);
        const double prod = f[0][t0] * f[1][t1] * f[2][t2];
        const double v = W * prod;
        L.val[sl][c][k] = v;
        if (jac) {
          const double dprod = df[0][t0] * f[1][t1] * f[2][t2] + f[0][t0] * df[1][t1] * f[2][t2] +
                               f[0][t0] * f[1][t1] * df[2][t2];
          L.jt[sl][c][k] = (W * ch * dprod + v * L.lat[k]) * L.dty[k] * is;
          L.ja[sl][c][k] = v * L.sa[k] * is;
        }
      }
    } else {
      for (int c = 0; c < kNcomp; ++c) {
        L.val[sl][c][k] = 0.0;
        if (jac) {
          L.jt[sl][c][k] = 0.0;
          L.ja[sl][c][k] = 0.0;
        }
      }
    }
    __syncthreads();
    if (tid < kFitSB * kNcomp) {
      const int rs = s0 + tid / kNcomp, c = tid % kNcomp;
      double r = 0.0;
      if (rs < S) {
        double sum = 0.0;
        for (int kk = 0; kk < R; ++kk) sum += L.val[tid / kNcomp][c][kk];
        r = (sum - Kref[(size_t(b) * S + rs) * kNcomp + c]) * residual_scale(L, rs, c);
      }
      L.res[tid] = r;
    }
    __syncthreads();
    if (tid == 0)
      for (int i = 0; i < kFitSB * kNcomp; ++i) e2 += L.res[i] * L.res[i];
    if (jac) {
      for (int i = 0; i < kFitSB * kNcomp; ++i) {
        const int il = i / kNcomp, c = i % kNcomp;
        const double jp = p < kRmax ? L.jt[il][c][p] : L.ja[il][c][p - kRmax];
        const double *rt = &L.jt[il][c][qj], *ra = &L.ja[il][c][qj];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) acc[cc] += jp * rt[4 * cc];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) acc[8 + cc] += jp * ra[4 * cc];
        if ((tid & 3) == 0) gacc += jp * L.res[i];
      }
    }
    __syncthreads();
  }
  if (jac) {
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) L.A[p][qj + 4 * cc] = acc[cc];
    if ((tid & 3) == 0) L.g[p] = gacc;
  }
  if (tid == 0) L.err2 = e2;
  __syncthreads();
}

// Levenberg-Marquardt fit per case (one 256-thread workgroup per case; every
// workgroup runs exactly `iters` iterations) in x = (u, v), held in L.y.
// y0: [B][65] network outputs or NULL (zeros: the base rule).
// Outputs: yout [B][65] (slot 64 = log10 err), t, alpha [B][32] (rule of
// the fitted outputs, zero past R), err [B].
__global__ __launch_bounds__(256) void k_quad_fit(const int *__restrict__ grids, const double *__restrict__ hmin,
                                                  const int *__restrict__ sent, const double *__restrict__ wts, int S,
                                                  const double *__restrict__ Kref, const int *__restrict__ Rv,
                                                  const float *__restrict__ y0, int iters, double mu0,
                                                  float *__restrict__ yout, double *__restrict__ xout,
                                                  float *__restrict__ Hout, double *__restrict__ tout,
                                                  double *__restrict__ aout, double *__restrict__ errout) {
  extern __shared__ double fit_smem[];
  FitLds &L = *reinterpret_cast<FitLds *>(fit_smem);
  const int b = blockIdx.x, tid = threadIdx.x;
  const int R = min(max(Rv[b], 1), kRmax);
  const double h = hmin[b];
  (void)grids;
  if (tid < kNP) {
    const double yv = y0 ? double(y0[size_t(b) * kOut + tid]) : 0.0;
    const double lim = tid < kRmax ? kUMax : kVMax;
    L.y[tid] = fmin(lim, fmax(-lim, tid < kRmax ? 0.45 * tanh(yv) : tanh(yv)));   // x = (u, v)
  }
  // weighted sums of squares of the reference's potential and field values
  if (tid < S) {
    const double w = wts[size_t(b) * S + tid];
    double dp = 0.0, dh = 0.0;
    for (int c = 0; c < kNcomp; ++c) {
      const double v = Kref[(size_t(b) * S + tid) * kNcomp + c];
      if (c < 3)
        dp += v * v;
      else
        dh += kmult(c) * v * v;
    }
    L.isig[tid][0] = w * dp;
    L.isig[tid][1] = w * dh;
  }
  __syncthreads();
  if (tid == 0) {
    double dp = 0.0, dh = 0.0;
    for (int i = 0; i < S; ++i) {
      dp += L.isig[i][0];
      dh += L.isig[i][1];
    }
    L.dsum[0] = dp;
    L.dsum[1] = dh;
    L.mu = mu0;
    L.err_cur = -1.0;
  }
  __syncthreads();
  if (tid < S) {
    const double w = wts[size_t(b) * S + tid];
    L.isig[tid][0] = sqrt(w / L.dsum[0]);
    L.isig[tid][1] = sqrt(w / L.dsum[1]);
  }
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    fit_nodes(L, L.y, R);
    __syncthreads();
    fit_pass(L, b, S, R, h, sent, Kref, true);
    if (tid == 0) {
      if (L.err_cur < 0.0) L.err_cur = sqrt(L.err2);
      L.ok = 1;
    }
    // damped normal equations; outputs of unused nodes stay fixed
    if (tid < kNP) {
      const bool act = (tid % kRmax) < R;
      if (!act) {
        for (int c = 0; c < kNP; ++c) {
          L.A[tid][c] = 0.0;
          L.A[c][tid] = 0.0;
        }
      }
    }
    __syncthreads();
    if (tid < kNP) {
      const bool act = (tid % kRmax) < R;
      L.A[tid][tid] = act ? L.A[tid][tid] * (1.0 + L.mu) : 1.0;
      if (!act) L.g[tid] = 0.0;
    }
    __syncthreads();
    // Cholesky factorization in place (lower triangle)
    for (int j = 0; j < kNP; ++j) {
      if (tid == 0) {
        const double v = L.A[j][j];
        if (!(v > 0.0)) L.ok = 0;
        L.A[j][j] = sqrt(v > 0.0 ? v : 1.0);
      }
      __syncthreads();
      for (int i = j + 1 + tid; i < kNP; i += blockDim.x) L.A[i][j] /= L.A[j][j];
      __syncthreads();
      const int m = kNP - 1 - j;
      for (int idx = tid; idx < m * m; idx += blockDim.x) {
        const int i = j + 1 + idx / m, l = j + 1 + idx % m;
        if (l <= i) L.A[i][l] -= L.A[i][j] * L.A[l][j];
      }
      __syncthreads();
    }
    if (tid == 0) {
      for (int i = 0; i < kNP; ++i) {
        double v = -L.g[i];
        for (int l = 0; l < i; ++l) v -= L.A[i][l] * L.d[l];
        L.d[i] = v / L.A[i][i];
      }
      for (int i = kNP - 1; i >= 0; --i) {
        double v = L.d[i];
        for (int l = i + 1; l < kNP; ++l) v -= L.A[l][i] * L.d[l];
        L.d[i] = v / L.A[i][i];
      }
    }
    __syncthreads();
    if (tid < kNP) {
      const double lim = tid < kRmax ? kUMax : kVMax;
      L.yc[tid] = fmin(lim, fmax(-lim, L.y[tid] + (L.ok ? L.d[tid] : 0.0)));
    }
    __syncthreads();
    fit_nodes(L, L.yc, R);
    __syncthreads();
    fit_pass(L, b, S, R, h, sent, Kref, false);
    if (tid == 0) {
      const double ec = sqrt(L.err2);
      if (L.ok && ec < L.err_cur) {
        L.err_cur = ec;
        L.mu = fmax(L.mu / 3.0, 1e-12);
        L.ok = 2;  // accepted
      } else {
        L.mu = fmin(L.mu * 4.0, 1e12);
      }
    }
    __syncthreads();
    if (L.ok == 2 && tid < kNP) L.y[tid] = L.yc[tid];
    __syncthreads();
  }
  // final rule, its error and (optionally) the Gauss-Newton matrix J^T J / err^2
  fit_nodes(L, L.y, R);
  __syncthreads();
  fit_pass(L, b, S, R, h, sent, Kref, Hout != nullptr);
  if (tid < kRmax) {
    tout[size_t(b) * kRmax + tid] = tid < R ? L.tp[tid] : 0.0;
    aout[size_t(b) * kRmax + tid] = tid < R ? L.ap[tid] : 0.0;
  }
  const double e = sqrt(L.err2);
  if (tid < kNP) {
    yout[size_t(b) * kOut + tid] = float(tid < kRmax ? atanh(L.y[tid] / 0.45) : atanh(L.y[tid]));
    if (xout) xout[size_t(b) * kNP + tid] = L.y[tid];
  }
  if (tid == 0) {
    yout[size_t(b) * kOut + 64] = float(log10(e));
    errout[b] = e;
  }
  if (Hout) {
    const double ie2 = 1.0 / (e * e);
    for (int idx = tid; idx < kNP * kNP; idx += blockDim.x) {
      const int pr = idx / kNP, pc = idx % kNP;
      const bool act = (pr % kRmax) < R && (pc % kRmax) < R;
      Hout[size_t(b) * kNP * kNP + idx] = act ? float(L.A[pr][pc] * ie2) : 0.0f;
    }
  }
}

// Distillation loss and output gradients (one 64-thread workgroup per case):
//   x(y) = (0.45 tanh y_k, tanh y_{32+k}),  d = x(y) - x*  (active outputs),
//   loss_b = ln(1 + d^T H d) + lambda (y_64 - t_64)^2,
// H = J^T J / err*^2 at the fitted x*, so d^T H d is the Gauss-Newton
// estimate of err(x)^2 / err*^2 - 1.  dY = d loss / d y / B.
__global__ __launch_bounds__(64) void k_distill_grads(const float *__restrict__ Y, const float *__restrict__ T,
                                                      const double *__restrict__ X, const float *__restrict__ H,
                                                      const int *__restrict__ Rv, int B, float lambda,
                                                      float *__restrict__ dY, float *__restrict__ loss) {
  __shared__ double d[kNP];
  __shared__ double part[kNP];
  const int b = blockIdx.x, k = threadIdx.x;
  if (b >= B) return;
  const int R = min(max(Rv[b], 1), kRmax);
  const bool act = (k % kRmax) < R;
  const double y = Y[size_t(b) * kOut + k];
  const double th = tanh(y);
  const double xk = k < kRmax ? 0.45 * th : th;
  const double dxdy = (k < kRmax ? 0.45 : 1.0) * (1.0 - th * th);
  d[k] = act ? xk - X[size_t(b) * kNP + k] : 0.0;
  __syncthreads();
  double hd = 0.0;
  const float *Hr = H + (size_t(b) * kNP + k) * kNP;
  for (int l = 0; l < kNP; ++l) hd += double(Hr[l]) * d[l];
  part[k] = d[k] * hd;
  __syncthreads();
  double q = 0.0;
  for (int l = 0; l < kNP; ++l) q += part[l];
  const float p = Y[size_t(b) * kOut + 64], tgt = T[size_t(b) * kOut + 64];
  dY[size_t(b) * kOut + k] = act ? float(2.0 * hd * dxdy / (1.0 + q) / B) : 0.0f;
  if (k == 0) {
    dY[size_t(b) * kOut + 64] = 2.0f * lambda * (p - tgt) / B;
    loss[b] = float(log1p(q)) + lambda * (p - tgt) * (p - tgt);
  }
}

template <class T>
demag_status dalloc(T **p, size_t n) {
  DEMAG_TRY_HIP(hipMalloc(p, sizeof(T) * std::max<size_t>(n, 1)));
  return DEMAG_OK;
}


demag_status reference_values(demag_ctx *ctx, const int *grids, const double *hmin, const int *sent, int S, int B,
                              double *Kref) {
  const int M = 96;
  double *t = nullptr, *a = nullptr;
  demag_status st = dalloc(&t, size_t(B) * M);
  if (st == DEMAG_OK) st = dalloc(&a, size_t(B) * M);
  if (st != DEMAG_OK) return st;
  k_ref_rules<<<B, 128, 0, ctx->stream>>>(hmin, B, M, t, a);
  k_judge_values<<<(B * S + 127) / 128, 128, 0, ctx->stream>>>(grids, hmin, sent, S, t, a, nullptr, M, B, Kref);
  DEMAG_TRY_HIP(hipGetLastError());
  DEMAG_TRY_HIP(hipStreamSynchronize(ctx->stream));
  (void)hipFree(t);
  (void)hipFree(a);
  return DEMAG_OK;
}

demag_status launch_fit(demag_ctx *ctx, int B, const int *grids, const double *hmin, const int *sent,
                        const double *wts, int S, const double *Kref, const int *R, const float *y0, int iters,
                        double mu0, float *yout, double *xout, float *H, double *t, double *alpha, double *err) {
  const size_t lds = sizeof(FitLds);
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_quad_fit),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  k_quad_fit<<<B, 256, lds, ctx->stream>>>(grids, hmin, sent, wts, S, Kref, R, y0, iters, mu0, yout, xout, H, t,
                                           alpha, err);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

// Offsets and weights of the fit on grid n (the recipe of the header
// comment of demag_quad_offsets); false if count cannot hold the near block.
bool fit_offsets_host(const int n[3], int count, int32_t *J, double *w) {
  static const double dirs[12][3] = {{1, 0, 0},   {0, 1, 0},   {0, 0, 1},   {1, 1, 1},   {1, 1, 0},   {0, 1, 1},
                                     {1, 0, 1},   {1, .5, .25}, {.5, 1, .25}, {.25, .5, 1}, {1, .25, .5}, {.5, .25, 1}};
  std::vector<double> c[3], cum[3];
  for (int d = 0; d < 3; ++d) {
    c[d].resize(n[d]);
    for (int j = 0; j < n[d]; ++j) c[d][j] = double((n[d] - j) * (j == 0 ? 1 : 2));
    cum[d].assign(1, 0.0);
    double acc = 0.0;
    for (double v : c[d]) {
      acc += v;
      cum[d].push_back(acc);
    }
  }
  int S = 0;
  for (int z = 0; z < std::min(4, n[2]); ++z)
    for (int y = 0; y < std::min(4, n[1]); ++y)
      for (int x = 0; x < std::min(4, n[0]); ++x) {
        if (S >= count) return false;
        J[3 * S] = x;
        J[3 * S + 1] = y;
        J[3 * S + 2] = z;
        w[S] = c[0][x] * c[1][y] * c[2][z];
        ++S;
      }
  auto total = [&](int sv) {
    return cum[0][std::min(sv, n[0])] * cum[1][std::min(sv, n[1])] * cum[2][std::min(sv, n[2])];
  };
  const int smax = std::max(n[0], std::max(n[1], n[2])) - 1;
  const int G = std::min((count - S) / 8, std::max(0, smax - 3));
  if (G > 0) {
    std::vector<int> edges{4};
    for (int g = 1; g < G; ++g)
      edges.push_back(std::max(edges.back() + 1,
                               int(std::nearbyint(4.0 * std::pow((smax + 1) / 4.0, double(g) / double(G))))));
    edges.push_back(smax + 1);
    std::vector<int> uniq;
    for (int v : edges) {
      v = std::min(v, smax + 1);
      if (uniq.empty() || v != uniq.back()) uniq.push_back(v);
    }
    for (size_t g = 0; g + 1 < uniq.size(); ++g) {
      const int lo = uniq[g], hi = uniq[g + 1];
      const double wg = (total(hi) - total(lo)) / 8.0;
      const int sg = int(std::nearbyint(std::sqrt(double(int64_t(lo) * (hi - 1)))));
      for (int i = 0; i < 8; ++i) {
        const double *u = dirs[(g + i) % 12];
        for (int d = 0; d < 3; ++d) J[3 * S + d] = std::min(int(std::nearbyint(sg * u[d])), n[d] - 1);
        w[S] = wg;
        ++S;
      }
    }
  }
  for (; S < count; ++S) {
    J[3 * S] = J[3 * S + 1] = J[3 * S + 2] = 0;
    w[S] = 0.0;
  }
  return true;
}

// Network input of one case (the layout of demag_quad_features).
void features_host(const int n[3], double h, double log10_tol, int R, float x[6]) {
  const double nmax = double(std::max(n[0], std::max(n[1], n[2])));
  for (int d = 0; d < 3; ++d) x[d] = float(double(n[d]) / nmax);
  x[3] = float(std::log2(1.0 / h) / 6.0 - 1.0);
  x[4] = float((log10_tol + 6.5) / 2.5);
  x[5] = float((double(R) - 24.0) / 8.0);
}

// Sample positions and weights of one axis for the certificate.
void cert_axis(int n, std::vector<int> &pos, std::vector<double> &w) {
  pos.clear();
  w.clear();
  auto c = [n](int j) { return double((n - j) * (j == 0 ? 1 : 2)); };
  for (int j = 0; j < std::min(n, kCertExact); ++j) {
    pos.push_back(j);
    w.push_back(c(j));
  }
  // octave [lo, 2 lo) in blocks of `blk` cells, blk = 4, 8, 16, ...
  for (int lo = kCertExact, blk = 4; lo < n; lo *= 2, blk *= 2)
    for (int b0 = lo; b0 < std::min(n, 2 * lo); b0 += blk) {
      const int b1 = std::min(std::min(n, 2 * lo), b0 + blk);
      double sw = 0.0;
      for (int j = b0; j < b1; ++j) sw += c(j);
      pos.push_back((b0 + b1 - 1) / 2);
      w.push_back(sw);
    }
}

// Certificate of the rule (t, alpha; M nodes, scaled domain) on grid n with
// scaled cell sizes hs (cubic cells: the factor tables use hs[d] per axis):
// out = (e_phi, e_h) against the reference rule of the smallest cell.
demag_status certify_rule(demag_ctx *ctx, const int n[3], const double hs[3], int M, const double *t,
                          const double *alpha, double out[2]) {
  const int Mref = 96;
  const int KT = M + Mref;
  const double hmin = std::min(hs[0], std::min(hs[1], hs[2]));
  std::vector<double> tau(KT), wcr(KT);
  {
    const double a = 2.0, bb = 0.25 * (0.5 * hmin) * (0.5 * hmin);
    const double theta = std::log(2.0 * kPi * a * Mref / bb) / (a * Mref);
    for (int k = 0; k < KT; ++k) {
      double tk, ak;
      if (k < M) {
        tk = t[k];
        ak = alpha[k];
      } else {
        tk = (k - M + 1) * theta;
        const double sh = std::sinh(tk);
        ak = 2.0 * theta * std::cosh(tk) * sh * sh;
      }
      tau[k] = std::sinh(tk);
      wcr[k] = std::cbrt(ak / (2.0 * std::pow(kPi, 1.5)));
    }
  }
  std::vector<int> pos[3];
  std::vector<double> wts[3];
  for (int d = 0; d < 3; ++d) cert_axis(n[d], pos[d], wts[d]);
  const int np[3] = {int(pos[0].size()), int(pos[1].size()), int(pos[2].size())};
  double *d_tau = nullptr, *d_wcr = nullptr, *d_T[3] = {nullptr, nullptr, nullptr},
         *d_w[3] = {nullptr, nullptr, nullptr}, *d_part = nullptr, *d_out = nullptr;
  int *d_pos[3] = {nullptr, nullptr, nullptr};
  const int nblk = std::max(1, std::min(np[1] * np[2], 4096));
  demag_status st = dalloc(&d_tau, KT);
  if (st == DEMAG_OK) st = dalloc(&d_wcr, KT);
  for (int d = 0; d < 3 && st == DEMAG_OK; ++d) {
    st = dalloc(&d_T[d], size_t(4) * KT * np[d]);
    if (st == DEMAG_OK) st = dalloc(&d_w[d], np[d]);
    if (st == DEMAG_OK) st = dalloc(&d_pos[d], np[d]);
  }
  if (st == DEMAG_OK) st = dalloc(&d_part, size_t(nblk) * 4);
  if (st == DEMAG_OK) st = dalloc(&d_out, 4);
  double sums[4] = {0, 0, 0, 0};
  if (st == DEMAG_OK) {
    hipError_t e = hipMemcpyAsync(d_tau, tau.data(), sizeof(double) * KT, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_wcr, wcr.data(), sizeof(double) * KT, hipMemcpyHostToDevice, ctx->stream);
    for (int d = 0; d < 3 && e == hipSuccess; ++d) {
      e = hipMemcpyAsync(d_pos[d], pos[d].data(), sizeof(int) * np[d], hipMemcpyHostToDevice, ctx->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(d_w[d], wts[d].data(), sizeof(double) * np[d], hipMemcpyHostToDevice, ctx->stream);
      if (e == hipSuccess) {
        dim3 g((np[d] + 127) / 128, KT);
        k_cert_factors<<<g, 128, 0, ctx->stream>>>(d_pos[d], np[d], d_tau, d_wcr, KT, hs[d], d_T[d]);
        e = hipGetLastError();
      }
    }
    if (e == hipSuccess) {
      k_cert_sums<<<nblk, 256, sizeof(double) * 6 * KT, ctx->stream>>>(d_T[0], d_T[1], d_T[2], d_w[0], d_w[1], d_w[2],
                                                                       np[0], np[1], np[2], KT, M, d_part);
      k_cert_final<<<1, 256, 0, ctx->stream>>>(d_part, nblk, d_out);
      e = hipGetLastError();
    }
    // the host vectors above stay alive until this synchronization
    if (e == hipSuccess) e = hipMemcpyAsync(sums, d_out, sizeof(sums), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      set_error(std::string("certificate: ") + hipGetErrorString(e));
      st = DEMAG_E_HIP;
    }
  }
  for (void *q : {(void *)d_tau, (void *)d_wcr, (void *)d_part, (void *)d_out, (void *)d_T[0], (void *)d_T[1],
                  (void *)d_T[2], (void *)d_w[0], (void *)d_w[1], (void *)d_w[2], (void *)d_pos[0], (void *)d_pos[1],
                  (void *)d_pos[2]})
    if (q) (void)hipFree(q);
  if (st == DEMAG_OK) {
    out[0] = std::sqrt(sums[0] / sums[1]);
    out[1] = std::sqrt(sums[2] / sums[3]);
  }
  return st;
}

}  // namespace
}  // namespace demag

using namespace demag;

extern "C" {

int32_t demag_mlp_param_count(void) { return kParams; }

demag_status demag_mlp_forward(demag_ctx *ctx, const float *params, const float *x, int32_t B, float *y,
                               float *z, float *a) {
  DEMAG_REQUIRE(ctx && params && x && y, "demag_mlp_forward: NULL argument");
  DEMAG_REQUIRE(B >= 1, "demag_mlp_forward: B must be >= 1");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  k_mlp_forward<<<B, 64, 0, ctx->stream>>>(params, x, B, y, z, a);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

demag_status demag_mlp_backward(demag_ctx *ctx, const float *params, const float *x, const float *z, const float *a,
                                const float *dy, int32_t B, float *delta, float *grad) {
  DEMAG_REQUIRE(ctx && params && x && z && a && dy && delta && grad, "demag_mlp_backward: NULL argument");
  DEMAG_REQUIRE(B >= 1, "demag_mlp_backward: B must be >= 1");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  k_mlp_delta<<<B, 64, 0, ctx->stream>>>(params, z, dy, B, delta);
  k_mlp_grad<<<(kParams + 255) / 256, 256, 0, ctx->stream>>>(x, a, delta, dy, B, grad);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

demag_status demag_adam_step(demag_ctx *ctx, float *params, const float *grad, float *m, float *v, int32_t count,
                             int32_t step, float lr, float b1, float b2, float eps) {
  DEMAG_REQUIRE(ctx && params && grad && m && v, "demag_adam_step: NULL argument");
  DEMAG_REQUIRE(count >= 1 && step >= 1, "demag_adam_step: count and step must be >= 1");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  k_adam<<<(count + 255) / 256, 256, 0, ctx->stream>>>(params, grad, m, v, count, step, lr, b1, b2, eps);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

demag_status demag_quad_judge(demag_ctx *ctx, int32_t B, const int32_t *grids, const double *hmin,
                              const int32_t *sent, const double *weights, int32_t S, const double *t,
                              const double *alpha, const int32_t *R, int32_t KM, double *err, double *parts,
                              double *dt, double *dalpha) {
  DEMAG_REQUIRE(ctx && grids && hmin && sent && weights && t && alpha && R && err, "demag_quad_judge: NULL argument");
  DEMAG_REQUIRE(B >= 1 && S >= 1 && KM >= 1 && KM <= 256, "demag_quad_judge: sizes out of range");
  DEMAG_REQUIRE((dt == nullptr) == (dalpha == nullptr), "demag_quad_judge: give both gradients or neither");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  double *Kref = nullptr, *K = nullptr, *resid = nullptr;
  demag_status st = dalloc(&Kref, size_t(B) * S * kNcomp);
  if (st == DEMAG_OK) st = dalloc(&K, size_t(B) * S * kNcomp);
  if (st == DEMAG_OK) st = dalloc(&resid, size_t(B) * S * kNcomp);
  if (st == DEMAG_OK) st = reference_values(ctx, grids, hmin, sent, S, B, Kref);
  if (st == DEMAG_OK) {
    k_judge_values<<<(B * S + 127) / 128, 128, 0, ctx->stream>>>(grids, hmin, sent, S, t, alpha, R, KM, B, K);
    k_judge_err<<<(B + 127) / 128, 128, 0, ctx->stream>>>(K, Kref, weights, B, S, err, parts, resid);
    if (dt)
      k_judge_grad<<<(B * KM + 127) / 128, 128, 0, ctx->stream>>>(grids, hmin, sent, S, t, alpha, R, KM, B, resid,
                                                                 err, dt, dalpha);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error(hipGetErrorString(e));
      st = DEMAG_E_HIP;
    } else if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
      set_error("demag_quad_judge: stream synchronization failed");
      st = DEMAG_E_HIP;
    }
  }
  for (double *q : {Kref, K, resid})
    if (q) (void)hipFree(q);
  return st;
}

demag_status demag_quad_rules(demag_ctx *ctx, const float *y, const int32_t *R, int32_t B, double *t,
                              double *alpha) {
  DEMAG_REQUIRE(ctx && R && t && alpha, "demag_quad_rules: NULL argument");
  DEMAG_REQUIRE(B >= 1, "demag_quad_rules: B must be >= 1");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  k_rules<<<B, kRmax, 0, ctx->stream>>>(y, R, B, kRmax, t, alpha);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

demag_status demag_quad_loss_grad(demag_ctx *ctx, const float *y, const float *targets, const double *xfit,
                                  const float *H, const int32_t *R, int32_t B, float lambda, float *dy,
                                  float *loss) {
  DEMAG_REQUIRE(ctx && y && targets && R && dy && loss, "demag_quad_loss_grad: NULL argument");
  DEMAG_REQUIRE((xfit == nullptr) == (H == nullptr), "demag_quad_loss_grad: give both xfit and H or neither");
  DEMAG_REQUIRE(B >= 1, "demag_quad_loss_grad: B must be >= 1");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  if (H)
    k_distill_grads<<<B, 64, 0, ctx->stream>>>(y, targets, xfit, H, R, B, lambda, dy, loss);
  else
    k_target_grads<<<B, 128, 0, ctx->stream>>>(y, targets, R, B, lambda, dy, loss);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

demag_status demag_quad_train(demag_ctx *ctx, float *params, float *adam_m, float *adam_v, const float *x,
                              const float *targets, const double *xfit, const float *H, const int32_t *R,
                              int32_t count, int32_t steps, int32_t batch, int32_t step0, float lr, float lambda,
                              float *loss_host) {
  DEMAG_REQUIRE(ctx && params && adam_m && adam_v && x && targets && R, "demag_quad_train: NULL argument");
  DEMAG_REQUIRE((xfit == nullptr) == (H == nullptr), "demag_quad_train: give both xfit and H or neither");
  DEMAG_REQUIRE(count >= 1 && steps >= 0 && batch >= 1 && batch <= count && step0 >= 0,
                "demag_quad_train: sizes out of range");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  float *Y = nullptr, *Z = nullptr, *A = nullptr, *D = nullptr, *dY = nullptr, *G = nullptr, *loss = nullptr;
  demag_status st = DEMAG_OK;
  for (auto pp : {&Y, &dY}) if (st == DEMAG_OK) st = dalloc(pp, size_t(batch) * kOut);
  for (auto pp : {&Z, &A, &D}) if (st == DEMAG_OK) st = dalloc(pp, size_t(batch) * 3 * kH);
  if (st == DEMAG_OK) st = dalloc(&G, kParams);
  if (st == DEMAG_OK) st = dalloc(&loss, size_t(steps) * batch);
  for (int it = 0; st == DEMAG_OK && it < steps; ++it) {
    // contiguous minibatch of the (caller-shuffled) cases, wrapping around
    const int first = int((int64_t(it) * batch) % count);
    const int nb = std::min(batch, count - first);
    const float *xb = x + size_t(first) * kIn;
    k_mlp_forward<<<nb, 64, 0, ctx->stream>>>(params, xb, nb, Y, Z, A);
    if (H)
      k_distill_grads<<<nb, 64, 0, ctx->stream>>>(Y, targets + size_t(first) * kOut, xfit + size_t(first) * kNP,
                                                  H + size_t(first) * kNP * kNP, R + first, nb, lambda, dY,
                                                  loss + size_t(it) * batch);
    else
      k_target_grads<<<nb, 128, 0, ctx->stream>>>(Y, targets + size_t(first) * kOut, R + first, nb, lambda, dY,
                                                 loss + size_t(it) * batch);
    k_mlp_delta<<<nb, 64, 0, ctx->stream>>>(params, Z, dY, nb, D);
    k_mlp_grad<<<(kParams + 255) / 256, 256, 0, ctx->stream>>>(xb, A, D, dY, nb, G);
    k_adam<<<(kParams + 255) / 256, 256, 0, ctx->stream>>>(params, G, adam_m, adam_v, kParams, step0 + it + 1, lr,
                                                          0.9f, 0.999f, 1e-8f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error(std::string("demag_quad_train: ") + hipGetErrorString(e));
      st = DEMAG_E_HIP;
    }
    if (loss_host && st == DEMAG_OK) {
      // mean loss of the step (host copy; the per-case values stay on the device)
      std::vector<float> lb(nb);
      if (hipMemcpyAsync(lb.data(), loss + size_t(it) * batch, sizeof(float) * nb, hipMemcpyDeviceToHost,
                         ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess) {
        set_error("demag_quad_train: loss copy failed");
        st = DEMAG_E_HIP;
      } else {
        double sum = 0;
        for (float v : lb) sum += v;
        loss_host[it] = float(sum / nb);
      }
    }
  }
  (void)hipStreamSynchronize(ctx->stream);
  for (float *p : {Y, Z, A, D, dY, G, loss})
    if (p) (void)hipFree(p);
  return st;
}

demag_status demag_quad_fit(demag_ctx *ctx, int32_t B, const int32_t *grids, const double *hmin,
                            const int32_t *sent, const double *weights, int32_t S, const int32_t *R, const float *y0,
                            int32_t iters, double mu0, float *yout, double *xout, float *H, double *t, double *alpha,
                            double *err) {
  DEMAG_REQUIRE(ctx && grids && hmin && sent && weights && R && yout && t && alpha && err,
                "demag_quad_fit: NULL argument");
  DEMAG_REQUIRE(B >= 1 && S >= 1 && S <= kMaxS && iters >= 0 && mu0 > 0, "demag_quad_fit: sizes out of range");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  double *Kref = nullptr;
  demag_status st = dalloc(&Kref, size_t(B) * S * kNcomp);
  if (st == DEMAG_OK) st = reference_values(ctx, grids, hmin, sent, S, B, Kref);
  if (st == DEMAG_OK)
    st = launch_fit(ctx, B, grids, hmin, sent, weights, S, Kref, R, y0, iters, mu0, yout, xout, H, t, alpha, err);
  if (st == DEMAG_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) {
    set_error("demag_quad_fit: stream synchronization failed");
    st = DEMAG_E_HIP;
  }
  if (Kref) (void)hipFree(Kref);
  return st;
}

demag_status demag_quad_offsets(const int32_t n[3], int32_t count, int32_t *J, double *w) {
  DEMAG_REQUIRE(n && J && w, "demag_quad_offsets: NULL argument");
  DEMAG_REQUIRE(n[0] >= 1 && n[1] >= 1 && n[2] >= 1 && n[0] <= 4096 && n[1] <= 4096 && n[2] <= 4096 && count >= 1,
                "demag_quad_offsets: sizes out of range");
  const int nn[3] = {n[0], n[1], n[2]};
  DEMAG_REQUIRE(fit_offsets_host(nn, count, J, w), "demag_quad_offsets: count too small for the near block");
  return DEMAG_OK;
}

demag_status demag_quad_features(const int32_t n[3], double h, double log10_tol, int32_t R, float *x) {
  DEMAG_REQUIRE(n && x, "demag_quad_features: NULL argument");
  DEMAG_REQUIRE(n[0] >= 1 && n[1] >= 1 && n[2] >= 1 && h > 0, "demag_quad_features: sizes out of range");
  const int nn[3] = {n[0], n[1], n[2]};
  features_host(nn, h, log10_tol, R, x);
  return DEMAG_OK;
}

namespace {
// Scaled grid of a demag_grid: n, the scaled cell sizes (longest extent 1).
demag_status scaled_grid(const demag_grid *g, int n[3], double hs[3], const char *where) {
  double L = 0.0;
  for (int d = 0; d < 3; ++d) {
    DEMAG_REQUIRE(g->n[d] >= 1 && g->n[d] <= 4096 && g->h[d] > 0 && std::isfinite(g->h[d]),
                  std::string(where) + ": grid out of range");
    n[d] = g->n[d];
    L = std::max(L, g->n[d] * g->h[d]);
  }
  for (int d = 0; d < 3; ++d) hs[d] = g->h[d] / L;
  return DEMAG_OK;
}
}  // namespace

demag_status demag_quad_certify(demag_ctx *ctx, const demag_grid *grid, int32_t M, const double *t,
                                const double *alpha, double err[2]) {
  DEMAG_REQUIRE(ctx && grid && t && alpha && err, "demag_quad_certify: NULL argument");
  DEMAG_REQUIRE(M >= 1 && M <= 256, "demag_quad_certify: M out of range");
  for (int k = 0; k < M; ++k)
    DEMAG_REQUIRE(std::isfinite(t[k]) && t[k] > 0 && std::isfinite(alpha[k]), "demag_quad_certify: bad node");
  int n[3];
  double hs[3];
  demag_status st = scaled_grid(grid, n, hs, "demag_quad_certify");
  if (st != DEMAG_OK) return st;
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  return certify_rule(ctx, n, hs, M, t, alpha, err);
}

// Shortened rule for one grid.  Modes:
//   DEMAG_PREDICT_NETWORK: the network's error head picks the smallest R'
//     (16..32) it expects to meet tol; the plain base rule with R' nodes is
//     fitted by fit_iters Levenberg-Marquardt steps on the grid's weighted
//     offsets and certified; on a miss R' + 1, R' + 2, ... (up to 32) follow;
//   DEMAG_PREDICT_NETWORK_PROPOSAL: the same R' schedule, fits started from
//     the network's proposed nodes and weights for that R' (measured to be
//     no better a start than the plain rule);
//   DEMAG_PREDICT_SEARCH: no network: bisection over R' = 16..32 for the
//     smallest R' whose fit (from the plain base rule) is certified within
//     tol (R' = 32 first; the certified error falls with R').
// If nothing meets tol, the sinc rule with the step of Thm. sinc_theo is
// returned with the fewest nodes in 33..64 whose certificate meets tol
// (fell_back = 1; with 64 nodes and DEMAG_E_ACCURACY if even 64 miss tol).
demag_status demag_quad_predict(demag_ctx *ctx, const float *params, const demag_grid *grid, double tol,
                                int32_t fit_iters, int32_t mode, demag_quad_result *out) {
  DEMAG_REQUIRE(ctx && grid && out, "demag_quad_predict: NULL argument");
  DEMAG_REQUIRE(mode == DEMAG_PREDICT_NETWORK || mode == DEMAG_PREDICT_NETWORK_PROPOSAL ||
                    mode == DEMAG_PREDICT_SEARCH,
                "demag_quad_predict: unknown mode");
  DEMAG_REQUIRE(params || mode == DEMAG_PREDICT_SEARCH, "demag_quad_predict: the network modes need params");
  DEMAG_REQUIRE(tol > 0 && fit_iters >= 0, "demag_quad_predict: tol or fit_iters out of range");
  int n[3];
  double hs[3];
  demag_status st = scaled_grid(grid, n, hs, "demag_quad_predict");
  if (st != DEMAG_OK) return st;
  if (!(std::fabs(hs[1] - hs[0]) <= 1e-12 * hs[0] && std::fabs(hs[2] - hs[0]) <= 1e-12 * hs[0])) {
    set_error("demag_quad_predict: the shortened rules are trained and judged for cubic cells");
    return DEMAG_E_UNSUPPORTED;
  }
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  const auto clock0 = std::chrono::steady_clock::now();
  const double hmin = hs[0];
  const int S = kMaxS, NC = 17;
  std::vector<int32_t> Jh(size_t(3) * S);
  std::vector<double> wh(S);
  (void)fit_offsets_host(n, S, Jh.data(), wh.data());
  std::vector<float> xh(size_t(NC) * kIn), yh(size_t(NC) * kOut, 0.0f);
  for (int c = 0; c < NC; ++c) features_host(n, hmin, std::log10(tol), 16 + c, xh.data() + size_t(c) * kIn);

  float *X = nullptr, *Y = nullptr, *yfit = nullptr;
  int32_t *dR = nullptr, *dgrid = nullptr, *dsent = nullptr;
  double *dh = nullptr, *dw = nullptr, *dt = nullptr, *da = nullptr, *derr = nullptr, *Kref = nullptr;
  st = dalloc(&X, xh.size());
  if (st == DEMAG_OK) st = dalloc(&Y, yh.size());
  if (st == DEMAG_OK) st = dalloc(&yfit, kOut);
  if (st == DEMAG_OK) st = dalloc(&dR, 1);
  if (st == DEMAG_OK) st = dalloc(&dgrid, 3);
  if (st == DEMAG_OK) st = dalloc(&dsent, size_t(3) * S);
  if (st == DEMAG_OK) st = dalloc(&dh, 1);
  if (st == DEMAG_OK) st = dalloc(&dw, S);
  if (st == DEMAG_OK) st = dalloc(&dt, kRmax);
  if (st == DEMAG_OK) st = dalloc(&da, kRmax);
  if (st == DEMAG_OK) st = dalloc(&derr, 1);
  if (st == DEMAG_OK) st = dalloc(&Kref, size_t(S) * kNcomp);
  auto copy_failed = [&](const char *what) {
    set_error(std::string("demag_quad_predict: ") + what);
    st = DEMAG_E_HIP;
  };
  if (st == DEMAG_OK) {
    const int32_t n32[3] = {n[0], n[1], n[2]};
    if (hipMemcpyAsync(dgrid, n32, sizeof(n32), hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(dh, &hmin, sizeof(double), hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(dsent, Jh.data(), sizeof(int32_t) * Jh.size(), hipMemcpyHostToDevice, ctx->stream) !=
            hipSuccess ||
        hipMemcpyAsync(dw, wh.data(), sizeof(double) * S, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(X, xh.data(), sizeof(float) * xh.size(), hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
      copy_failed("copy failed");
  }
  if (st == DEMAG_OK) st = reference_values(ctx, dgrid, dh, dsent, S, 1, Kref);   // synchronizes
  out->predicted = std::nan("");
  if (st == DEMAG_OK && mode != DEMAG_PREDICT_SEARCH) {
    k_mlp_forward<<<NC, 64, 0, ctx->stream>>>(params, X, NC, Y, nullptr, nullptr);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(yh.data(), Y, sizeof(float) * yh.size(), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      copy_failed("network forward failed");
  }
  int fits = 0;
  // fit R' nodes from the network's outputs (use_net) or the plain base rule,
  // then certify: (t, alpha, e_phi, e_h)
  struct Cand {
    int R = 0;
    std::vector<double> t, a;
    double e[2] = {0, 0};
    bool ok = false;
  };
  auto run = [&](int Rp, bool use_net, Cand &c) -> demag_status {
    c.R = Rp;
    if (hipMemcpyAsync(dR, &Rp, sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream) != hipSuccess) {
      copy_failed("copy failed");
      return st;
    }
    demag_status s2 = launch_fit(ctx, 1, dgrid, dh, dsent, dw, S, Kref, dR,
                                 use_net ? Y + size_t(Rp - 16) * kOut : nullptr, fit_iters, 1e-3, yfit, nullptr,
                                 nullptr, dt, da, derr);
    if (s2 != DEMAG_OK) return s2;
    ++fits;
    std::vector<double> th(kRmax), ah(kRmax);
    if (hipMemcpyAsync(th.data(), dt, sizeof(double) * kRmax, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(ah.data(), da, sizeof(double) * kRmax, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      copy_failed("copy failed");
      return st;
    }
    c.t.assign(th.begin(), th.begin() + Rp);
    c.a.assign(ah.begin(), ah.begin() + Rp);
    s2 = certify_rule(ctx, n, hs, Rp, c.t.data(), c.a.data(), c.e);
    c.ok = (s2 == DEMAG_OK) && std::max(c.e[0], c.e[1]) <= tol;
    return s2;
  };
  Cand best;
  if (st == DEMAG_OK) {
    if (mode == DEMAG_PREDICT_SEARCH) {
      Cand c;
      st = run(32, false, c);
      if (st == DEMAG_OK && c.ok) {
        best = c;
        int lo = 16, hi = 32;
        while (st == DEMAG_OK && lo < hi) {
          const int mid = (lo + hi) / 2;
          st = run(mid, false, c);
          if (st != DEMAG_OK) break;
          if (c.ok) {
            hi = mid;
            best = c;
          } else {
            lo = mid + 1;
          }
        }
      }
    } else {
      int pick = NC - 1;
      for (int c = 0; c < NC; ++c)
        if (yh[size_t(c) * kOut + 64] <= std::log10(tol)) {
          pick = c;
          break;
        }
      out->predicted = yh[size_t(pick) * kOut + 64];
      for (int Rp = 16 + pick; st == DEMAG_OK && Rp <= 32; ++Rp) {
        Cand c;
        st = run(Rp, mode == DEMAG_PREDICT_NETWORK_PROPOSAL, c);
        if (st == DEMAG_OK && c.ok) {
          best = c;
          break;
        }
      }
    }
  }
  if (st == DEMAG_OK) {
    if (best.ok) {
      out->fell_back = 0;
    } else {
      // fallback: the sinc rule with the step of Thm. sinc_theo, the fewest
      // nodes in 33..64 whose certificate meets tol (64 first; then
      // bisection, keeping only certified candidates), 64 if none does
      auto theorem_rule = [&](int M, Cand &c) -> demag_status {
        const double a = 2.0, bb = 0.25 * (0.5 * hmin) * (0.5 * hmin);
        const double theta = std::log(2.0 * kPi * a * M / bb) / (a * M);
        c.R = M;
        c.t.resize(M);
        c.a.resize(M);
        for (int k = 0; k < M; ++k) {
          const double tk = (k + 1) * theta, sh = std::sinh(tk);
          c.t[k] = tk;
          c.a[k] = 2.0 * theta * std::cosh(tk) * sh * sh;
        }
        demag_status s2 = certify_rule(ctx, n, hs, M, c.t.data(), c.a.data(), c.e);
        c.ok = (s2 == DEMAG_OK) && std::max(c.e[0], c.e[1]) <= tol;
        return s2;
      };
      st = theorem_rule(64, best);
      if (st == DEMAG_OK && best.ok) {
        int lo = 33, hi = 63;
        while (st == DEMAG_OK && lo <= hi) {
          const int mid = (lo + hi) / 2;
          Cand c;
          st = theorem_rule(mid, c);
          if (st != DEMAG_OK) break;
          if (c.ok) {
            best = c;
            hi = mid - 1;
          } else {
            lo = mid + 1;
          }
        }
      }
      out->fell_back = 1;
    }
  }
  if (st == DEMAG_OK) {
    out->R = best.R;
    out->mode = mode;
    out->fits = fits;
    out->err_phi = best.e[0];
    out->err_h = best.e[1];
    for (int k = 0; k < 64; ++k) {
      out->t[k] = k < best.R ? best.t[k] : 0.0;
      out->alpha[k] = k < best.R ? best.a[k] : 0.0;
    }
  }
  for (void *q : {(void *)X, (void *)Y, (void *)yfit, (void *)dR, (void *)dgrid, (void *)dsent, (void *)dh,
                  (void *)dw, (void *)dt, (void *)da, (void *)derr, (void *)Kref})
    if (q) (void)hipFree(q);
  out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - clock0).count();
  if (st == DEMAG_OK && !best.ok) {
    set_error("demag_quad_predict: the fallback rule misses tol as well");
    return DEMAG_E_ACCURACY;
  }
  return st;
}

}  // extern "C"
