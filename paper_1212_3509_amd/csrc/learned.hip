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
// Judge: at S sentinel offsets J, nine kernel values per rule
//   [K^x, K^y, K^z, F_xx, F_yy, F_zz, F_xy, F_xz, F_yz]
//   K^q  = W prod_d f_d with f = X along q, E elsewhere;
//   F_pq = the same for h_p <- m_q with axis p differentiated (X -> P = -X',
//          E -> Q = 2 tau^2 X), W = alpha / (2 pi^(3/2)),
// err = sqrt(mean_J |K - K_ref|^2 / |K_ref|^2), K_ref from the sinc rule with
// the step of Thm. sinc_theo and 96 nodes.
// Fit: residuals r = (K - K_ref)(J) / sqrt(S |K_ref(J)|^2) (|r| = err);
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

// err per case and the scaled residuals (K - K_ref)/|K_ref|^2 per sentinel.
__global__ void k_judge_err(const double *__restrict__ K, const double *__restrict__ Kref, int B, int S,
                            double *__restrict__ err, double *__restrict__ resid) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double sum = 0.0;
  for (int s = 0; s < S; ++s) {
    const double *k = K + (size_t(b) * S + s) * kNcomp;
    const double *r = Kref + (size_t(b) * S + s) * kNcomp;
    double num = 0.0, den = 0.0;
    for (int c = 0; c < kNcomp; ++c) {
      num += (k[c] - r[c]) * (k[c] - r[c]);
      den += r[c] * r[c];
    }
    sum += num / den;
    if (resid)
      for (int c = 0; c < kNcomp; ++c) resid[(size_t(b) * S + s) * kNcomp + c] = (k[c] - r[c]) / den;
  }
  err[b] = sqrt(sum / S);
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
    const double scale = 1.0 / (S * err[b]);
    gt *= scale;
    ga *= scale;
  }
  dt[idx] = gt;
  dalpha[idx] = ga;
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
  double sig[kMaxS];
  double err2, err_cur, mu;
  int ok;
};

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
      const double is = 1.0 / L.sig[s];
#pragma unroll
      for (int c = 0; c < kNcomp; ++c) {
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
        r = (sum - Kref[(size_t(b) * S + rs) * kNcomp + c]) / L.sig[rs];
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
                                                  const int *__restrict__ sent, int S,
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
  if (tid < S) {
    double den = 0.0;
    for (int c = 0; c < kNcomp; ++c) {
      const double v = Kref[(size_t(b) * S + tid) * kNcomp + c];
      den += v * v;
    }
    L.sig[tid] = sqrt(den * S);
  }
  if (tid == 0) {
    L.mu = mu0;
    L.err_cur = -1.0;
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

demag_status launch_fit(demag_ctx *ctx, int B, const int *grids, const double *hmin, const int *sent, int S,
                        const double *Kref, const int *R, const float *y0, int iters, double mu0, float *yout,
                        double *xout, float *H, double *t, double *alpha, double *err) {
  const size_t lds = sizeof(FitLds);
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_quad_fit),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  k_quad_fit<<<B, 256, lds, ctx->stream>>>(grids, hmin, sent, S, Kref, R, y0, iters, mu0, yout, xout, H, t, alpha,
                                           err);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
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
                              const int32_t *sent, int32_t S, const double *t, const double *alpha, const int32_t *R,
                              int32_t KM, double *err, double *dt, double *dalpha) {
  DEMAG_REQUIRE(ctx && grids && hmin && sent && t && alpha && R && err, "demag_quad_judge: NULL argument");
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
    k_judge_err<<<(B + 127) / 128, 128, 0, ctx->stream>>>(K, Kref, B, S, err, resid);
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
  for (double *p : {Kref, K, resid})
    if (p) (void)hipFree(p);
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
                            const int32_t *sent, int32_t S, const int32_t *R, const float *y0, int32_t iters,
                            double mu0, float *yout, double *xout, float *H, double *t, double *alpha,
                            double *err) {
  DEMAG_REQUIRE(ctx && grids && hmin && sent && R && yout && t && alpha && err, "demag_quad_fit: NULL argument");
  DEMAG_REQUIRE(B >= 1 && S >= 1 && S <= kMaxS && iters >= 0 && mu0 > 0, "demag_quad_fit: sizes out of range");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  double *Kref = nullptr;
  demag_status st = dalloc(&Kref, size_t(B) * S * kNcomp);
  if (st == DEMAG_OK) st = reference_values(ctx, grids, hmin, sent, S, B, Kref);
  if (st == DEMAG_OK)
    st = launch_fit(ctx, B, grids, hmin, sent, S, Kref, R, y0, iters, mu0, yout, xout, H, t, alpha, err);
  if (st == DEMAG_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) {
    set_error("demag_quad_fit: stream synchronization failed");
    st = DEMAG_E_HIP;
  }
  if (Kref) (void)hipFree(Kref);
  return st;
}

// Shortened rule for one grid: the network's predicted-error head picks the
// smallest R' (16..32) it expects to meet tol; that proposal (and the plain
// base rule, as a guard) is polished by `fit_iters` Levenberg-Marquardt
// steps on the grid's fit offsets, and the better one is judged on the
// check offsets (not seen by the fit); if it misses tol, R' + 4, R' + 8, ... (up to 32) are tried the
// same way, and if none meets tol the sinc rule with the step of
// Thm. sinc_theo and 64 nodes is returned (*fell_back = 1).
demag_status demag_quad_predict(demag_ctx *ctx, const float *params, const float *features, const int32_t n[3],
                                double hmin, const int32_t *sent, int32_t S, const int32_t *check, int32_t Sc,
                                double tol, int32_t fit_iters, double *t_out, double *alpha_out, int32_t *R_out,
                                double *judged, double *predicted, int32_t *fell_back) {
  DEMAG_REQUIRE(ctx && params && features && n && sent && check && t_out && alpha_out && R_out && judged &&
                    predicted && fell_back,
                "demag_quad_predict: NULL argument");
  DEMAG_REQUIRE(tol > 0 && hmin > 0 && S >= 1 && S <= kMaxS && Sc >= 1 && fit_iters >= 0,
                "demag_quad_predict: tol, hmin, S, Sc or fit_iters out of range");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  const int NC = 17;
  float *Y = nullptr, *yfit = nullptr;
  int32_t *dR = nullptr, *dgrid = nullptr;
  double *dh = nullptr, *dt = nullptr, *da = nullptr, *derr = nullptr, *Kref = nullptr, *KrefC = nullptr,
         *Kc = nullptr;
  demag_status st = dalloc(&Y, size_t(NC) * kOut);
  if (st == DEMAG_OK) st = dalloc(&yfit, kOut);
  if (st == DEMAG_OK) st = dalloc(&dR, 1);
  if (st == DEMAG_OK) st = dalloc(&dgrid, 3);
  if (st == DEMAG_OK) st = dalloc(&dh, 1);
  if (st == DEMAG_OK) st = dalloc(&dt, kRmax);
  if (st == DEMAG_OK) st = dalloc(&da, kRmax);
  if (st == DEMAG_OK) st = dalloc(&derr, 1);
  if (st == DEMAG_OK) st = dalloc(&Kref, size_t(S) * kNcomp);
  if (st == DEMAG_OK) st = dalloc(&KrefC, size_t(Sc) * kNcomp);
  if (st == DEMAG_OK) st = dalloc(&Kc, size_t(Sc) * kNcomp);
  std::vector<float> yh(size_t(NC) * kOut);
  if (st == DEMAG_OK) {
    k_mlp_forward<<<NC, 64, 0, ctx->stream>>>(params, features, NC, Y, nullptr, nullptr);
    if (hipMemcpyAsync(yh.data(), Y, sizeof(float) * yh.size(), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(dgrid, n, sizeof(int32_t) * 3, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(dh, &hmin, sizeof(double), hipMemcpyHostToDevice, ctx->stream) != hipSuccess) {
      set_error("demag_quad_predict: copy failed");
      st = DEMAG_E_HIP;
    }
  }
  if (st == DEMAG_OK) st = reference_values(ctx, dgrid, dh, sent, S, 1, Kref);
  if (st == DEMAG_OK) st = reference_values(ctx, dgrid, dh, check, Sc, 1, KrefC);
  int pick = NC - 1;
  if (st == DEMAG_OK) {
    for (int c = 0; c < NC; ++c)
      if (yh[size_t(c) * kOut + 64] <= std::log10(tol)) {
        pick = c;
        break;
      }
    *predicted = yh[size_t(pick) * kOut + 64];
  }
  bool done = false;
  for (int c = pick; st == DEMAG_OK && !done; c = (c == NC - 1) ? NC : std::min(c + 4, NC - 1)) {
    if (c >= NC) break;
    const int Rp = 16 + c;
    double e = 0;
    std::vector<double> th(kRmax), ah(kRmax);
    if (hipMemcpyAsync(dR, &Rp, sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream) != hipSuccess) {
      set_error("demag_quad_predict: copy failed");
      st = DEMAG_E_HIP;
      break;
    }
    // polish the network's proposal and, as a guard, the plain base rule;
    // keep the better of the two
    for (int start = 0; start < 2 && st == DEMAG_OK; ++start) {
      st = launch_fit(ctx, 1, dgrid, dh, sent, S, Kref, dR, start == 0 ? Y + size_t(c) * kOut : nullptr, fit_iters,
                      1e-3, yfit, nullptr, nullptr, dt, da, derr);
      if (st != DEMAG_OK) break;
      double es = 0;
      std::vector<double> ts(kRmax), as(kRmax);
      if (hipMemcpyAsync(&es, derr, sizeof(double), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
          hipMemcpyAsync(ts.data(), dt, sizeof(double) * kRmax, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
          hipMemcpyAsync(as.data(), da, sizeof(double) * kRmax, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess) {
        set_error("demag_quad_predict: copy failed");
        st = DEMAG_E_HIP;
        break;
      }
      if (start == 0 || es < e) {
        e = es;
        th = ts;
        ah = as;
      }
    }
    if (st != DEMAG_OK) break;
    // judge the kept rule on the check offsets, which the fit never saw
    if (hipMemcpyAsync(dt, th.data(), sizeof(double) * kRmax, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(da, ah.data(), sizeof(double) * kRmax, hipMemcpyHostToDevice, ctx->stream) != hipSuccess) {
      set_error("demag_quad_predict: copy failed");
      st = DEMAG_E_HIP;
      break;
    }
    k_judge_values<<<(Sc + 127) / 128, 128, 0, ctx->stream>>>(dgrid, dh, check, Sc, dt, da, dR, kRmax, 1, Kc);
    k_judge_err<<<1, 128, 0, ctx->stream>>>(Kc, KrefC, 1, Sc, derr, nullptr);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&e, derr, sizeof(double), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      set_error("demag_quad_predict: judge failed");
      st = DEMAG_E_HIP;
      break;
    }
    *judged = e;
    if (e <= tol) {
      done = true;
      *fell_back = 0;
      *R_out = Rp;
      for (int k = 0; k < Rp; ++k) {
        t_out[k] = th[k];
        alpha_out[k] = ah[k];
      }
    }
  }
  if (st == DEMAG_OK && !done) {
    // fallback: the sinc rule with the step of Thm. sinc_theo, 64 nodes
    *fell_back = 1;
    const int M = 64;
    const double a = 2.0, bb = 0.25 * (0.5 * hmin) * (0.5 * hmin);
    const double theta = std::log(2.0 * kPi * a * M / bb) / (a * M);
    *R_out = M;
    for (int k = 0; k < M; ++k) {
      const double tk = (k + 1) * theta, sh = std::sinh(tk);
      t_out[k] = tk;
      alpha_out[k] = 2.0 * theta * std::cosh(tk) * sh * sh;
    }
  }
  for (void *p : {(void *)Y, (void *)yfit, (void *)dR, (void *)dgrid, (void *)dh, (void *)dt, (void *)da,
                  (void *)derr, (void *)Kref, (void *)KrefC, (void *)Kc})
    if (p) (void)hipFree(p);
  return st;
}

}  // extern "C"
