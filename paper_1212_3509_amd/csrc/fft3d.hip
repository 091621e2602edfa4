// Full-format apply by 3D FFT convolution (Sec. 4.2: for unstructured
// tensors the Toeplitz-structured operator is best evaluated with FFTs).
//
// The operator is the same separable sinc-quadrature kernel as the mode
// products of demag_apply_full: for each (output, input component) pair,
//   K(J) = sum_k f_x[k](Jx) f_y[k](Jy) f_z[k](Jz),
// embedded per axis in a circulant of length L_d = 2^p >= 2 n_d - 1.  Its 3D
// spectrum is separable per node: K^(fx, fy, fz) = sum_k G_x(fx) G_y(fy)
// G_z(fz), with G the 1D spectra of the structured path (real for E and P,
// imaginary for X and Q).  With one odd factor (potential kernels) the 3D
// spectrum is imaginary, with none (F_pp) real, with two (F_pq) real and
// negated; it is stored as one real array per component.
//
// Layout of a spectrum: [fz < Lz][fy < Ly][fx <= Lx/2] complex FP64 (real
// transform along x).  Passes, all FP64 in LDS (Stockham radix 16/8/4/2,
// several lines per workgroup, 4096 points at most per workgroup):
//   x: real rows (z < nz, y < ny) -> half spectra;  y: lines along y for
//   z < nz (rows y >= ny are zero, not read);  z: lines along z for all
//   (fy, fx) (planes z >= nz are zero, not read);  pointwise products with
//   the nine kernel spectra; then the inverse passes, each storing only the
//   part of the next input that is needed (z < nz, then y < ny, then x < nx).
#include "internal.h"

#include <cmath>

namespace demag {

namespace {

constexpr int kT = 256;          // threads per workgroup
constexpr int kPts = 4096;       // points per workgroup

struct alignas(16) cplx {
  double x, y;
};
__device__ inline cplx cadd(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline cplx csub(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline cplx cconj(cplx a) { return {a.x, -a.y}; }
template <bool INV> __device__ inline cplx mul_mi(cplx a) { return INV ? cplx{-a.y, a.x} : cplx{a.y, -a.x}; }

// LDS slot of point i of line b: b * LS + pd(i), with one pad slot after
// every 16 points and an odd line stride LS, so that stride-R butterfly
// accesses within a line and accesses across lines (the transposed global
// loads of the strided passes) both spread over the banks.
__device__ inline int pd(int i) { return i + (i >> 4); }
__host__ __device__ inline int line_stride(int N) { return (N + (N - 1) / 16 + 1) | 1; }
constexpr int kCap = kPts + kPts / 16 + 64;   // LDS points per workgroup
// lines per workgroup for lines of N points
__host__ __device__ inline int lines_per_wg(int N) {
  int nl = kPts / N;
  while (nl > 1 && nl * line_stride(N) > kCap) nl /= 2;
  return nl;
}

template <bool INV> __device__ inline void dft2(cplx *v) {
  const cplx t = v[0];
  v[0] = cadd(t, v[1]);
  v[1] = csub(t, v[1]);
}
template <bool INV> __device__ inline void dft4(cplx *v) {
  const cplx s0 = cadd(v[0], v[2]), d0 = csub(v[0], v[2]);
  const cplx s1 = cadd(v[1], v[3]), d1 = mul_mi<INV>(csub(v[1], v[3]));
  v[0] = cadd(s0, s1);
  v[2] = csub(s0, s1);
  v[1] = cadd(d0, d1);
  v[3] = csub(d0, d1);
}
// cos and sin of 2 pi e / 16 (compile-time constants after unrolling)
__device__ constexpr double cos16(int e) {
  constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                            -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                            0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
  return c[e & 15];
}
__device__ constexpr double sin16(int e) { return cos16(e + 12); }   // sin x = cos(x - pi/2)

// radix 8 = 4 x 2 and 16 = 4 x 4 (Cooley-Tukey split with constant twiddles)
template <bool INV, int R1, int R2> __device__ inline void dft_split(cplx *v) {
  cplx t[R1 * R2];
#pragma unroll
  for (int b = 0; b < R2; ++b) {
    cplx col[R1];
#pragma unroll
    for (int a = 0; a < R1; ++a) col[a] = v[R2 * a + b];
    dft4<INV>(col);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      if (b * k1 == 0) {
        t[b * R1 + k1] = col[k1];
      } else {
        const int e = (b * k1 * (16 / (R1 * R2))) & 15;   // angle 2 pi e / 16
        t[b * R1 + k1] = cmul(col[k1], cplx{cos16(e), INV ? sin16(e) : -sin16(e)});
      }
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cplx row[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) row[b] = t[b * R1 + k1];
    if (R2 == 2) dft2<INV>(row);
    else dft4<INV>(row);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = row[k2];
  }
}
template <bool INV, int R> __device__ inline void dftR(cplx *v) {
  if (R == 2) dft2<INV>(v);
  else if (R == 4) dft4<INV>(v);
  else if (R == 8) dft_split<INV, 4, 2>(v);
  else dft_split<INV, 4, 4>(v);
}

// W_N^e (forward sign) from two LDS tables: lo[i] = W_N^i, hi[i] = W_N^(64 i).
__device__ inline cplx twid(int e, const cplx *lo, const cplx *hi) {
  const cplx a = lo[e & 63];
  return (e >> 6) ? cmul(a, hi[e >> 6]) : a;
}
__device__ inline void make_twiddles(cplx *lo, cplx *hi, int N) {
  const int t = threadIdx.x;
  double s, c;
  if (t < 64) {
    sincospi(-2.0 * double(t) / double(N), &s, &c);
    lo[t] = cplx{c, s};
  } else if (t < 128) {
    sincospi(-2.0 * double(64 * (t - 64)) / double(N), &s, &c);
    hi[t - 64] = cplx{c, s};
  }
}

// One Stockham pass of radix R over nl lines of N points.  Butterfly g:
// line g % nl, index g / nl (lines fastest across threads).
template <bool INV, int R>
__device__ inline void pass(cplx *buf, int N, int nl, int LS, int Ns, const cplx *tlo, const cplx *thi) {
  const int per = N / R;                 // butterflies per line
  const int nb = nl * per;
  constexpr int kMaxB = (kPts / R + kT - 1) / kT;
  cplx v[kMaxB][R];
  int jj[kMaxB];
#pragma unroll
  for (int q = 0; q < kMaxB; ++q) {
    const int g = threadIdx.x + q * kT;
    jj[q] = g;
    if (g < nb) {
      const int j = g / nl, line = g - j * nl;
      cplx *lb = buf + line * LS;
      const int k = j & (Ns - 1);
      cplx w = twid((k * (N / (Ns * R))) & (N - 1), tlo, thi);
      if (INV) w = cconj(w);
      cplx wr = w;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cplx x = lb[pd(j + r * per)];
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
    const int g = jj[q];
    if (g < nb) {
      const int j = g / nl, line = g - j * nl;
      const int k = j & (Ns - 1);
      const int o = (j / Ns) * Ns * R + k;
      cplx *lb = buf + line * LS;
#pragma unroll
      for (int r = 0; r < R; ++r) lb[pd(o + r * Ns)] = v[q][r];
    }
  }
  __syncthreads();
}

// Complex FFTs of nl lines of N points (power of 2) in LDS.
template <bool INV>
__device__ void fft_lines(cplx *buf, int N, int nl, const cplx *tlo, const cplx *thi) {
  const int LS = line_stride(N);
  int Ns = 1;
  while (Ns < N) {
    const int left = N / Ns;
    if (left >= 16) {
      pass<INV, 16>(buf, N, nl, LS, Ns, tlo, thi);
      Ns *= 16;
    } else if (left == 8) {
      pass<INV, 8>(buf, N, nl, LS, Ns, tlo, thi);
      Ns *= 8;
    } else if (left == 4) {
      pass<INV, 4>(buf, N, nl, LS, Ns, tlo, thi);
      Ns *= 4;
    } else {
      pass<INV, 2>(buf, N, nl, LS, Ns, tlo, thi);
      Ns *= 2;
    }
  }
}

// W_L^f for the real-transform (un)packing, L = 2N: W_N^(f/2), times W_L^1 for odd f.
__device__ inline cplx wl(int f, int N, const cplx *tlo, const cplx *thi, cplx w1) {
  cplx w = twid((f >> 1) & (N - 1), tlo, thi);
  if (f & 1) w = cmul(w, w1);
  return w;
}

// ---------------------------------------------------------------- x pass
// Real rows r = z * ny + y (z < nz, y < ny) of in[3][nz][ny][nx] (component
// c = blockIdx.y) -> S_c[z][y][0..Lx/2].  nl rows per workgroup.
__global__ __launch_bounds__(kT) void k_x_fwd(const double *__restrict__ in, cplx *__restrict__ S, int nx, int ny,
                                              int nz, int Lx, int Ly, int Lz, int nl) {
  extern __shared__ cplx sm[];
  cplx *buf = sm, *tlo = sm + kCap, *thi = tlo + 64;
  const int N = Lx / 2, H = N + 1;
  const int comp = blockIdx.y;
  const int rows = ny * nz;
  const int r0 = blockIdx.x * nl;
  const int nr = min(nl, rows - r0);
  make_twiddles(tlo, thi, N);
  const double *src = in + size_t(comp) * nx * ny * nz;
  const int LS = line_stride(N);
  for (int i = threadIdx.x; i < nl * N; i += kT) {
    const int line = i / N, m = i - line * N;
    cplx v{0.0, 0.0};
    if (line < nr) {
      const double *row = src + size_t(r0 + line) * nx;
      const int a = 2 * m, b = 2 * m + 1;
      v = cplx{a < nx ? row[a] : 0.0, b < nx ? row[b] : 0.0};
    }
    buf[line * LS + pd(m)] = v;
  }
  __syncthreads();
  fft_lines<false>(buf, N, nl, tlo, thi);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const cplx w1{cw, sw};
  cplx *dst = S + size_t(comp) * Lz * Ly * H;
  for (int i = threadIdx.x; i < nl * H; i += kT) {
    const int line = i / H, f = i - line * H;
    if (line >= nr) continue;
    const int r = r0 + line, z = r / ny, y = r - z * ny;
    const cplx zf = buf[line * LS + pd(f & (N - 1))];
    const cplx zcc = cconj(buf[line * LS + pd((N - f) & (N - 1))]);
    const cplx D{0.5 * (zf.x - zcc.x), 0.5 * (zf.y - zcc.y)};
    dst[(size_t(z) * Ly + y) * H + f] =
        cadd(cplx{0.5 * (zf.x + zcc.x), 0.5 * (zf.y + zcc.y)}, cmul(wl(f, N, tlo, thi, w1), cplx{D.y, -D.x}));
  }
}

// ---------------------------------------------------------------- y, z passes
// Complex FFTs of length N along a strided axis, in place: workgroup
// (blockIdx.x = fx tile, blockIdx.y = outer index o, blockIdx.z = array)
// handles nl lines fx = fx0 .. fx0 + nl - 1 of elements
//   A[arr][o * so + i * si + fx],  i < N,
// reading only i < nin (the rest is zero) and writing only i < nout.
template <bool INV>
__global__ __launch_bounds__(kT) void k_lines(cplx *__restrict__ A, size_t arr_stride, int N, int H, size_t so,
                                              size_t si, int nin, int nout, int nl) {
  extern __shared__ cplx sm[];
  cplx *buf = sm, *tlo = sm + kCap, *thi = tlo + 64;
  const int fx0 = blockIdx.x * nl;
  const int nf = min(nl, H - fx0);
  cplx *base = A + size_t(blockIdx.z) * arr_stride + size_t(blockIdx.y) * so + fx0;
  make_twiddles(tlo, thi, N);
  // global accesses run along fx (coalesced); line stride LS is odd
  const int LS = line_stride(N);
  for (int e = threadIdx.x; e < nl * N; e += kT) {
    const int i = e / nl, b = e - i * nl;
    cplx v{0.0, 0.0};
    if (i < nin && b < nf) v = base[size_t(i) * si + b];
    buf[b * LS + pd(i)] = v;
  }
  __syncthreads();
  fft_lines<INV>(buf, N, nl, tlo, thi);
  for (int e = threadIdx.x; e < nl * nout; e += kT) {
    const int i = e / nl, b = e - i * nl;
    if (b < nf) base[size_t(i) * si + b] = buf[b * LS + pd(i)];
  }
}

// ---------------------------------------------------------------- kernel spectra
// Kspec[c][fz][fy][fx] (real; component c: 0..2 potential K^q, 3..8 field
// (0,0) (1,1) (2,2) (0,1) (0,2) (1,2)) = sign_c * sum_k s_x(fx) s_y(fy) s_z(fz),
// s the stored 1D spectra ([type][M][L/2+1], the imaginary part for odd
// types; s(L - f) = s(f) for even, -s(f) for odd types).
__device__ inline double spec1(const double *sp, int type, int k, int M, int L, int f) {
  const bool odd = (type == F_X || type == F_Q);
  const int h = L / 2;
  const double *s = sp + size_t(type * M + k) * (h + 1);
  if (f <= h) return s[f];
  return odd ? -s[L - f] : s[L - f];
}

__device__ inline void comp_types(int c, int t[3]) {
  // potential K^q: X along q, E elsewhere; field h_p <- m_q: differentiate along p
  const int p = c < 3 ? -1 : (c < 6 ? c - 3 : (c == 6 ? 0 : (c == 7 ? 0 : 1)));
  const int q = c < 3 ? c : (c < 6 ? c - 3 : (c == 6 ? 1 : 2));
  for (int d = 0; d < 3; ++d) t[d] = (d == q) ? F_X : F_E;
  if (p >= 0) t[p] = (t[p] == F_X) ? F_P : F_Q;
}

__global__ void k_kernel_spectra(const double *__restrict__ sx, const double *__restrict__ sy,
                                 const double *__restrict__ sz, double *__restrict__ K, int M, int Lx, int Ly,
                                 int Lz) {
  const int H = Lx / 2 + 1;
  const size_t np = size_t(Lz) * Ly * H;
  const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= np) return;
  const int fx = int(idx % H);
  const int fy = int((idx / H) % Ly);
  const int fz = int(idx / (size_t(H) * Ly));
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < M; ++k) {
    double vx[4], vy[4], vz[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      vx[t] = spec1(sx, t, k, M, Lx, fx);
      vy[t] = spec1(sy, t, k, M, Ly, fy);
      vz[t] = spec1(sz, t, k, M, Lz, fz);
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      int t[3];
      comp_types(c, t);
      acc[c] += vx[t[0]] * vy[t[1]] * vz[t[2]];
    }
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) K[size_t(c) * np + idx] = (c >= 6) ? -acc[c] : acc[c];
}

// ---------------------------------------------------------------- products
// S[0..2] = m^ (x, y, z); writes phi^ to S[3] and h^_p to S[p] (in place),
// scaled by 1/(Lx Ly Lz) (and the length scale for phi).  Potential kernels
// are imaginary (times i), field kernels real.
__global__ void k_products(cplx *__restrict__ S, const double *__restrict__ K, size_t np, double scale,
                           double phi_scale) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const cplx m0 = S[i], m1 = S[np + i], m2 = S[2 * np + i];
  const cplx mq[3] = {m0, m1, m2};
  double kv[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) kv[c] = K[size_t(c) * np + i];
  // phi^ = i sum_q K^q m^_q
  cplx ph{0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 3; ++q) ph = cadd(ph, cplx{-kv[q] * mq[q].y, kv[q] * mq[q].x});
  // field: symmetric pairs 3..8 = (0,0) (1,1) (2,2) (0,1) (0,2) (1,2)
  const double F[3][3] = {{kv[3], kv[6], kv[7]}, {kv[6], kv[4], kv[8]}, {kv[7], kv[8], kv[5]}};
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    cplx hp{0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 3; ++q) hp = cadd(hp, cplx{F[p][q] * mq[q].x, F[p][q] * mq[q].y});
    S[size_t(p) * np + i] = cplx{scale * hp.x, scale * hp.y};
  }
  S[3 * np + i] = cplx{scale * phi_scale * ph.x, scale * phi_scale * ph.y};
}

// ---------------------------------------------------------------- x inverse
// Half spectra S[a][z][y][0..Lx/2] (z < nz, y < ny) -> real rows out[a] (x < nx),
// output a = blockIdx.y: 0..2 field components to h[a], 3 potential to phi.
__global__ __launch_bounds__(kT) void k_x_inv(const cplx *__restrict__ S, double *__restrict__ phi,
                                              double *__restrict__ hout, int nx, int ny, int nz, int Lx, int Ly,
                                              int Lz, int nl) {
  extern __shared__ cplx sm[];
  cplx *buf = sm, *tlo = sm + kCap, *thi = tlo + 64;
  const int N = Lx / 2, H = N + 1;
  const int a = blockIdx.y;
  const int rows = ny * nz;
  const int r0 = blockIdx.x * nl;
  const int nr = min(nl, rows - r0);
  make_twiddles(tlo, thi, N);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const cplx w1{cw, sw};
  const cplx *src = S + size_t(a) * Lz * Ly * H;
  // pack Z[f] = E[f] + i O[f] from X[f], X[N - f]: E = X[f] + conj X[N-f],
  // O = (X[f] - conj X[N-f]) conj(W_L^f); the unnormalized inverse complex
  // transform of Z then holds Lx x[2m] + i Lx x[2m+1]
  const int LS = line_stride(N);
  for (int i = threadIdx.x; i < nl * N; i += kT) {
    const int line = i / N, f = i - line * N;
    cplx v{0.0, 0.0};
    if (line < nr) {
      const int r = r0 + line, z = r / ny, y = r - z * ny;
      const cplx *row = src + (size_t(z) * Ly + y) * H;
      const cplx xf = row[f], xcc = cconj(row[N - f]);
      const cplx E = cadd(xf, xcc);
      const cplx O = cmul(csub(xf, xcc), cconj(wl(f, N, tlo, thi, w1)));
      v = cplx{E.x - O.y, E.y + O.x};
    }
    buf[line * LS + pd(f)] = v;
  }
  __syncthreads();
  fft_lines<true>(buf, N, nl, tlo, thi);
  double *dst = (a < 3) ? hout + size_t(a) * nx * ny * nz : phi;
  for (int i = threadIdx.x; i < nl * N; i += kT) {
    const int line = i / N, m = i - line * N;
    if (line >= nr) continue;
    const cplx v = buf[line * LS + pd(m)];
    double *row = dst + size_t(r0 + line) * nx;
    const int xa = 2 * m, xb = 2 * m + 1;
    if (xa < nx) row[xa] = v.x;
    if (xb < nx) row[xb] = v.y;
  }
}

}  // namespace

demag_status prepare_fft3d(demag_ctx *ctx, demag_factors *f) {
  if (f->k3) return DEMAG_OK;
  demag_status st = prepare_spectra(ctx, f);
  if (st != DEMAG_OK) return st;
  const int Lx = fft_length(f->n[0]), Ly = fft_length(f->n[1]), Lz = fft_length(f->n[2]);
  const size_t np = size_t(Lz) * Ly * (Lx / 2 + 1);
  DEMAG_TRY_HIP(hipMalloc(&f->k3, 9 * np * sizeof(double)));
  k_kernel_spectra<<<unsigned((np + 255) / 256), 256, 0, ctx->stream>>>(f->spec[0], f->spec[1], f->spec[2], f->k3,
                                                                       f->M, Lx, Ly, Lz);
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

size_t fft3d_workspace_bytes(const demag_factors *f) {
  const int Lx = fft_length(f->n[0]), Ly = fft_length(f->n[1]), Lz = fft_length(f->n[2]);
  return 4 * size_t(Lz) * Ly * (Lx / 2 + 1) * sizeof(cplx);
}

demag_status launch_fft3d(demag_ctx *ctx, const demag_factors *f, const double *m, double *phi, double *h,
                          void *ws) {
  const int nx = f->n[0], ny = f->n[1], nz = f->n[2];
  const int Lx = fft_length(nx), Ly = fft_length(ny), Lz = fft_length(nz);
  const int Nx = Lx / 2, H = Nx + 1;
  const size_t np = size_t(Lz) * Ly * H;
  cplx *S = static_cast<cplx *>(ws);
  const size_t lds = sizeof(cplx) * (kCap + 128);
  for (const void *k : {reinterpret_cast<const void *>(&k_x_fwd), reinterpret_cast<const void *>(&k_x_inv),
                        reinterpret_cast<const void *>(&k_lines<false>), reinterpret_cast<const void *>(&k_lines<true>)})
    DEMAG_TRY_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipEvent_t ev = nullptr;
  demag_status st = prof_begin(ctx, &ev);
  if (st != DEMAG_OK) return st;
  const int rows = ny * nz;
  const int nlx = lines_per_wg(Nx);                // real rows per workgroup
  const int nly = lines_per_wg(Ly), nlz = lines_per_wg(Lz);   // strided lines per workgroup
  // forward: x (real rows), y (z < nz), z (all fy)
  k_x_fwd<<<dim3((rows + nlx - 1) / nlx, 3), kT, lds, ctx->stream>>>(m, S, nx, ny, nz, Lx, Ly, Lz, nlx);
  k_lines<false><<<dim3((H + nly - 1) / nly, nz, 3), kT, lds, ctx->stream>>>(S, np, Ly, H, size_t(Ly) * H, H, ny,
                                                                             Ly, nly);
  k_lines<false><<<dim3((H + nlz - 1) / nlz, Ly, 3), kT, lds, ctx->stream>>>(S, np, Lz, H, H, size_t(Ly) * H, nz,
                                                                             Lz, nlz);
  // products with the kernel spectra (4 outputs), normalization folded in
  k_products<<<unsigned((np + 255) / 256), 256, 0, ctx->stream>>>(S, f->k3, np, 1.0 / (double(Lx) * Ly * Lz), f->L);
  // inverse: z (keep z < nz), y (z < nz, keep y < ny), x (rows -> real, x < nx)
  k_lines<true><<<dim3((H + nlz - 1) / nlz, Ly, 4), kT, lds, ctx->stream>>>(S, np, Lz, H, H, size_t(Ly) * H, Lz, nz,
                                                                            nlz);
  k_lines<true><<<dim3((H + nly - 1) / nly, nz, 4), kT, lds, ctx->stream>>>(S, np, Ly, H, size_t(Ly) * H, H, Ly, ny,
                                                                            nly);
  k_x_inv<<<dim3((rows + nlx - 1) / nlx, 4), kT, lds, ctx->stream>>>(S, phi, h, nx, ny, nz, Lx, Ly, Lz, nlx);
  DEMAG_TRY_HIP(hipGetLastError());
  if (ev) {
    // real FFTs ~2.5 L log2 L per line point... counted per 3D transform as
    // 2.5 Lx Ly Lz log2(Lx Ly Lz) (half for the real direction) x 7 transforms
    const double vol = double(Lx) * Ly * Lz;
    const double flops = 7.0 * 2.5 * vol * std::log2(vol) / 2.0 + np * (9.0 * 8.0);
    // compulsory traffic: m, the nine kernel spectra, the outputs
    const double bytes = 8.0 * (7.0 * nx * ny * nz) + 8.0 * 9.0 * np;
    st = prof_end(ctx, ev, "fft3d/fp64", flops, bytes);
  }
  return st;
}

}  // namespace demag
