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
// negated; it is stored as one real array per component, and since each 1D
// spectrum is even or odd in f, only the octant fy <= Ly/2, fz <= Lz/2.
//
// Layout of a spectrum: [fz < Lz][fy < Ly][fx <= Lx/2] complex FP64 (real
// transform along x), rows padded to a multiple of 8 points (128 B).
// Passes, all FP64 in LDS (Stockham radix 16/8/4/2, several lines per
// workgroup):
//   x: real rows (z < nz, y < ny) -> half spectra;  y: lines along y for
//   z < nz (rows y >= ny are zero, not read);  z, fused with the products:
//   per column group, forward transforms of the three magnetization spectra
//   (planes z >= nz zero, not read), pointwise products with the kernel
//   spectra, inverse transforms of the four outputs, stored for z < nz; then
//   the inverse y pass (stores y < ny) and the inverse real x pass (x < nx).
#include "fft_core.h"
#include "internal.h"

#include <cmath>
#include <cstdint>

namespace demag {

namespace {

using namespace fftc;

// ---------------------------------------------------------------- x pass
// Work index of a workgroup: the hardware places workgroup lin on XCD
// lin % 8; this gives the workgroups of one XCD consecutive work indices, so
// that neighbouring column tiles (which share cache lines) meet in one L2.
__device__ inline unsigned xcd_work_index(unsigned lin, unsigned total) {
  const unsigned x = lin & 7u, slot = lin >> 3;
  const unsigned per = total >> 3, rem = total & 7u;
  return x * per + min(x, rem) + slot;
}

// Real rows r = z * ny + y (z < nz, y < ny) of in[3][nz][ny][nx] (component
// c = blockIdx.y) -> S_c[z][y][0..Lx/2] (row pitch P).  2^lnl rows per
// workgroup.
template <int KT, int KP>
__global__ __launch_bounds__(KT) void k_x_fwd(const double *__restrict__ in, cplx *__restrict__ S, size_t astride,
                                              int nx, int ny, int nz, int Lx, int Ly, int P, int lnl) {
  extern __shared__ cplx sm[];
  cplx *buf = sm, *tlo = sm + cap(KP), *thi = tlo + 64;
  const int N = Lx / 2, H = N + 1, lN = __builtin_ctz(N);
  const int nl = 1 << lnl;
  const int comp = blockIdx.y;
  const int rows = ny * nz;
  const int r0 = blockIdx.x << lnl;
  const int nr = min(nl, rows - r0);
  make_twiddles(tlo, thi, N);
  const double *src = in + size_t(comp) * nx * ny * nz;
  const int LS = line_stride(N, nl);
  // all loads of a thread in flight before the LDS stores (nl N <= KP)
  constexpr int kE = KP / KT;
  // (x, x + 1) pairs are 16-byte aligned for an even row length and base
  const bool even = (nx & 1) == 0 && (reinterpret_cast<uintptr_t>(in) & 15) == 0;
  cplx v[kE];
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int i = threadIdx.x + q * KT;
    const int line = i >> lN, m = i & (N - 1);
    v[q] = cplx{0.0, 0.0};
    if (i < nl * N && line < nr) {
      const double *row = src + size_t(r0 + line) * nx;
      const int a = 2 * m, b = 2 * m + 1;
      if (even && b < nx) {
        const double2 t = *reinterpret_cast<const double2 *>(row + a);
        v[q] = cplx{t.x, t.y};
      } else {
        v[q] = cplx{a < nx ? row[a] : 0.0, b < nx ? row[b] : 0.0};
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int i = threadIdx.x + q * KT;
    if (i < nl * N) buf[(i >> lN) * LS + pd(i & (N - 1))] = v[q];
  }
  __syncthreads();
  fft_lines<false, KT, KP>(buf, N, LS, nl, tlo, thi);
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const cplx w1{cw, sw};
  cplx *dst = S + size_t(comp) * astride;
  // X[f] = (Z[f] + conj Z[N-f]) / 2 - i W_L^f (Z[f] - conj Z[N-f]) / 2 for
  // f < N; the thread of f = 0 also writes f = N (same two points, W_L^N = -1)
  for (int i = threadIdx.x; i < nl * N; i += KT) {
    const int line = i >> lN, f = i & (N - 1);
    if (line >= nr) continue;
    const int r = r0 + line, z = r / ny, y = r - z * ny;
    cplx *drow = dst + (size_t(z) * Ly + y) * P;
    const cplx zf = buf[line * LS + pd(f)];
    const cplx zcc = cconj(buf[line * LS + pd((N - f) & (N - 1))]);
    const cplx Sm{0.5 * (zf.x + zcc.x), 0.5 * (zf.y + zcc.y)};
    const cplx D{0.5 * (zf.x - zcc.x), 0.5 * (zf.y - zcc.y)};
    drow[f] = cadd(Sm, cmul(wl(f, N, tlo, thi, w1), cplx{D.y, -D.x}));
    if (f == 0) drow[N] = cplx{Sm.x - D.y, Sm.y + D.x};
  }
}

// ---------------------------------------------------------------- y pass
// Complex FFTs of length N along y, in place, for the planes z < nz: the
// workgroup with work index w (XCD-grouped) handles array w / (tiles nz),
// plane z, and the 2^lnl lines fx = fx0 .. (fx < H) of elements
//   A[arr][(z Ly + i) P + fx],  i < N,
// reading only i < nin (the rest is zero) and writing only i < nout.
template <bool INV, int KT, int KP>
__global__ __launch_bounds__(KT) void k_lines(cplx *__restrict__ A, size_t astride, int N, int H, int P, int nz,
                                              int nin, int nout, int lnl) {
  extern __shared__ cplx sm[];
  cplx *buf = sm, *tlo = sm + cap(KP), *thi = tlo + 64;
  const int nl = 1 << lnl;
  const int tiles = (H + nl - 1) >> lnl;
  const unsigned w = xcd_work_index(blockIdx.x, gridDim.x);
  const int tile = int(w % unsigned(tiles)), rest = int(w / unsigned(tiles));
  const int z = rest % nz, arr = rest / nz;
  const int fx0 = tile << lnl;
  const int nf = min(nl, H - fx0);
  cplx *base = A + size_t(arr) * astride + size_t(z) * N * P + fx0;
  make_twiddles(tlo, thi, N);
  // global accesses run along fx (coalesced)
  const int LS = line_stride(N, nl);
  // all loads of a thread in flight before the LDS stores (nl N <= KP)
  constexpr int kE = KP / KT;
  cplx v[kE];
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = threadIdx.x + q * KT;
    const int i = e >> lnl, b = e & (nl - 1);
    v[q] = cplx{0.0, 0.0};
    if (e < nl * N && i < nin && b < nf) v[q] = base[size_t(i) * P + b];
  }
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = threadIdx.x + q * KT;
    if (e < nl * N) buf[(e & (nl - 1)) * LS + pd(e >> lnl)] = v[q];
  }
  __syncthreads();
  fft_lines<INV, KT, KP>(buf, N, LS, nl, tlo, thi);
  for (int e = threadIdx.x; e < nl * nout; e += KT) {
    const int i = e >> lnl, b = e & (nl - 1);
    if (b < nf) base[size_t(i) * P + b] = buf[b * LS + pd(i)];
  }
}

// ---------------------------------------------------------------- kernel spectra
// 1D spectra s(f) of the factors ([type][M][L/2+1], the imaginary part for
// odd types): s(L - f) = s(f) for even, -s(f) for odd types.  The 3D kernel
// spectra inherit this per axis, so only the octant fy <= Ly/2, fz <= Lz/2 is
// stored: Kspec[fz][fy][fx][c] (row pitch P, kKC = 10 doubles per frequency,
// 16-byte aligned; component c: 0..2 potential K^q, 3..8 field (0,0) (1,1)
// (2,2) (0,1) (0,2) (1,2), 9 unused) = sign_c sum_k s_x s_y s_z.
__device__ inline void comp_types(int c, int t[3]) {
  // potential K^q: X along q, E elsewhere; field h_p <- m_q: differentiate along p
  const int p = c < 3 ? -1 : (c < 6 ? c - 3 : (c == 6 ? 0 : (c == 7 ? 0 : 1)));
  const int q = c < 3 ? c : (c < 6 ? c - 3 : (c == 6 ? 1 : 2));
  for (int d = 0; d < 3; ++d) t[d] = (d == q) ? F_X : F_E;
  if (p >= 0) t[p] = (t[p] == F_X) ? F_P : F_Q;
}
__host__ __device__ constexpr bool odd_type(int t) { return t == F_X || t == F_Q; }
constexpr int kKC = 10;   // doubles per frequency of the kernel spectra

__global__ void k_kernel_spectra(const double *__restrict__ sx, const double *__restrict__ sy,
                                 const double *__restrict__ sz, double *__restrict__ K, int M, int Lx, int Ly,
                                 int Lz, int P) {
  const int H = Lx / 2 + 1, hy = Ly / 2 + 1, hz = Lz / 2 + 1;
  const size_t npk = size_t(hz) * hy * P;
  const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= npk) return;
  const int fx = int(idx % P);
  const int fy = int((idx / P) % hy);
  const int fz = int(idx / (size_t(P) * hy));
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (fx < H) {
    for (int k = 0; k < M; ++k) {
      double vx[4], vy[4], vz[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        vx[t] = sx[size_t(t * M + k) * H + fx];
        vy[t] = sy[size_t(t * M + k) * hy + fy];
        vz[t] = sz[size_t(t * M + k) * hz + fz];
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        int t[3];
        comp_types(c, t);
        acc[c] += vx[t[0]] * vy[t[1]] * vz[t[2]];
      }
    }
  }
  double *out = K + idx * kKC;
#pragma unroll
  for (int c = 0; c < 9; ++c) out[c] = (c >= 6) ? -acc[c] : acc[c];
  out[9] = 0.0;
}

// ---------------------------------------------------------------- z pass + products
// For the columns (fx0 .. fx0 + nl - 1, fy), nl = 2^lnl: forward transforms
// along z of m^_0..2 (planes z >= nz are zero), products with the kernel
// spectra (phi^ = i sum_q K^q m^_q, h^_p = sum_q F_pq m^_q, scaled by
// 1 / (Lx Ly Lz) and the length scale for phi), inverse transforms along z
// of the four outputs, stored for z < nz only: S[0..2] <- h^, S[3] <- phi^.
// LDS holds 4 nl lines: array a, column b at line a * nl + b.  Work order
// (XCD-grouped): fy = 0, Ly/2, 1, Ly - 1, 2, Ly - 2, ..., fx tiles fastest,
// so that fy and Ly - fy, which read the same kernel spectra, run together.
template <int KT, int KP>
__global__ __launch_bounds__(KT) void k_z_conv(cplx *__restrict__ S, size_t astride, const double *__restrict__ K,
                                               int Lz, int nz, int Ly, int P, int H, int lnl, double scale,
                                               double phi_scale) {
  extern __shared__ cplx sm[];
  cplx *buf = sm, *tlo = sm + cap(KP), *thi = tlo + 64;
  const int nl = 1 << lnl;
  const int tiles = (H + nl - 1) >> lnl;
  const unsigned w = xcd_work_index(blockIdx.x, gridDim.x);
  const int tile = int(w % unsigned(tiles)), q = int(w / unsigned(tiles));
  const int fy = q == 0 ? 0 : (q == 1 ? Ly / 2 : ((q & 1) ? Ly - (q - 1) / 2 : q / 2));
  const int fx0 = tile << lnl;
  const int nf = min(nl, H - fx0);
  make_twiddles(tlo, thi, Lz);
  const int LS = line_stride(Lz, nl);
  const size_t col = size_t(fy) * P + fx0;      // offset of (z = 0, fy, fx0)
  const size_t zs = size_t(Ly) * P;             // z stride
  // all loads of a thread in flight before the LDS stores (4 nl Lz <= KP)
  constexpr int kE = KP / 4 / KT;
  {
    cplx v[3][kE];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int q = 0; q < kE; ++q) {
        const int e = threadIdx.x + q * KT;
        const int i = e >> lnl, b = e & (nl - 1);
        v[a][q] = cplx{0.0, 0.0};
        if (e < nl * Lz && i < nz && b < nf) v[a][q] = S[size_t(a) * astride + i * zs + col + b];
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int q = 0; q < kE; ++q) {
        const int e = threadIdx.x + q * KT;
        if (e < nl * Lz) buf[(a * nl + (e & (nl - 1))) * LS + pd(e >> lnl)] = v[a][q];
      }
    }
  }
  __syncthreads();
  fft_lines<false, KT, KP>(buf, Lz, LS, 3 * nl, tlo, thi);
  // kernel spectra octant index and per-component signs for this fy
  const int hy = Ly / 2 + 1, hz = Lz / 2 + 1;
  const bool fy_hi = fy >= hy;
  const int fyk = fy_hi ? Ly - fy : fy;
  const double ps = scale * phi_scale;
  // Frequencies fz and Lz - fz share one stored kernel entry: item (p, b)
  // handles fz = p and Lz - p for 0 < p < Lz/2, item (0, b) handles fz = 0
  // and Lz/2.  The kernel spectra of all the thread's items are in flight at
  // once.
  constexpr int kI = (kE + 1) / 2;   // items per thread (nl Lz / 2 <= kI KT)
  double2 kr[kI][kKC / 2], k2[kKC / 2];
#pragma unroll
  for (int q = 0; q < kI; ++q) {
    const int e = threadIdx.x + q * KT;
    const int p = e >> lnl, b = e & (nl - 1);
    if (e < nl * (Lz / 2) && b < nf) {
      const double2 *kp = reinterpret_cast<const double2 *>(K + ((size_t(p) * hy + fyk) * P + fx0 + b) * kKC);
#pragma unroll
      for (int c = 0; c < kKC / 2; ++c) kr[q][c] = kp[c];
    }
  }
  if (int(threadIdx.x) < nf && Lz > 1) {   // items (0, b) also need fz = Lz/2
    const double2 *kp =
        reinterpret_cast<const double2 *>(K + ((size_t(Lz / 2) * hy + fyk) * P + fx0 + threadIdx.x) * kKC);
#pragma unroll
    for (int c = 0; c < kKC / 2; ++c) k2[c] = kp[c];
  }
  // products at point (i, b) with the kernel entry kr (fz_hi: i > Lz/2)
  auto product = [&](int i, int b, const double2 *kraw, bool fz_hi) {
    double kv[kKC];
#pragma unroll
    for (int c = 0; c < kKC / 2; ++c) {
      kv[2 * c] = kraw[c].x;
      kv[2 * c + 1] = kraw[c].y;
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      int t[3];
      comp_types(c, t);
      if ((fy_hi && odd_type(t[1])) != (fz_hi && odd_type(t[2]))) kv[c] = -kv[c];
    }
    const cplx m0 = buf[(0 * nl + b) * LS + pd(i)];
    const cplx m1 = buf[(1 * nl + b) * LS + pd(i)];
    const cplx m2 = buf[(2 * nl + b) * LS + pd(i)];
    // potential: i (K^0 m0 + K^1 m1 + K^2 m2)
    const double pr = kv[0] * m0.x + kv[1] * m1.x + kv[2] * m2.x;
    const double pi = kv[0] * m0.y + kv[1] * m1.y + kv[2] * m2.y;
    buf[(3 * nl + b) * LS + pd(i)] = cplx{-ps * pi, ps * pr};
    // field: symmetric F with pairs 3..8 = (0,0) (1,1) (2,2) (0,1) (0,2) (1,2)
    const double F[3][3] = {{kv[3], kv[6], kv[7]}, {kv[6], kv[4], kv[8]}, {kv[7], kv[8], kv[5]}};
#pragma unroll
    for (int a = 0; a < 3; ++a)
      buf[(a * nl + b) * LS + pd(i)] = cplx{scale * (F[a][0] * m0.x + F[a][1] * m1.x + F[a][2] * m2.x),
                                           scale * (F[a][0] * m0.y + F[a][1] * m1.y + F[a][2] * m2.y)};
  };
#pragma unroll
  for (int q = 0; q < kI; ++q) {
    const int e = threadIdx.x + q * KT;
    const int p = e >> lnl, b = e & (nl - 1);
    if (e >= nl * (Lz / 2) || b >= nf) continue;
    product(p, b, kr[q], false);
    if (p > 0) product(Lz - p, b, kr[q], true);
    else if (Lz > 1) product(Lz / 2, b, k2, false);
  }
  __syncthreads();
  fft_lines<true, KT, KP>(buf, Lz, LS, 4 * nl, tlo, thi);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    for (int e = threadIdx.x; e < nl * nz; e += KT) {
      const int i = e >> lnl, b = e & (nl - 1);
      if (b < nf) S[size_t(a) * astride + i * zs + col + b] = buf[(a * nl + b) * LS + pd(i)];
    }
  }
}

// ---------------------------------------------------------------- x inverse
// Half spectra S[a][z][y][0..Lx/2] (z < nz, y < ny) -> real rows out[a] (x < nx),
// output a = blockIdx.y: 0..2 field components to h[a], 3 potential to phi.
template <int KT, int KP>
__global__ __launch_bounds__(KT) void k_x_inv(const cplx *__restrict__ S, size_t astride, double *__restrict__ phi,
                                              double *__restrict__ hout, int nx, int ny, int nz, int Lx, int Ly,
                                              int P, int lnl) {
  extern __shared__ cplx sm[];
  cplx *buf = sm, *tlo = sm + cap(KP), *thi = tlo + 64;
  const int N = Lx / 2, lN = __builtin_ctz(N);
  const int nl = 1 << lnl;
  const int a = blockIdx.y;
  const int rows = ny * nz;
  const int r0 = blockIdx.x << lnl;
  const int nr = min(nl, rows - r0);
  make_twiddles(tlo, thi, N);
  __syncthreads();   // the unpacking below reads the twiddle tables
  double sw, cw;
  sincospi(-1.0 / double(N), &sw, &cw);
  const cplx w1{cw, sw};
  const cplx *src = S + size_t(a) * astride;
  // pack Z[f] = E[f] + i O[f] from X[f], X[N - f]: E = X[f] + conj X[N-f],
  // O = (X[f] - conj X[N-f]) conj(W_L^f); the unnormalized inverse complex
  // transform of Z then holds Lx x[2m] + i Lx x[2m+1]
  const int LS = line_stride(N, nl);
  // two batches of kE / 2 points per thread, all their loads in flight at once
  constexpr int kE = KP / KT, kB = kE / 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    cplx xf[kB], xc[kB];
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int i = threadIdx.x + (h * kB + q) * KT;
      const int line = i >> lN, f = i & (N - 1);
      xf[q] = xc[q] = cplx{0.0, 0.0};
      if (i < nl * N && line < nr) {
        const int r = r0 + line, z = r / ny, y = r - z * ny;
        const cplx *row = src + (size_t(z) * Ly + y) * P;
        xf[q] = row[f];
        xc[q] = row[N - f];
      }
    }
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int i = threadIdx.x + (h * kB + q) * KT;
      if (i >= nl * N) continue;
      const int f = i & (N - 1);
      const cplx xcc = cconj(xc[q]);
      const cplx E = cadd(xf[q], xcc);
      const cplx O = cmul(csub(xf[q], xcc), cconj(wl(f, N, tlo, thi, w1)));
      buf[(i >> lN) * LS + pd(f)] = cplx{E.x - O.y, E.y + O.x};
    }
  }
  __syncthreads();
  fft_lines<true, KT, KP>(buf, N, LS, nl, tlo, thi);
  double *dst = (a < 3) ? hout + size_t(a) * nx * ny * nz : phi;
  // (x, x + 1) pairs are 16-byte aligned for an even row length and base
  const bool even = (nx & 1) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0;
  for (int i = threadIdx.x; i < nl * N; i += KT) {
    const int line = i >> lN, m = i & (N - 1);
    if (line >= nr) continue;
    const cplx v = buf[line * LS + pd(m)];
    double *row = dst + size_t(r0 + line) * nx;
    const int xa = 2 * m, xb = 2 * m + 1;
    if (even && xb < nx) {
      *reinterpret_cast<double2 *>(row + xa) = make_double2(v.x, v.y);
    } else {
      if (xa < nx) row[xa] = v.x;
      if (xb < nx) row[xb] = v.y;
    }
  }
}

// Row pitch of the half spectra: Lx/2 + 1 rounded up to 8 points (128 B).
int pitch(int Lx) { return (Lx / 2 + 1 + 7) & ~7; }

template <typename Kern> demag_status allow_lds(Kern k, size_t lds) {
  DEMAG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    int(lds)));
  return DEMAG_OK;
}

// Passes along x and y with workgroups of shape <KT, KP>.
template <int KT, int KP> struct xy_passes {
  static constexpr size_t lds = sizeof(cplx) * (cap(KP) + 128);
  static demag_status fwd(hipStream_t s, const double *m, cplx *S, size_t as, int nx, int ny, int nz, int Lx,
                          int Ly, int P) {
    demag_status st = allow_lds(k_x_fwd<KT, KP>, lds);
    if (st == DEMAG_OK) st = allow_lds(k_lines<false, KT, KP>, lds);
    if (st != DEMAG_OK) return st;
    const int H = Lx / 2 + 1, rows = ny * nz;
    const int lx = ilog2(lines_per_wg(Lx / 2, KP)), ly = ilog2(lines_per_wg(Ly, KP));
    const unsigned ytiles = unsigned((H + (1 << ly) - 1) >> ly);
    k_x_fwd<KT, KP><<<dim3((rows + (1 << lx) - 1) >> lx, 3), KT, lds, s>>>(m, S, as, nx, ny, nz, Lx, Ly, P, lx);
    k_lines<false, KT, KP><<<ytiles * nz * 3, KT, lds, s>>>(S, as, Ly, H, P, nz, ny, Ly, ly);
    return DEMAG_OK;
  }
  static demag_status inv(hipStream_t s, cplx *S, size_t as, double *phi, double *h, int nx, int ny, int nz,
                          int Lx, int Ly, int P) {
    demag_status st = allow_lds(k_x_inv<KT, KP>, lds);
    if (st == DEMAG_OK) st = allow_lds(k_lines<true, KT, KP>, lds);
    if (st != DEMAG_OK) return st;
    const int H = Lx / 2 + 1, rows = ny * nz;
    const int lx = ilog2(lines_per_wg(Lx / 2, KP)), ly = ilog2(lines_per_wg(Ly, KP));
    const unsigned ytiles = unsigned((H + (1 << ly) - 1) >> ly);
    k_lines<true, KT, KP><<<ytiles * nz * 4, KT, lds, s>>>(S, as, Ly, H, P, nz, Ly, ny, ly);
    k_x_inv<KT, KP><<<dim3((rows + (1 << lx) - 1) >> lx, 4), KT, lds, s>>>(S, as, phi, h, nx, ny, nz, Lx, Ly, P, lx);
    return DEMAG_OK;
  }
};

template <int KT, int KP>
demag_status z_conv(hipStream_t s, cplx *S, size_t as, const double *K, int Lz, int nz, int Ly, int P, int H,
                    double scale, double phi_scale) {
  constexpr size_t lds = sizeof(cplx) * (cap(KP) + 128);
  demag_status st = allow_lds(k_z_conv<KT, KP>, lds);
  if (st != DEMAG_OK) return st;
  const int l = ilog2(lines_per_wg(Lz, KP, 4));
  const unsigned tiles = unsigned((H + (1 << l) - 1) >> l);
  k_z_conv<KT, KP><<<tiles * Ly, KT, lds, s>>>(S, as, K, Lz, nz, Ly, P, H, l, scale, phi_scale);
  return DEMAG_OK;
}

}  // namespace

demag_status prepare_fft3d(demag_ctx *ctx, demag_factors *f) {
  if (f->k3) return DEMAG_OK;
  demag_status st = prepare_spectra(ctx, f);
  if (st != DEMAG_OK) return st;
  const int Lx = fft_length(f->n[0]), Ly = fft_length(f->n[1]), Lz = fft_length(f->n[2]);
  const size_t npk = size_t(Lz / 2 + 1) * (Ly / 2 + 1) * pitch(Lx);
  DEMAG_TRY_HIP(hipMalloc(&f->k3, kKC * npk * sizeof(double)));
  k_kernel_spectra<<<unsigned((npk + 255) / 256), 256, 0, ctx->stream>>>(f->spec[0], f->spec[1], f->spec[2], f->k3,
                                                                        f->M, Lx, Ly, Lz, pitch(Lx));
  DEMAG_TRY_HIP(hipGetLastError());
  return DEMAG_OK;
}

size_t fft3d_workspace_bytes(const demag_factors *f) {
  const int Lx = fft_length(f->n[0]), Ly = fft_length(f->n[1]), Lz = fft_length(f->n[2]);
  return 4 * size_t(Lz) * Ly * pitch(Lx) * sizeof(cplx);
}

demag_status launch_fft3d(demag_ctx *ctx, const demag_factors *f, const double *m, double *phi, double *h,
                          void *ws) {
  const int nx = f->n[0], ny = f->n[1], nz = f->n[2];
  const int Lx = fft_length(nx), Ly = fft_length(ny), Lz = fft_length(nz);
  const int H = Lx / 2 + 1, P = pitch(Lx);
  const size_t as = size_t(Lz) * Ly * P;        // array stride
  cplx *S = static_cast<cplx *>(ws);
  hipStream_t s = ctx->stream;
  hipEvent_t ev = nullptr;
  demag_status st = prof_begin(ctx, &ev);
  if (st != DEMAG_OK) return st;
  // x and y lines in 4096-point workgroups; the fused z pass in column groups
  // of at least four lines (8192-point workgroups beyond Lz = 256)
  const double scale = 1.0 / (double(Lx) * Ly * Lz);
  st = xy_passes<256, 4096>::fwd(s, m, S, as, nx, ny, nz, Lx, Ly, P);
  if (st == DEMAG_OK)
    st = Lz > 256 ? z_conv<512, 8192>(s, S, as, f->k3, Lz, nz, Ly, P, H, scale, f->L)
                  : z_conv<256, 4096>(s, S, as, f->k3, Lz, nz, Ly, P, H, scale, f->L);
  if (st == DEMAG_OK) st = xy_passes<256, 4096>::inv(s, S, as, phi, h, nx, ny, nz, Lx, Ly, P);
  if (st != DEMAG_OK) return st;
  DEMAG_TRY_HIP(hipGetLastError());
  if (ev) {
    // FFT flops 2.5 L log2 L per complex line of L points (half for the real
    // x transforms): 3 forward and 4 inverse 3D transforms; 18 flops per
    // frequency and component pair in the products
    const double vol = double(Lx) * Ly * Lz;
    const double flops = 7.0 * 2.5 * vol * std::log2(vol) / 2.0 + double(Lz) * Ly * H * 36.0;
    // compulsory traffic: m, the nine kernel spectra (one octant), the outputs
    const double bytes = 8.0 * (7.0 * nx * ny * nz) + 8.0 * 9.0 * double(Lz / 2 + 1) * (Ly / 2 + 1) * H;
    st = prof_end(ctx, ev, "fft3d/fp64", flops, bytes);
  }
  return st;
}

}  // namespace demag
