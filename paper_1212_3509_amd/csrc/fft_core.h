// Complex FFTs in LDS shared by the structured apply and the 3D FFT route:
// radix 16/8/4/2 Stockham passes over one or several lines, with sizes known
// at compile time per line length.  Templated on the real type: FP64
// (cplx) throughout the 3D route and the structured forward transforms, FP32
// (cplx32) for the structured inverse transforms of the FP32 apply.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace demag {
namespace fftc {

template <class T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};
using cplx = cx<double>;
using cplx32 = cx<float>;
template <class T> __device__ inline cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T> __device__ inline cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T> __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T> __device__ inline cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
template <bool INV, class T> __device__ inline cx<T> mul_mi(cx<T> a) {
  return INV ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

// LDS slot of point i of line b: b * LS + pd(i), with one pad slot after
// every 16 points.  16-byte LDS writes are served eight lanes at a time,
// conflict-free when those lanes hit distinct slots modulo 8 (reads: see
// slot below).  Butterflies
// run along a line across lanes (consecutive points: distinct, thanks to the
// pad for the Stockham stride-R stores); the transposed accesses of the
// strided passes put nl lines across lanes (fx fastest, then the point), and
// are conflict-free for a line stride LS = 8 / min(nl, 8) modulo 8.
__device__ inline int pd(int i) { return i + (i >> 4); }
// Single-line transforms (XS) use an unpadded layout instead: point i at
// slot i ^ ((i >> 4) & 15).  16-byte reads are served 16 lanes per cycle
// (within each half-wave, the 4-lane blocks (lane >> 2) & 7 of even and of
// odd bit parity together) and are conflict-free for slots distinct modulo
// 16: the pad of pd puts two lanes of such a group on one bank when lanes
// read consecutive points, the swizzle does not, and the Stockham stride-R
// stores stay distinct modulo 8.
// XS = 2: the same with bit 6 of i also folded into bit 3, for the radix-8
// plan of 4096-point FP32 lines (8-byte points: groups of 16 lanes,
// conflict-free for slots distinct modulo 16): its Ns = 8 pass stores the
// two halves of a group 64 points apart, on the same banks under XS = 1.
template <int XS> __device__ inline int slot(int i) {
  if constexpr (XS == 2) return i ^ (((i >> 4) ^ ((i >> 3) & 8)) & 15);
  else return XS ? (i ^ ((i >> 4) & 15)) : pd(i);
}
__host__ __device__ constexpr int line_stride(int N, int nl) {
  const int base = N + (N - 1) / 16;                  // pd(N - 1) + 1
  const int t = nl >= 8 ? 1 : 8 / nl;                 // wanted residue modulo 8
  return nl == 1 ? base : base + ((t - base % 8) + 8) % 8;
}
__host__ __device__ constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
// LDS points of a workgroup of shape <KT threads, KP points> (KP / KT = 16:
// one radix-16 butterfly per thread and pass)
__host__ __device__ constexpr int cap(int KP) { return KP + KP / 16 + 128; }
// lines of N points (N <= KP) per workgroup, in groups of g lines that share
// a column (g = 1, or 4 for the fused z pass); returns the lines per group
__host__ __device__ inline int lines_per_wg(int N, int KP, int g = 1) {
  int nl = KP / (N * g);
  while (nl > 1 && g * nl * line_stride(N, nl) > cap(KP)) nl /= 2;
  return nl;
}

template <bool INV, class T> __device__ inline void dft2(cx<T> *v) {
  const cx<T> t = v[0];
  v[0] = cadd(t, v[1]);
  v[1] = csub(t, v[1]);
}
template <bool INV, class T> __device__ inline void dft4(cx<T> *v) {
  const cx<T> s0 = cadd(v[0], v[2]), d0 = csub(v[0], v[2]);
  const cx<T> s1 = cadd(v[1], v[3]), d1 = mul_mi<INV>(csub(v[1], v[3]));
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
template <bool INV, int R1, int R2, class T> __device__ inline void dft_split(cx<T> *v) {
  cx<T> t[R1 * R2];
#pragma unroll
  for (int b = 0; b < R2; ++b) {
    cx<T> col[R1];
#pragma unroll
    for (int a = 0; a < R1; ++a) col[a] = v[R2 * a + b];
    dft4<INV>(col);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      if (b * k1 == 0) {
        t[b * R1 + k1] = col[k1];
      } else {
        const int e = (b * k1 * (16 / (R1 * R2))) & 15;   // angle 2 pi e / 16
        t[b * R1 + k1] = cmul(col[k1], cx<T>{T(cos16(e)), T(INV ? sin16(e) : -sin16(e))});
      }
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cx<T> row[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) row[b] = t[b * R1 + k1];
    if (R2 == 2) dft2<INV>(row);
    else dft4<INV>(row);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = row[k2];
  }
}
template <bool INV, int R, class T> __device__ inline void dftR(cx<T> *v) {
  if (R == 2) dft2<INV>(v);
  else if (R == 4) dft4<INV>(v);
  else if (R == 8) dft_split<INV, 4, 2>(v);
  else dft_split<INV, 4, 4>(v);
}

// W_N^e (forward sign).  FP64: from two LDS tables lo[i] = W_N^i, hi[i] =
// W_N^(64 i) (one product).  FP32: lo is the whole table W_N^e, e < N, each
// entry rounded once from FP64 (hi unused), so every twiddle is within half
// an ulp; products of rounded entries would double that.
template <class T> __device__ inline cx<T> twid(int e, const cx<T> *lo, const cx<T> *hi) {
  if constexpr (std::is_same_v<T, float>) {
    (void)hi;
    return lo[e];
  } else {
    const cx<T> a = lo[e & 63];
    return (e >> 6) ? cmul(a, hi[e >> 6]) : a;
  }
}
template <class T> __device__ inline void make_twiddles(cx<T> *lo, cx<T> *hi, int N) {
  for (int t = threadIdx.x; t < 128; t += blockDim.x) {
    double s, c;
    sincospi(-2.0 * double(t < 64 ? t : 64 * (t - 64)) / double(N), &s, &c);
    (t < 64 ? lo[t] : hi[t - 64]) = cx<T>{T(c), T(s)};
  }
}

// One Stockham pass of radix R over nlines lines of N points at line stride
// LS (input sub-transform length Ns).  Butterfly g: line g / (N / R), index
// g % (N / R).  The first pass (Ns = 1) has no twiddles.
// Destination of the results of a pass: the LDS lines (ToLds), or, for the
// last pass of a transform, a functor sink(line, index, value).
struct ToLds {};

// FP32 twiddles in pass-major order (PM = 16) for the inverse transforms whose
// first radix-16 pass runs in registers: the pass of sub-transform length
// Ns and radix R reads entry pm_offset(Ns) + (r - 1) Ns + k = W_N^(k r N /
// (Ns R)), k < Ns, 1 <= r < R, so the 16 lanes of a read group (consecutive
// k) read consecutive entries.  The whole table W_N^e, indexed by e = k r N
// / (Ns R), puts those lanes N R / (Ns R) entries apart: on one bank for
// Ns = 16.  Passes: Ns = 16 (R = 16, 240 entries), then Ns = 256 (R = N / 256).
// PM = 8: the radix-8 plan of 4096-point lines (first pass in registers,
// then Ns = 8, 64, 512, radix 8 each; 56 + 448 + 3584 entries).
__host__ __device__ constexpr int pm_offset(int PM, int Ns) {
  return PM == 16 ? (Ns == 16 ? 0 : 15 * 16) : (Ns == 8 ? 0 : Ns == 64 ? 7 * 8 : 7 * 8 + 7 * 64);
}
__host__ __device__ constexpr int pm_twiddle_count(int N) { return N >= 256 ? 15 * 16 + (N / 256 - 1) * 256 : 0; }
__host__ __device__ constexpr int pm8_twiddle_count(int N) { return N == 4096 ? 7 * 8 + 7 * 64 + 7 * 512 : 0; }

template <bool INV, int R, int KT, int KP, int N, int Ns, typename Sink = ToLds, int XS = 0, int PM = 0,
          class T>
__device__ inline void pass(cx<T> *buf, int LS, int nlines, const cx<T> *tlo, const cx<T> *thi,
                            const Sink &sink = Sink{}) {
  constexpr int per = N / R;             // butterflies per line
  constexpr int lper = ilog2(per);
  constexpr int kMaxB = (KP / R + KT - 1) / KT;
  const int nb = nlines << lper;
  cx<T> v[kMaxB][R];
#pragma unroll
  for (int q = 0; q < kMaxB; ++q) {
    const int g = threadIdx.x + q * KT;
    if (g < nb) {
      const int j = g & (per - 1), line = g >> lper;
      const cx<T> *lb = buf + line * LS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = lb[slot<XS>(j + r * per)];
      if constexpr (Ns > 1 && std::is_same_v<T, float> && PM != 0) {
        static_assert(PM == 16 ? (Ns == 16 || Ns == 256) : (N == 4096 && R == 8 && (Ns == 8 || Ns == 64 || Ns == 512)),
                      "pass-major twiddles: passes of the radix-16 or the radix-8 plan");
        const int k = j & (Ns - 1);
        const cx<T> *tp = tlo + pm_offset(PM, Ns) + k;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tp[(r - 1) * Ns];
          if (INV) w = cconj(w);
          v[q][r] = cmul(v[q][r], w);
        }
      } else if constexpr (Ns > 1 && std::is_same_v<T, float>) {
        // FP32: every power w^r straight from the table (one rounded entry
        // each); a chain of products would compound FP32 roundoff over the
        // passes
        const int k = j & (Ns - 1);
        const int e = k * (N / (Ns * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = twid((e * r) & (N - 1), tlo, thi);
          if (INV) w = cconj(w);
          v[q][r] = cmul(v[q][r], w);
        }
      } else if constexpr (Ns > 1) {
        const int k = j & (Ns - 1);
        cx<T> w = twid(k * (N / (Ns * R)), tlo, thi);
        if (INV) w = cconj(w);
        // powers w^r, r < R, as w^(4a + b) = (w^4)^a w^b: dependency depth 5
        cx<T> wp[R];
        wp[1] = w;
        if constexpr (R > 2) {
          wp[2] = cmul(w, w);
          wp[3] = cmul(wp[2], w);
        }
        if constexpr (R > 4) {
          wp[4] = cmul(wp[2], wp[2]);
#pragma unroll
          for (int r = 5; r < 8; ++r) wp[r] = cmul(wp[4], wp[r - 4]);
        }
        if constexpr (R > 8) {
          wp[8] = cmul(wp[4], wp[4]);
          wp[12] = cmul(wp[8], wp[4]);
#pragma unroll
          for (int r = 9; r < 12; ++r) wp[r] = cmul(wp[8], wp[r - 8]);
#pragma unroll
          for (int r = 13; r < 16; ++r) wp[r] = cmul(wp[12], wp[r - 12]);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], wp[r]);
      }
      dftR<INV, R>(v[q]);
    }
  }
  if constexpr (std::is_same_v<Sink, ToLds>) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaxB; ++q) {
      const int g = threadIdx.x + q * KT;
      if (g < nb) {
        const int j = g & (per - 1), line = g >> lper;
        const int k = j & (Ns - 1);
        const int o = (j / Ns) * Ns * R + k;
        cx<T> *lb = buf + line * LS;
#pragma unroll
        for (int r = 0; r < R; ++r) lb[slot<XS>(o + r * Ns)] = v[q][r];
      }
    }
    __syncthreads();
  } else {
    // no LDS writes: callers synchronize before reusing the lines
#pragma unroll
    for (int q = 0; q < kMaxB; ++q) {
      const int g = threadIdx.x + q * KT;
      if (g < nb) {
        const int j = g & (per - 1), line = g >> lper;
        const int k = j & (Ns - 1);
        const int o = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) sink(line, o + r * Ns, v[q][r]);
      }
    }
  }
}

// Complex FFTs of nlines lines of N points at line stride LS (power of 2, N <= 4096,
// or 8192 in workgroups of KP >= 8192 points) in LDS: a fixed pass plan per length (radix 16 first), each pass inlined with
// its sizes known at compile time, so that the register allocation and the
// index arithmetic are per pass.
template <bool INV, int KT, int KP, int N, int Ns, typename Sink, bool XS, int R0, int... Rs, class T>
__device__ inline void run_passes(cx<T> *buf, int LS, int nlines, const cx<T> *tlo, const cx<T> *thi,
                                  const Sink &sink) {
  if constexpr (sizeof...(Rs) > 0) {
    pass<INV, R0, KT, KP, N, Ns, ToLds, XS>(buf, LS, nlines, tlo, thi);
    run_passes<INV, KT, KP, N, Ns * R0, Sink, XS, Rs...>(buf, LS, nlines, tlo, thi, sink);
  } else {
    pass<INV, R0, KT, KP, N, Ns, Sink, XS>(buf, LS, nlines, tlo, thi, sink);
  }
}
// Transforms whose last pass hands its results to sink (ToLds: in place).
template <bool INV, int KT, int KP, typename Sink, bool XS = false, class T = double>
__device__ __noinline__ void fft_lines_to(cx<T> *buf, int N, int LS, int nlines, const cx<T> *tlo, const cx<T> *thi,
                                          Sink sink) {
  switch (N) {
    case 2: run_passes<INV, KT, KP, 2, 1, Sink, XS, 2>(buf, LS, nlines, tlo, thi, sink); break;
    case 4: run_passes<INV, KT, KP, 4, 1, Sink, XS, 4>(buf, LS, nlines, tlo, thi, sink); break;
    case 8: run_passes<INV, KT, KP, 8, 1, Sink, XS, 8>(buf, LS, nlines, tlo, thi, sink); break;
    case 16: run_passes<INV, KT, KP, 16, 1, Sink, XS, 16>(buf, LS, nlines, tlo, thi, sink); break;
    case 32: run_passes<INV, KT, KP, 32, 1, Sink, XS, 16, 2>(buf, LS, nlines, tlo, thi, sink); break;
    case 64: run_passes<INV, KT, KP, 64, 1, Sink, XS, 16, 4>(buf, LS, nlines, tlo, thi, sink); break;
    case 128: run_passes<INV, KT, KP, 128, 1, Sink, XS, 16, 8>(buf, LS, nlines, tlo, thi, sink); break;
    case 256: run_passes<INV, KT, KP, 256, 1, Sink, XS, 16, 16>(buf, LS, nlines, tlo, thi, sink); break;
    case 512: run_passes<INV, KT, KP, 512, 1, Sink, XS, 16, 16, 2>(buf, LS, nlines, tlo, thi, sink); break;
    case 1024: run_passes<INV, KT, KP, 1024, 1, Sink, XS, 16, 16, 4>(buf, LS, nlines, tlo, thi, sink); break;
    case 2048: run_passes<INV, KT, KP, 2048, 1, Sink, XS, 16, 16, 8>(buf, LS, nlines, tlo, thi, sink); break;
    case 4096: run_passes<INV, KT, KP, 4096, 1, Sink, XS, 16, 16, 16>(buf, LS, nlines, tlo, thi, sink); break;
    case 8192:
      if constexpr (KP >= 8192) run_passes<INV, KT, KP, 8192, 1, Sink, XS, 16, 16, 16, 2>(buf, LS, nlines, tlo, thi, sink);
      break;
    default:   // N = 1: identity
      if constexpr (!std::is_same_v<Sink, ToLds>) {
        for (int line = threadIdx.x; line < nlines; line += KT) sink(line, 0, buf[line * LS]);
      }
      break;
  }
}
template <bool INV, int KT, int KP, bool XS = false, class T>
__device__ inline void fft_lines(cx<T> *buf, int N, int LS, int nlines, const cx<T> *tlo, const cx<T> *thi) {
  fft_lines_to<INV, KT, KP, ToLds, XS, T>(buf, N, LS, nlines, tlo, thi, ToLds{});
}

// W_L^f for the real-transform (un)packing, L = 2N: W_N^(f/2), times W_L^1 for odd f.
template <class T> __device__ inline cx<T> wl(int f, int N, const cx<T> *tlo, const cx<T> *thi, cx<T> w1) {
  cx<T> w = twid((f >> 1) & (N - 1), tlo, thi);
  if (f & 1) w = cmul(w, w1);
  return w;
}

}  // namespace fftc
}  // namespace demag
