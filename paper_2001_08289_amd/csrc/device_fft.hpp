// Device-side complex arithmetic and a workgroup-cooperative Stockham FFT
// staged in LDS, for CDNA4 (gfx950, wave64).
//
// The FFT is the transform the paper's schemes use to go back and forth
// between real space (where the local conductivity acts) and Fourier space
// (where Gamma_1 of eq. J11 acts).  Unnormalised: forward uses
// exp(-2 pi i j k/n), inverse exp(+2 pi i j k/n).
//
// Algorithm: self-sorting Stockham, one radix-R pass at a time (R in
// {2,3,4,5,8}); pass p with stride Ns = product of the earlier radices maps
//   in[j + q n/R]  ->  twiddle exp(-+2 pi i (j mod Ns) q/(Ns R)), DFT_R,
//   out[(j div Ns) Ns R + (j mod Ns) + q Ns]          (q = 0..R-1).
// Every thread loads all of its butterflies' inputs into registers, the
// workgroup synchronises, then every thread writes its outputs, so one LDS
// buffer serves in place.  A workgroup transforms `nl` lines at once; a line's
// element k sits at lds[l*lstride + k*estride].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scfft {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk<T>(s * a.x, s * a.y); }
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return a.x * a.x + a.y * a.y; }
// multiply by i*s (s = +-1)
template <typename T>
__device__ __forceinline__ cx<T> mul_is(cx<T> a, T s) { return mk<T>(-s * a.y, s * a.x); }
template <typename T>
__device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  T d = b.x * b.x + b.y * b.y;
  return mk<T>((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
template <typename T, typename U>
__device__ __forceinline__ cx<T> cvt(cx<U> a) { return mk<T>((T)a.x, (T)a.y); }

// ----------------------------------------------------------------- butterflies
// In-place DFT of R registers with exponent sign s (-1 forward, +1 inverse).
template <typename T, int R>
struct Dft;

template <typename T>
struct Dft<T, 2> {
  __device__ __forceinline__ static void run(cx<T>* v, T) {
    cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T>
struct Dft<T, 3> {
  __device__ __forceinline__ static void run(cx<T>* v, T s) {
    const T h = (T)0.86602540378443864676;  // sqrt(3)/2
    cx<T> t1 = v[1] + v[2];
    cx<T> t2 = v[0] - (T)0.5 * t1;
    cx<T> t3 = mul_is(v[1] - v[2], s * h);
    v[0] = v[0] + t1;
    v[1] = t2 + t3;
    v[2] = t2 - t3;
  }
};

template <typename T>
struct Dft<T, 4> {
  __device__ __forceinline__ static void run(cx<T>* v, T s) {
    cx<T> a = v[0] + v[2], b = v[0] - v[2];
    cx<T> c = v[1] + v[3], d = mul_is(v[1] - v[3], s);
    v[0] = a + c;
    v[2] = a - c;
    v[1] = b + d;
    v[3] = b - d;
  }
};

template <typename T>
struct Dft<T, 5> {
  __device__ __forceinline__ static void run(cx<T>* v, T s) {
    const T c1 = (T)0.30901699437494742410;   // cos(2pi/5)
    const T c2 = (T)-0.80901699437494742410;  // cos(4pi/5)
    const T s1 = (T)0.95105651629515357212;   // sin(2pi/5)
    const T s2 = (T)0.58778525229247312917;   // sin(4pi/5)
    cx<T> t1 = v[1] + v[4], t2 = v[2] + v[3];
    cx<T> t3 = v[1] - v[4], t4 = v[2] - v[3];
    cx<T> a1 = v[0] + c1 * t1 + c2 * t2;
    cx<T> a2 = v[0] + c2 * t1 + c1 * t2;
    cx<T> b1 = mul_is(s1 * t3 + s2 * t4, s);
    cx<T> b2 = mul_is(s2 * t3 - s1 * t4, s);
    v[0] = v[0] + t1 + t2;
    v[1] = a1 + b1;
    v[4] = a1 - b1;
    v[2] = a2 + b2;
    v[3] = a2 - b2;
  }
};

template <typename T>
struct Dft<T, 8> {
  __device__ __forceinline__ static void run(cx<T>* v, T s) {
    const T r = (T)0.70710678118654752440;
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4>::run(e, s);
    Dft<T, 4>::run(o, s);
    // w8^k = exp(s i pi k / 4)
    cx<T> w1 = mk<T>(r, s * r);
    cx<T> w3 = mk<T>(-r, s * r);
    o[1] = o[1] * w1;
    o[2] = mul_is(o[2], s);
    o[3] = o[3] * w3;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = e[k] + o[k];
      v[k + 4] = e[k] - o[k];
    }
  }
};

// 16 points as 4 x 4: DFT4 over the stride-4 subsequences, the internal
// twiddles exp(s 2 pi i n2 k1/16), then DFT4 across them.
template <typename T>
struct Dft<T, 16> {
  __device__ __forceinline__ static void run(cx<T>* v, T s) {
    const T c1 = (T)0.92387953251128675613;  // cos(pi/8)
    const T s1 = (T)0.38268343236508977173;  // sin(pi/8)
    const T r = (T)0.70710678118654752440;
    cx<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cx<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Dft<T, 4>::run(t, s);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
    }
    // twiddles w^(n2 k1), w = exp(s 2 pi i/16); exponents 0..9
    y[1][1] = y[1][1] * mk<T>(c1, s * s1);
    y[1][2] = y[1][2] * mk<T>(r, s * r);
    y[1][3] = y[1][3] * mk<T>(s1, s * c1);
    y[2][1] = y[2][1] * mk<T>(r, s * r);
    y[2][2] = mul_is(y[2][2], s);
    y[2][3] = y[2][3] * mk<T>(-r, s * r);
    y[3][1] = y[3][1] * mk<T>(s1, s * c1);
    y[3][2] = y[3][2] * mk<T>(-r, s * r);
    y[3][3] = y[3][3] * mk<T>(-c1, -s * s1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cx<T> t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<T, 4>::run(t, s);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

// ------------------------------------------------------------- LDS Stockham
constexpr int kMaxPass = 16;

struct FftDesc {
  int n;
  int npass;
  int radix[kMaxPass];
};

// One radix-R pass over nl lines.  NT threads; each handles up to
// ceil(EMAX/R) butterflies, so nl*n <= NT*EMAX must hold.
template <typename T, int NT, int EMAX, int R>
__device__ __forceinline__ void stockham_pass(cx<T>* lds, int nl, int n, int ns, int lstride,
                                              int estride, bool line_fast, const cx<T>* __restrict__ tw,
                                              T sign, int tid) {
  constexpr int BPT = (EMAX + R - 1) / R;
  const int nbl = n / R;
  const int nb = nl * nbl;
  const int step = n / (ns * R);
  cx<T> v[BPT][R];
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int b = tid + u * NT;
    if (b < nb) {
      int l, j;
      if (line_fast) {
        l = b % nl;
        j = b / nl;
      } else {
        l = b / nbl;
        j = b - l * nbl;
      }
      const cx<T>* base = lds + l * lstride;
#pragma unroll
      for (int q = 0; q < R; ++q) v[u][q] = base[(j + q * nbl) * estride];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int b = tid + u * NT;
    if (b < nb) {
      int l, j;
      if (line_fast) {
        l = b % nl;
        j = b / nl;
      } else {
        l = b / nbl;
        j = b - l * nbl;
      }
      const int k = j % ns;
      if (ns > 1) {
        // one table load per butterfly; the powers w^q follow by products
        cx<T> w1 = tw[k * step];
        if (sign > 0) w1.y = -w1.y;
        cx<T> wq[R];
        wq[1] = w1;
#pragma unroll
        for (int q = 2; q < R; ++q) wq[q] = (q & 1) ? wq[q - 1] * w1 : wq[q / 2] * wq[q / 2];
#pragma unroll
        for (int q = 1; q < R; ++q) v[u][q] = v[u][q] * wq[q];
      }
      Dft<T, R>::run(v[u], sign);
      const int idxd = (j / ns) * ns * R + k;
      cx<T>* base = lds + l * lstride;
#pragma unroll
      for (int q = 0; q < R; ++q) base[(idxd + q * ns) * estride] = v[u][q];
    }
  }
  __syncthreads();
}

// Full transform of nl lines of length fd.n in LDS (callers synchronise before).
template <typename T, int NT, int EMAX>
__device__ void fft_lines(cx<T>* lds, int nl, const FftDesc& fd, int lstride, int estride,
                          bool line_fast, const cx<T>* __restrict__ tw, T sign, int tid) {
  int ns = 1;
  for (int p = 0; p < fd.npass; ++p) {
    const int r = fd.radix[p];
    switch (r) {
      case 8:
        stockham_pass<T, NT, EMAX, 8>(lds, nl, fd.n, ns, lstride, estride, line_fast, tw, sign, tid);
        break;
      case 4:
        stockham_pass<T, NT, EMAX, 4>(lds, nl, fd.n, ns, lstride, estride, line_fast, tw, sign, tid);
        break;
      case 2:
        stockham_pass<T, NT, EMAX, 2>(lds, nl, fd.n, ns, lstride, estride, line_fast, tw, sign, tid);
        break;
      case 3:
        stockham_pass<T, NT, EMAX, 3>(lds, nl, fd.n, ns, lstride, estride, line_fast, tw, sign, tid);
        break;
      default:
        stockham_pass<T, NT, EMAX, 5>(lds, nl, fd.n, ns, lstride, estride, line_fast, tw, sign, tid);
        break;
    }
    ns *= r;
  }
}

}  // namespace scfft
