// Lanczos process with full reorthogonalisation (fp64) for the spectral
// measure behind the singularities of sigma*(sigma1): A = Gamma_1 chi Gamma_1
// from v_0 = Gamma_1 chi e0 (section "Estimating the parameters alpha and
// beta").
//
// Every Lanczos vector is kept in the stored form the iteration passes
// exchange: X, the x-direction spectrum of the real-space field (half
// spectrum for real rows).  A is then one x pass (inverse x-FFT, chi, forward
// x-FFT) plus one Gamma pass, and the Gram-Schmidt steps work on that form.
// By Parseval the real-space inner product is, up to one factor common to all
// vectors, the spectral one with each stored element weighted by the number
// of real-space DFT coefficients it stands for: 1 for kx = 0 and kx = n0/2
// (real for real rows; in the packed column they are its real and imaginary
// parts), 2 for the other columns of a half spectrum, 1 everywhere in the
// full-spectrum form, and 0 in the pad of a row pitch.
#pragma once

#include "kernels.hpp"

namespace scfft {

struct LzArgs {
  cx<double>* X;       // current vector (vlen elements)
  cx<double>* Q;       // basis, [slot][vlen]
  double* part;        // [k][block][2] partial sums
  double* red;         // [k][2] reduced sums
  long long vlen;      // elements of one vector: d components of the stored grid
  int H, HP;           // stored columns per row, row pitch
  int half, packed;    // half spectrum (real rows); kx = 0 and n0/2 packed in column 0
  int nk;              // basis vectors 0..nk-1 taking part
  int slot;            // lz_scale_kernel: slot that receives the normalised X
  double* save;        // lz_reduce_kernel: where red[save_k].re is also written
  int save_k;
};

constexpr int kLzGroup = 8;   // basis vectors per workgroup row of lz_dots_kernel
constexpr int kLzThreads = 256;

__device__ __forceinline__ double lz_weight(const LzArgs& a, long long e) {
  const int col = (int)(e % a.HP);
  if (col >= a.H) return 0.0;
  if (!a.half || col == 0) return 1.0;
  if (!a.packed && col == a.H - 1) return 1.0;
  return 2.0;
}

// Sums NV values over the workgroup (wave64 shuffles, then LDS); thread t <
// NV then holds value t's sum in *out.
template <int NV>
__device__ __forceinline__ void lz_block_sum(const double* v, double* out) {
  __shared__ double sh[NV][kLzThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) sh[i][wave] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double s = 0;
    for (int w = 0; w < kLzThreads / 64; ++w) s += sh[threadIdx.x][w];
    *out = s;
  }
}

// Partial inner products (q_k, X) = sum w conj(q_k) X for the basis vectors
// k = kLzGroup * blockIdx.y + 0..kLzGroup-1, each workgroup over a
// grid-stride share of the elements.
__global__ __launch_bounds__(kLzThreads) void lz_dots_kernel(LzArgs a) {
  const int k0 = blockIdx.y * kLzGroup;
  const int nk = min(kLzGroup, a.nk - k0);
  double v[2 * kLzGroup];
#pragma unroll
  for (int i = 0; i < 2 * kLzGroup; ++i) v[i] = 0.0;
  for (long long e = (long long)blockIdx.x * kLzThreads + threadIdx.x; e < a.vlen;
       e += (long long)gridDim.x * kLzThreads) {
    const double w = lz_weight(a, e);
    if (w == 0.0) continue;
    const cx<double> x = a.X[e];
#pragma unroll
    for (int kk = 0; kk < kLzGroup; ++kk) {
      if (kk < nk) {
        const cx<double> q = a.Q[(long long)(k0 + kk) * a.vlen + e];
        v[2 * kk] += w * (q.x * x.x + q.y * x.y);
        v[2 * kk + 1] += w * (q.x * x.y - q.y * x.x);
      }
    }
  }
  double s = 0;
  lz_block_sum<2 * kLzGroup>(v, &s);
  if ((int)threadIdx.x < 2 * nk) {
    const int k = k0 + (int)threadIdx.x / 2;
    a.part[((long long)k * gridDim.x + blockIdx.x) * 2 + (threadIdx.x & 1)] = s;
  }
}

// red[k] = the sum of part[k][0..nblocks) in a fixed order (one workgroup per
// k); red[save_k].re is also stored at *save.
__global__ __launch_bounds__(kLzThreads) void lz_reduce_kernel(LzArgs a, int nblocks) {
  const int k = blockIdx.x;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kLzThreads) {
    v[0] += a.part[((long long)k * nblocks + b) * 2];
    v[1] += a.part[((long long)k * nblocks + b) * 2 + 1];
  }
  double s = 0;
  lz_block_sum<2>(v, &s);
  if (threadIdx.x < 2) {
    a.red[2 * k + threadIdx.x] = s;
    if (threadIdx.x == 0 && k == a.save_k && a.save) *a.save = s;
  }
}

// X <- X - sum_{k < nk} c_k q_k with c_k = red[k] (real parts only for half
// spectra, whose vectors stand for real fields).
__global__ __launch_bounds__(kLzThreads) void lz_update_kernel(LzArgs a) {
  for (long long e = (long long)blockIdx.x * kLzThreads + threadIdx.x; e < a.vlen;
       e += (long long)gridDim.x * kLzThreads) {
    if ((int)(e % a.HP) >= a.H) continue;
    cx<double> x = a.X[e];
    for (int k = 0; k < a.nk; ++k) {
      const cx<double> c = mk<double>(a.red[2 * k], a.half ? 0.0 : a.red[2 * k + 1]);
      x = x - c * a.Q[(long long)k * a.vlen + e];
    }
    a.X[e] = x;
  }
}

// Partial sums of the weighted |X|^2 (into part[0][block]).
__global__ __launch_bounds__(kLzThreads) void lz_norm_kernel(LzArgs a) {
  double v[2] = {0.0, 0.0};
  for (long long e = (long long)blockIdx.x * kLzThreads + threadIdx.x; e < a.vlen;
       e += (long long)gridDim.x * kLzThreads) {
    const double w = lz_weight(a, e);
    if (w == 0.0) continue;
    const cx<double> x = a.X[e];
    v[0] += w * (x.x * x.x + x.y * x.y);
  }
  double s = 0;
  lz_block_sum<2>(v, &s);
  if (threadIdx.x < 2) a.part[(long long)blockIdx.x * 2 + threadIdx.x] = s;
}

// X <- X / sqrt(red[0]) and Q[slot] <- X.
__global__ __launch_bounds__(kLzThreads) void lz_scale_kernel(LzArgs a) {
  const double inv = 1.0 / sqrt(a.red[0]);
  cx<double>* q = a.Q + (long long)a.slot * a.vlen;
  for (long long e = (long long)blockIdx.x * kLzThreads + threadIdx.x; e < a.vlen;
       e += (long long)gridDim.x * kLzThreads) {
    const cx<double> x = inv * a.X[e];
    a.X[e] = x;
    q[e] = x;
  }
}

}  // namespace scfft
