// Real-field mode (real sigma1, real graded medium).
//
// With real sigma1 every scheme keeps its fields real: MS, EM and the power /
// adjoint iterations have real local coefficients, and in H'' (eqs. J27-J37)
// p1 is real while p2, p3 are imaginary, so Q stays real and S, T stay
// imaginary; they are stored as S' = S/i, T' = T/i with
//   s = p1 Q - q2 S' - q3 T'   (q2 = Im p2, q3 = Im p3),
//   S' <- -z (2 q2 s - S'),  T' <- z (2 q3 s - T'),
// the same algebra as the complex form of eq. J36 / J44.
//
// Layout: real-space arrays (E_prev, S', T') are real [b][c][N^d]; the iterate
// X is stored as the Hermitian half of its x-direction spectrum, kx = 0..n0/2.
// In 3D a row holds H = n0/2 + 1 complex values.  In 2D (when that removes a
// Gamma-pass tile from the busiest CU) the two coefficients that are real
// for a real row, kx = 0 and kx = n0/2, share column 0 (real and imaginary
// part), so a row holds H = n0/2 values.  Rows start every hp >= H elements
// ([b][c][hp n1 n2]; the pad is never read); in 3D hp is a whole number of
// 128-byte cache lines, so that a strided pass's tile of adjacent columns
// shares cache lines only with the neighbouring tiles of the same row.  Two real rows of one component share one complex FFT of length
// n0: w = a + i b, and a, b are recovered from w(k) and w(n0 - k).
#pragma once

#include "kernels_p2.hpp"

namespace scfft {

// Loads and stores of the streams only the x pass uses (phase map, E_prev,
// H'' slots).  NT marks them nontemporal: where an iteration's arrays do not
// fit in the 256 MB Infinity Cache, that keeps the half spectrum the x pass
// writes there for the next pass (256^3 fp32: forward y pass 107 -> 62 us);
// where they fit it costs (2048^2 fp32 x pass 41 -> 47 us), so it is chosen
// per plan.
template <bool NT, typename U>
__device__ __forceinline__ U ld_x(const U* p) {
  if (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT, typename U>
__device__ __forceinline__ void st_x(U* p, U v) {
  if (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <typename T, int MK, bool NT = false>
struct LocalMapR {
  int iter, kind;
  T cE[2], cO[2], cJ[2], cS[2];
  T s1, s0, p1, q2, q3, z, inv1w, p1kap;
  T invM, e0c;
  const uint8_t* phase;
  const double* dens;
  T* S;
  T* Tt;
  T* Ep;

  __device__ __forceinline__ void load(const XArgs& a, int solve, int comp, long long rbase) {
    const SolveCoef& cf = a.coef[solve];
    const SolveCtl& ctl = a.ctl[solve];
    iter = ctl.iter;
    kind = cf.kind;
    for (int ph = 0; ph < 2; ++ph) {
      cE[ph] = (T)cf.cE[ph][0];
      cO[ph] = (T)cf.cO[ph][0];
      cJ[ph] = (T)cf.cJ[ph][0];
      cS[ph] = (T)cf.cS[ph][0];
    }
    s1 = (T)cf.s1[0];
    s0 = (T)cf.s0[0];
    p1 = (T)cf.p[0][0];
    q2 = (T)cf.p[1][1];
    q3 = (T)cf.p[2][1];
    z = (T)cf.z[0];
    inv1w = (T)cf.inv1w[0];
    p1kap = (T)cf.p1kap[0];
    invM = (T)a.invM;
    e0c = (T)ctl.e0[comp];
    phase = a.phase;
    dens = a.density;
    S = a.Sslot ? reinterpret_cast<T*>(a.Sslot) + rbase : nullptr;
    Tt = a.Tslot ? reinterpret_cast<T*>(a.Tslot) + rbase : nullptr;
    Ep = reinterpret_cast<T*>(a.Eprev) + rbase;
  }

  // Row-relative form: pointers advanced to the row start (uniform per
  // workgroup), k the 32-bit position in the row.
  struct Row {
    const uint8_t* ph;
    const double* rho;
    T* S;
    T* Tt;
    T* Ep;
  };
  __device__ __forceinline__ Row row(long long r0) const {
    Row w;
    w.ph = phase ? phase + r0 : nullptr;
    w.rho = dens ? dens + r0 : nullptr;
    w.S = S ? S + r0 : nullptr;
    w.Tt = Tt ? Tt + r0 : nullptr;
    w.Ep = Ep + r0;
    return w;
  }

  __device__ __forceinline__ T apply(T raw, const Row& w, unsigned int k, Acc& acc) const {
    const bool ph = MK == MAP_LIN_DENS ? false : w.ph[k] != 0;
    return apply_pf<false>(raw, ph, w.Ep[k], (T)0, (T)0, w, k, acc);
  }

  // Same step with the phase and the old E_prev value already in registers
  // (loaded before the inverse FFT, so their latency hides under it).
  // With SLOTS the H'' slots sv, tv (phase-1 voxels) are prefetched as well.
  template <bool SLOTS>
  __device__ __forceinline__ T apply_pf(T raw, bool phk, T epo, T sv, T tv, const Row& w,
                                        unsigned int k, Acc& acc) const {
    const T x = invM * raw;
    T E, J, out;
    if (MK == MAP_ACC_EM) {
      if (phk) {
        if (!SLOTS) {
          sv = ld_x<NT>(&w.S[k]);
          tv = ld_x<NT>(&w.Tt[k]);
        }
        const T s = p1 * x - q2 * sv - q3 * tv;
        E = inv1w * x + p1kap * s;
        J = s1 * E;
        out = z * ((T)2 * p1 * s - x);
        st_x<NT>(&w.S[k], -z * ((T)2 * q2 * s - sv));
        st_x<NT>(&w.Tt[k], z * ((T)2 * q3 * s - tv));
      } else {
        E = inv1w * x;
        J = E;
        out = -z * x;
      }
    } else if (MK == MAP_ACC_MS) {
      E = x;
      if (phk) {
        if (!SLOTS) sv = ld_x<NT>(&w.S[k]);
        const T s = p1 * x - q2 * sv;
        J = s1 * E;
        out = z * (x - (T)2 * p1 * s);
        st_x<NT>(&w.S[k], z * (sv - (T)2 * q2 * s));
      } else {
        J = E;
        out = z * x;
      }
    } else {
      T ce, co, cj, cs;
      if (MK == MAP_LIN_DENS) {
        const T rho = (T)w.rho[k];
        const T sig = (T)1 + (s1 - (T)1) * rho;
        if (kind == K_MS) {
          ce = (T)1;
          co = (T)1 - sig / s0;
          cj = sig;
          cs = (T)0;
        } else if (kind == K_EM) {
          ce = (T)1 / (sig + s0);
          co = (sig - s0) * ce;
          cj = sig;
          cs = (T)0;
        } else {   // adjoint
          ce = (T)1;
          co = (sig - s0) / (sig + s0);
          cj = (T)0;
          cs = sig / (sig + s0);
        }
      } else {
        const bool ph = phk != 0;
        ce = ph ? cE[1] : cE[0];
        co = ph ? cO[1] : cO[0];
        cj = ph ? cJ[1] : cJ[0];
        cs = ph ? cS[1] : cS[0];
      }
      E = ce * x;
      J = cj * E;
      out = co * x + cs * e0c;
    }
    acc.Jr += (double)J;
    acc.e2 += (double)(E * E);
    acc.eJ += (double)(E * J);
    if (iter >= 1) {
      const T dE = E - epo;
      acc.d2 += (double)(dE * dE);
    }
    st_x<NT>(&w.Ep[k], E);
    return out;
  }

};

// x pass, real mode: LINES complex lines = 2*LINES real rows of one component.
template <typename T, int N, int R, int MK, bool NT>
__global__ __launch_bounds__((XPassShape<N, R>::NTH)) void xpass_r2c_kernel(XArgs a) {
  using SH = XPassShape<N, R>;
  constexpr int TL = SH::TL, LINES = SH::LINES, NTH = SH::NTH;
  constexpr int LP = P2Plan<N, R>::LP;
  const int solve = blockIdx.z;
  const int comp = blockIdx.y;
  if (!a.ignore_done && a.ctl[solve].done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int line = tid / TL;
  const int j = tid - line * TL;
  const long long pr = (long long)blockIdx.x * LINES + line;
  const bool valid = pr < a.nlines / 2;
  const long long rowA = 2 * pr, rowB = 2 * pr + 1;
  const long long cbase = (long long)solve * a.d + comp;
  cx<T>* XA = reinterpret_cast<cx<T>*>(a.X) + cbase * a.Mh + rowA * a.hp;
  cx<T>* XB = XA + a.hp;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  cx<T> v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int k = j + TL * i;
    cx<T> av = mk<T>(0, 0), bv = mk<T>(0, 0);
    if (valid) {
      if (a.packed && (k == 0 || k == N / 2)) {
        const cx<T> pa = XA[0], pb = XB[0];
        av = mk<T>(k == 0 ? pa.x : pa.y, (T)0);
        bv = mk<T>(k == 0 ? pb.x : pb.y, (T)0);
      } else if (k <= N / 2) {
        av = XA[k];
        bv = XB[k];
      } else {
        av = conj(XA[N - k]);
        bv = conj(XB[N - k]);
      }
    }
    v[i] = mk<T>(av.x - bv.y, av.y + bv.x);   // a + i b
  }
  LocalMapR<T, MK, NT> lm;
  lm.load(a, solve, comp, cbase * a.M);
  const auto wa = lm.row(rowA * N);
  const auto wb = lm.row(rowB * N);
  // the phase maps and E_prev do not depend on the FFT: load them first
  constexpr bool PF = MK == MAP_LIN || MK == MAP_ACC_EM || MK == MAP_ACC_MS;
  // the H'' slots too where registers allow (fp32 with radix 4: measured
  // faster; at radix 8 or fp64 the extra registers cost a wave per SIMD)
  constexpr bool PSL = sizeof(T) == 4 && R <= 4;
  constexpr bool PS = PSL && (MK == MAP_ACC_EM || MK == MAP_ACC_MS);
  constexpr bool PT = PSL && MK == MAP_ACC_EM;
  // voxel-by-voxel fp64 accumulation where the map branches per voxel and
  // the slots are not already in registers (fewer VGPRs there; elsewhere
  // it measured neutral or a few registers worse)
  constexpr bool SETTLE = (MK == MAP_LIN_DENS || MK == MAP_ACC_EM || MK == MAP_ACC_MS) && !PSL;
  bool pha[R], phb[R];
  T epa[R], epb[R], sa[R], sb[R], ta[R], tb[R];
  if (PF && valid) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const unsigned int k = (unsigned int)(j + TL * i);
      pha[i] = ld_x<NT>(&wa.ph[k]) != 0;
      phb[i] = ld_x<NT>(&wb.ph[k]) != 0;
      epa[i] = ld_x<NT>(&wa.Ep[k]);
      epb[i] = ld_x<NT>(&wb.Ep[k]);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const unsigned int k = (unsigned int)(j + TL * i);
      sa[i] = (PS && pha[i]) ? ld_x<NT>(&wa.S[k]) : (T)0;
      sb[i] = (PS && phb[i]) ? ld_x<NT>(&wb.S[k]) : (T)0;
      ta[i] = (PT && pha[i]) ? ld_x<NT>(&wa.Tt[k]) : (T)0;
      tb[i] = (PT && phb[i]) ? ld_x<NT>(&wb.Tt[k]) : (T)0;
    }
  }
  cx<T>* slot = lds + line * LP;
  reg_fft<T, N, R>(v, slot, j, (T)1, tw);
  Acc acc;
  if (valid) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const unsigned int k = (unsigned int)(j + TL * i);
      T oa, ob;
      if (PF) {
        oa = lm.template apply_pf<PSL>(v[i].x, pha[i], epa[i], sa[i], ta[i], wa, k, acc);
        ob = lm.template apply_pf<PSL>(v[i].y, phb[i], epb[i], sb[i], tb[i], wb, k, acc);
      } else {
        oa = lm.apply(v[i].x, wa, k, acc);
        ob = lm.apply(v[i].y, wb, k, acc);
      }
      v[i] = mk<T>(oa, ob);
      if (SETTLE) acc_settle<false>(acc);
    }
  }
  reg_fft<T, N, R>(v, slot, j, (T)-1, tw);
  // split w(k) into the half spectra of the two rows: needs w(N - k)
  __syncthreads();
#pragma unroll
  for (int i = 0; i < R; ++i) slot[lpad<true>(j + TL * i)] = v[i];
  __syncthreads();
  if (valid) {
    T a0 = 0, b0 = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int k = j + TL * i;
      if (k <= N / 2) {
        const cx<T> wn = conj(slot[lpad<true>((N - k) & (N - 1))]);
        const cx<T> s = v[i] + wn, dd = v[i] - wn;
        const cx<T> xa = mk<T>((T)0.5 * s.x, (T)0.5 * s.y);
        const cx<T> xb = mk<T>((T)0.5 * dd.y, (T)-0.5 * dd.x);
        if (a.packed && (k == 0 || k == N / 2)) {
          // thread j = 0 holds both k = 0 (i = 0) and k = N/2 (i = R/2)
          if (k == 0) {
            a0 = xa.x;
            b0 = xb.x;
          } else {
            XA[0] = mk<T>(a0, xa.x);
            XB[0] = mk<T>(b0, xb.x);
          }
        } else {
          XA[k] = xa;
          XB[k] = xb;
        }
      }
    }
  }
  __syncthreads();
  block_reduce5<NTH>(acc, reinterpret_cast<double*>(smem_raw),
                     a.part + cbase * 5 * gridDim.x + blockIdx.x, gridDim.x, tid);
}

struct InitRArgs {
  void* X;
  void* Sslot;
  void* Tslot;
  SolveCtl* ctl;
  const SolveCoef* coef;
  long long M, Mh;
  int d, H, nsolve, has_st;   // H: the row pitch of X
};

// X^0 = constant c per component: half spectrum M*c at kx = 0 of every row.
template <typename T>
__global__ void init_real_kernel(InitRArgs a) {
  const long long totx = (long long)a.nsolve * a.d * a.Mh;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < totx;
       i += (long long)gridDim.x * blockDim.x) {
    const long long f = i / a.Mh;
    const long long g = i - f * a.Mh;
    const int c = (int)(f % a.d);
    const int s = (int)(f / a.d);
    cx<T> v = mk<T>(0, 0);
    if (g % a.H == 0) v = mk<T>((T)a.coef[s].init_src[c][0], (T)0);
    reinterpret_cast<cx<T>*>(a.X)[i] = v;
  }
  if (a.has_st) {
    const long long tot = (long long)a.nsolve * a.d * a.M;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (long long)gridDim.x * blockDim.x) {
      reinterpret_cast<T*>(a.Sslot)[i] = (T)0;
      reinterpret_cast<T*>(a.Tslot)[i] = (T)0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < a.nsolve) {
    SolveCtl* c = a.ctl + threadIdx.x;
    c->iter = 0;
    c->done = 0;
    c->status = -3;
    c->since_min = 0;
    c->min_r = __builtin_inf();
    c->res = __builtin_nan("");
  }
}

template <typename T>
__global__ void extract_real_kernel(ExtractArgs a) {
  const long long tot = (long long)a.d * a.M;
  const SolveCoef& cf = a.coef[a.solve];
  const T* src = reinterpret_cast<const T*>(a.Eprev) + (long long)a.solve * a.d * a.M;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x) {
    const long long g = i % a.M;
    const double e = (double)src[i];
    if (a.E) {
      a.E[2 * i] = e;
      a.E[2 * i + 1] = 0.0;
    }
    if (a.J) {
      double sig;
      if (cf.density) sig = 1.0 + (cf.s1[0] - 1.0) * a.density[g];
      else sig = a.phase[g] ? cf.s1[0] : 1.0;
      a.J[2 * i] = sig * e;
      a.J[2 * i + 1] = 0.0;
    }
  }
}

}  // namespace scfft
