// Kernels of one solver iteration (CDNA4 / gfx950).
//
// Data layout in HBM, per solve b (a batch stacks solves):
//   X     [b][c][N^d] complex T: the iterate between passes, held as the
//         (unnormalised) x-direction DFT of N^d * X_real, i.e. x in Fourier
//         space and y (, z) in real space;
//   Eprev [b][c][N^d] complex T: physical field of the last iterate (used for
//         the relative increment and returned as the solution);
//   S, T  [b][c][N^d] complex T: the two extra slots of H'' (eq. J27), only
//         touched at phase-1 voxels (H'' schemes only);
//   part  [b][c][xblocks][5] double: per-workgroup partial sums.
//
// One iteration (2D): x pass (inverse x-FFT, physical field, reductions,
// local map, forward x-FFT) -> Gamma pass (forward y-FFT, Gamma_1 of eq. J11 /
// J44-J45 fused with the scheme's k = 0 source term, inverse y-FFT; one extra
// workgroup per solve reduces the x pass's fp64 partials and applies the stop
// rules).  3D adds a forward y pass before and an inverse y pass after the
// Gamma pass (which then runs along z).
#pragma once

#include "device_fft.hpp"

namespace scfft {

enum Kind { K_MS = 0, K_EM = 1, K_ACC_EM = 2, K_ACC_MS = 3, K_POWER = 4, K_ADJ = 5 };
enum Sym { SYM_ROTATED = 0, SYM_SPECTRAL = 1, SYM_NETWORK = 2 };

// Per-solve control block (device resident).  The host writes the parameter
// part before a solve; finalize_solve owns the state part afterwards.
struct SolveCtl {
  double tol, div_factor;
  int max_iter, stag_window;
  double e0[3];
  double inv_e0n2;
  int d, kind;
  // state
  int iter, done, status, since_min;
  double min_r, res, sstar_re, sstar_im, lam;
  double meanJ[6];
};

// Per-solve coefficients of the local real-space map (device resident).
// Phase-map media use the per-phase tables (index 0 = matrix, 1 = inclusion);
// graded media recompute them per voxel from sigma(x).
struct SolveCoef {
  int kind, density;
  double cE[2][2];   // physical field E = cE * X
  double cO[2][2];   // local-map output = cO * X + cS * e0_c
  double cJ[2][2];   // current J = cJ * E
  double cS[2][2];
  double s1[2], s0[2];
  double p[3][2];    // H'': p1, p2, p3 (eq. J24)
  double z[2];       // H'': z'' (EM) or z_M (MS)
  double inv1w[2];   // H'' EM: 1/(1 + sqrt t)
  double p1kap[2];   // H'' EM: p1 (1/(t + sqrt t) - 1/(1 + sqrt t))
  double ga, gb;     // Gamma pass: out = ga*in + gb*Gamma_1 in   (k != 0)
  double kz_keep;    //             out = kz_keep*in + kz_src[c] (k = 0)
  double pad;
  double kz_src[3][2];
  double init_src[3][2];   // N^d * (the constant source field X^0)
};

struct XArgs {
  void* X;
  void* Eprev;
  void* Sslot;
  void* Tslot;
  const uint8_t* phase;
  const double* density;
  double* part;
  SolveCtl* ctl;
  const SolveCoef* coef;
  const void* tw;       // twiddles for n0
  FftDesc fd;
  long long M;          // voxels per field
  long long Mh;         // stored elements of one component of X (real mode: H n1 n2)
  int n0, nlines, lines_per_block, d;
  double invM;
  int ignore_done;
  int packed;           // real mode, 2D: rows of n0/2 values, column 0 = X(0) + i X(n0/2)
  int hp;               // real mode: elements between consecutive rows of X (>= n0/2 + 1)
};

// Reduction inputs of the stop rules (see finalize_solve).
struct FArgs {
  const double* part;
  SolveCtl* ctl;
  double* hist_r;
  double* hist_s;
  int hist_cap;
  int nblocks;     // x-pass workgroups per component
  double invM;
  int ignore_done;
};

struct GArgs {
  void* X;
  SolveCtl* ctl;
  const SolveCoef* coef;
  const void* tw;       // twiddles for the line length
  const double* symtab[3];  // per-axis symbol tables (double2 per index)
  FftDesc fd;
  long long M;
  int n[3];
  int d, C, stride, symbol;
  int ignore_done;
  int mode;             // 0: Gamma pass; 1: forward FFT only; 2: inverse FFT only
  int fin;              // 1: one extra workgroup per solve runs finalize_solve
  int packed;           // 2D real mode: column 0 holds kx = 0 (real part) and kx = n0/2 (imaginary)
  FArgs f;
  int rp;               // elements between consecutive rows of X (the row pitch)
};

__device__ __forceinline__ void finalize_solve(const FArgs& a, int solve, int tid, int nth);

template <typename T>
__device__ __forceinline__ cx<T> ld2(const double* p) { return mk<T>((T)p[0], (T)p[1]); }

// ------------------------------------------------------- local real-space map
struct Acc {
  double Jr = 0, Ji = 0, e2 = 0, d2 = 0, eJ = 0;
};

// Makes the fp64 accumulation happen voxel by voxel in an unrolled loop.
// Without it the compiler sinks every voxel's conversions and adds below the
// map's last per-voxel branch (the H'' slots of phase-1 voxels), so all the
// voxels' E and J values stay live at once: the 2048-point fp32 x pass then
// needs 134 VGPRs (three waves per SIMD) instead of 120 (four).  The empty asm
// emits nothing; it only marks the accumulators as used and redefined here.
template <bool CPLX>
__device__ __forceinline__ void acc_settle(Acc& acc) {
  if (CPLX) asm volatile("" : "+v"(acc.Jr), "+v"(acc.Ji), "+v"(acc.e2), "+v"(acc.d2), "+v"(acc.eJ));
  else asm volatile("" : "+v"(acc.Jr), "+v"(acc.e2), "+v"(acc.d2), "+v"(acc.eJ));
}

// The scheme's pointwise step at one voxel: from the scaled iterate x it
// forms the physical field E (the Q-slot of E'' in H''), the current J, the
// fp64 reduction terms (sum J, |E|^2, |E - E_prev|^2, Re conj(E) J), stores E
// as the new E_prev, updates the S/T slots (H''), and returns the value the
// forward FFT receives: MS tau = (1 - sigma/sigma0) E; EM R = Z P; H'' the
// Q-slot of Z'' P'' (eq. J36 form) or of (I - sigma''/sigma0'') E''; the
// power and adjoint kinds their own linear maps.
enum MapKind { MAP_LIN = 0, MAP_LIN_DENS = 1, MAP_ACC_EM = 2, MAP_ACC_MS = 3, MAP_ANY = 4 };

// MK fixes the branch at compile time (MAP_ANY decides at run time).
template <typename T, int MK = MAP_ANY>
struct LocalMap {
  int kind, density, iter;
  cx<T> cE[2], cO[2], cJ[2], cS[2];
  cx<T> s1, s0, p1, p2, p3, z, inv1w, p1kap;
  T invM, e0c;
  const uint8_t* phase;
  const double* dens;
  cx<T>* S;
  cx<T>* Tt;
  cx<T>* Ep;

  __device__ __forceinline__ void load(const XArgs& a, int solve, int comp, long long fbase) {
    const SolveCoef& cf = a.coef[solve];
    const SolveCtl& ctl = a.ctl[solve];
    kind = cf.kind;
    density = cf.density;
    iter = ctl.iter;
    for (int ph = 0; ph < 2; ++ph) {
      cE[ph] = ld2<T>(cf.cE[ph]);
      cO[ph] = ld2<T>(cf.cO[ph]);
      cJ[ph] = ld2<T>(cf.cJ[ph]);
      cS[ph] = ld2<T>(cf.cS[ph]);
    }
    s1 = ld2<T>(cf.s1);
    s0 = ld2<T>(cf.s0);
    p1 = ld2<T>(cf.p[0]);
    p2 = ld2<T>(cf.p[1]);
    p3 = ld2<T>(cf.p[2]);
    z = ld2<T>(cf.z);
    inv1w = ld2<T>(cf.inv1w);
    p1kap = ld2<T>(cf.p1kap);
    invM = (T)a.invM;
    e0c = (T)ctl.e0[comp];
    phase = a.phase;
    dens = a.density;
    S = a.Sslot ? reinterpret_cast<cx<T>*>(a.Sslot) + fbase : nullptr;
    Tt = a.Tslot ? reinterpret_cast<cx<T>*>(a.Tslot) + fbase : nullptr;
    Ep = reinterpret_cast<cx<T>*>(a.Eprev) + fbase;
  }

  __device__ __forceinline__ cx<T> apply(cx<T> raw, long long g, Acc& acc) const {
    return apply_core<false>(raw, g, false, mk<T>(0, 0), acc);
  }

  // Same step with the phase and the old E_prev value already in registers
  // (loaded before the inverse FFT, so their latency hides under it).
  __device__ __forceinline__ cx<T> apply_pf(cx<T> raw, long long g, bool phv, cx<T> epo,
                                            Acc& acc) const {
    return apply_core<true>(raw, g, phv, epo, acc);
  }

  template <bool PF>
  __device__ __forceinline__ cx<T> apply_core(cx<T> raw, long long g, bool phv, cx<T> epo,
                                              Acc& acc) const {
    const cx<T> x = invM * raw;
    cx<T> E, J, out;
    const bool acc_kind = MK == MAP_ANY ? (kind == K_ACC_EM || kind == K_ACC_MS)
                                        : (MK == MAP_ACC_EM || MK == MAP_ACC_MS);
    const bool acc_em = MK == MAP_ANY ? kind == K_ACC_EM : MK == MAP_ACC_EM;
    const bool dens_kind = MK == MAP_ANY ? density != 0 : MK == MAP_LIN_DENS;
    if (acc_kind) {
      const T two = (T)2;
      const int ph = PF ? (int)phv : phase[g];
      if (acc_em) {
        if (ph) {
          // phase 1 of H'': s = p^T (Q, S, T); Z'' = z (2 p p^T - I)
          const cx<T> sv = S[g], tv = Tt[g];
          const cx<T> s = p1 * x + p2 * sv + p3 * tv;
          E = inv1w * x + p1kap * s;
          J = s1 * E;
          out = z * (two * (p1 * s) - x);
          S[g] = mk<T>(0, 0) - z * (two * (p2 * s) - sv);   // W'' flips S (eq. J44)
          Tt[g] = z * (two * (p3 * s) - tv);
        } else {
          E = inv1w * x;
          J = E;
          out = mk<T>(0, 0) - z * x;
        }
      } else {
        E = x;
        if (ph) {
          const cx<T> sv = S[g];
          const cx<T> s = p1 * x + p2 * sv;      // the T-slot of E'' is zero
          J = s1 * E;
          out = z * (x - two * (p1 * s));
          S[g] = z * (sv - two * (p2 * s));
        } else {
          J = E;
          out = z * x;
        }
      }
    } else {
      cx<T> ce, co, cj, cs;
      if (dens_kind) {
        // graded medium: sigma(x) = 1 + (sigma1 - 1) rho(x)
        const T rho = (T)dens[g];
        const cx<T> sig = mk<T>((T)1 + (s1.x - (T)1) * rho, s1.y * rho);
        const cx<T> one = mk<T>(1, 0);
        if (kind == K_MS) {
          ce = one;
          co = one - cdiv(sig, s0);
          cj = sig;
          cs = mk<T>(0, 0);
        } else {
          const cx<T> inv = cdiv(one, sig + s0);
          co = (sig - s0) * inv;
          if (kind == K_EM) {
            ce = inv;
            cj = sig;
            cs = mk<T>(0, 0);
          } else {  // K_ADJ
            ce = one;
            cj = mk<T>(0, 0);
            cs = sig * inv;
          }
        }
      } else {
        const bool ph = PF ? phv : phase[g] != 0;
        ce = ph ? cE[1] : cE[0];
        co = ph ? cO[1] : cO[0];
        cj = ph ? cJ[1] : cJ[0];
        cs = ph ? cS[1] : cS[0];
      }
      E = ce * x;
      J = cj * E;
      out = co * x + e0c * cs;
    }
    acc.Jr += (double)J.x;
    acc.Ji += (double)J.y;
    acc.e2 += (double)norm2(E);
    acc.eJ += (double)(E.x * J.x + E.y * J.y);
    if (iter >= 1) acc.d2 += (double)norm2(E - (PF ? epo : Ep[g]));
    Ep[g] = E;
    return out;
  }
};

// ------------------------------------------------------------------ x pass
template <typename T, int NT, int EMAX>
__global__ __launch_bounds__(NT) void xpass_kernel(XArgs a) {
  const int solve = blockIdx.z;
  const int comp = blockIdx.y;
  SolveCtl* ctl = a.ctl + solve;
  if (!a.ignore_done && ctl->done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int n0 = a.n0;
  const long long line0 = (long long)blockIdx.x * a.lines_per_block;
  const int nl = (int)min((long long)a.lines_per_block, (long long)a.nlines - line0);
  const int cnt = nl * n0;
  const long long M = a.M;
  const long long fbase = ((long long)solve * a.d + comp) * M;
  const long long base = line0 * n0;
  cx<T>* X = reinterpret_cast<cx<T>*>(a.X) + fbase;
  cx<T>* Ep = reinterpret_cast<cx<T>*>(a.Eprev) + fbase;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);

  for (int i = tid; i < cnt; i += NT) lds[i] = X[base + i];
  __syncthreads();
  fft_lines<T, NT, EMAX>(lds, nl, a.fd, n0, 1, false, tw, (T)1, tid);

  LocalMap<T> lm;
  lm.load(a, solve, comp, fbase);
  Acc acc;
  for (int i = tid; i < cnt; i += NT) lds[i] = lm.apply(lds[i], base + i, acc);
  __syncthreads();
  fft_lines<T, NT, EMAX>(lds, nl, a.fd, n0, 1, false, tw, (T)-1, tid);
  for (int i = tid; i < cnt; i += NT) X[base + i] = lds[i];

  // deterministic workgroup reduction (wave64 shuffles, then across waves)
  double v[5] = {acc.Jr, acc.Ji, acc.e2, acc.d2, acc.eJ};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double s = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    v[k] = s;
  }
  // the FFT buffer is free again once every thread has stored its outputs
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem_raw);   // [5][NT/64]
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 5; ++k) red[k * (NT / 64) + wave] = v[k];
  }
  __syncthreads();
  if (tid < 5) {
    double s = 0;
    for (int w = 0; w < NT / 64; ++w) s += red[tid * (NT / 64) + w];
    a.part[(((long long)solve * a.d + comp) * 5 + tid) * gridDim.x + blockIdx.x] = s;
  }
}

// ------------------------------------------------------- Gamma / y passes
// Symbol vector n(m) for one mode (eq. J11 on a grid); returns |n|^2.
template <typename T>
__device__ __forceinline__ T mode_symbol(const GArgs& a, const int* m, cx<T>* nv) {
  const int d = a.d;
  if (a.symbol == SYM_ROTATED) {
    T s[3], c[3];
    for (int j = 0; j < d; ++j) {
      const double* t = a.symtab[j] + 2 * m[j];
      s[j] = (T)t[0];
      c[j] = (T)t[1];
    }
    T nrm = 0;
    for (int j = 0; j < d; ++j) {
      T v = s[j];
      for (int l = 0; l < d; ++l)
        if (l != j) v *= c[l];
      nv[j] = mk<T>(v, 0);
      nrm += v * v;
    }
    if (nrm == (T)0) {
      // n = 0 at m != 0 (two or more Nyquist indices): the Nyquist-indicator
      // direction, scaled per axis (s[j] = n_j at a Nyquist index)
      for (int j = 0; j < d; ++j) {
        const T v = (c[j] == (T)0) ? s[j] : (T)0;
        nv[j] = mk<T>(v, 0);
        nrm += v * v;
      }
    }
    return nrm;
  } else if (a.symbol == SYM_SPECTRAL) {
    T v[3];
    bool nyq[3];
    bool has_nyq = false, has_other = false;
    for (int j = 0; j < d; ++j) {
      const double* t = a.symtab[j] + 2 * m[j];
      v[j] = (T)t[0];
      nyq[j] = t[1] != 0.0;
      has_nyq |= nyq[j];
      has_other |= (!nyq[j]) && (v[j] != (T)0);
    }
    T nrm = 0;
    for (int j = 0; j < d; ++j) {
      const T w = (has_nyq && has_other && nyq[j]) ? (T)0 : v[j];
      nv[j] = mk<T>(w, 0);
      nrm += w * w;
    }
    return nrm;
  } else {
    T nrm = 0;
    for (int j = 0; j < d; ++j) {
      const double* t = a.symtab[j] + 2 * m[j];
      nv[j] = mk<T>((T)t[0], (T)t[1]);
      nrm += norm2(nv[j]);
    }
    return nrm;
  }
}

// Tile of C lines (adjacent along x) of the last axis (mode 0, all d
// components, Gamma_1 fused) or of the y axis in 3D (modes 1/2, blockIdx.z =
// solve*d + comp).  LDS layout [k][line], line = comp*C + l.
template <typename T, int NT, int EMAX>
__global__ __launch_bounds__(NT) void line_pass_kernel(GArgs a) {
  const int d = a.d;
  const bool gam = (a.mode == 0);
  const int solve = gam ? blockIdx.z : blockIdx.z / d;
  const int comp0 = gam ? 0 : blockIdx.z % d;
  const int ncomp = gam ? d : 1;
  SolveCtl* ctl = a.ctl + solve;
  // done was set by an earlier kernel (or, harmlessly, by this one's
  // finalizing workgroup: a stale read only costs a wasted tile)
  if (!a.ignore_done && ctl->done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  if (a.fin && blockIdx.x == 0 && blockIdx.y == 0 && comp0 == 0) finalize_solve(a.f, solve, tid, NT);
  const int C = a.C;
  const int N = a.fd.n;
  const int x0 = blockIdx.x * C;
  const int nlc = min(C, a.n[0] - x0);
  const long long off = x0 + (long long)blockIdx.y * a.rp * (gam ? 1 : a.n[1]);
  // gam: 2D off = x0 (blockIdx.y = 0); 3D off = x0 + y*n0.  y pass: off = x0 + z*n0*n1.
  const long long M = a.M;
  cx<T>* X = reinterpret_cast<cx<T>*>(a.X) + ((long long)solve * d + comp0) * M;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  const int W = ncomp * C;
  const int tot = N * W;
  for (int i = tid; i < tot; i += NT) {
    const int k = i / W;
    const int r = i - k * W;
    const int c = r / C;
    const int l = r - c * C;
    cx<T> v = mk<T>(0, 0);
    if (l < nlc) v = X[c * M + off + (long long)k * a.stride + l];
    lds[i] = v;
  }
  __syncthreads();
  if (a.mode != 2) fft_lines<T, NT, EMAX>(lds, W, a.fd, 1, W, true, tw, (T)-1, tid);
  if (gam) {
    const SolveCoef& cf = a.coef[solve];
    const T ga = (T)cf.ga, gb = (T)cf.gb, keep = (T)cf.kz_keep;
    const int yidx = blockIdx.y;
    for (int i = tid; i < N * C; i += NT) {
      const int k = i / C;
      const int l = i - k * C;
      int m[3];
      m[0] = x0 + l;
      if (d == 2) {
        m[1] = k;
      } else {
        m[1] = yidx;
        m[2] = k;
      }
      if (m[0] >= a.n[0]) continue;
      cx<T> xv[3];
      for (int c = 0; c < d; ++c) xv[c] = lds[k * W + c * C + l];
      const bool zero = (m[0] == 0) && (m[1] == 0) && (d == 2 || m[2] == 0);
      if (zero) {
        for (int c = 0; c < d; ++c) lds[k * W + c * C + l] = keep * xv[c] + ld2<T>(cf.kz_src[c]);
      } else {
        cx<T> nv[3];
        const T nrm = mode_symbol<T>(a, m, nv);
        cx<T> dot = mk<T>(0, 0);
        if (a.symbol == SYM_NETWORK) {
          for (int c = 0; c < d; ++c) dot = dot + conj(nv[c]) * xv[c];
        } else {
          for (int c = 0; c < d; ++c) dot = dot + nv[c] * xv[c];
        }
        const T inv = (T)1 / nrm;
        for (int c = 0; c < d; ++c) {
          const cx<T> gv = inv * (nv[c] * dot);
          lds[k * W + c * C + l] = ga * xv[c] + gb * gv;
        }
      }
    }
    __syncthreads();
  }
  if (a.mode != 1) fft_lines<T, NT, EMAX>(lds, W, a.fd, 1, W, true, tw, (T)1, tid);
  for (int i = tid; i < tot; i += NT) {
    const int k = i / W;
    const int r = i - k * W;
    const int c = r / C;
    const int l = r - c * C;
    if (l < nlc) X[c * M + off + (long long)k * a.stride + l] = lds[i];
  }
}

// ---------------------------------------------------------------- finalize

// Stop rules (converged / diverged / stagnated / max_iter) from the sums.
__device__ __forceinline__ void finalize_status(const FArgs& a, SolveCtl* ctl, const double* tot) {
  const int d = ctl->d;
  const int solve = (int)(ctl - a.ctl);
  const int n = ctl->iter;
  double sr = 0, si = 0;
  for (int c = 0; c < d; ++c) {
    const double jr = tot[2 * c] * a.invM, ji = tot[2 * c + 1] * a.invM;
    ctl->meanJ[2 * c] = jr;
    ctl->meanJ[2 * c + 1] = ji;
    sr += jr * ctl->e0[c];
    si += ji * ctl->e0[c];
  }
  sr *= ctl->inv_e0n2;
  si *= ctl->inv_e0n2;
  const double e2 = tot[6], d2 = tot[7], eJ = tot[8];
  const double lam = eJ / e2;
  double r = __builtin_nan("");
  if (n >= 1) r = (e2 > 0) ? sqrt(d2 / e2) : __builtin_inf();
  if (n < a.hist_cap) {
    a.hist_r[(long long)solve * a.hist_cap + n] = r;
    a.hist_s[((long long)solve * a.hist_cap + n) * 2] = (ctl->kind == K_POWER) ? lam : sr;
    a.hist_s[((long long)solve * a.hist_cap + n) * 2 + 1] = (ctl->kind == K_POWER) ? 0.0 : si;
  }
  ctl->res = r;
  ctl->sstar_re = sr;
  ctl->sstar_im = si;
  ctl->lam = lam;
  if (a.ignore_done) {
    ctl->iter = n + 1;
    return;
  }
  bool stop = false;
  int status = -3;
  if (n >= 1) {
    const bool finite = isfinite(r) && isfinite(sr) && isfinite(si);
    if (!finite) {
      stop = true;
      status = -4;
    } else if (r <= ctl->tol) {
      stop = true;
      status = 0;
    } else if (ctl->div_factor > 0 && r > ctl->div_factor * ctl->min_r) {
      stop = true;
      status = -4;
    } else {
      if (r < ctl->min_r) {
        ctl->min_r = r;
        ctl->since_min = 0;
      } else {
        ctl->since_min += 1;
      }
      if (ctl->stag_window > 0 && ctl->since_min >= ctl->stag_window) {
        stop = true;
        status = -5;
      }
    }
  }
  if (!stop && n >= ctl->max_iter) {
    stop = true;
    status = -3;
  }
  if (stop) {
    ctl->status = status;
    ctl->done = 1;
  } else {
    ctl->iter = n + 1;
  }
}

// Reduction of the x-pass partials and the stop rules for one solve, run by
// one workgroup (all its threads call it).  The partials come from the
// previous kernel; the control block is read by the next x pass.  The sums
// run in a fixed order, so sigma* and the residual are bit-reproducible.
__device__ __forceinline__ void finalize_solve(const FArgs& a, int solve, int tid, int nth) {
  SolveCtl* ctl = a.ctl + solve;
  const int d = ctl->d;
  __shared__ double fred[9][16];
  __shared__ double tot[9];
  // workgroups that are not whole waves (tiny grids) sum on one thread
  const int nt = (nth >= 64 && nth % 64 == 0) ? nth : 1;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (tid < nt) {
    // partials are [solve][component][quantity][block]: every quantity is one
    // contiguous run, read coalesced, with 4 blocks x 5 quantities in flight
    for (int c = 0; c < d; ++c) {
      const double* p = a.part + ((long long)solve * d + c) * 5 * a.nblocks;
      constexpr int U = 4;
      for (int b0 = tid; b0 < a.nblocks; b0 += U * nt) {
        double v[U][5];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            const int b = b0 + u * nt;
            v[u][q] = b < a.nblocks ? p[(long long)q * a.nblocks + b] : 0.0;
          }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          acc[2 * c] += v[u][0];
          acc[2 * c + 1] += v[u][1];
          acc[6] += v[u][2];
          acc[7] += v[u][3];
          acc[8] += v[u][4];
        }
      }
    }
  }
  if (nt == 1) {
    if (tid == 0)
      for (int q = 0; q < 9; ++q) tot[q] = acc[q];
  } else {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      double v = acc[q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((tid & 63) == 0) fred[q][tid >> 6] = v;
    }
    __syncthreads();
    if (tid < 9) {
      double v = 0;
      for (int w = 0; w < nt / 64; ++w) v += fred[tid][w];
      tot[tid] = v;
    }
  }
  __syncthreads();
  if (tid == 0) finalize_status(a, ctl, tot);
  __syncthreads();
}

// -------------------------------------------------------------------- init
struct InitArgs {
  void* X;
  void* Sslot;
  void* Tslot;
  SolveCtl* ctl;
  const SolveCoef* coef;
  long long M;
  int d, n0, nsolve;
  int has_st;
  double src_scale;   // N^d
};

// X^0 is the constant source field c (e0, 2 sigma0 e0 or 0): its stored form
// is N^d c at kx = 0 of every x-line and 0 elsewhere.
template <typename T>
__global__ void init_kernel(InitArgs a) {
  const long long tot = (long long)a.nsolve * a.d * a.M;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x) {
    const long long f = i / a.M;
    const long long g = i - f * a.M;
    const int c = (int)(f % a.d);
    const int s = (int)(f / a.d);
    cx<T> v = mk<T>(0, 0);
    if (g % a.n0 == 0) {
      const SolveCoef& cf = a.coef[s];
      v = mk<T>((T)cf.init_src[c][0], (T)cf.init_src[c][1]);
    }
    reinterpret_cast<cx<T>*>(a.X)[i] = v;
    if (a.has_st) {
      reinterpret_cast<cx<T>*>(a.Sslot)[i] = mk<T>(0, 0);
      reinterpret_cast<cx<T>*>(a.Tslot)[i] = mk<T>(0, 0);
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

// ----------------------------------------------------------------- outputs
struct ExtractArgs {
  const void* Eprev;
  const uint8_t* phase;
  const double* density;
  const SolveCoef* coef;
  double* E;   // [d][M] complex double or null
  double* J;
  long long M;
  int d, solve;
};

template <typename T>
__global__ void extract_kernel(ExtractArgs a) {
  const long long tot = (long long)a.d * a.M;
  const SolveCoef& cf = a.coef[a.solve];
  const cx<T>* src = reinterpret_cast<const cx<T>*>(a.Eprev) + (long long)a.solve * a.d * a.M;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x) {
    const long long g = i % a.M;
    const cx<T> e = src[i];
    const double er = (double)e.x, ei = (double)e.y;
    if (a.E) {
      a.E[2 * i] = er;
      a.E[2 * i + 1] = ei;
    }
    if (a.J) {
      double sr, si;
      if (cf.density) {
        const double rho = a.density[g];
        sr = 1.0 + (cf.s1[0] - 1.0) * rho;
        si = cf.s1[1] * rho;
      } else if (a.phase[g]) {
        sr = cf.s1[0];
        si = cf.s1[1];
      } else {
        sr = 1.0;
        si = 0.0;
      }
      a.J[2 * i] = sr * er - si * ei;
      a.J[2 * i + 1] = sr * ei + si * er;
    }
  }
}

// ---------------------------------------------------------------- gradient
struct GradArgs {
  const double* E;       // forward field [d][M] complex double
  const void* Y;         // adjoint y = W m, [d][M] complex T (solve 0)
  const uint8_t* phase;
  const double* density;
  double* g;             // [M] complex or null
  double* drho;          // [M] complex or null
  double* part;          // [blocks][2]
  double s1[2], s0[2];
  double e0[3];
  double scale;          // 1/(N^d |e0|^2)
  long long M;
  int d;
};

template <typename T, bool REAL>
__global__ __launch_bounds__(256) void gradient_kernel(GradArgs a) {
  __shared__ double red[2][4];
  const cx<T>* Y = reinterpret_cast<const cx<T>*>(a.Y);
  const T* Yr = reinterpret_cast<const T*>(a.Y);
  double accr = 0, acci = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.M;
       i += (long long)gridDim.x * blockDim.x) {
    const double rho = a.density ? a.density[i] : (double)(a.phase[i] ? 1 : 0);
    const double sr = 1.0 + (a.s1[0] - 1.0) * rho, si = a.s1[1] * rho;
    const double ar = sr + a.s0[0], ai = si + a.s0[1];   // sigma + sigma0
    double ypr = 0, ypi = 0, per = 0, pei = 0;
    for (int c = 0; c < a.d; ++c) {
      const double er = a.E[2 * (c * a.M + i)], ei = a.E[2 * (c * a.M + i) + 1];
      const double pr = ar * er - ai * ei, pi = ar * ei + ai * er;    // P = (sigma+sigma0) E
      const cx<T> y = REAL ? mk<T>(Yr[c * a.M + i], (T)0) : Y[c * a.M + i];
      ypr += (double)y.x * pr - (double)y.y * pi;
      ypi += (double)y.x * pi + (double)y.y * pr;
      per += pr * a.e0[c];
      pei += pi * a.e0[c];
    }
    const double br = ypr + 0.5 * per, bi = ypi + 0.5 * pei;
    // 2 sigma0/(sigma+sigma0)^2
    const double a2r = ar * ar - ai * ai, a2i = 2 * ar * ai;
    const double den = a2r * a2r + a2i * a2i;
    const double fr = 2.0 * (a.s0[0] * a2r + a.s0[1] * a2i) / den;
    const double fi = 2.0 * (a.s0[1] * a2r - a.s0[0] * a2i) / den;
    const double gr = (fr * br - fi * bi) * a.scale, gi = (fr * bi + fi * br) * a.scale;
    if (a.g) {
      a.g[2 * i] = gr;
      a.g[2 * i + 1] = gi;
    }
    if (a.drho) {
      const double dr = a.s1[0] - 1.0, di = a.s1[1];
      a.drho[2 * i] = dr * gr - di * gi;
      a.drho[2 * i + 1] = dr * gi + di * gr;
    }
    accr += gr * rho;
    acci += gi * rho;
  }
  for (int off = 32; off > 0; off >>= 1) {
    accr += __shfl_down(accr, off, 64);
    acci += __shfl_down(acci, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = accr;
    red[1][wave] = acci;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0;
    for (int w = 0; w < 4; ++w) s += red[threadIdx.x][w];
    a.part[2 * blockIdx.x + threadIdx.x] = s;
  }
}

static __global__ void sum_pairs_kernel(const double* part, int n, double* out) {
  __shared__ double red[2][256];
  double s0 = 0, s1 = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    s0 += part[2 * i];
    s1 += part[2 * i + 1];
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

// ------------------------------------------------------------ setup tables
// tw[k] = exp(-2 pi i k / n), computed in fp64 and rounded once.
template <typename T>
__global__ void twiddle_kernel(cx<T>* tw, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)n, &s, &c);
  tw[k] = mk<T>((T)c, (T)-s);
}

// Per-axis symbol tables (double pairs).  The cell is the unit square
// (cube): a voxel is 1/n wide along an axis of n voxels, so the difference
// quotients carry the factor n.
//   rotated : (n sin(pi m/n), cos(pi m/n)) with the exact zeros at m = 0 / 2m = n
//   spectral: (signed m in (-n/2, n/2], 1 if 2m = n else 0)
//   network : (n (cos(2 pi m/n) - 1), n sin(2 pi m/n))
static __global__ void symbol_table_kernel(double* tab, int n, int symbol) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double a, b;
  if (symbol == SYM_ROTATED) {
    sincospi((double)m / (double)n, &a, &b);
    if (m == 0) a = 0.0;
    if (2 * m == n) b = 0.0;
    a *= (double)n;
  } else if (symbol == SYM_SPECTRAL) {
    a = (2 * m > n) ? (double)(m - n) : (double)m;
    b = (2 * m == n) ? 1.0 : 0.0;
  } else {
    double s, c;
    sincospi(2.0 * (double)m / (double)n, &s, &c);
    a = (double)n * (c - 1.0);
    b = (double)n * s;
  }
  tab[2 * m] = a;
  tab[2 * m + 1] = b;
}

}  // namespace scfft
