// Seed-system COCG step and per-shift scalar recurrences (Appendix D,
// Algorithm 1, in the reading: bilinear products r^T r (Appendix A,
// r~ = r*), zeta recurrence with (1 - alpha_m w) and beta_{m-1}).
//
// One iteration m of the seed runs as these launches on `nsys` systems:
//   k_cocg_p: p_m = r_m + beta_{m-1} p_{m-1}  (beta_{-1} = 0 gives p_0 = r_0)
//   apply   : v = A_s p,  sigma = r_m^T v, |v|^2           (k_apply.hip)
//   k_cocg_r: alpha_m = rho_m / sigma,  r_{m+1} = r_m - alpha_m v  (new bank
//             slot), partial rho_{m+1} = r^T r and |r_{m+1}|^2;
//   k_cocg_book (one workgroup per system): beta_m = rho_{m+1}/rho_m, every
//             shift's zeta, freeze of converged shifts
//             (|r_{m+1}|/|zeta_{m+1}| <= tol |E|) and the next status.
// The x / p vectors of the shifted systems are not touched here: the
// residuals r_m stay in the bank and the shifted solutions are assembled
// from them in k_shift.hip.
// Recurred form (not with the dual form, whose shadow vectors need p~):
// k_cocg_p is skipped.  The apply (kModeSelf) reads r_m in place from its
// bank slot and writes
//   v_m = A r_m + beta_{m-1} v_{m-1} = A (r_m + beta_{m-1} p_{m-1}) = A p_m
// over v_{m-1}, with sigma = r_m^T v_m as before; k_cocg_r and the
// bookkeeping are unchanged.  Where residual replacement needs the seed
// solution, x_m and p_{m-1} are rebuilt from the bank slots at each
// replacement (k_seed_rebuild) instead of being updated every iteration.
// Dual-space form (non-symmetric A; CocgArgs::rt set): the shadow residual
// r~ and direction p~ follow the same recurrences with v~ = A^T p~ (a second
// apply, plain mode), sigma = r~^T A p (the apply reads r~ instead of the bank
// slot) and rho_{m+1} = r~_{m+1}^T r_{m+1}; the shift recurrences are unchanged.
#include "k_common.h"

namespace msb {

constexpr int kEptStream = 4;   // elements per thread per step of the streaming kernels
constexpr int kPerStep = kBlock * kEptStream;

int cocg_nbx(int64_t D, int nsys) { return stream_nbx(D, nsys, kPerStep); }

// Element offset of (system s, index i) in p and v: one vector per system, or
// groups of il systems interleaved ([nsys / il][D][il]).  With il the grid is
// (system, block) so that the systems of a group stream the same lines together.
__device__ __forceinline__ int64_t pv_index(int il, int64_t D, int s, int64_t i) {
  return il ? ((int64_t)(s / il) * D + i) * il + s % il : (int64_t)s * D + i;
}
__device__ __forceinline__ int grid_sys(int il) { return il ? blockIdx.x : blockIdx.y; }
__device__ __forceinline__ int grid_blk(int il) { return il ? blockIdx.y : blockIdx.x; }

__device__ __forceinline__ bool sigma_breakdown(const SysState& st, const double* red1, int s,
                                                cv<double>& alpha) {
  const cv<double> sigma = {red1[s * 4 + 0], red1[s * 4 + 1]};
  const double vnorm = sqrt(red1[s * 4 + 2]);
  const double sabs = cabs(sigma);
  if (!(sabs > 1e-14 * st.rtnorm * vnorm)) return true;   // also catches NaN (r~ = r unless dual)
  alpha = cdiv({st.rho_re, st.rho_im}, sigma);
  return false;
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_cocg_init(InitArgs a) {
  using Ax = Access<S, true>;
  using A64 = Access<double, true>;
  const int s = grid_sys(a.il), bx = grid_blk(a.il);
  double part[3] = {0.0, 0.0, 0.0};
  void* r0 = Ax::offset(a.bank, (int64_t)s * a.cap * a.D);
  for (int64_t base = (int64_t)bx * kPerStep; base < a.D; base += (int64_t)a.nbx * kPerStep) {
#pragma unroll
    for (int e = 0; e < kEptStream; ++e) {
      const int64_t i = base + e * kBlock + threadIdx.x;
      if (i < a.D) {
        const cv<double> x = A64::template load<double>(a.E, (int64_t)s * a.D + i);
        const cv<double> xs = {(double)(S)x.re, (double)(S)x.im};
        Ax::store(r0, i, xs);
        Ax::store(a.pvec, pv_index(a.il, a.D, s, i), xs);
        if (a.rt) {                     // dual-space form: r~_0 = p~_0 = E
          Ax::store(Ax::offset(a.rt, (int64_t)s * a.D), i, xs);
          Ax::store(Ax::offset(a.pt, (int64_t)s * a.D), i, xs);
        }
        if (a.xseed) A64::store(a.xseed, (int64_t)s * a.D + i, cv<double>{0.0, 0.0});
        if (a.psnap) Ax::store(Ax::offset(a.psnap, (int64_t)s * a.D), i, xs);
        part[0] += xs.re * xs.re - xs.im * xs.im;
        part[1] += 2.0 * xs.re * xs.im;
        part[2] += xs.re * xs.re + xs.im * xs.im;
      }
    }
  }
  block_partial<3>(part, a.partials, a.nbx, s, bx);
}

// One workgroup per system: rho_0 = E^T E, |E|, initial state and shift scalars.
__global__ __launch_bounds__(kBlock) void k_cocg_init_fin(InitArgs a) {
  const int s = blockIdx.x;
  __shared__ double red[4];
  reduce_partials<3>(a.partials, a.nbx, s, red);
  if (threadIdx.x == 0) {
    SysState st;
    st.rho_re = red[0];
    st.rho_im = red[1];
    st.rnorm = sqrt(red[2]);
    st.rtnorm = st.rnorm;
    st.normE = st.rnorm;
    st.ap_re = 1.0; st.ap_im = 0.0;     // alpha_{-1} = 1
    st.bp_re = 0.0; st.bp_im = 0.0;     // beta_{-1} = 0
    st.al_re = st.al_im = st.be_re = st.be_im = 0.0;
    st.m = 0;
    st.rbest = st.normE;
    st.n_stall = 0;
    st.pad = 0;
    st.n_active = a.n_shift;
    st.breakdown_iter = -1;
    if (st.normE == 0.0) {
      st.status = kDone;                // E = 0: Psi = 0 for every shift
      st.n_active = 0;
    } else if (!(cabs({st.rho_re, st.rho_im}) > 1e-14 * st.normE * st.normE)) {
      st.status = kBreakdown;           // E^T E = 0: COCG cannot start
      st.breakdown_iter = 0;
    } else if (a.maxit <= 0) {
      st.status = kMaxit;
    } else {
      st.status = kActive;
    }
    a.st[s] = st;
    a.rnorm_log[(int64_t)s * (a.maxit + 1)] = st.rnorm;
  }
  const bool zero = (red[2] == 0.0);
  for (int k = threadIdx.x; k < a.n_shift; k += kBlock) {
    const int64_t t = (int64_t)s * a.n_shift + k;
    a.zeta[2 * t] = 1.0; a.zeta[2 * t + 1] = 0.0;
    a.zeta_prev[2 * t] = 1.0; a.zeta_prev[2 * t + 1] = 0.0;
    a.conv_iter[t] = zero ? 0 : -1;
  }
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_cocg_r(CocgArgs a) {
  using Ax = Access<S, true>;
  const int s = grid_sys(a.il), bx = grid_blk(a.il);
  // rho_{m+1} (bilinear: r~^T r, or r^T r), |r_{m+1}|^2, |r~_{m+1}|^2
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  const SysState st = a.st[s];
  if (st.status == kActive) {
    cv<double> alpha;
    if (!sigma_breakdown(st, a.red1, s, alpha)) {
      const int slot = st.m - *a.base;
      void* rt = a.rt ? Ax::offset(a.rt, (int64_t)s * a.D) : nullptr;
      const void* vt = a.rt ? Ax::offset(a.vt, (int64_t)s * a.D) : nullptr;
      const void* r = Ax::offset((const void*)a.bank, ((int64_t)s * a.cap + slot) * a.D);
      void* rn = Ax::offset(a.bank, ((int64_t)s * a.cap + slot + 1) * a.D);
      for (int64_t base = (int64_t)bx * kPerStep; base < a.D; base += (int64_t)a.nbx * kPerStep) {
#pragma unroll
        for (int e = 0; e < kEptStream; ++e) {
          const int64_t i = base + e * kBlock + threadIdx.x;
          if (i < a.D) {
            const cv<double> ri = Ax::template load<double>(r, i);
            const cv<double> vi = Ax::template load<double>(a.vvec, pv_index(a.il, a.D, s, i));
            if (a.xseed) {          // seed solution for residual replacement: x += alpha p
              using A64 = Access<double, true>;
              const cv<double> pi = Ax::template load<double>(a.pvec, pv_index(a.il, a.D, s, i));
              cv<double> xs = A64::template load<double>(a.xseed, (int64_t)s * a.D + i);
              xs = cadd(xs, cmul(alpha, pi));
              A64::store(a.xseed, (int64_t)s * a.D + i, xs);
            }
            cv<double> x = {ri.re - (alpha.re * vi.re - alpha.im * vi.im),
                            ri.im - (alpha.re * vi.im + alpha.im * vi.re)};
            x.re = (double)(S)x.re;
            x.im = (double)(S)x.im;
            Ax::store(rn, i, x);
            cv<double> xt = x;
            if (rt) {               // dual-space form: r~ <- r~ - alpha A^T p~
              const cv<double> rti = Ax::template load<double>(rt, i);
              const cv<double> vti = Ax::template load<double>(vt, i);
              xt = {rti.re - (alpha.re * vti.re - alpha.im * vti.im),
                    rti.im - (alpha.re * vti.im + alpha.im * vti.re)};
              xt.re = (double)(S)xt.re;
              xt.im = (double)(S)xt.im;
              Ax::store(rt, i, xt);
            }
            part[0] += xt.re * x.re - xt.im * x.im;
            part[1] += xt.re * x.im + xt.im * x.re;
            part[2] += x.re * x.re + x.im * x.im;
            part[3] += xt.re * xt.re + xt.im * xt.im;
          }
        }
      }
    }
  }
  block_partial<4>(part, a.partials, a.nbx, s, bx);
}

// One workgroup per system: rho_{m+1}, |r_{m+1}|, beta_m, every shift's zeta,
// the freeze test and the status for the next iteration.
__global__ __launch_bounds__(kBlock) void k_cocg_book(CocgArgs a) {
  const int s = blockIdx.x;
  __shared__ double red2[4];
  reduce_partials<4>(a.partials, a.nbx, s, red2);
  SysState t = a.st[s];
  if (t.status != kActive) return;
  cv<double> alpha;
  if (sigma_breakdown(t, a.red1, s, alpha)) {
    if (threadIdx.x == 0) {
      a.st[s].status = kBreakdown;
      a.st[s].breakdown_iter = t.m;
    }
    return;
  }
  const int base = *a.base;
  const cv<double> rho_new = {red2[0], red2[1]};
  const double rn = sqrt(red2[2]);
  const double rtn = a.rt ? sqrt(red2[3]) : rn;
  const cv<double> beta = cdiv(rho_new, {t.rho_re, t.rho_im});
  // zeta_{m+1} = (1 - alpha_m w) zeta_m + (alpha_m beta_{m-1} / alpha_{m-1}) (zeta_m - zeta_{m-1})
  const cv<double> cshift = cdiv(cmul(alpha, {t.bp_re, t.bp_im}), {t.ap_re, t.ap_im});
  const double thresh = a.tol * t.normE;
  int active = 0;
  for (int k = threadIdx.x; k < a.n_shift; k += kBlock) {
    const int64_t idx = (int64_t)s * a.n_shift + k;
    if (a.conv_iter[idx] >= 0) continue;
    const double w = a.wshift[k];
    const cv<double> z = {a.zeta[2 * idx], a.zeta[2 * idx + 1]};
    const cv<double> zp = {a.zeta_prev[2 * idx], a.zeta_prev[2 * idx + 1]};
    const cv<double> f = {1.0 - alpha.re * w, -alpha.im * w};
    const cv<double> zn = cadd(cmul(f, z), cmul(cshift, csub(z, zp)));
    a.zeta_prev[2 * idx] = z.re;
    a.zeta_prev[2 * idx + 1] = z.im;
    a.zeta[2 * idx] = zn.re;
    a.zeta[2 * idx + 1] = zn.im;
    if (rn / cabs(zn) <= thresh) {
      a.conv_iter[idx] = t.m + 1;
    } else {
      ++active;
    }
  }
  double cnt[1] = {(double)active};
  __shared__ double shc[1][kBlock / kWave];
  block_sum<1>(cnt, shc);
  if (threadIdx.x == 0) {
    const int m = t.m;
    a.alpha_log[((int64_t)s * a.maxit + m) * 2] = alpha.re;
    a.alpha_log[((int64_t)s * a.maxit + m) * 2 + 1] = alpha.im;
    a.beta_log[((int64_t)s * a.maxit + m) * 2] = beta.re;
    a.beta_log[((int64_t)s * a.maxit + m) * 2 + 1] = beta.im;
    a.rnorm_log[(int64_t)s * (a.maxit + 1) + m + 1] = rn;
    t.n_active = (int)cnt[0];
    t.al_re = alpha.re; t.al_im = alpha.im;
    t.be_re = beta.re; t.be_im = beta.im;
    t.ap_re = alpha.re; t.ap_im = alpha.im;
    t.bp_re = beta.re; t.bp_im = beta.im;
    t.rho_re = rho_new.re; t.rho_im = rho_new.im;
    t.rnorm = rn;
    t.rtnorm = rtn;
    t.m = m + 1;
    if (t.n_active == 0) {
      t.status = kDone;
    } else if (!(rn > kSeedFloor * t.normE) || !isfinite(beta.re) || !isfinite(beta.im)) {
      t.status = kExhausted;
    } else if (!(cabs(rho_new) > 1e-14 * rn * rtn)) {
      t.status = kBreakdown;            // rho_{m+1} = 0 with shifts still open
      t.breakdown_iter = m + 1;
    } else if (t.m >= a.maxit) {
      t.status = kMaxit;
    } else if (t.m + 1 - base >= a.cap) {
      t.status = kPaused;               // no bank slot for r_{m+1} of the next iteration
    }
    a.st[s] = t;
  }
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_cocg_p(CocgArgs a) {
  using Ax = Access<S, true>;
  const int s = grid_sys(a.il), bx = grid_blk(a.il);
  const SysState st = a.st[s];
  if (st.status != kActive) return;
  const int slot = st.m - *a.base;
  const void* r = Ax::offset((const void*)a.bank, ((int64_t)s * a.cap + slot) * a.D);
  const cv<double> beta = {st.be_re, st.be_im};
  const void* rt = a.rt ? Ax::offset((const void*)a.rt, (int64_t)s * a.D) : nullptr;
  void* pt = a.rt ? Ax::offset(a.pt, (int64_t)s * a.D) : nullptr;
  for (int64_t base = (int64_t)bx * kPerStep; base < a.D; base += (int64_t)a.nbx * kPerStep) {
#pragma unroll
    for (int e = 0; e < kEptStream; ++e) {
      const int64_t i = base + e * kBlock + threadIdx.x;
      if (i < a.D) {
        const int64_t pi_ = pv_index(a.il, a.D, s, i);
        const cv<double> ri = Ax::template load<double>(r, i);
        const cv<double> pi = Ax::template load<double>(a.pvec, pi_);
        const cv<double> x = {ri.re + beta.re * pi.re - beta.im * pi.im,
                              ri.im + beta.re * pi.im + beta.im * pi.re};
        Ax::store(a.pvec, pi_, x);
        if (pt) {                       // p~ = r~ + beta p~
          const cv<double> rti = Ax::template load<double>(rt, i);
          const cv<double> pti = Ax::template load<double>(pt, i);
          const cv<double> y = {rti.re + beta.re * pti.re - beta.im * pti.im,
                                rti.im + beta.re * pti.im + beta.im * pti.re};
          Ax::store(pt, i, y);
        }
      }
    }
  }
}

// Seed solution and last direction rebuilt from the bank slots at a residual
// replacement (recurred form: into p itself; direct form: into a copy of p
// kept for the next rebuild); one pass over the L slots per element.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_seed_rebuild(RebuildArgs a) {
  using Ax = Access<S, true>;
  using A64 = Access<double, true>;
  const int s = blockIdx.y, bx = blockIdx.x;
  const int status = a.st[s].status;
  if (status != kActive && status != kPaused) return;
  extern __shared__ double cf[];                          // [2][L + 1] complex
  const double* src = a.coef + (int64_t)s * 2 * (a.L + 1) * 2;
  for (int k = threadIdx.x; k < 4 * (a.L + 1); k += kBlock) cf[k] = src[k];
  __syncthreads();
  const double* cx = cf;
  const double* cp = cf + 2 * (a.L + 1);
  const void* b0 = Ax::offset(a.bank, ((int64_t)s * a.cap + a.slot0) * a.D);
  void* p = Ax::offset(a.p, (int64_t)s * a.D);
  for (int64_t i = (int64_t)bx * kBlock + threadIdx.x; i < a.D; i += (int64_t)a.nbx * kBlock) {
    cv<double> ax = {0.0, 0.0}, ap = {0.0, 0.0};
    for (int l = 0; l < a.L; ++l) {
      const cv<double> r = Ax::template load<double>(b0, (int64_t)l * a.D + i);
      ax = cadd(ax, cmul({cx[2 * l], cx[2 * l + 1]}, r));
      ap = cadd(ap, cmul({cp[2 * l], cp[2 * l + 1]}, r));
    }
    const cv<double> po = Ax::template load<double>(p, i);
    const cv<double> xo = A64::template load<double>(a.x, (int64_t)s * a.D + i);
    const cv<double> xn = cadd(cadd(xo, ax), cmul({cx[2 * a.L], cx[2 * a.L + 1]}, po));
    cv<double> pn = cadd(ap, cmul({cp[2 * a.L], cp[2 * a.L + 1]}, po));
    pn.re = (double)(S)pn.re;
    pn.im = (double)(S)pn.im;
    A64::store(a.x, (int64_t)s * a.D + i, xn);
    Ax::store(p, i, pn);
  }
}

// A system's residual is replaced while it is iterating and its recurrence
// residual is above rep_floor |E|.  Below that the seed is as accurate as the
// FP64 product can show (or already at tol), and the shifted systems, whose
// residuals are r_m / zeta_m, need the recurrence to go on unperturbed.
__device__ __forceinline__ bool wants_replace(const SysState& t, const CocgArgs& a) {
  return t.status == kActive && t.m > 0 && t.rnorm > a.rep_floor * t.normE;
}

// r_m <- E - w for the systems that want it (w = A_s x_m in complex128); partial rho, |r|^2
template <typename S>
__global__ __launch_bounds__(kBlock) void k_cocg_replace(CocgArgs a, const double* E, const double* w) {
  using Ax = Access<S, true>;
  using A64 = Access<double, true>;
  const int s = blockIdx.y, bx = blockIdx.x;
  double part[3] = {0.0, 0.0, 0.0};
  const SysState st = a.st[s];
  if (wants_replace(st, a)) {
    void* r = Ax::offset(a.bank, ((int64_t)s * a.cap + (st.m - *a.base)) * a.D);
    for (int64_t base = (int64_t)bx * kPerStep; base < a.D; base += (int64_t)a.nbx * kPerStep) {
#pragma unroll
      for (int e = 0; e < kEptStream; ++e) {
        const int64_t i = base + e * kBlock + threadIdx.x;
        if (i < a.D) {
          const cv<double> ei = A64::template load<double>(E, (int64_t)s * a.D + i);
          const cv<double> wi = A64::template load<double>(w, (int64_t)s * a.D + i);
          cv<double> x = csub(ei, wi);
          x.re = (double)(S)x.re;
          x.im = (double)(S)x.im;
          Ax::store(r, i, x);
          part[0] += x.re * x.re - x.im * x.im;
          part[1] += 2.0 * x.re * x.im;
          part[2] += x.re * x.re + x.im * x.im;
        }
      }
    }
  }
  block_partial<3>(part, a.partials, a.nbx, s, bx);
}

__global__ __launch_bounds__(kBlock) void k_cocg_replace_fin(CocgArgs a) {
  const int s = blockIdx.x;
  __shared__ double red[4];
  reduce_partials<3>(a.partials, a.nbx, s, red);
  if (threadIdx.x != 0) return;
  SysState t = a.st[s];
  if (!wants_replace(t, a)) return;
  const cv<double> rho_new = {red[0], red[1]};
  const double rn = sqrt(red[2]);
  const double rn_rec = t.rnorm;    // recurrence residual before the replacement
  // beta_{m-1} = rho_m / rho_{m-1}: rescale by rho_m(new) / rho_m(old)
  const cv<double> ratio = cdiv(rho_new, {t.rho_re, t.rho_im});
  const cv<double> beta = cmul({t.be_re, t.be_im}, ratio);
  t.be_re = t.bp_re = beta.re;
  t.be_im = t.bp_im = beta.im;
  a.beta_log[((int64_t)s * a.maxit + t.m - 1) * 2] = beta.re;
  a.beta_log[((int64_t)s * a.maxit + t.m - 1) * 2 + 1] = beta.im;
  t.rho_re = rho_new.re;
  t.rho_im = rho_new.im;
  t.rnorm = rn;
  t.rtnorm = rn;                      // replacement runs in the complex-symmetric form only
  a.rnorm_log[(int64_t)s * (a.maxit + 1) + t.m] = rn;
  if (!(cabs(rho_new) > 1e-14 * rn * rn)) {
    t.status = kBreakdown;
    t.breakdown_iter = t.m;
  } else if (rn > kFloorGap * rn_rec) {
    t.status = kFloor;                // the recurrence went below what its precision can attain
  } else if (rn < kStall * t.rbest) {
    t.rbest = rn;                     // real progress
    t.n_stall = 0;
  } else if (rn_rec < kStall * t.rbest) {
    if (++t.n_stall >= kStallMax) t.status = kFloor;   // claimed progress that the truth does not show
  }
  a.st[s] = t;
}

hipError_t launch_cocg_init(Elem e, const InitArgs& a, hipStream_t st) {
  const dim3 grid = a.il ? dim3(a.nsys, a.nbx) : dim3(a.nbx, a.nsys);
  if (e == Elem::C128) hipLaunchKernelGGL(k_cocg_init<double>, grid, dim3(kBlock), 0, st, a);
  else if (e == Elem::C64) hipLaunchKernelGGL(k_cocg_init<float>, grid, dim3(kBlock), 0, st, a);
  else return hipErrorInvalidValue;
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_cocg_init_fin, dim3(a.nsys), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_cocg_r(Elem e, const CocgArgs& a, hipStream_t st) {
  const dim3 grid = a.il ? dim3(a.nsys, a.nbx) : dim3(a.nbx, a.nsys);
  if (e == Elem::C128) hipLaunchKernelGGL(k_cocg_r<double>, grid, dim3(kBlock), 0, st, a);
  else if (e == Elem::C64) hipLaunchKernelGGL(k_cocg_r<float>, grid, dim3(kBlock), 0, st, a);
  else return hipErrorInvalidValue;
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_cocg_book, dim3(a.nsys), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_seed_rebuild(Elem e, const RebuildArgs& a, hipStream_t st) {
  if (a.L < 0 || a.slot0 < 0 || a.slot0 + a.L > a.cap) return hipErrorInvalidValue;
  dim3 grid(a.nbx, a.nsys);
  const size_t lds = (size_t)4 * (a.L + 1) * sizeof(double);
  if (e == Elem::C128) hipLaunchKernelGGL(k_seed_rebuild<double>, grid, dim3(kBlock), lds, st, a);
  else if (e == Elem::C64) hipLaunchKernelGGL(k_seed_rebuild<float>, grid, dim3(kBlock), lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_cocg_p(Elem e, const CocgArgs& a, hipStream_t st) {
  const dim3 grid = a.il ? dim3(a.nsys, a.nbx) : dim3(a.nbx, a.nsys);
  if (e == Elem::C128) hipLaunchKernelGGL(k_cocg_p<double>, grid, dim3(kBlock), 0, st, a);
  else if (e == Elem::C64) hipLaunchKernelGGL(k_cocg_p<float>, grid, dim3(kBlock), 0, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace msb

namespace msb {
hipError_t launch_cocg_replace(Elem e, const CocgArgs& a, const double* E, const double* w,
                               hipStream_t st) {
  dim3 grid(a.nbx, a.nsys);
  if (e == Elem::C128) hipLaunchKernelGGL(k_cocg_replace<double>, grid, dim3(kBlock), 0, st, a, E, w);
  else if (e == Elem::C64) hipLaunchKernelGGL(k_cocg_replace<float>, grid, dim3(kBlock), 0, st, a, E, w);
  else return hipErrorInvalidValue;
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_cocg_replace_fin, dim3(a.nsys), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}
}  // namespace msb
