// Field solve of the fine burst: Newton iterations for the Poisson-Boltzmann
// equation -phi'' + exp(phi) = rho (eq. 3.15; Boltzmann electrons of eqs. 3.2 and
// 3.16) on the node grid, then the node field E_k = -(phi_{k+1} - phi_{k-1}) / 2h.
//
// One workgroup per replica, FP64.  Rows are scaled by the node volume so that
// the Jacobian is symmetric with constant off-diagonals alpha = -1/h^2:
//   interior rows:  (2 phi_k - phi_{k-1} - phi_{k+1}) / h^2 + exp(phi_k) - Q_k / h
//   wall rows:      (phi_0 - phi_1) / h^2 + exp(phi_0) / 2 - Q_0 / h   (and row N)
// (Q in charge units: interior nodes own h, wall nodes h/2, which is the Neumann
// condition phi' = 0).  Each Newton step J delta = -F is solved by a partition
// method: thread t owns M consecutive rows; the M-1 interior rows are eliminated
// in registers (downward and upward sweeps), leaving one tridiagonal equation per
// thread for its last row, solved by parallel cyclic reduction in LDS; then the
// interior rows follow by one Thomas pass.  Periodic grids give cyclic systems; on
// walls, node N is eliminated into row N-1 first so every system has N rows.
#include "efpi_internal.h"

namespace efpi {
namespace {

constexpr int kMaxT = 1024;

__device__ __forceinline__ double clamp2(double x) { return fmin(2.0, fmax(-2.0, x)); }

// 1/b from the hardware reciprocal estimate and two Newton-Raphson corrections
// (the error squares each time); the solver only needs full FP64 precision,
// not correct rounding.
__device__ __forceinline__ double rcp(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return fma(r, fma(-b, r, 1.0), r);
}

template <int M, int THREADS>
__global__ __launch_bounds__(THREADS) void k_newton(const RepDev* __restrict__ reps,
                                                   const int32_t* __restrict__ list, int iters,
                                                   int cold, int qsel, int save_en,
                                                   int zero_bins, double tol,
                                                   uint32_t* __restrict__ status) {
  __shared__ double s_first[kMaxT], s_last[kMaxT];
  __shared__ double s_a[kMaxT], s_b[kMaxT], s_c[kMaxT], s_d[kMaxT];
  __shared__ double s_y0[kMaxT], s_gl0[kMaxT], s_gr0[kMaxT];
  __shared__ double s_phin;
  __shared__ unsigned long long s_maxd;
  __shared__ int s_nan;

  const RepDev& R = reps[list[blockIdx.x]];
  const int n = R.n_cells;
  const int T = n / M;
  const int t = threadIdx.x;
  const bool act = t < T;
  const bool periodic = R.bc == 0;
  const double h = R.h;
  const double ih2 = 1.0 / (h * h);
  const double alpha = -ih2;
  const double qscale = kFxInv / h;
  const long long* __restrict__ Q = reinterpret_cast<const long long*>(R.q[qsel]);
  const bool owns_n = !periodic && act && t == T - 1;
  const double aL = (periodic || t > 0) ? alpha : 0.0;
  const double aR = (periodic || t < T - 1) ? alpha : 0.0;

  if (t == 0) {
    s_maxd = 0ull;
    s_nan = 0;
  }

  double phi[M];
  double phin = 0.0;
  if (R.closure != 2) {
    if (act) {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const int g = t * M + j;
        if (cold) {
          const double s = (!periodic && g == 0) ? 0.5 : 1.0;
          phi[j] = log(fmax((double)Q[g] * qscale / s, 1e-8));
        } else {
          phi[j] = R.phi[g];
        }
      }
      if (owns_n) phin = cold ? log(fmax((double)Q[n] * qscale / 0.5, 1e-8)) : R.phi[n];
    }

    for (int it = 0; it < iters; ++it) {
      // --- neighbours of the chunk ends
      if (act) {
        s_first[t] = phi[0];
        s_last[t] = phi[M - 1];
      }
      if (owns_n) s_phin = phin;
      __syncthreads();
      double b[M], d[M];
      double bn = 1.0, dn = 0.0;
      if (act) {
        const double pl = t > 0 ? s_last[t - 1] : (periodic ? s_last[T - 1] : 0.0);
        const double pr = t < T - 1 ? s_first[t + 1] : (periodic ? s_first[0] : s_phin);
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const int g = t * M + j;
          const double left = j > 0 ? phi[j - 1] : pl;
          const double right = j < M - 1 ? phi[j + 1] : pr;
          const double ex = exp(phi[j]);
          const double qv = (double)Q[g] * qscale;
          double lap, s, diag;
          if (!periodic && g == 0) {
            lap = (phi[j] - right) * ih2;
            s = 0.5;
            diag = ih2;
          } else {
            lap = (2.0 * phi[j] - left - right) * ih2;
            s = 1.0;
            diag = 2.0 * ih2;
          }
          d[j] = -(lap + s * ex - qv);
          b[j] = diag + s * ex;
        }
        if (owns_n) {
          const double ex = exp(phin);
          dn = -((phin - phi[M - 1]) * ih2 + 0.5 * ex - (double)Q[n] * qscale);
          bn = ih2 + 0.5 * ex;
          // eliminate node N into row N-1
          const double rbn = rcp(bn);
          b[M - 1] -= alpha * alpha * rbn;
          d[M - 1] -= alpha * dn * rbn;
        }
      }

      // --- local elimination of the interior rows 0..M-2
      double yl = 0.0, gll = 0.0, grl = 0.0;  // row M-2 in terms of (X_{t-1}, X_t)
      double y0 = 0.0, gl0 = 0.0, gr0 = 0.0;  // row 0
      if (M >= 2 && act) {
        double den = b[0];
        const double r0 = rcp(den);
        double c = alpha * r0;
        double y = d[0] * r0;
        double gl = -aL * r0;
#pragma unroll
        for (int j = 1; j <= M - 2; ++j) {
          den = b[j] - alpha * c;
          const double rj = rcp(den);
          y = (d[j] - alpha * y) * rj;
          gl = (-alpha * gl) * rj;
          c = alpha * rj;
        }
        yl = y;
        gll = gl;
        grl = -alpha * rcp(den);
        // upward sweep for row 0
        double dn2 = b[M - 2];
        double rh = rcp(dn2);
        double ch = -alpha * rh;
        double yh = d[M - 2] * rh;
        double grh = -alpha * rh;
#pragma unroll
        for (int j = M - 3; j >= 0; --j) {
          dn2 = b[j] + alpha * ch;
          rh = rcp(dn2);
          yh = (d[j] - alpha * yh) * rh;
          grh = (-alpha * grh) * rh;
          ch = -alpha * rh;
        }
        y0 = yh;
        gr0 = grh;
        gl0 = -aL * rh;
        s_y0[t] = y0;
        s_gl0[t] = gl0;
        s_gr0[t] = gr0;
      }
      __syncthreads();

      // --- one equation per thread for its last row
      double A = 0.0, B = 1.0, C = 0.0, D = 0.0;
      if (act) {
        if (M >= 2) {
          const int tn = t < T - 1 ? t + 1 : 0;
          const double yn = s_y0[tn], gln = s_gl0[tn], grn = s_gr0[tn];
          A = alpha * gll;
          B = b[M - 1] + alpha * grl + aR * gln;
          C = aR * grn;
          D = d[M - 1] - alpha * yl - aR * yn;
        } else {
          A = aL;
          B = b[0];
          C = aR;
          D = d[0];
        }
        s_a[t] = A;
        s_b[t] = B;
        s_c[t] = C;
        s_d[t] = D;
      }
      // --- parallel cyclic reduction over the T separator rows
      for (int st = 1; st < T; st <<= 1) {
        __syncthreads();
        double nA = A, nB = B, nC = C, nD = D;
        if (act) {
          int im = t - st, ip = t + st;
          bool vm = true, vp = true;
          if (periodic) {
            im &= (T - 1);
            ip &= (T - 1);
          } else {
            vm = im >= 0;
            vp = ip < T;
          }
          nA = 0.0;
          nC = 0.0;
          if (vm) {
            const double k1 = A * rcp(s_b[im]);
            nA = -s_a[im] * k1;
            nB -= s_c[im] * k1;
            nD -= s_d[im] * k1;
          }
          if (vp) {
            const double k2 = C * rcp(s_b[ip]);
            nC = -s_c[ip] * k2;
            nB -= s_a[ip] * k2;
            nD -= s_d[ip] * k2;
          }
        }
        __syncthreads();
        if (act) {
          A = nA;
          B = nB;
          C = nC;
          D = nD;
          s_a[t] = A;
          s_b[t] = B;
          s_c[t] = C;
          s_d[t] = D;
        }
      }
      double X = 0.0;
      if (act) {
        X = D * rcp(A + B + C);
        s_first[t] = X;  // reuse as the separator values
      }
      __syncthreads();

      // --- interior rows by one Thomas pass with both ends known
      double local_max = 0.0;
      bool bad = false;
      if (act) {
        const double XL = t > 0 ? s_first[t - 1] : (periodic ? s_first[T - 1] : 0.0);
        if (M >= 2) {
          d[0] -= aL * XL;
          d[M - 2] -= alpha * X;
          // forward: b[j] <- c'_j, d[j] <- z'_j
          double rd = rcp(b[0]);
          b[0] = alpha * rd;
          d[0] = d[0] * rd;
#pragma unroll
          for (int j = 1; j <= M - 2; ++j) {
            rd = rcp(b[j] - alpha * b[j - 1]);
            d[j] = (d[j] - alpha * d[j - 1]) * rd;
            b[j] = alpha * rd;
          }
#pragma unroll
          for (int j = M - 3; j >= 0; --j) d[j] -= b[j] * d[j + 1];
        }
        d[M - 1] = X;
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double dl = clamp2(d[j]);
          bad |= !(fabs(d[j]) < 1e300);
          local_max = fmax(local_max, fabs(dl));
          phi[j] += dl;
        }
        if (owns_n) {
          const double dN = clamp2((dn - alpha * X) * rcp(bn));
          bad |= !(fabs(dN) < 1e300);
          local_max = fmax(local_max, fabs(dN));
          phin += dN;
        }
      }
      if (it == iters - 1) {
        if (bad) atomicOr(&s_nan, 1);
        if (local_max > 0.0) atomicMax(&s_maxd, (unsigned long long)__double_as_longlong(local_max));
      }
      __syncthreads();
    }
  } else if (act) {
#pragma unroll
    for (int j = 0; j < M; ++j) phi[j] = 0.0;
  }

  // --- store phi, then the centred-difference field
  if (act) {
#pragma unroll
    for (int j = 0; j < M; ++j) R.phi[t * M + j] = phi[j];
    if (owns_n) R.phi[n] = phin;
    s_first[t] = phi[0];
    s_last[t] = phi[M - 1];
  }
  if (owns_n) s_phin = phin;
  __syncthreads();
  if (act) {
    const double pl = t > 0 ? s_last[t - 1] : (periodic ? s_last[T - 1] : 0.0);
    const double pr = t < T - 1 ? s_first[t + 1] : (periodic ? s_first[0] : s_phin);
    const double inv2h = 0.5 / h;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int g = t * M + j;
      const double left = j > 0 ? phi[j - 1] : pl;
      const double right = j < M - 1 ? phi[j + 1] : pr;
      float ev = (float)(-(right - left) * inv2h);
      if (!periodic && g == 0) ev = 0.f;
      R.e[g] = ev;
      if (save_en) R.en[g] = ev;
    }
    if (owns_n) {
      R.e[n] = 0.f;
      if (save_en) R.en[n] = 0.f;
    }
  }
  // --- clear the next deposit buffer and, at a burst start, the snapshot bins
  {
    long long* other = reinterpret_cast<long long*>(R.q[qsel ^ 1]);
    for (int k = t; k < R.n_nodes; k += blockDim.x) other[k] = 0;
    if (zero_bins) {
      const int nb = (R.burst_steps + 1) * 2 * R.n_coarse;
      long long* rb = reinterpret_cast<long long*>(R.rbins);
      for (int k = t; k < nb; k += blockDim.x) rb[k] = 0;
    }
  }
  if (t == 0 && R.closure != 2) {
    const double md = __longlong_as_double((long long)s_maxd);
    if (s_nan) atomicOr(status, 2u);
    if (md > tol || s_nan) atomicOr(status, 1u);
  }
}

// Burst start when the field is already current: store E_n and clear the bins.
__global__ void k_prep_burst(const RepDev* __restrict__ reps) {
  const RepDev& R = reps[blockIdx.x];
  for (int k = threadIdx.x; k < R.n_nodes; k += blockDim.x) R.en[k] = R.e[k];
  const int nb = (R.burst_steps + 1) * 2 * R.n_coarse;
  long long* rb = reinterpret_cast<long long*>(R.rbins);
  for (int k = threadIdx.x; k < nb; k += blockDim.x) rb[k] = 0;
}

}  // namespace

void launch_newton(const RepDev* d_reps, const int32_t* d_list, int n_list, int M, int threads,
                   int iters, int cold, int qsel, int save_en, int zero_bins, double tol,
                   uint32_t* d_status, hipStream_t stream) {
  if (n_list <= 0) return;
  const dim3 grid(n_list);
#define EFPI_NEWTON(MM, TT)                                                                   \
  hipLaunchKernelGGL((k_newton<MM, TT>), grid, dim3(threads), 0, stream, d_reps, d_list, iters, \
                     cold, qsel, save_en, zero_bins, tol, d_status)
  if (M == 1) EFPI_NEWTON(1, 256);
  else if (M == 2) EFPI_NEWTON(2, 256);
  else if (M == 4) EFPI_NEWTON(4, 256);
  else if (M == 8) EFPI_NEWTON(8, 256);
  else if (M == 16) EFPI_NEWTON(16, 256);
  else EFPI_NEWTON(32, 512);
#undef EFPI_NEWTON
}

void launch_prep_burst(const RepDev* d_reps, int n_reps, hipStream_t stream) {
  hipLaunchKernelGGL(k_prep_burst, dim3(n_reps), dim3(256), 0, stream, d_reps);
}

}  // namespace efpi
