// Field solve of the fine burst: Newton iterations for the Poisson-Boltzmann
// equation -phi'' + exp(phi) = rho (eq. 3.15; Boltzmann electrons of eqs. 3.2 and
// 3.16) on the node grid, then the node field E_k = -(phi_{k+1} - phi_{k-1}) / 2h.
//
// One workgroup per replica.  The residual F and the potential are FP64; each
// Newton correction J delta = -F is solved in FP32 (the Jacobian is diagonally
// dominant, so the FP32 solve adds a relative error of ~1e-7 to delta, which the
// next iteration removes with the FP64 residual: the iteration still converges
// to the FP64 solution).  Rows are scaled by the node volume so that
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

// 1/b for the FP32 correction solve: the hardware reciprocal (1 ulp).
__device__ __forceinline__ float rcp(float b) { return __builtin_amdgcn_rcpf(b); }

// Tridiagonal separator system a_i X_{i-1} + b_i X_i + c_i X_{i+1} = d_i,
// i = 0..T-1 (cyclic when periodic; a_0 = c_{T-1} = 0 otherwise), solved by the
// 64 lanes of one wave.  Lane l owns rows [l S, (l + 1) S) with W = min(T, 64)
// lanes and S = T / W: it eliminates its first S - 1 rows (expressing them by
// the last row of the previous lane and its own last row), which leaves one
// equation per lane for its last row; those W equations are solved by cyclic
// reduction with lane shuffles, and the eliminated rows follow by one Thomas
// pass with both ends known.  Writes x to sx[0..T).  Call with all 64 lanes.
__device__ void solve_separators(int l, int T, bool periodic, const float* sa, const float* sb,
                                 const float* sc, const float* sd, float* scp, float* syp,
                                 float* sx) {
  const int W = T < kWave ? T : kWave;
  const int S = T / W;
  const bool on = l < W;
  const int i0 = on ? l * S : 0;
  // rows 0..S-2 of the chunk in terms of XL (previous lane's X) and XR (own X)
  float yl = 0.f, gll = 0.f, grl = 0.f, y0 = 0.f, gl0 = 0.f, gr0 = 0.f;
  if (on && S >= 2) {
    float r = rcp(sb[i0]);
    float cp = sc[i0] * r, yp = sd[i0] * r, glp = -sa[i0] * r;
    for (int j = 1; j <= S - 2; ++j) {
      const float aj = sa[i0 + j];
      r = rcp(sb[i0 + j] - aj * cp);
      yp = (sd[i0 + j] - aj * yp) * r;
      glp = -aj * glp * r;
      cp = sc[i0 + j] * r;
    }
    yl = yp;
    gll = glp;
    grl = -cp;
    r = rcp(sb[i0 + S - 2]);
    float ch = sa[i0 + S - 2] * r, yh = sd[i0 + S - 2] * r, grh = -sc[i0 + S - 2] * r;
    for (int j = S - 3; j >= 0; --j) {
      const float cj = sc[i0 + j];
      r = rcp(sb[i0 + j] - cj * ch);
      yh = (sd[i0 + j] - cj * yh) * r;
      grh = -cj * grh * r;
      ch = sa[i0 + j] * r;
    }
    y0 = yh;
    gl0 = -ch;
    gr0 = grh;
  }
  // one equation per lane for its last row
  const int nxt = (l + 1) & (W - 1);
  const float y0n = __shfl(y0, nxt), gl0n = __shfl(gl0, nxt), gr0n = __shfl(gr0, nxt);
  float A = 0.f, B = 1.f, C = 0.f, D = 0.f;
  if (on) {
    const int il = i0 + S - 1;
    const float al = sa[il], bl = sb[il], cl = sc[il], dl = sd[il];
    if (S >= 2) {
      A = al * gll;
      B = bl + al * grl + cl * gl0n;
      C = cl * gr0n;
      D = dl - al * yl - cl * y0n;
    } else {
      A = al;
      B = bl;
      C = cl;
      D = dl;
    }
  }
  // cyclic reduction over the W lane equations
  for (int st = 1; st < W; st <<= 1) {
    int im = l - st, ip = l + st;
    bool vm = true, vp = true;
    if (periodic) {
      im &= (W - 1);
      ip &= (W - 1);
    } else {
      vm = im >= 0;
      vp = ip < W;
      im = vm ? im : l;
      ip = vp ? ip : l;
    }
    const float Am = __shfl(A, im), Bm = __shfl(B, im), Cm = __shfl(C, im), Dm = __shfl(D, im);
    const float Ap = __shfl(A, ip), Bp = __shfl(B, ip), Cp = __shfl(C, ip), Dp = __shfl(D, ip);
    float nA = 0.f, nB = B, nC = 0.f, nD = D;
    if (vm) {
      const float k1 = A * rcp(Bm);
      nA = -Am * k1;
      nB -= Cm * k1;
      nD -= Dm * k1;
    }
    if (vp) {
      const float k2 = C * rcp(Bp);
      nC = -Cp * k2;
      nB -= Ap * k2;
      nD -= Dp * k2;
    }
    A = nA;
    B = nB;
    C = nC;
    D = nD;
  }
  // after the reduction the couplings reach the lane itself (cyclic) or vanish
  const float X = D * rcp(A + B + C);
  const float XL = __shfl(X, (l - 1) & (W - 1));
  if (!on) return;
  sx[i0 + S - 1] = X;
  if (S >= 2) {
    // rows 0..S-2 with x_{-1} = XL and x_{S-1} = X known
    float dj = sd[i0] - sa[i0] * XL;
    if (S == 2) dj -= sc[i0] * X;
    float r = rcp(sb[i0]);
    float cp = sc[i0] * r;
    float yp = dj * r;
    scp[i0] = cp;
    syp[i0] = yp;
    for (int j = 1; j <= S - 2; ++j) {
      dj = sd[i0 + j];
      if (j == S - 2) dj -= sc[i0 + j] * X;
      const float aj = sa[i0 + j];
      r = rcp(sb[i0 + j] - aj * cp);
      yp = (dj - aj * yp) * r;
      cp = sc[i0 + j] * r;
      scp[i0 + j] = cp;
      syp[i0 + j] = yp;
    }
    float x = syp[i0 + S - 2];
    sx[i0 + S - 2] = x;
    for (int j = S - 3; j >= 0; --j) {
      x = syp[i0 + j] - scp[i0 + j] * x;
      sx[i0 + j] = x;
    }
  }
}

template <int M, int THREADS>
__global__ __launch_bounds__(THREADS) void k_newton(const RepDev* __restrict__ reps,
                                                   const int32_t* __restrict__ list, int iters,
                                                   int cold, int qsel, int save_en,
                                                   int zero_bins, double tol,
                                                   uint32_t* __restrict__ status) {
  __shared__ double s_first[kMaxT], s_last[kMaxT];
  __shared__ float s_a[kMaxT], s_b[kMaxT], s_c[kMaxT], s_d[kMaxT];
  __shared__ float s_y0[kMaxT], s_gl0[kMaxT], s_gr0[kMaxT], s_x[kMaxT];
  __shared__ float s_cp[kMaxT], s_yp[kMaxT];
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
  const float alpha = (float)-ih2;
  const double qscale = kFxInv / h;
  const long long* __restrict__ Q = reinterpret_cast<const long long*>(R.q[qsel]);
  const bool owns_n = !periodic && act && t == T - 1;
  const float aL = (periodic || t > 0) ? alpha : 0.f;
  const float aR = (periodic || t < T - 1) ? alpha : 0.f;

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
      float b[M], d[M];
      float bn = 1.f, dn = 0.f;
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
          d[j] = (float)-(lap + s * ex - qv);
          b[j] = (float)(diag + s * ex);
        }
        if (owns_n) {
          const double ex = exp(phin);
          dn = (float)-((phin - phi[M - 1]) * ih2 + 0.5 * ex - (double)Q[n] * qscale);
          bn = (float)(ih2 + 0.5 * ex);
          // eliminate node N into row N-1
          const float rbn = rcp(bn);
          b[M - 1] -= alpha * alpha * rbn;
          d[M - 1] -= alpha * dn * rbn;
        }
      }

      // --- local elimination of the interior rows 0..M-2
      float yl = 0.f, gll = 0.f, grl = 0.f;  // row M-2 in terms of (X_{t-1}, X_t)
      float y0 = 0.f, gl0 = 0.f, gr0 = 0.f;  // row 0
      if (M >= 2 && act) {
        float den = b[0];
        const float r0 = rcp(den);
        float c = alpha * r0;
        float y = d[0] * r0;
        float gl = -aL * r0;
#pragma unroll
        for (int j = 1; j <= M - 2; ++j) {
          den = b[j] - alpha * c;
          const float rj = rcp(den);
          y = (d[j] - alpha * y) * rj;
          gl = (-alpha * gl) * rj;
          c = alpha * rj;
        }
        yl = y;
        gll = gl;
        grl = -alpha * rcp(den);
        // upward sweep for row 0
        float dn2 = b[M - 2];
        float rh = rcp(dn2);
        float ch = -alpha * rh;
        float yh = d[M - 2] * rh;
        float grh = -alpha * rh;
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
      float A = 0.f, B = 1.f, C = 0.f, D = 0.f;
      if (act) {
        if (M >= 2) {
          const int tn = t < T - 1 ? t + 1 : 0;
          const float yn = s_y0[tn], gln = s_gl0[tn], grn = s_gr0[tn];
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
      __syncthreads();
      // --- the T separator rows: wave 0 solves them (no workgroup barriers inside)
      if (t < kWave) solve_separators(t, T, periodic, s_a, s_b, s_c, s_d, s_cp, s_yp, s_x);
      __syncthreads();
      float X = 0.f;
      if (act) X = s_x[t];

      // --- interior rows by one Thomas pass with both ends known
      double local_max = 0.0;
      bool bad = false;
      if (act) {
        const float XL = t > 0 ? s_x[t - 1] : (periodic ? s_x[T - 1] : 0.f);
        if (M >= 2) {
          d[0] -= aL * XL;
          d[M - 2] -= alpha * X;
          // forward: b[j] <- c'_j, d[j] <- z'_j
          float rd = rcp(b[0]);
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
          const double dl = clamp2((double)d[j]);
          bad |= !(fabsf(d[j]) < 3e38f);
          local_max = fmax(local_max, fabs(dl));
          phi[j] += dl;
        }
        if (owns_n) {
          const float dNf = (dn - alpha * X) * rcp(bn);
          const double dN = clamp2((double)dNf);
          bad |= !(fabsf(dNf) < 3e38f);
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
  else if (M == 16 && threads <= 256) EFPI_NEWTON(16, 256);
  else if (M == 16) EFPI_NEWTON(16, 512);
  else EFPI_NEWTON(32, 512);
#undef EFPI_NEWTON
}

void launch_prep_burst(const RepDev* d_reps, int n_reps, hipStream_t stream) {
  hipLaunchKernelGGL(k_prep_burst, dim3(n_reps), dim3(256), 0, stream, d_reps);
}

}  // namespace efpi
