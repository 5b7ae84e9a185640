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
// thread for its last row.  Those T equations are split again by wave: the last
// lane of each wave is a separator, the other lanes are reduced by parallel
// cyclic reduction over lane shuffles (in terms of the two separators around the
// wave), and the small cyclic system of the separators is solved redundantly by
// every wave, so a Newton step takes three workgroup barriers.  The interior rows
// then follow by one Thomas pass.  Periodic grids give cyclic systems; on walls,
// node N is eliminated into row N-1 first so every system has N rows.
#include "efpi_internal.h"

namespace efpi {
namespace {

// 16-byte vector types for the row loads and stores
typedef long long i64x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double clamp2(double x) { return fmin(2.0, fmax(-2.0, x)); }

// 1/b for the FP32 correction solve: the hardware reciprocal (1 ulp).
__device__ __forceinline__ float rcp(float b) { return __builtin_amdgcn_rcpf(b); }

// Wave-level solve of the thread equations.  Lane l of wave w (thread t = 64 w + l)
// holds the equation A X_{t-1} + B X_t + C X_{t+1} = D of its last row.  The last
// active lane of each wave is that wave's separator G_w; lanes 0..L-2 are solved
// by parallel cyclic reduction over lane shuffles in terms of the two separators
// around them, X_t = y + gl G_{w-1} + gr G_w (three right-hand sides: D, and the
// couplings of lane 0 to G_{w-1} and of lane L-2 to G_w moved to the right).
// Rows outside 0..L-2 act as identity rows.  Returns (y, gl, gr).
__device__ __forceinline__ void wave_pcr(int lane, int L, bool inb, float A, float B, float C,
                                         float D, float& y, float& gl, float& gr) {
  float pa = lane == 0 ? 0.f : A;
  float pc = lane == L - 2 ? 0.f : C;
  float pb = B, r0 = D;
  float r1 = lane == 0 ? -A : 0.f;
  float r2 = lane == L - 2 ? -C : 0.f;
  if (!inb) {
    pa = pc = r0 = r1 = r2 = 0.f;
    pb = 1.f;
  }
  for (int st = 1; st < L - 1; st <<= 1) {
    const bool vm = lane - st >= 0 && inb;
    const bool vp = lane + st <= L - 2 && inb;
    const int im = vm ? lane - st : lane;
    const int ip = vp ? lane + st : lane;
    const float Am = __shfl(pa, im), Bm = __shfl(pb, im), Cm = __shfl(pc, im);
    const float Rm0 = __shfl(r0, im), Rm1 = __shfl(r1, im), Rm2 = __shfl(r2, im);
    const float Ap = __shfl(pa, ip), Bp = __shfl(pb, ip), Cp = __shfl(pc, ip);
    const float Rp0 = __shfl(r0, ip), Rp1 = __shfl(r1, ip), Rp2 = __shfl(r2, ip);
    const float k1 = vm ? pa * rcp(Bm) : 0.f;
    const float k2 = vp ? pc * rcp(Bp) : 0.f;
    pa = -Am * k1;
    pc = -Cp * k2;
    pb = pb - Cm * k1 - Ap * k2;
    r0 = r0 - Rm0 * k1 - Rp0 * k2;
    r1 = r1 - Rm1 * k1 - Rp1 * k2;
    r2 = r2 - Rm2 * k1 - Rp2 * k2;
  }
  const float inv = rcp(pb);
  y = r0 * inv;
  gl = r1 * inv;
  gr = r2 * inv;
}

// Separator system of the waves: lane i < nw holds alpha G_{i-1} + beta G_i +
// gamma G_{i+1} = delta (cyclic when periodic), solved by cyclic reduction over
// lane shuffles; returns G_i in lane i.
__device__ __forceinline__ float wave_cr(int lane, int nw, bool periodic, float A, float B,
                                         float C, float D) {
  if (lane >= nw) {
    A = C = D = 0.f;
    B = 1.f;
  }
  for (int st = 1; st < nw; st <<= 1) {
    int im = lane - st, ip = lane + st;
    bool vm = lane < nw, vp = lane < nw;
    if (periodic) {
      im &= (nw - 1);
      ip &= (nw - 1);
    } else {
      vm = vm && im >= 0;
      vp = vp && ip < nw;
    }
    im = vm ? im : lane;
    ip = vp ? ip : lane;
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
  return D * rcp(A + B + C);
}

// Every field solve runs one workgroup of kFieldThreads threads per replica, all
// replicas of a context in one launch; a replica's rows per thread M (its
// descriptor's field_m) selects the compiled body, and threads past N / M only
// take part in the barriers.
constexpr int kFieldThreads = 512;
constexpr int kFieldWaves = kFieldThreads / kWave;

struct NewtonLds {
  double s_first[kFieldThreads], s_last[kFieldThreads];
  float s_row0[kFieldWaves][3];  // row 0 of each wave's lane 0, in terms of (X_{t-1}, X_t)
  float s_sol0[kFieldWaves][3];  // lane 0's X in terms of the separators around its wave
  float s_if[kFieldWaves][4];    // separator equation of each wave
  double s_wmax[kFieldWaves];
  int s_wbad[kFieldWaves];
  double s_phin;
};

template <int M>
__device__ __forceinline__ void newton_body(const RepDev& R, NewtonLds& S, int iters, int cold,
                                            int qsel, int save_en, int zero_bins, double tol,
                                            uint32_t* __restrict__ status) {
  constexpr int THREADS = kFieldThreads;
  double* const s_first = S.s_first;
  double* const s_last = S.s_last;
  auto& s_row0 = S.s_row0;
  auto& s_sol0 = S.s_sol0;
  auto& s_if = S.s_if;
  auto& s_wmax = S.s_wmax;
  auto& s_wbad = S.s_wbad;
  double& s_phin = S.s_phin;
  const int n = R.n_cells;
  const int T = n / M;
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  const int w = t / kWave;
  const int L = T < kWave ? T : kWave;      // active lanes of an active wave
  const int nw = (T + kWave - 1) / kWave;   // active waves
  const bool act = t < T;
  const bool periodic = R.bc == 0;
  const double h = R.h;
  const double ih2 = 1.0 / (h * h);
  const float alpha = (float)-ih2;
  const double qscale = kFxInv / h;
  const auto Q = gmem(reinterpret_cast<const long long*>(R.q[qsel]));
  const auto phig = gmem(R.phi);
  // fields used only after the iterations, read now with the others (a scalar
  // load issued at the end would cost one more memory round trip there)
  const int n_nodes = R.n_nodes;
  const auto other = gmem(reinterpret_cast<long long*>(R.q[qsel ^ 1]));
  const int n_bins = zero_bins ? (R.burst_steps + 1) * R.moments * R.n_coarse : 0;
  const auto bins = gmem(reinterpret_cast<long long*>(R.rbins));
  const auto eg = gmem(R.e);
  const auto eng = gmem(R.en);
  const bool no_field = R.closure == 2;
  // the convergence check's arguments are needed only at the end; have them in
  // registers from the start as well
  asm volatile("" ::"s"(status), "s"(tol));
  const bool owns_n = !periodic && act && t == T - 1;
  const float aL = (periodic || t > 0) ? alpha : 0.f;
  const float aR = (periodic || t < T - 1) ? alpha : 0.f;

  // the charge is held in registers up to 16 rows per thread (above, it is
  // re-read from L2 each iteration to keep the kernel free of spills)
  constexpr bool kHoist = M <= 16;
  double phi[M];
  double qv[kHoist ? M : 1];
  auto charge = [&](int j) -> double {
    if constexpr (kHoist) return qv[j];
    else return (double)Q[t * M + j] * qscale;
  };
  double phin = 0.0;
  if (!no_field) {
    if (act) {
      if constexpr (!kHoist) {
      } else if constexpr (M >= 2) {
        const auto q2 = gmem(reinterpret_cast<const i64x2*>(R.q[qsel])) + t * (M / 2);
#pragma unroll
        for (int j = 0; j < M / 2; ++j) {
          const i64x2 v = q2[j];
          qv[2 * j] = (double)v.x * qscale;
          qv[2 * j + 1] = (double)v.y * qscale;
        }
      } else {
        qv[0] = (double)Q[t] * qscale;
      }
      if (cold) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double s = (!periodic && t * M + j == 0) ? 0.5 : 1.0;
          phi[j] = log(fmax(charge(j) / s, 1e-8));
        }
      } else if constexpr (M >= 2) {
        // storage order of phi_slot: pair j of thread t at pair slot j T + t
        const auto p2 = gmem(reinterpret_cast<const f64x2*>(R.phi)) + t;
#pragma unroll
        for (int j = 0; j < M / 2; ++j) {
          const f64x2 v = p2[j * T];
          phi[2 * j] = v.x;
          phi[2 * j + 1] = v.y;
        }
      } else {
        phi[0] = phig[t];
      }
      if (owns_n) phin = cold ? log(fmax((double)Q[n] * qscale / 0.5, 1e-8)) : phig[n];
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
          d[j] = (float)-(lap + s * ex - charge(j));
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
      }

      // --- one equation per thread for its last row (row 0 of the next thread
      // comes from the next lane; the wave's last lane takes it after the barrier)
      const float yn = __shfl(y0, lane + 1), gln = __shfl(gl0, lane + 1);
      const float grn = __shfl(gr0, lane + 1);
      float A = 0.f, B = 1.f, C = 0.f, D = 0.f;
      if (act) {
        if (M >= 2) {
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
      }
      // --- lanes 0..L-2 of every wave in terms of the separators G_{w-1}, G_w
      float xy, xgl, xgr;
      wave_pcr(lane, L, act && lane <= L - 2, A, B, C, D, xy, xgl, xgr);
      const float py = __shfl(xy, L - 2), pgl = __shfl(xgl, L - 2), pgr = __shfl(xgr, L - 2);
      if (act && lane == 0) {
        s_row0[w][0] = y0;
        s_row0[w][1] = gl0;
        s_row0[w][2] = gr0;
        s_sol0[w][0] = xy;
        s_sol0[w][1] = xgl;
        s_sol0[w][2] = xgr;
      }
      __syncthreads();
      // --- separator equation of each wave (its last lane)
      if (act && lane == L - 1) {
        const int wn = w + 1 < nw ? w + 1 : 0;
        float Aw = aL, Bw = b[0], Cw = aR, Dw = d[0];
        if (M >= 2) {
          Aw = alpha * gll;
          Bw = b[M - 1] + alpha * grl + aR * s_row0[wn][1];
          Cw = aR * s_row0[wn][2];
          Dw = d[M - 1] - alpha * yl - aR * s_row0[wn][0];
        }
        const float y2 = s_sol0[wn][0], gl2 = s_sol0[wn][1], gr2 = s_sol0[wn][2];
        s_if[w][0] = Aw * pgl;
        s_if[w][1] = Bw + Aw * pgr + Cw * gl2;
        s_if[w][2] = Cw * gr2;
        s_if[w][3] = Dw - Aw * py - Cw * y2;
      }
      __syncthreads();
      // --- the nw separators, solved redundantly by every wave
      float IA = 0.f, IB = 1.f, IC = 0.f, ID = 0.f;
      if (lane < nw) {
        IA = s_if[lane][0];
        IB = s_if[lane][1];
        IC = s_if[lane][2];
        ID = s_if[lane][3];
      }
      const float G = wave_cr(lane, nw, periodic, IA, IB, IC, ID);
      const int wl = w > 0 ? w - 1 : (periodic ? nw - 1 : 0);
      const float Gw = __shfl(G, w < nw ? w : 0);
      const float Gl = (w > 0 || periodic) ? __shfl(G, wl) : 0.f;
      const float X = lane == L - 1 ? Gw : xy + xgl * Gl + xgr * Gw;
      const float Xp = __shfl(X, lane > 0 ? lane - 1 : 0);

      // --- interior rows by one Thomas pass with both ends known
      double local_max = 0.0;
      bool bad = false;
      if (act) {
        const float XL = lane > 0 ? Xp : Gl;
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
        // largest correction and NaN flag of the wave, one LDS slot per wave
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) local_max = fmax(local_max, __shfl_xor(local_max, o));
        const bool wbad = __any(bad);
        if (lane == 0) {
          s_wmax[w] = local_max;
          s_wbad[w] = wbad ? 1 : 0;
        }
      }
    }
  } else if (act) {
#pragma unroll
    for (int j = 0; j < M; ++j) phi[j] = 0.0;
  }

  // --- centred-difference field (the potential is stored after the barrier)
  if (act) {
    s_first[t] = phi[0];
    s_last[t] = phi[M - 1];
  }
  if (owns_n) s_phin = phin;
  __syncthreads();
  if (act) {
    if constexpr (M >= 2) {
      const auto p2 = reinterpret_cast<EFPI_GLOBAL f64x2*>(phig) + t;  // phi_slot order
#pragma unroll
      for (int j = 0; j < M / 2; ++j) p2[j * T] = f64x2{phi[2 * j], phi[2 * j + 1]};
    } else {
      phig[t] = phi[0];
    }
    if (owns_n) phig[n] = phin;
    const double pl = t > 0 ? s_last[t - 1] : (periodic ? s_last[T - 1] : 0.0);
    const double pr = t < T - 1 ? s_first[t + 1] : (periodic ? s_first[0] : s_phin);
    const double inv2h = 0.5 / h;
    float ev[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int g = t * M + j;
      const double left = j > 0 ? phi[j - 1] : pl;
      const double right = j < M - 1 ? phi[j + 1] : pr;
      ev[j] = (float)(-(right - left) * inv2h);
      if (!periodic && g == 0) ev[j] = 0.f;
    }
    if constexpr (M >= 4) {
      const auto e4 = reinterpret_cast<EFPI_GLOBAL f32x4*>(eg) + t * (M / 4);
      const auto n4 = reinterpret_cast<EFPI_GLOBAL f32x4*>(eng) + t * (M / 4);
#pragma unroll
      for (int j = 0; j < M / 4; ++j) {
        const f32x4 v = {ev[4 * j], ev[4 * j + 1], ev[4 * j + 2], ev[4 * j + 3]};
        e4[j] = v;
        if (save_en) n4[j] = v;
      }
    } else {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        eg[t * M + j] = ev[j];
        if (save_en) eng[t * M + j] = ev[j];
      }
    }
    if (owns_n) {
      eg[n] = 0.f;
      if (save_en) eng[n] = 0.f;
    }
  }
  // --- clear the next deposit buffer (n_nodes = M T + 1 <= M THREADS + 1: at
  // most M + 1 stores per thread) and, at a burst start, the snapshot bins
#pragma unroll
  for (int j = 0; j <= M; ++j) {
    const int k = t + j * THREADS;
    if (k < n_nodes) other[k] = 0;
  }
  for (int k = t; k < n_bins; k += THREADS) bins[k] = 0;
  if (t == 0 && !no_field) {
    double md = 0.0;
    int nan = 0;
    for (int k = 0; k < nw; ++k) {
      md = fmax(md, s_wmax[k]);
      nan |= s_wbad[k];
    }
    if (nan) atomicOr(status, 2u);
    if (md > tol || nan) atomicOr(status, 1u);
  }
}

__global__ __launch_bounds__(kFieldThreads) void k_newton(const RepDev* __restrict__ reps,
                                                         int iters, int cold, int qsel,
                                                         int save_en, int zero_bins, double tol,
                                                         uint32_t* __restrict__ status) {
  __shared__ NewtonLds S;
  const RepDev& R = reps[blockIdx.x];
  switch (R.field_m) {
    case 1: newton_body<1>(R, S, iters, cold, qsel, save_en, zero_bins, tol, status); break;
    case 2: newton_body<2>(R, S, iters, cold, qsel, save_en, zero_bins, tol, status); break;
    case 4: newton_body<4>(R, S, iters, cold, qsel, save_en, zero_bins, tol, status); break;
    case 8: newton_body<8>(R, S, iters, cold, qsel, save_en, zero_bins, tol, status); break;
    case 16: newton_body<16>(R, S, iters, cold, qsel, save_en, zero_bins, tol, status); break;
    default: newton_body<32>(R, S, iters, cold, qsel, save_en, zero_bins, tol, status); break;
  }
}

// Burst start when the field is already current: store E_n and clear the bins.
__global__ void k_prep_burst(const RepDev* __restrict__ reps) {
  const RepDev& R = reps[blockIdx.x];
  const auto e = gmem(R.e);
  const auto en = gmem(R.en);
  for (int k = threadIdx.x; k < R.n_nodes; k += blockDim.x) en[k] = e[k];
  const int nb = (R.burst_steps + 1) * R.moments * R.n_coarse;
  const auto rb = gmem(reinterpret_cast<long long*>(R.rbins));
  for (int k = threadIdx.x; k < nb; k += blockDim.x) rb[k] = 0;
}

// ---------------------------------------------------------- linear Poisson --
// Periodic -phi'' = rho - mean(rho) (eq. 2.2) for the kinetic-electron closure,
// solved exactly by prefix sums.  With S_k = sum_{j<=k} (rho_j - mean) and
// g_k = phi_{k+1} - phi_k, the second difference gives g_k = c - h^2 S_k, and
// periodicity (sum_k g_k = 0) fixes c = h^2 Q_N / N with Q_k = sum_{j<k} S_j.  So
// phi_k = sum_{j<k} g_j = h^2 (k Q_N / N - Q_k), and the mean of phi is removed.
// One workgroup per replica, each thread owning M consecutive nodes (M and the
// workgroup size fixed at compile time, as for Newton, so that a thread's loads
// are issued together): two scans (of rho, then of S) and one sum, each in a
// fixed order (reproducible bits).

// Exclusive scan of x over the workgroup (thread order) and the total.
template <int THREADS>
__device__ double block_excl_scan(double x, double* s_w, double& total) {
  constexpr int kW = THREADS / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  double inc = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  double ex = __shfl_up(inc, 1, kWave);
  if (lane == 0) ex = 0.0;
  if (lane == kWave - 1) s_w[wid] = inc;
  __syncthreads();
  double before = 0.0, all = 0.0;
#pragma unroll
  for (int k = 0; k < kW; ++k) {
    const double t = s_w[k];
    if (k < wid) before += t;
    all += t;
  }
  total = all;
  __syncthreads();  // s_w is reused by the next scan
  return before + ex;
}

struct PoissonLds {
  double s_w[kFieldWaves];
  double s_first[kFieldThreads], s_last[kFieldThreads];
  int s_bad;
};

template <int M>
__device__ __forceinline__ void poisson_body(const RepDev& R, PoissonLds& S, int qsel,
                                             int save_en, int zero_bins,
                                             uint32_t* __restrict__ status) {
  constexpr int THREADS = kFieldThreads;
  double* const s_w = S.s_w;
  double* const s_first = S.s_first;
  double* const s_last = S.s_last;
  int& s_bad = S.s_bad;
  const int n = R.n_cells;
  const int T = n / M;
  const int t = threadIdx.x;
  const bool act = t < T;
  const double h = R.h;
  const double h2 = h * h;
  const double qscale = kFxInv / h;
  if (t == 0) s_bad = 0;
  double r[M];
  double loc = 0.0;
  if (act) {
    if constexpr (M >= 2) {
      const auto q2 = gmem(reinterpret_cast<const i64x2*>(R.q[qsel])) + t * (M / 2);
#pragma unroll
      for (int j = 0; j < M / 2; ++j) {
        const i64x2 v = q2[j];
        r[2 * j] = (double)v.x * qscale;
        r[2 * j + 1] = (double)v.y * qscale;
      }
    } else {
      r[0] = (double)gmem(reinterpret_cast<const long long*>(R.q[qsel]))[t] * qscale;
    }
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) r[j] = 0.0;
  }
#pragma unroll
  for (int j = 0; j < M; ++j) loc += r[j];
  double tot;
  double run = block_excl_scan<THREADS>(loc, s_w, tot);
  const double mean = tot / n;
  // S_k = (sum_{j<=k} rho_j) - (k + 1) mean
  loc = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    run += r[j];
    r[j] = act ? run - (double)(t * M + j + 1) * mean : 0.0;
    loc += r[j];
  }
  double qn;
  run = block_excl_scan<THREADS>(loc, s_w, qn);
  const double cq = qn / n;
  // phi_k = h^2 (k Q_N / N - Q_k), Q_k the exclusive running sum of S
  loc = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double sk = r[j];
    r[j] = act ? h2 * ((double)(t * M + j) * cq - run) : 0.0;
    run += sk;
    loc += r[j];
  }
  double ptot;
  block_excl_scan<THREADS>(loc, s_w, ptot);
  const double pmean = ptot / n;
#pragma unroll
  for (int j = 0; j < M; ++j) r[j] -= pmean;
  if (act) {
    s_first[t] = r[0];
    s_last[t] = r[M - 1];
  }
  __syncthreads();
  if (act) {
    const double pl = s_last[t > 0 ? t - 1 : T - 1];
    const double pr = s_first[t < T - 1 ? t + 1 : 0];
    const double inv2h = 0.5 / h;
    bool bad = false;
    float ev[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const double left = j > 0 ? r[j - 1] : pl;
      const double right = j < M - 1 ? r[j + 1] : pr;
      ev[j] = (float)(-(right - left) * inv2h);
      bad |= !(fabs(r[j]) < 1e300);
    }
    const auto phig = gmem(R.phi);
    const auto eg = gmem(R.e);
    const auto eng = gmem(R.en);
    if constexpr (M >= 4) {
      const auto p2 = reinterpret_cast<EFPI_GLOBAL f64x2*>(phig) + t;  // phi_slot order
#pragma unroll
      for (int j = 0; j < M / 2; ++j) p2[j * T] = f64x2{r[2 * j], r[2 * j + 1]};
      const auto e4 = reinterpret_cast<EFPI_GLOBAL f32x4*>(eg) + t * (M / 4);
      const auto n4 = reinterpret_cast<EFPI_GLOBAL f32x4*>(eng) + t * (M / 4);
#pragma unroll
      for (int j = 0; j < M / 4; ++j) {
        const f32x4 v = {ev[4 * j], ev[4 * j + 1], ev[4 * j + 2], ev[4 * j + 3]};
        e4[j] = v;
        if (save_en) n4[j] = v;
      }
    } else {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        phig[t * M + j] = r[j];
        eg[t * M + j] = ev[j];
        if (save_en) eng[t * M + j] = ev[j];
      }
    }
    if (bad) s_bad = 1;
  }
  // clear the next deposit buffer and, at a burst start, the snapshot bins
  const auto other = gmem(reinterpret_cast<long long*>(R.q[qsel ^ 1]));
  for (int k = t; k < R.n_nodes; k += THREADS) other[k] = 0;
  if (zero_bins) {
    const int nb = (R.burst_steps + 1) * R.moments * R.n_coarse;
    const auto bins = gmem(reinterpret_cast<long long*>(R.rbins));
    for (int k = t; k < nb; k += THREADS) bins[k] = 0;
  }
  __syncthreads();
  if (t == 0 && s_bad) atomicOr(status, 2u);
}

__global__ __launch_bounds__(kFieldThreads) void k_poisson(const RepDev* __restrict__ reps,
                                                          int qsel, int save_en, int zero_bins,
                                                          uint32_t* __restrict__ status) {
  __shared__ PoissonLds S;
  const RepDev& R = reps[blockIdx.x];
  switch (R.field_m) {
    case 1: poisson_body<1>(R, S, qsel, save_en, zero_bins, status); break;
    case 2: poisson_body<2>(R, S, qsel, save_en, zero_bins, status); break;
    case 4: poisson_body<4>(R, S, qsel, save_en, zero_bins, status); break;
    case 8: poisson_body<8>(R, S, qsel, save_en, zero_bins, status); break;
    default: poisson_body<16>(R, S, qsel, save_en, zero_bins, status); break;
  }
}

}  // namespace

namespace {
// A replica's potential between the natural node order and the solve's (phi_slot).
__global__ void k_phi_copy(const RepDev* __restrict__ reps, int rep, const double* __restrict__ src,
                           double* __restrict__ dst, int to_natural) {
  const RepDev& R = reps[rep];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < R.n_nodes;
       k += gridDim.x * blockDim.x) {
    const int64_t s = phi_slot(k, R.n_cells, R.field_m);
    if (to_natural) dst[k] = src[s];
    else dst[s] = src[k];
  }
}

// Every replica's charge buffer q[which] cleared in one launch (block row r: replica r).
__global__ void k_zero_charge(const RepDev* __restrict__ reps, int which) {
  const RepDev& R = reps[blockIdx.y];
  const auto q = gmem(reinterpret_cast<long long*>(R.q[which]));
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < R.n_nodes; k += gridDim.x * blockDim.x)
    q[k] = 0;
}
}  // namespace

void launch_zero_charge(const RepDev* d_reps, int n_reps, int which, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_charge, dim3(8, n_reps), dim3(256), 0, stream, d_reps, which);
}

void launch_phi_copy(const RepDev* d_reps, int rep, const double* d_src, double* d_dst,
                     int to_natural, hipStream_t stream) {
  hipLaunchKernelGGL(k_phi_copy, dim3(64), dim3(256), 0, stream, d_reps, rep, d_src, d_dst,
                     to_natural);
}

void launch_poisson(const RepDev* d_reps, int n_reps, int qsel, int save_en, int zero_bins,
                    uint32_t* d_status, hipStream_t stream) {
  if (n_reps <= 0) return;
  hipLaunchKernelGGL(k_poisson, dim3(n_reps), dim3(kFieldThreads), 0, stream, d_reps, qsel,
                     save_en, zero_bins, d_status);
}

void launch_newton(const RepDev* d_reps, int n_reps, int iters, int cold, int qsel, int save_en,
                   int zero_bins, double tol, uint32_t* d_status, hipStream_t stream) {
  if (n_reps <= 0) return;
  hipLaunchKernelGGL(k_newton, dim3(n_reps), dim3(kFieldThreads), 0, stream, d_reps, iters, cold,
                     qsel, save_en, zero_bins, tol, d_status);
}

void launch_prep_burst(const RepDev* d_reps, int n_reps, hipStream_t stream) {
  hipLaunchKernelGGL(k_prep_burst, dim3(n_reps), dim3(256), 0, stream, d_reps);
}

}  // namespace efpi
