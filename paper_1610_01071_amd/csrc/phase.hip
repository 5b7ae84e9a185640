// Phase-space coarse variables of the wavelet-based scheme (Sec. 3.3, App. A):
// the ions' CIC-in-x, nearest-bin-in-v histogram after l full-weighting levels,
// accumulated exactly in int64, then the periodized wavelet transform of every
// velocity column down to 2^jc scaling coefficients.
//
// Full weighting composes, over l levels, into a hat: fine node i = 2^l K + d
// contributes (2^l - d) / 4^l to coarse node K and d / 4^l to K + 1.  An ion's
// two CIC shares therefore reach at most three coarse nodes, with integer
// weights over the implicit denominator 4^l, so the histogram is exact and does
// not depend on the order of the atomics.  Work items of cell-ordered ions
// accumulate in an LDS window of coarse nodes around their first ion (the
// co-evolving shift tau v moves ions by a few coarse cells at most); anything
// outside the window goes straight to the global histogram.
#include <cmath>

#include "efpi_internal.h"

namespace efpi {
namespace {

constexpr int kPhThreads = 256;
constexpr int kPhTile = 4096;  // ions per work item
constexpr int kPhWin = 8;      // coarse x nodes of a work item's LDS window

struct PhaseHistArg {
  double v_min, inv_dv;
  float tau;
  int levels, n_vf, win, fresh;
};

__global__ __launch_bounds__(kPhThreads) void k_phase_hist(const RepDev* __restrict__ reps,
                                                           int rep, PhaseHistArg a,
                                                           long long* __restrict__ hist) {
  extern __shared__ long long s_h[];  // [win][n_vf]
  const RepDev& R = reps[rep];
  const int n = R.n_cells;
  const int nmask = n - 1;
  const int nxc = n >> a.levels;
  const int span = 1 << a.levels;
  const int64_t np = *gmem(R.np);
  const int64_t items = (np + kPhTile - 1) / kPhTile;
  const EFPI_GLOBAL float* __restrict__ e = gmem(R.e);
  const EFPI_GLOBAL int16_t* __restrict__ cellp = gmem(R.cell);
  const EFPI_GLOBAL float* __restrict__ fracp = gmem(R.frac);
  const EFPI_GLOBAL float* __restrict__ velp = gmem(R.v);
  const EFPI_GLOBAL float* __restrict__ wp = gmem(R.w);
  const float half_dt = 0.5f * (float)R.dt;
  const float tau_inv_h = a.tau * (float)R.inv_h;
  const int cells = a.win * a.n_vf;
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
    const int64_t i0 = item * kPhTile;
    const int64_t i1 = min(i0 + (int64_t)kPhTile, np);
    const int c_first = min(max((int)cellp[i0], 0), nmask);
    const int base = ((c_first >> a.levels) - a.win / 2 + 1 + nxc) % nxc;
    for (int k = threadIdx.x; k < cells; k += kPhThreads) s_h[k] = 0;
    __syncthreads();
    auto add = [&](int K, int kv, long long val) {
      const int slot = (K - base + nxc) % nxc;
      if (slot < a.win)
        atomicAdd(reinterpret_cast<unsigned long long*>(&s_h[slot * a.n_vf + kv]),
                  (unsigned long long)val);
      else
        atomicAdd(reinterpret_cast<unsigned long long*>(&hist[(int64_t)K * a.n_vf + kv]),
                  (unsigned long long)val);
    };
    auto node_share = [&](int node, int kv, long long s) {
      const int K = node >> a.levels;
      const int d = node & (span - 1);
      add(K, kv, s * (long long)(span - d));
      if (d) add(K + 1 == nxc ? 0 : K + 1, kv, s * (long long)d);
    };
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kPhThreads) {
      const int c = cellp[i];
      if (c < 0 || c >= n) continue;
      const float f = fracp[i];
      const float w = wp[i];
      float v = velp[i];
      float ep = 0.f;
      if (!a.fresh || a.tau != 0.f) ep = (1.f - f) * e[c] + f * e[(c + 1) & nmask];
      if (!a.fresh) v += half_dt * ep;  // time-centred velocity after a burst
      // co-evolving frame: X + tau v, V = v + tau E(X) (App. B)
      const float xs = f + tau_inv_h * v;
      const float fl = floorf(xs);
      const bool wrap_up = (xs - fl) >= 1.f;
      const float fn = wrap_up ? 0.f : xs - fl;
      const int cn = (c + (int)fl + (wrap_up ? 1 : 0)) & nmask;
      const float vt = v + a.tau * ep;
      const double bin = floor(((double)vt - a.v_min) * a.inv_dv);
      if (!(bin >= 0.0 && bin < (double)a.n_vf)) continue;
      const int kv = (int)bin;
      const double q = __builtin_rint((double)w * kFxScale);
      const double qr = __builtin_rint((double)fn * q);
      node_share(cn, kv, (long long)(q - qr));
      node_share((cn + 1) & nmask, kv, (long long)qr);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < cells; k += kPhThreads) {
      const long long val = s_h[k];
      if (val != 0) {
        const int K = (base + k / a.n_vf) % nxc;
        atomicAdd(reinterpret_cast<unsigned long long*>(&hist[(int64_t)K * a.n_vf + k % a.n_vf]),
                  (unsigned long long)val);
      }
    }
    __syncthreads();  // the window is reused by the next work item
  }
}

struct PhaseDwtArg {
  double scale;  // histogram value -> finest scaling coefficient
  int n_vf, levels_v, n_taps;
  double taps[16];
};

// One workgroup per coarse x node: the column in LDS, levels_v levels of the
// periodized low-pass filter a_k = sum_m h_m x_{(2k + m) mod N}.
__global__ __launch_bounds__(kPhThreads) void k_phase_dwt(const long long* __restrict__ hist,
                                                          PhaseDwtArg a,
                                                          double* __restrict__ out) {
  extern __shared__ double s_col[];  // [2][n_vf]
  const int K = blockIdx.x;
  double* cur = s_col;
  double* nxt = s_col + a.n_vf;
  for (int k = threadIdx.x; k < a.n_vf; k += kPhThreads)
    cur[k] = (double)hist[(int64_t)K * a.n_vf + k] * a.scale;
  __syncthreads();
  int len = a.n_vf;
  for (int lev = 0; lev < a.levels_v; ++lev) {
    const int half = len >> 1;
    for (int k = threadIdx.x; k < half; k += kPhThreads) {
      double acc = 0.0;
      for (int m = 0; m < a.n_taps; ++m) acc += a.taps[m] * cur[(2 * k + m) & (len - 1)];
      nxt[k] = acc;
    }
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
    len = half;
  }
  for (int k = threadIdx.x; k < len; k += kPhThreads) out[(int64_t)K * len + k] = cur[k];
}

}  // namespace

void launch_phase_restrict(const RepDev* d_reps, int rep, int n_cells, int levels_x, double v_min,
                           double v_max, int jf, int jc, const double* h_taps, int n_taps,
                           double tau, int fresh, double h, long long* d_hist, double* d_out,
                           hipStream_t stream) {
  const int n_vf = 1 << jf;
  const int nxc = n_cells >> levels_x;
  PhaseHistArg ha;
  ha.v_min = v_min;
  ha.inv_dv = (double)n_vf / (v_max - v_min);
  ha.tau = (float)tau;
  ha.levels = levels_x;
  ha.n_vf = n_vf;
  ha.win = nxc < kPhWin ? nxc : kPhWin;
  ha.fresh = fresh;
  launch_fill_u8(d_hist, sizeof(long long) * (size_t)nxc * n_vf, stream);
  const size_t lds = sizeof(long long) * (size_t)ha.win * n_vf;
  hipLaunchKernelGGL(k_phase_hist, dim3(2048), dim3(kPhThreads), lds, stream, d_reps, rep, ha,
                     d_hist);
  PhaseDwtArg da;
  const double dv = (v_max - v_min) / n_vf;
  da.scale = kFxInv / ((double)(1LL << (2 * levels_x)) * h * dv) * std::pow(2.0, -0.5 * jf) *
             (v_max - v_min);
  da.n_vf = n_vf;
  da.levels_v = jf - jc;
  da.n_taps = n_taps;
  for (int m = 0; m < 16; ++m) da.taps[m] = m < n_taps ? h_taps[m] : 0.0;
  hipLaunchKernelGGL(k_phase_dwt, dim3(nxc), dim3(kPhThreads), sizeof(double) * 2 * n_vf, stream,
                     d_hist, da, d_out);
}

}  // namespace efpi
