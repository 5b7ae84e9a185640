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
// At 2^8 bins, 2048 ions per work item and a window of 4 coarse nodes: 34 us per
// restriction of 4,096,000 ions against 41 us at 4096 ions and 8 nodes (the result
// is the same integer histogram for any tile and window)
constexpr int kPhTile = 2048;  // ions per work item (at least)
constexpr int kPhWin = 4;      // coarse x nodes of a work item's LDS window (at most)
constexpr int kPhGrid = 8192;  // workgroups, striding over the work items
// Histogram workgroups of 512 threads: at 2^11 bins (a 48 KB window, three
// workgroups per CU) 47 us per restriction of 4,096,000 ions against 59 us with
// 256 threads; at 2^8 bins the same (33 us); 1024 threads: 47 and 41 us.  (Since
// the ion loop lost its integer divisions and issues its field gathers first:
// 41 us at 2^11 bins, 28 us at 2^8.)
#ifndef EFPI_HIST_THREADS
#define EFPI_HIST_THREADS 512
#endif
constexpr int kHistThreads = EFPI_HIST_THREADS;
static_assert(kPhWin * 2048 * sizeof(long long) <= 65536, "window of 2^11 bins over 64 KB");

struct PhaseHistArg {
  double v_min, inv_dv;
  float tau;
  int levels, n_vf, win, tile, fresh, stored_field;
};

__global__ __launch_bounds__(kHistThreads) void k_phase_hist(const RepDev* __restrict__ reps,
                                                           int rep, PhaseHistArg a,
                                                           long long* __restrict__ hist) {
  extern __shared__ long long s_h[];  // [win][n_vf]
  const RepDev& R = reps[rep];
  const int n = R.n_cells;
  const int nmask = n - 1;
  const int nxc = n >> a.levels;
  const int span = 1 << a.levels;
  const int64_t np = *gmem(R.np);
  const int64_t items = (np + a.tile - 1) / a.tile;
  const EFPI_GLOBAL float* __restrict__ e = gmem(R.e);
  const EFPI_GLOBAL float* __restrict__ en_ = gmem(R.en);
  const EFPI_GLOBAL int16_t* __restrict__ cellp = gmem(R.cell);
  const EFPI_GLOBAL float* __restrict__ fracp = gmem(R.frac);
  const EFPI_GLOBAL float* __restrict__ velp = gmem(R.v);
  const EFPI_GLOBAL float* __restrict__ wp = gmem(R.w);
  const float half_dt = 0.5f * (float)R.dt;
  const float tau_inv_h = a.tau * (float)R.inv_h;
  const int cells = a.win * a.n_vf;
  const int lvf = __builtin_ctz(a.n_vf);
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
    const int64_t i0 = item * a.tile;
    const int64_t i1 = min(i0 + (int64_t)a.tile, np);
    const int c_first = min(max((int)cellp[i0], 0), nmask);
    const int base = ((c_first >> a.levels) - a.win / 2 + 1 + nxc) % nxc;
    for (int k = threadIdx.x; k < cells; k += kHistThreads) s_h[k] = 0;
    __syncthreads();
    // no integer division in the ion loop: K and base lie in [0, nxc)
    auto add = [&](int K, int kv, long long val) {
      int slot = K - base;
      if (slot < 0) slot += nxc;
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
    const bool need_e = !a.fresh || a.tau != 0.f;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kHistThreads) {
      // every load of the ion, its field gathers included, is issued before the
      // ion is tested (an ion outside the grid gathers at node 0 and is skipped)
      const int c = cellp[i];
      const float f = fracp[i];
      const float w = wp[i];
      float v = velp[i];
      const int cc = (c >= 0 && c < n) ? c : 0;
      const float e0 = need_e ? e[cc] : 0.f;
      const float e1 = need_e ? e[(cc + 1) & nmask] : 0.f;
      const float n0 = a.stored_field ? en_[cc] : 0.f;
      const float n1 = a.stored_field ? en_[(cc + 1) & nmask] : 0.f;
      if (c < 0 || c >= n) continue;
      float ep = 0.f;
      if (need_e) ep = (1.f - f) * e0 + f * e1;
      if (!a.fresh) v += half_dt * ep;  // time-centred velocity after a burst
      // co-evolving frame: X + tau v, V = v + tau E_n(X) (App. B), E_n the field
      // stored at the burst start or the current one
      const float en = a.stored_field ? (1.f - f) * n0 + f * n1 : ep;
      const float xs = f + tau_inv_h * v;
      const float fl = floorf(xs);
      const bool wrap_up = (xs - fl) >= 1.f;
      const float fn = wrap_up ? 0.f : xs - fl;
      const int cn = (c + (int)fl + (wrap_up ? 1 : 0)) & nmask;
      const float vt = v + a.tau * en;
      const double bin = floor(((double)vt - a.v_min) * a.inv_dv);
      if (!(bin >= 0.0 && bin < (double)a.n_vf)) continue;
      const int kv = (int)bin;
      const double q = __builtin_rint((double)w * kFxScale);
      const double qr = __builtin_rint((double)fn * q);
      node_share(cn, kv, (long long)(q - qr));
      node_share((cn + 1) & nmask, kv, (long long)qr);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < cells; k += kHistThreads) {
      const long long val = s_h[k];
      if (val != 0) {
        int K = base + (k >> lvf);  // n_vf = 2^lvf; a window slot is below win <= nxc
        if (K >= nxc) K -= nxc;
        atomicAdd(reinterpret_cast<unsigned long long*>(&hist[(int64_t)K * a.n_vf +
                                                             (k & (a.n_vf - 1))]),
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

// ------------------------------------------------------------------ lift --
// The lift repeats the oracle's arithmetic operation by operation (the CDF
// repair takes decisions on compared sums), so nothing here is contracted into
// fused multiply-adds.
#pragma clang fp contract(off)
// Columns of the coarse nodes back at J_f with zero details: level by level,
// x_t = sum over taps m = t (mod 2), in ascending m, of h_m a_{((t - m) / 2) mod N/2},
// then scaled to the phase-space density.
__global__ __launch_bounds__(kPhThreads) void k_phase_refine(const double* __restrict__ coarse,
                                                            PhaseDwtArg a, double up_scale,
                                                            double* __restrict__ cols) {
  extern __shared__ double s_col[];  // [2][n_vf]
  const int K = blockIdx.x;
  double* cur = s_col;
  double* nxt = s_col + a.n_vf;
  int len = a.n_vf >> a.levels_v;
  for (int k = threadIdx.x; k < len; k += kPhThreads) cur[k] = coarse[(int64_t)K * len + k];
  __syncthreads();
  for (int lev = 0; lev < a.levels_v; ++lev) {
    const int n2 = 2 * len;
    for (int t = threadIdx.x; t < n2; t += kPhThreads) {
      double acc = 0.0;
      for (int m = 0; m < a.n_taps; ++m) {
        const int r = t - m;
        if (r & 1) continue;
        const int k = (r & (n2 - 1)) >> 1;  // r mod n2 (n2 a power of two, r >= -15)
        acc = acc + a.taps[m] * cur[k];
      }
      nxt[t] = acc;
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
    len = n2;
  }
  for (int k = threadIdx.x; k < a.n_vf; k += kPhThreads)
    cols[(int64_t)K * a.n_vf + k] = up_scale * cur[k];
}

// The repair of App. C below runs on a whole wave over one node's LDS arrays.
// Every search that the method defines as "the first index in a given order with
// a property" tests 64 candidates at once and takes the first set lane of the
// ballot; each candidate is computed with the same operations as in a sequential
// scan, so the chosen index and every stored value are those of the sequential
// method.  Sums over the array stay sequential in index order (the same on all
// lanes, from broadcast LDS reads), since the method's decisions compare them.

// s + A[lo] + A[lo + 1] + ... + A[hi - 1], added in index order; the loads are
// issued eight at a time ahead of the additions.
__device__ double seq_sum(const double* A, int lo, int hi, double s) {
  int k = lo;
  for (; k + 8 <= hi; k += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = A[k + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) s = s + v[u];
  }
  for (; k < hi; ++k) s = s + A[k];
  return s;
}

// Index of the first set lane of a ballot (m != 0).
__device__ __forceinline__ int first_lane(unsigned long long m) { return __ffsll(m) - 1; }

// Edge reconstruction of App. C for entries below 0 of the array A[0..nf]: k0 is
// the last negative entry; for each right end kp rising from k0 + 1 the first left
// end km (falling from k0 - 1 to 0) whose momentum-conserving ramp from 0 stays in
// [0, A[kp]] is taken; the right end nf is taken unconditionally.
__device__ void edge_low(double* A, int nf, int lane) {
  int k0 = -1;
  for (int top = nf; top >= 0; top -= kWave) {
    const int k = top - lane;
    const unsigned long long m = __ballot(k >= 0 && A[k] < 0.0);
    if (m) {
      k0 = top - first_lane(m);
      break;
    }
  }
  if (k0 < 0) return;
  // A[1] + ... + A[kp - 1] in index order, one term more per step of kp
  double sum = seq_sum(A, 1, k0 + 1, 0.0);
  const int n_cand = k0 >= 1 ? k0 : 1;  // km = k0 - 1 - j, j < n_cand (km = -1 if k0 = 0)
  int km = k0 - 1, kp = k0 + 1;
  for (;; ++kp) {
    if (kp >= nf) {
      km = k0 - 1;
      break;
    }
    bool found = false;
    for (int j0 = 0; j0 < n_cand; j0 += kWave) {
      const int j = j0 + lane;
      bool ok = false;
      if (j < n_cand) {
        const int span = kp - (k0 - 1 - j);
        const double d = 2.0 * sum / (double)(span * (span - 1));
        ok = 0.0 <= (span - 1) * d && (span - 1) * d <= A[kp];
      }
      const unsigned long long m = __ballot(ok);
      if (m) {
        km = k0 - 1 - (j0 + first_lane(m));
        found = true;
        break;
      }
    }
    if (found) break;
    sum = sum + A[kp];
  }
  const int span = kp - km;
  const double dF = 2.0 * sum / (double)(span * (span - 1));
  const int k_lo = km > 0 ? km : 0;
  __syncthreads();  // every lane has read A before any lane writes the ramp
  for (int k = lane; k < kp; k += kWave) A[k] = k < k_lo ? 0.0 : (k - km) * dF;
  __syncthreads();
}

// Interior reconstruction of App. C from the lower indexes on A[0..nf]: at each
// first decrease k0 the ramp starts at k_- (the last earlier entry not above
// A[k_+]) and ends at k_+ (the first minimum before the array climbs back to
// A[k0]), and k_+ moves right until the momentum-conserving ramp is monotone.
__device__ void interior_forward(double* A, int nf, int lane) {
  int k0 = 0;
  while (true) {
    int j = -1;
    for (int b = k0; b < nf; b += kWave) {
      const int k = b + lane;
      const unsigned long long m = __ballot(k < nf && A[k] > A[k + 1]);
      if (m) {
        j = b + first_lane(m);
        break;
      }
    }
    if (j < 0) return;
    k0 = j;
    const double fk0 = A[k0];
    int k1 = nf;
    for (int b = k0 + 1; b <= nf; b += kWave) {
      const int k = b + lane;
      const unsigned long long m = __ballot(k <= nf && A[k] >= fk0);
      if (m) {
        k1 = b + first_lane(m);
        break;
      }
    }
    // first index of the minimum over [k0 + 1, k1]: (value, index) reduced over the wave
    double best = A[k0 + 1];
    int at = k0 + 1;
    for (int k = k0 + 1 + lane; k <= k1; k += kWave) {
      const double a = A[k];
      if (a < best || (a == best && k < at)) {
        best = a;
        at = k;
      }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oa = __shfl_xor(at, off);
      if (ob < best || (ob == best && oa < at)) {
        best = ob;
        at = oa;
      }
    }
    int kp = at;
    const double fkp = A[kp];
    int km = 0;
    for (int top = k0 - 1; top >= 0; top -= kWave) {
      const int k = top - lane;
      const unsigned long long m = __ballot(k >= 0 && A[k] <= fkp);
      if (m) {
        km = top - first_lane(m);
        break;
      }
    }
    // sum of A[km .. kp - 1] in index order, extended by one term as kp moves right.
    // The lanes test the next 64 right ends at once: lane l takes kp + l with the sum
    // extended term by term up to it (the sequential sums, bit for bit), and the first
    // lane whose ramp is monotone, or that reaches nf, decides.
    double dF, sum = seq_sum(A, km, kp, 0.0);
    const double akm = A[km];
    while (true) {
      const int kq = kp + lane;
      const bool valid = kq <= nf;  // the method never moves kp past nf
      double s = sum;
      for (int t = kp; t < kq && valid; ++t) s = s + A[t];
      bool ok = false;
      double d = 0.0;
      if (valid) {
        const int span = kq - km;
        d = 2.0 / (span - 1) * (s / span - akm);
        ok = 0.0 <= (span - 1) * d && akm + (span - 1) * d <= A[kq];
      }
      const unsigned long long m = __ballot(valid && (ok || kq >= nf));
      if (m) {
        const int l = first_lane(m);
        const bool ok_l = __shfl(ok ? 1 : 0, l) != 0;
        dF = __shfl(d, l);
        kp += l;
        if (!ok_l) {  // kp = nf without a monotone ramp: the straight line to A[nf]
          dF = (A[nf] - akm) / (nf - km);
          kp = nf;
        }
        break;
      }
      // no lane stopped: all 64 right ends lie below nf
      sum = __shfl(s, kWave - 1) + A[kp + kWave - 1];
      kp += kWave;
    }
    const double base = A[km];
    __syncthreads();
    for (int k = km + 1 + lane; k < kp; k += kWave) A[k] = base + (k - km) * dF;
    __syncthreads();
    k0 = kp;
  }
}

// One wave per fine node, the node's array in LDS: the lanes build the column
// from its two coarse columns by l levels of midpoint interpolation (eq. 3.7);
// lane 0 takes the density and CDF sums in index order; the repair of App. C
// follows (edges, forward and backward interior passes, averaged) on the whole
// wave.  One LDS array of n_vf + 1 doubles serves every stage (the reflections
// are done in place), so nine workgroups share a CU: the edge-repaired CDF is
// kept in registers (entry k in lane k mod 64) for the backward pass, and the
// forward pass's result goes to rf and is read back for the average.  The
// lanes write the repaired CDF rf[i][0..n_vf] and lane 0 the density to
// R.prof_n.
constexpr int kMaxVfPerLane = ((1 << 11) + 1 + kWave - 1) / kWave;  // n_vf <= 2^11

__device__ __forceinline__ void reflect_in_place(double* A, int nf, int lane) {
  // A[k] <- 1 - A[nf - k] for every k, as one reads and one writes per pair
  for (int k = lane; 2 * k <= nf; k += kWave) {
    const double a = A[k], b = A[nf - k];
    A[k] = 1.0 - b;
    A[nf - k] = 1.0 - a;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kWave) void k_phase_cdf(const RepDev* __restrict__ reps, int rep,
                                                    const double* __restrict__ cols, int levels,
                                                    int n_vf, double dv,
                                                    double* __restrict__ rf) {
  extern __shared__ double s_cdf[];  // [n_vf + 1]: the column at 1..n_vf, then the CDF
  const RepDev& R = reps[rep];
  const int n = R.n_cells;
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const int nf = n_vf;
  double* sA = s_cdf;
  const int nxc = n >> levels;
  const int K = i >> levels;
  const int K1 = K + 1 == nxc ? 0 : K + 1;
  for (int k = lane; k < nf; k += kWave) {
    double A = cols[(int64_t)K * nf + k];
    double B = cols[(int64_t)K1 * nf + k];
    for (int j = levels - 1; j >= 0; --j) {  // bits of i below the coarse node, top first
      const double mid = 0.5 * (A + B);
      if ((i >> j) & 1) A = mid;
      else B = mid;
    }
    sA[k + 1] = A;
  }
  __syncthreads();
  __shared__ double s_dens;
  if (lane == 0) {
    double run = 0.0;
    for (int k = 0; k < nf; k += 8) {  // nf is a power of two >= 16
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = sA[k + u + 1];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        run = run + v[u];
        sA[k + u + 1] = run;
      }
    }
    const double dens = run * dv;
    s_dens = dens;
    gmem(R.prof_n)[i] = dens;
  }
  __syncthreads();
  const double dens = s_dens;
  if (!(dens > R.n_floor)) return;  // the same for every lane of the workgroup
  // normalisation on all lanes; the repair below runs on the whole wave
  for (int k = 1 + lane; k < nf; k += kWave) sA[k] = (sA[k] * dv) / dens;
  if (lane == 0) {
    sA[0] = 0.0;
    sA[nf] = 1.0;
  }
  __syncthreads();
  edge_low(sA, nf, lane);  // entries below 0
  // entries above 1: the same rule on the reflected array
  reflect_in_place(sA, nf, lane);
  edge_low(sA, nf, lane);
  reflect_in_place(sA, nf, lane);
  // the edge-repaired CDF, kept for the backward pass
  double e0[kMaxVfPerLane];
#pragma unroll
  for (int j = 0; j < kMaxVfPerLane; ++j) {
    const int k = lane + j * kWave;
    e0[j] = k <= nf ? sA[k] : 0.0;
  }
  // forward pass in place; its result goes to rf
  interior_forward(sA, nf, lane);
  double* out = rf + (int64_t)i * (nf + 1);
  for (int k = lane; k <= nf; k += kWave) out[k] = sA[k];
  __syncthreads();  // every lane has read the forward pass before the array is refilled
  // backward pass on the reflection of the edge-repaired CDF
#pragma unroll
  for (int j = 0; j < kMaxVfPerLane; ++j) {
    const int k = lane + j * kWave;
    if (k <= nf) sA[nf - k] = 1.0 - e0[j];
  }
  __syncthreads();
  interior_forward(sA, nf, lane);
  for (int k = lane; k <= nf; k += kWave) out[k] = 0.5 * (out[k] + (1.0 - sA[nf - k]));
}

// v with RF(v) = b in node i's repaired CDF rf[i][0..nf]: the last bin k with
// RF[k] <= b (binary search), linear inside it.
__device__ double inverse_cdf(const double* F, int nf, double b, double v_min, double dv) {
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (F[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const double f0 = F[lo], f1 = F[lo + 1];
  const double t = f1 > f0 ? (b - f0) / (f1 - f0) : 0.5;
  return v_min + (lo + t) * dv;
}

// Quiet start from the repaired CDFs: ion m of occupied cell c (rank order) at
// offset (m + 1/2)/ppc, velocity the inverse CDFs of the cell's two nodes at the
// Hammersley b, interpolated in x, weight n(X) h / ppc.  One workgroup per
// occupied cell stages the two nodes' CDFs in LDS for its ions' binary searches.
__global__ __launch_bounds__(kPhThreads) void k_phase_load(const RepDev* __restrict__ reps,
                                                          int rep, const double* __restrict__ rf,
                                                          int n_vf, double v_min, double dv,
                                                          uint32_t shift) {
  extern __shared__ double s_rf[];  // CDFs of the cell's left and right node: 2 x (n_vf + 1)
  const RepDev& R = reps[rep];
  const int n = R.n_cells;
  const int nf = n_vf;
  const int ppc = R.ppc;
  const int64_t total = *gmem(R.np);
  const int64_t ranks = (total + ppc - 1) / ppc;
  const auto prof_n = gmem(R.prof_n);
  const auto cell_of_rank = gmem(R.cell_of_rank);
  double* FL = s_rf;
  double* FR = s_rf + (nf + 1);
  for (int64_t r = blockIdx.x; r < ranks; r += gridDim.x) {
    const int c = cell_of_rank[r];
    const int cr = (c + 1) & (n - 1);
    const double nl = prof_n[c], nr = prof_n[cr];
    const bool okl = nl > R.n_floor, okr = nr > R.n_floor;
    __syncthreads();  // the previous cell's rows are no longer read
    for (int k = threadIdx.x; k <= nf; k += kPhThreads) {
      if (okl) FL[k] = rf[(int64_t)c * (nf + 1) + k];
      if (okr) FR[k] = rf[(int64_t)cr * (nf + 1) + k];
    }
    __syncthreads();
    for (int m = threadIdx.x; m < ppc; m += kPhThreads) {
      const int64_t j = r * ppc + m;
      if (j >= total) break;
      const float frac = (float)(((double)m + 0.5) / (double)ppc);
      const double th = (double)frac;
      const uint32_t idx = (uint32_t)c * (uint32_t)ppc + (uint32_t)m;
      const uint32_t u = __brev(idx) + shift;
      const double b = ((double)u + 0.5) * 2.3283064365386963e-10;  // 2^-32
      double vl = okl ? inverse_cdf(FL, nf, b, v_min, dv) : 0.0;
      double vr = okr ? inverse_cdf(FR, nf, b, v_min, dv) : vl;
      if (!okl) vl = vr;
      const double v = (1.0 - th) * vl + th * vr;
      const double nx = (1.0 - th) * fmax(nl, 0.0) + th * fmax(nr, 0.0);
      gmem(R.cell)[j] = (int16_t)c;
      gmem(R.frac)[j] = frac;
      gmem(R.v)[j] = (float)v;
      gmem(R.w)[j] = (float)(nx * R.h / ppc);
    }
  }
}

// Least squares over the snapshots (eq. 3.18) and forward-Euler projection
// (eq. 3.17) of arbitrary coefficient arrays snap[0..ne][count].
__global__ void k_phase_project(const double* __restrict__ snap, int64_t count, int ne, double dt,
                                double macro_dt, double* __restrict__ out) {
#pragma clang fp contract(off)
  const double den = (double)ne * (ne + 1) * (ne + 2) * dt;
  const double leap = macro_dt - ne * dt;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x) {
    double slope = 0.0;
    for (int p = 0; p <= ne / 2; ++p) {
      const double coef = 6.0 * (double)(ne - 2 * p) / den;
      slope += coef * (snap[(int64_t)(ne - p) * count + k] - snap[(int64_t)p * count + k]);
    }
    out[k] = snap[(int64_t)ne * count + k] + leap * slope;
  }
}

}  // namespace

void launch_phase_lift(const RepDev* d_reps, int rep, int n_cells, int levels_x, double v_min,
                       double v_max, int jf, int jc, const double* h_taps, int n_taps,
                       const double* d_coarse, double* d_cols, double* d_cdf,
                       uint32_t* d_status, uint32_t shift, hipStream_t stream) {
  const int n_vf = 1 << jf;
  const int nxc = n_cells >> levels_x;
  const double dv = (v_max - v_min) / n_vf;
  PhaseDwtArg da;
  da.scale = 0.0;
  da.n_vf = n_vf;
  da.levels_v = jf - jc;
  da.n_taps = n_taps;
  for (int m = 0; m < 16; ++m) da.taps[m] = m < n_taps ? h_taps[m] : 0.0;
  const double up_scale = std::pow(2.0, 0.5 * jf) / (v_max - v_min);
  hipLaunchKernelGGL(k_phase_refine, dim3(nxc), dim3(kPhThreads), sizeof(double) * 2 * n_vf,
                     stream, d_coarse, da, up_scale, d_cols);
  hipLaunchKernelGGL(k_phase_cdf, dim3(n_cells), dim3(kWave), sizeof(double) * (n_vf + 1),
                     stream, d_reps, rep, d_cols, levels_x, n_vf, dv, d_cdf);
  launch_occupancy(d_reps, 0, rep, d_status, stream);
  hipLaunchKernelGGL(k_phase_load, dim3(4096), dim3(kPhThreads), sizeof(double) * 2 * (n_vf + 1),
                     stream, d_reps, rep, d_cdf, n_vf, v_min, dv, shift);
}

void launch_phase_project(const double* d_snap, int64_t count, int ne, double dt, double macro_dt,
                          double* d_out, hipStream_t stream) {
  const int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_phase_project, dim3((unsigned)(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024)),
                     dim3(256), 0, stream, d_snap, count, ne, dt, macro_dt, d_out);
}

void launch_phase_restrict(const RepDev* d_reps, int rep, int n_cells, int levels_x, double v_min,
                           double v_max, int jf, int jc, const double* h_taps, int n_taps,
                           double tau, int fresh, int stored_field, double h, long long* d_hist,
                           double* d_out, hipStream_t stream) {
  const int n_vf = 1 << jf;
  const int nxc = n_cells >> levels_x;
  PhaseHistArg ha;
  ha.v_min = v_min;
  ha.inv_dv = (double)n_vf / (v_max - v_min);
  ha.tau = (float)tau;
  ha.levels = levels_x;
  ha.n_vf = n_vf;
  // the window's clear and flush grow with 2^jf, so wider columns take longer work
  // items: 4 x 2^jf ions, at least kPhTile (at 2^11 bins: 68 us per restriction with
  // 8192 ions and a 3-node window, against 88 us with 2048 ions)
  const int tile = 4 * n_vf > kPhTile ? 4 * n_vf : kPhTile;
  const int win = n_vf > 1024 ? 3 : kPhWin;
  ha.win = nxc < win ? nxc : win;
  ha.tile = tile;
  ha.fresh = fresh;
  ha.stored_field = stored_field;
  launch_fill_u8(d_hist, sizeof(long long) * (size_t)nxc * n_vf, stream);
  const size_t lds = sizeof(long long) * (size_t)ha.win * n_vf;
  hipLaunchKernelGGL(k_phase_hist, dim3(kPhGrid), dim3(kHistThreads), lds, stream, d_reps, rep, ha,
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
