// Coarse side of the projective cycle: lifting (Sec. 3.3 "Lifting", App. C
// particle loading), conversion of the restriction bins to Haar coefficients,
// least-squares projection (eqs. 3.17-3.18) and ensemble means.
#include "efpi_internal.h"

namespace efpi {
namespace {

// Lift workgroups: 256 threads, each keeping the velocity and weight of its first
// EFPI_LIFT_KEEP ions in registers between the correction sums and the stores.  A
// work item is one coarse block (a few thousand ions), so several workgroups per CU
// hide each other's dependent loads and barriers: on the 64-replica ensemble the
// lift takes 0.65 ms against 1.0 ms with 1024-thread workgroups.  The two-moment
// kernel is held to 96 VGPRs, so five waves share a SIMD (568 against 615 us on
// the ensemble, fused deposit included).
#ifndef EFPI_LIFT_KEEP
#define EFPI_LIFT_KEEP 8
#endif
#ifndef EFPI_LIFT_THREADS
#define EFPI_LIFT_THREADS 256
#endif
constexpr int kLiftThreads = EFPI_LIFT_THREADS;
constexpr int kProfThreads = 1024;

// Inverse standard normal CDF at the Hammersley coordinate b = (u + 1/2) 2^-32, in
// FP32 (the velocity is stored in FP32).  With p = min(b, 1 - b), x = 1 - 2p and
// w = -log(4 p (1 - p)), Phi^{-1}(b) = -/+ sqrt(2) x r(w) with r = erfinv(x) / x, a
// smooth function of w (the change of variable of Giles's erfinv approximation): a
// degree-9 polynomial in w - 2.5 for w < 5 and in sqrt(w) - 3 above, with
// coefficients fitted by least squares (fit_inverse_normal.py).  p and x come from
// the integers: p = (min(u, ~u) + 1/2) 2^-32 and x = |u - ~u| 2^-32, so neither tail
// loses precision in FP32; the result is within 1.3e-6 (3.6e-7 relative) of the
// exact value for every u.  The central polynomial is always evaluated; the tail
// one only in waves with a lane in a tail (w >= 5, about one point in 300: four
// waves in five skip it), which took the ensemble's lift from 556 to 542 us.
__device__ __forceinline__ float inv_normal(uint32_t u) {
  constexpr float kC[10] = {1.501409411e+00f, 2.466402948e-01f, -4.177389666e-03f,
                            -1.252748421e-03f, 2.183469187e-04f, -4.959743364e-06f,
                            -3.463356052e-06f, 4.654287409e-07f, 2.328584436e-08f,
                            -8.739831081e-09f};
  constexpr float kT[10] = {2.832977057e+00f, 1.001676440e+00f, 9.434493259e-03f,
                            -7.654667366e-03f, 5.764349364e-03f, -3.560388228e-03f,
                            1.293608337e-03f, -3.136037049e-05f, -1.542049431e-04f,
                            3.841022772e-05f};
  constexpr float k2m32 = 2.3283064365386963e-10f;  // 2^-32
  const uint32_t nu = ~u;
  const bool lower = u < nu;                       // b < 1/2
  const uint32_t lo = lower ? u : nu;
  const float p = ((float)lo + 0.5f) * k2m32;
  const float x = (float)(lower ? nu - u : u - nu) * k2m32;
  // 4 p (1 - p) >= 2^-31: log2 of the hardware is exact enough there
  const float w = -0.693147180560f * __builtin_amdgcn_logf(4.0f * p * (1.0f - p));
  const float tc = w - 2.5f;
  float rc = kC[9];
#pragma unroll
  for (int k = 8; k >= 0; --k) rc = fmaf(rc, tc, kC[k]);
  float r = rc;
  if (w >= 5.0f) {  // p < 0.0017: most waves have no such lane and skip the tail
    const float tt = __builtin_amdgcn_sqrtf(w) - 3.0f;
    float rt = kT[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) rt = fmaf(rt, tt, kT[k]);
    r = rt;
  }
  const float z = -1.41421356237f * x * r;
  return lower ? z : -z;
}

// ---------------------------------------------------------------- profile --
// Nodes of a replica (n_cells <= 16384, checked at init): the profile kernels keep
// one byte per node in LDS, "density above n_floor".
constexpr int kMaxNodes = 16385;

// Fine node density and mean velocity (and, with three moments, temperature)
// from the coarse coefficients: inverse Haar with zero details (block means
// 2^{-l/2} c_B), optionally linearly interpolated between block centres
// (periodic wrap; constant past the end centres on walls).  The temperature is
// T = s / n - u^2, clipped at 0, and 0 where the density is at most n_floor.
// s_above[k] records n_k > n_floor for the occupancy count.
__device__ void profile_of(const RepDev& R, const double* __restrict__ cn,
                           uint8_t* __restrict__ s_above) {
  const int nc = R.n_coarse;
  const double* cj = cn + nc;
  const bool third = R.moments == 3;
  const double* cs = third ? cn + 2 * nc : cn;  // second moments (read only with three)
  const int bs = 1 << R.levels;
  const double inv_s = 1.0 / sqrt((double)bs);
  const bool periodic = R.bc == 0;
#pragma unroll 4
  for (int k = threadIdx.x; k < R.n_nodes; k += blockDim.x) {
    int b0, b1;
    double w0, w1;
    if (!R.lift_linear) {
      b0 = b1 = min(k >> R.levels, nc - 1);
      w0 = 1.0;
      w1 = 0.0;
    } else {
      const double u = ((double)k - 0.5 * (bs - 1)) / (double)bs;
      const double fb = floor(u);
      b0 = (int)fb;
      const double th = u - fb;
      b1 = b0 + 1;
      w0 = 1.0 - th;
      w1 = th;
      if (periodic) {
        b0 &= nc - 1;  // nc is a power of two: the periodic index without dividing
        b1 &= nc - 1;
      } else {
        if (b0 < 0) { b0 = 0; b1 = 0; w0 = 1.0; w1 = 0.0; }
        if (b1 > nc - 1) { b0 = nc - 1; b1 = nc - 1; w0 = 1.0; w1 = 0.0; }
      }
    }
    const double dn = R.lift_linear ? (w0 * cn[b0] + w1 * cn[b1]) * inv_s : cn[b0] * inv_s;
    const double dj = R.lift_linear ? (w0 * cj[b0] + w1 * cj[b1]) * inv_s : cj[b0] * inv_s;
    const double nn = fmax(dn, 0.0);
    const bool ok = nn > R.n_floor;
    const double u = ok ? dj / nn : 0.0;
    gmem(R.prof_n)[k] = nn;
    gmem(R.prof_u)[k] = u;
    s_above[k] = ok ? 1 : 0;
    if (third) {
      const double ds = R.lift_linear ? (w0 * cs[b0] + w1 * cs[b1]) * inv_s : cs[b0] * inv_s;
      gmem(R.prof_t)[k] = ok ? fmax(ds / nn - u * u, 0.0) : 0.0;
    }
  }
}

// -------------------------------------------------------------- occupancy --
// A cell is occupied when one of its nodes exceeds n_floor (s_above, filled and
// synchronised by the caller).  Thread t takes a run of consecutive cells; an
// exclusive scan of the runs' counts (waves by shuffles, then the wave totals)
// gives each occupied cell its rank, and the lift puts ppc ions per rank.
__device__ void occupancy_of(const RepDev& R, uint32_t* __restrict__ status,
                             const uint8_t* __restrict__ s_above, int* __restrict__ s_wave) {
  const int n = R.n_cells;
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  const int wid = t / kWave;
  const int per = (n + kProfThreads - 1) / kProfThreads;
  const int c0 = t * per;
  const int c1 = min(c0 + per, n);
  const bool periodic = R.bc == 0;
  auto occupied = [&](int c) {
    const int cr = periodic ? ((c + 1) & (n - 1)) : c + 1;
    return (s_above[c] | s_above[cr]) != 0;
  };
  const auto block_rank = gmem(R.block_rank);
  const auto cell_of_rank = gmem(R.cell_of_rank);
  int cnt = 0;
  for (int c = c0; c < c1; ++c) cnt += occupied(c) ? 1 : 0;
  int inc = cnt;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) s_wave[wid] = inc;
  __syncthreads();
  int before = 0, total = 0;
  for (int k = 0; k < kProfThreads / kWave; ++k) {
    const int v = s_wave[k];
    before += k < wid ? v : 0;
    total += v;
  }
  const int64_t max_cells = R.capacity / R.ppc;
  int rank = before + inc - cnt;
  const int lmask = (1 << R.levels) - 1;
  for (int c = c0; c < c1; ++c) {
    if ((c & lmask) == 0) block_rank[c >> R.levels] = (int32_t)min((int64_t)rank, max_cells);
    if (occupied(c)) {
      if (rank < max_cells) cell_of_rank[rank] = c;
      ++rank;
    }
  }
  if (t == 0) {
    const int64_t kept = min((int64_t)total, max_cells);
    block_rank[R.n_coarse] = (int32_t)kept;
    *gmem(R.np) = kept * R.ppc;
    if (total > max_cells) atomicOr(status, 4u);
  }
}

__global__ __launch_bounds__(kProfThreads) void k_occupancy(const RepDev* __restrict__ reps,
                                                            int only_rep,
                                                            uint32_t* __restrict__ status) {
  __shared__ uint8_t s_above[kMaxNodes];
  __shared__ int s_wave[kProfThreads / kWave];
  const RepDev& R = reps[only_rep >= 0 ? only_rep : (int)blockIdx.x];
  const auto prof_n = gmem(R.prof_n);
  for (int k = threadIdx.x; k < R.n_nodes; k += blockDim.x) s_above[k] = prof_n[k] > R.n_floor;
  __syncthreads();
  occupancy_of(R, status, s_above, s_wave);
}

__global__ __launch_bounds__(kProfThreads) void k_lift_prep(const RepDev* __restrict__ reps,
                                                            const double* __restrict__ coarse,
                                                            const int64_t* __restrict__ coff,
                                                            uint32_t* __restrict__ status,
                                                            int set_shift, const ShiftArg shifts) {
  __shared__ uint8_t s_above[kMaxNodes];
  __shared__ int s_wave[kProfThreads / kWave];
  const RepDev& R = reps[blockIdx.x];
  profile_of(R, coarse + coff[blockIdx.x], s_above);
  __syncthreads();  // s_above is read by other threads below
  occupancy_of(R, status, s_above, s_wave);
  if (set_shift && threadIdx.x == 0) gmem(R.aux)[1] = (int64_t)shifts.s[blockIdx.x];
}

// ---------------------------------------------------------- lift particles --
// Standard normal deviate of ion m of cell c from its Hammersley point (quiet
// start): b = ((bitrev32(c ppc + m) + shift) mod 2^32 + 1/2) 2^-32.
__device__ __forceinline__ float normal_of(int c, int m, int ppc, uint32_t shift) {
  const uint32_t idx = (uint32_t)c * (uint32_t)ppc + (uint32_t)m;
  return inv_normal(__brev(idx) + shift);
}

__device__ __forceinline__ int right_node(const RepDev& R, int c) {
  return R.bc == 0 ? ((c + 1) & (R.n_cells - 1)) : c + 1;
}

// Occupied cells of a block staged in LDS (one round of loads per block), and
// the in-cell offsets (m + 1/2) / ppc as FP32 for ppc up to kFracTable.
constexpr int kLiftCache = 256;
constexpr int kFracTable = 4096;
// The lift's charge deposit: a block of 2^l cells touches 2^l + 1 nodes, held in
// LDS with 16 slots per node (threads t and t + 16k share one) as integer-valued
// binary64, as in the particle pass.
constexpr int kLiftNodes = 65;
#ifndef EFPI_LIFT_SLOTS
#define EFPI_LIFT_SLOTS 16
#endif
constexpr int kLiftSlots = EFPI_LIFT_SLOTS;

__device__ double block_sum(double x, double* s_red) {
  // fixed-order tree: waves by shuffles, then the wave totals in index order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[wid] = x;
  __syncthreads();
  double tot = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tot += s_red[k];
  return tot;
}

__device__ __forceinline__ int find_rep(const int64_t* prefix, int n, int64_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One work item per (replica, coarse block): generate the block's ions, and
// with coarse targets rescale weights to the block mass h 2^{l/2} max(c^n_B, 0)
// and shift velocities to the block momentum h 2^{l/2} c^j_B.  Ion j of the block
// is ion m = j mod ppc of its (j / ppc)-th occupied cell; thread t walks
// j = t, t + kLiftThreads, ... and steps (j / ppc, m) without dividing.  Offsets are
// (float)((m + 1/2) / ppc); n and u are linear in the cell from its two nodes;
// v = u + vth z, w = n h / ppc, formed in FP32 (the stored precision), summed
// over the block in binary64 in a fixed order.  With three coarse moments and
// coarse targets, the thermal speed is sqrt(T) with T linear in the cell, and the
// velocities are also stretched about the block's mean velocity u_g: v <- a v +
// (J / M - a u_g), a = sqrt(max(S - J^2 / M, 0) / G), G = sum w (v - u_g)^2 of the
// rescaled weights, so that sum w v^2 meets the block's second moment S = h 2^{l/2}
// c^s_B (a = 1 without spread).  With qsel >= 0 (every replica's
// blocks of at most 64 cells) the ions' charge is deposited into R.q[qsel] as the
// particle pass deposits it (the same fixed-point shares of the stored w and
// offset), so the burst needs no separate deposit pass.
template <bool kThird>
__global__ __launch_bounds__(kLiftThreads) __attribute__((amdgpu_waves_per_eu(kThird ? 4 : 5)))
void k_lift(const RepDev* __restrict__ reps,
                                                       const int64_t* __restrict__ block_prefix,
                                                       int n_reps, int64_t total, int only_rep,
                                                       const double* __restrict__ coarse,
                                                       const int64_t* __restrict__ coff,
                                                       int qsel, uint32_t* __restrict__ status) {
  __shared__ double s_red[kLiftThreads / 64];
  __shared__ double s_q[kLiftNodes][kLiftSlots];
  __shared__ int s_c[kLiftCache];
  __shared__ float s_nl[kLiftCache], s_dn[kLiftCache], s_ul[kLiftCache], s_du[kLiftCache];
  __shared__ float s_tl[kLiftCache], s_dt[kLiftCache];
  __shared__ float s_frac[kFracTable];
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int r = only_rep >= 0 ? only_rep : find_rep(block_prefix, n_reps, item);
    const RepDev& R = reps[r];
    const int B = (int)(item - (only_rep >= 0 ? 0 : R.block_begin));
    const auto block_rank = gmem(R.block_rank);
    const auto cell_of_rank = gmem(R.cell_of_rank);
    const auto prof_n = gmem(R.prof_n);
    const auto prof_u = gmem(R.prof_u);
    const auto prof_t = gmem(R.prof_t);
    constexpr bool third = kThird;  // thermal speed from T (three moments, coarse targets)
    const int rb0 = block_rank[B];
    const int rb1 = block_rank[B + 1];
    const int ppc = R.ppc;
    const int count = (rb1 - rb0) * ppc;  // at most 2^l cells * ppc < 2^31 (checked at init)
    const int64_t slot0 = (int64_t)rb0 * ppc;
    const uint32_t shift = (uint32_t)gmem(R.aux)[1];  // Cranley-Patterson rotation of this lift
    const int ncell = rb1 - rb0;
    const bool cached = ncell <= kLiftCache;
    const bool table = ppc <= kFracTable;
    const float vth = (float)R.vth;
    const float hp = (float)(R.h / (double)ppc);
    if (cached) {
      for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int c = cell_of_rank[rb0 + k];
        const int cr = right_node(R, c);
        const float nl = (float)prof_n[c], ul = (float)prof_u[c];
        s_c[k] = c;
        s_nl[k] = nl;
        s_dn[k] = (float)prof_n[cr] - nl;
        s_ul[k] = ul;
        s_du[k] = (float)prof_u[cr] - ul;
        if (third) {
          const float tl = (float)prof_t[c];
          s_tl[k] = tl;
          s_dt[k] = (float)prof_t[cr] - tl;
        }
      }
    }
    if (table)
      for (int m = threadIdx.x; m < ppc; m += blockDim.x)
        s_frac[m] = (float)(((double)m + 0.5) / (double)ppc);
    const bool dep = qsel >= 0;
    if (dep)
      for (int k = threadIdx.x; k < kLiftNodes * kLiftSlots; k += blockDim.x) (&s_q[0][0])[k] = 0.0;
    __syncthreads();
    // the thread's first ion and its stride, as (cell rank, index in the cell)
    const int q0 = (int)threadIdx.x / ppc, m0 = (int)threadIdx.x - q0 * ppc;
    const int qs = kLiftThreads / ppc, ms = kLiftThreads - qs * ppc;
    auto advance = [&](int& jr, int& m) {
      jr += qs;
      m += ms;
      if (m >= ppc) {
        m -= ppc;
        ++jr;
      }
    };
    auto cell_at = [&](int jr) { return cached ? s_c[jr] : cell_of_rank[rb0 + jr]; };
    auto offset_at = [&](int m) {
      return table ? s_frac[m] : (float)(((double)m + 0.5) / (double)ppc);
    };
    // ion (jr, m) of cell c at offset fr: velocity and weight before the correction
    auto ion = [&](int jr, int c, int m, float fr, float& v, float& w) {
      float nl, dn, ul, du, sig = vth;
      if (cached) {
        nl = s_nl[jr];
        dn = s_dn[jr];
        ul = s_ul[jr];
        du = s_du[jr];
        if (third) sig = sqrtf(fmaxf(fmaf(fr, s_dt[jr], s_tl[jr]), 0.0f));
      } else {
        const int cr = right_node(R, c);
        nl = (float)prof_n[c];
        dn = (float)prof_n[cr] - nl;
        ul = (float)prof_u[c];
        du = (float)prof_u[cr] - ul;
        if (third) {
          const float tl = (float)prof_t[c];
          sig = sqrtf(fmaxf(fmaf(fr, (float)prof_t[cr] - tl, tl), 0.0f));
        }
      }
      v = fmaf(sig, normal_of(c, m, ppc, shift), fmaf(fr, du, ul));
      w = fmaf(fr, dn, nl) * hp;
    };
    // the first kKeep ions of every thread keep (v, w) in registers
    constexpr int kKeep = EFPI_LIFT_KEEP;
    float keep_v[kKeep], keep_w[kKeep];
    float ratio = 1.0f, stretch = 1.0f, dv = 0.0f;
    if (coarse != nullptr) {
      double sw = 0.0, swv = 0.0, swvv = 0.0;
      int jr = q0, m = m0;
#pragma unroll
      for (int k = 0; k < kKeep; ++k) {
        if ((int)threadIdx.x + k * kLiftThreads < count) {
          ion(jr, cell_at(jr), m, offset_at(m), keep_v[k], keep_w[k]);
          sw += (double)keep_w[k];
          swv += (double)keep_w[k] * (double)keep_v[k];
          if (third) swvv += (double)keep_w[k] * (double)keep_v[k] * (double)keep_v[k];
        }
        advance(jr, m);
      }
#pragma unroll 1
      for (int j = threadIdx.x + kKeep * kLiftThreads; j < count; j += kLiftThreads) {
        float v, w;
        ion(jr, cell_at(jr), m, offset_at(m), v, w);
        sw += (double)w;
        swv += (double)w * (double)v;
        if (third) swvv += (double)w * (double)v * (double)v;
        advance(jr, m);
      }
      sw = block_sum(sw, s_red);
      swv = block_sum(swv, s_red);
      if (third) swvv = block_sum(swvv, s_red);
      const double scale = R.h * sqrt((double)(1 << R.levels));
      const auto cc = gmem(coarse + coff[r]);
      const double mt = fmax(cc[B], 0.0) * scale;
      const double jt = cc[R.n_coarse + B] * scale;
      const double rd = sw > 0.0 ? mt / sw : 1.0;
      ratio = (float)rd;
      if (mt > 0.0 && !third) dv = (float)((jt - rd * swv) / mt);
      if (mt > 0.0 && third) {
        const double st = cc[2 * R.n_coarse + B] * scale;
        const double ug = rd * swv / mt, ut = jt / mt;
        const double spread = rd * (swvv - 2.0 * ug * swv + ug * ug * sw);
        const double a = spread > 0.0 ? sqrt(fmax(st - jt * jt / mt, 0.0) / spread) : 1.0;
        stretch = (float)a;
        dv = (float)(ut - a * ug);
      }
    }
    const auto cell = gmem(R.cell);
    const auto frac = gmem(R.frac);
    const auto vel = gmem(R.v);
    const auto wgt = gmem(R.w);
    const int c0 = B << R.levels;  // first cell of the block: node c0 + d is bin d
    const int slot = threadIdx.x & (kLiftSlots - 1);
    bool big = false;
    auto put = [&](int j, int c, float fr, float v, float w) {
      const int64_t s = slot0 + j;
      const float ws = w * ratio;
      // nontemporal: the ions are not read again before the lift ends (0.76 -> 0.72 ms
      // per ensemble lift against plain stores)
      __builtin_nontemporal_store((int16_t)c, &cell[s]);
      __builtin_nontemporal_store(fr, &frac[s]);
      __builtin_nontemporal_store(fmaf(stretch, v, dv), &vel[s]);  // v + dv when stretch = 1
      __builtin_nontemporal_store(ws, &wgt[s]);
      if (dep) {
        const double q = fx_charge(ws);
        const double qr = fx_share(fr, q);
        const int d = c - c0;
        __hip_atomic_fetch_add(&s_q[d][slot], q - qr, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&s_q[d + 1][slot], qr, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        big |= !(fabsf(ws) < 16.0f);
      }
    };
    {
      int jr = q0, m = m0;
#pragma unroll
      for (int k = 0; k < kKeep; ++k) {
        const int j = threadIdx.x + k * kLiftThreads;
        if (j < count) {
          const int c = cell_at(jr);
          const float fr = offset_at(m);
          if (coarse == nullptr) ion(jr, c, m, fr, keep_v[k], keep_w[k]);
          put(j, c, fr, keep_v[k], keep_w[k]);
        }
        advance(jr, m);
      }
#pragma unroll 1
      for (int j = threadIdx.x + kKeep * kLiftThreads; j < count; j += kLiftThreads) {
        const int c = cell_at(jr);
        const float fr = offset_at(m);
        float v, w;
        ion(jr, c, m, fr, v, w);
        put(j, c, fr, v, w);
        advance(jr, m);
      }
    }
    if (dep) {
      // node totals (the slots in a fixed order; exact integer sums) to the grid
      if (__any(big) && (threadIdx.x & 63) == 0) atomicOr(status, (uint32_t)EFPI_DEV_WEIGHT);
      __syncthreads();
      const int nodes = (1 << R.levels) + 1;
      const int nmask = R.n_cells - 1;
      const auto qg = reinterpret_cast<unsigned long long*>(R.q[qsel]);
      for (int d = threadIdx.x; d < nodes; d += blockDim.x) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < kLiftSlots; ++k) t += s_q[d][k];
        if (t != 0.0) {
          const int node = R.bc == 0 ? ((c0 + d) & nmask) : c0 + d;
          atomicAdd(qg + node, (unsigned long long)rint_i64(t));
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- restrict/project --
__global__ void k_restrict(const RepDev* __restrict__ reps, int steps, double* __restrict__ snap,
                           const int64_t* __restrict__ soff) {
  const RepDev& R = reps[blockIdx.y];
  const int nc = R.n_coarse;
  const int64_t count = (int64_t)(steps + 1) * R.moments * nc;
  const double scale = kFxInv / R.h / sqrt((double)(1 << R.levels));
  double* out = snap + soff[blockIdx.y];
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    out[k] = (double)gmem(R.rbins)[k] * scale;
}

// LS slope (eq. 3.18) of one coefficient from its snapshot values v(p), p = 0..ne,
// and the forward-Euler projective step (eq. 3.17).  Products and sums are never
// fused into FMAs here, so every kernel that calls these gives the same bits for
// the same snapshots.
template <class V>
__device__ __forceinline__ double ls_slope_value(V v, int ne, double dt) {
#pragma clang fp contract(off)
  const double den = (double)ne * (ne + 1) * (ne + 2) * dt;
  double slope = 0.0;
  for (int p = 0; p <= ne / 2; ++p) {
    const double coef = 6.0 * (double)(ne - 2 * p) / den;
    slope += coef * (v(ne - p) - v(p));
  }
  return slope;
}

template <class V>
__device__ __forceinline__ double project_value(V v, int ne, double dt, double macro_dt) {
#pragma clang fp contract(off)
  const double leap = macro_dt - ne * dt;
  return v(ne) + leap * ls_slope_value(v, ne, dt);
}

__global__ void k_project(const RepDev* __restrict__ reps, const double* __restrict__ snap,
                          const int64_t* __restrict__ soff, double* __restrict__ out,
                          const int64_t* __restrict__ coff, uint32_t* __restrict__ status) {
  const RepDev& R = reps[blockIdx.y];
  const int nk = R.moments * R.n_coarse;  // coefficients of one snapshot
  const int nc = R.n_coarse;
  const int ne = R.burst_steps;
  const double* s = snap + soff[blockIdx.y];
  double* o = out + coff[blockIdx.y];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nk; k += gridDim.x * blockDim.x) {
    auto snapshot = [&](int p) { return s[(int64_t)p * nk + k]; };
    const double val = project_value(snapshot, ne, R.dt, R.macro_dt);
    o[k] = val;
    if (!(fabs(val) < 1e300)) atomicOr(status, 2u);
    if (k < nc && val < 0.0) atomicOr(status, 8u);
  }
}

// Restriction of every snapshot of the burst into coefficients and, in the same
// pass, the least-squares slope (eq. 3.18) and projective step (eq. 3.17): the
// thread of coefficient k converts that coefficient of all K + 1 snapshots, so
// the projection needs no second launch.  The same arithmetic as k_restrict
// followed by k_project.
__global__ void k_restrict_project(const RepDev* __restrict__ reps, double* __restrict__ snap,
                                   const int64_t* __restrict__ soff, double* __restrict__ out,
                                   const int64_t* __restrict__ coff,
                                   uint32_t* __restrict__ status) {
  const RepDev& R = reps[blockIdx.y];
  const int nk = R.moments * R.n_coarse;  // coefficients of one snapshot
  const int nc = R.n_coarse;
  const int ne = R.burst_steps;
  const double scale = kFxInv / R.h / sqrt((double)(1 << R.levels));
  const auto rb = gmem(R.rbins);
  double* s = snap + soff[blockIdx.y];
  double* o = out + coff[blockIdx.y];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nk; k += gridDim.x * blockDim.x) {
    // the snapshot value as k_restrict stores it (one rounded product)
    auto snapshot = [&](int p) { return (double)rb[(int64_t)p * nk + k] * scale; };
    for (int p = 0; p <= ne; ++p) s[(int64_t)p * nk + k] = snapshot(p);
    const double v = project_value(snapshot, ne, R.dt, R.macro_dt);
    o[k] = v;
    if (!(fabs(v) < 1e300)) atomicOr(status, 2u);
    if (k < nc && v < 0.0) atomicOr(status, 8u);
  }
}

// Second-order projective step.  The LS slope f of this burst estimates the time
// derivative at the burst's centre, and f_prev (the previous burst's) at the centre
// one macro step of length `gap` earlier; their linear extrapolation to the middle
// of the projection leap [t + N_e dt, t + Delta t] is f + (f - f_prev) Delta t /
// (2 gap) (Adams-Bashforth 2 for equal steps: 3/2 f - 1/2 f_prev), and the state
// advances from the last snapshot over the leap with it.  Writes the slope, the
// forward-Euler projection (eq. 3.17, as k_project) and the second-order one
// (equal to Euler when f_prev is absent).
__global__ void k_project2(const RepDev* __restrict__ reps, const double* __restrict__ snap,
                           const int64_t* __restrict__ soff, const double* __restrict__ slope_prev,
                           double gap, double* __restrict__ slope_out,
                           double* __restrict__ euler_out, double* __restrict__ out,
                           const int64_t* __restrict__ coff, uint32_t* __restrict__ status) {
#pragma clang fp contract(off)
  const RepDev& R = reps[blockIdx.y];
  const int nk = R.moments * R.n_coarse;  // coefficients of one snapshot
  const int nc = R.n_coarse;
  const int ne = R.burst_steps;
  const double* s = snap + soff[blockIdx.y];
  const int64_t co = coff[blockIdx.y];
  const double leap = R.macro_dt - ne * R.dt;
  const double w = slope_prev ? R.macro_dt / (2.0 * gap) : 0.0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nk; k += gridDim.x * blockDim.x) {
    auto snapshot = [&](int p) { return s[(int64_t)p * nk + k]; };
    const double f = ls_slope_value(snapshot, ne, R.dt);
    const double last = snapshot(ne);
    const double euler = last + leap * f;
    const double fm = slope_prev ? f + (f - slope_prev[co + k]) * w : f;
    const double val = last + leap * fm;
    slope_out[co + k] = f;
    if (euler_out) euler_out[co + k] = euler;
    out[co + k] = val;
    if (!(fabs(val) < 1e300)) atomicOr(status, 2u);
    if (k < nc && val < 0.0) atomicOr(status, 8u);
  }
}

__global__ void k_ensemble_mean(const RepDev* __restrict__ reps, int n_reps,
                                const int32_t* __restrict__ group, double* __restrict__ coarse,
                                const int64_t* __restrict__ coff) {
  // one block row per group leader; members share n_cells, hence moments N_c entries
  const int r = blockIdx.y;
  if (group[r] != r) return;
  const int count = reps[r].moments * reps[r].n_coarse;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) {
    double acc = 0.0;
    int m = 0;
    for (int q = 0; q < n_reps; ++q)
      if (group[q] == r) {
        acc += coarse[coff[q] + k];
        ++m;
      }
    const double mean = acc / m;
    for (int q = 0; q < n_reps; ++q)
      if (group[q] == r) coarse[coff[q] + k] = mean;
  }
}

// Store each replica's lift rotation where the lift kernel reads it.
__global__ void k_set_shifts(const RepDev* __restrict__ reps, int n_reps, int only_rep,
                             const ShiftArg shifts) {
  const int r = threadIdx.x;
  if (r < n_reps && (only_rep < 0 || r == only_rep)) gmem(reps[r].aux)[1] = (int64_t)shifts.s[r];
}

__global__ void k_set_profile(const RepDev* __restrict__ reps, int rep,
                              const double* __restrict__ dn, const double* __restrict__ du) {
  const RepDev& R = reps[rep];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < R.n_nodes; k += gridDim.x * blockDim.x) {
    gmem(R.prof_n)[k] = fmax(dn[k], 0.0);
    gmem(R.prof_u)[k] = du[k];
  }
}

}  // namespace

void launch_set_profile(const RepDev* d_reps, int rep, const double* d_n, const double* d_u,
                        hipStream_t stream) {
  hipLaunchKernelGGL(k_set_profile, dim3(16), dim3(256), 0, stream, d_reps, rep, d_n, d_u);
}

void launch_lift_prep(const RepDev* d_reps, int n_reps, const double* d_coarse,
                      const int64_t* d_coff, uint32_t* d_status, const ShiftArg* shifts,
                      hipStream_t stream) {
  const ShiftArg none{};
  hipLaunchKernelGGL(k_lift_prep, dim3(n_reps), dim3(kProfThreads), 0, stream, d_reps, d_coarse,
                     d_coff, d_status, shifts ? 1 : 0, shifts ? *shifts : none);
}

void launch_occupancy(const RepDev* d_reps, int n_reps, int only_rep, uint32_t* d_status,
                      hipStream_t stream) {
  hipLaunchKernelGGL(k_occupancy, dim3(only_rep >= 0 ? 1 : n_reps), dim3(kProfThreads), 0,
                     stream, d_reps, only_rep, d_status);
}

void launch_set_shifts(const RepDev* d_reps, int n_reps, int only_rep, const ShiftArg& shifts,
                       hipStream_t stream) {
  hipLaunchKernelGGL(k_set_shifts, dim3(1), dim3(kMaxShiftReplicas), 0, stream, d_reps, n_reps,
                     only_rep, shifts);
}

void launch_lift_particles(const RepDev* d_reps, const int64_t* d_block_prefix, int n_reps,
                           int64_t total_blocks, int only_rep, const double* d_coarse,
                           const int64_t* d_coff, const ShiftArg* shifts, int grid_blocks,
                           hipStream_t stream, int qsel, uint32_t* d_status, bool third) {
  if (total_blocks <= 0) return;
  if (shifts) launch_set_shifts(d_reps, n_reps, only_rep, *shifts, stream);
  const int64_t g = grid_blocks > 0 ? min((int64_t)grid_blocks, total_blocks) : total_blocks;
  if (third && d_coarse != nullptr)
    hipLaunchKernelGGL(k_lift<true>, dim3((unsigned)g), dim3(kLiftThreads), 0, stream, d_reps,
                       d_block_prefix, n_reps, total_blocks, only_rep, d_coarse, d_coff, qsel,
                       d_status);
  else
    hipLaunchKernelGGL(k_lift<false>, dim3((unsigned)g), dim3(kLiftThreads), 0, stream, d_reps,
                       d_block_prefix, n_reps, total_blocks, only_rep, d_coarse, d_coff, qsel,
                       d_status);
}

void launch_restrict(const RepDev* d_reps, int n_reps, int steps, double* d_snap,
                     const int64_t* d_soff, hipStream_t stream) {
  hipLaunchKernelGGL(k_restrict, dim3(16, n_reps), dim3(256), 0, stream, d_reps, steps, d_snap,
                     d_soff);
}

void launch_project(const RepDev* d_reps, int n_reps, const double* d_snap,
                    const int64_t* d_soff, double* d_out, const int64_t* d_coff,
                    uint32_t* d_status, hipStream_t stream) {
  hipLaunchKernelGGL(k_project, dim3(4, n_reps), dim3(256), 0, stream, d_reps, d_snap, d_soff,
                     d_out, d_coff, d_status);
}

void launch_restrict_project(const RepDev* d_reps, int n_reps, double* d_snap,
                             const int64_t* d_soff, double* d_out, const int64_t* d_coff,
                             uint32_t* d_status, hipStream_t stream) {
  hipLaunchKernelGGL(k_restrict_project, dim3(4, n_reps), dim3(256), 0, stream, d_reps, d_snap,
                     d_soff, d_out, d_coff, d_status);
}

void launch_project2(const RepDev* d_reps, int n_reps, const double* d_snap,
                     const int64_t* d_soff, const double* d_slope_prev, double gap,
                     double* d_slope, double* d_euler, double* d_out, const int64_t* d_coff,
                     uint32_t* d_status, hipStream_t stream) {
  hipLaunchKernelGGL(k_project2, dim3(4, n_reps), dim3(256), 0, stream, d_reps, d_snap, d_soff,
                     d_slope_prev, gap, d_slope, d_euler, d_out, d_coff, d_status);
}

void launch_ensemble_mean(const RepDev* d_reps, int n_reps, const int32_t* d_group,
                          double* d_coarse, const int64_t* d_coff, hipStream_t stream) {
  hipLaunchKernelGGL(k_ensemble_mean, dim3(4, n_reps), dim3(256), 0, stream, d_reps, n_reps,
                     d_group, d_coarse, d_coff);
}

}  // namespace efpi
