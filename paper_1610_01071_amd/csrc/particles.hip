// Particle pass of the fine burst: field gather, leapfrog push, boundaries,
// fixed-point CIC charge deposit (Sec. 2.2) and the co-evolving restriction
// snapshot of the density and momentum moments (App. B, eqs. B.4-B.5), fused in
// one streaming pass over the structure-of-arrays ion store.
//
// Work decomposition: every replica's particle slots are cut into tiles of
// `tile` consecutive particles; a persistent grid walks the (replica, tile)
// items.  The node field around the tile is staged in LDS.  Inside a tile, each
// wave takes runs of 512 consecutive ions (8 per lane), so that in a cell-sorted
// store its ions touch few distinct nodes.  It merges all of its ions that hit
// the same node (deposit) or coarse block (restriction) with fixed-order wave
// reductions, and adds the merged value to a register owned by one lane (lane s
// holds node or block base + s).  At the end of the tile the four waves' registers are summed
// through LDS and flushed with one 64-bit integer atomic per non-zero target.
// Rare targets outside a wave's 64 slots go to an LDS window (deposit) or to
// global atomics.  Every sum that reaches memory is an integer sum, so the
// result does not depend on scheduling order.
#include "efpi_internal.h"

#include <hip/hip_ext.h>

#include <type_traits>

namespace efpi {
namespace {

typedef EFPI_GLOBAL unsigned long long gu64;

// A value that is the same in every lane, read so that the compiler knows it is
// uniform (scalar registers, uniform control flow).
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ void gatomic_add(long long* p, long long v) {
  __hip_atomic_fetch_add((gu64*)p, (unsigned long long)v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kBatch = 8;       // particles per thread loaded ahead of use
constexpr int kQWin = 256;      // node window (int64 bins)
constexpr int kQMargin = 16;
constexpr int kQSlotMargin = 4;  // node slots per wave start this far below the tile
constexpr int kRWin = kWave;    // coarse block slots per wave (one per lane)
constexpr int kRMargin = 8;
constexpr int kEWin = 128;      // node field window staged in LDS (cells)
constexpr int kEMargin = 32;

// Wave-wide sums with a fixed pattern: inside each 16-lane row an inclusive scan
// by row shifts 1, 2, 3 of the input, then 4 and 8 (lanes shifted in from
// outside the row read 0), which leaves each row's total in its lane 15; the
// four row totals are read into scalar registers and added as (r3 + r2) + (r1 +
// r0).  The order of every addition is fixed, so FP32 sums are reproducible bit
// for bit.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_shr(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, true);
}

__device__ __forceinline__ int row_scan_i32(int x) {
  int t = x + dpp_shr<0x111>(x);
  t += dpp_shr<0x112>(x);
  t += dpp_shr<0x113>(x);
  t += dpp_shr<0x114>(t);
  t += dpp_shr<0x118>(t);
  return t;
}

__device__ __forceinline__ int wave_sum_i32(int x) {
  const int t = row_scan_i32(x);
  const int r0 = __builtin_amdgcn_readlane(t, 15), r1 = __builtin_amdgcn_readlane(t, 31);
  const int r2 = __builtin_amdgcn_readlane(t, 47), r3 = __builtin_amdgcn_readlane(t, 63);
  return (r3 + r2) + (r1 + r0);
}

__device__ __forceinline__ float wave_sum_f32(float x) {
  float t = x + __int_as_float(dpp_shr<0x111>(__float_as_int(x)));
  t += __int_as_float(dpp_shr<0x112>(__float_as_int(x)));
  t += __int_as_float(dpp_shr<0x113>(__float_as_int(x)));
  t += __int_as_float(dpp_shr<0x114>(__float_as_int(t)));
  t += __int_as_float(dpp_shr<0x118>(__float_as_int(t)));
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 15));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 31));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 47));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 63));
  return (r3 + r2) + (r1 + r0);
}

// Exact wave sum of int64 values with |v| < 2^49: the low 24 bits and the rest
// are summed separately as int32 (64 * 2^24 and 64 * 2^25 both fit) and recombined.
__device__ __forceinline__ long long wave_sum_i64(long long v) {
  const int lo = (int)(v & 0xFFFFFF);
  const int hi = (int)(v >> 24);
  return (long long)wave_sum_i32(hi) * (1ll << 24) + (long long)wave_sum_i32(lo);
}

// rint(x) as int64 for |x| < 2^51: adding 1.5 * 2^52 leaves the integer part
// rounded to nearest (ties to even, the IEEE default) in the low mantissa bits.
__device__ __forceinline__ long long rint_i64(double x) {
  const double magic = 6755399441055744.0;
  return (long long)(__double_as_longlong(x + magic) - __double_as_longlong(magic));
}

// rint(x) for |x| < 2^51 as a binary64 value (the same rounding as rint_i64).
__device__ __forceinline__ double rint_d(double x) { return __builtin_rint(x); }

// q = rint(w 2^40): the particle's charge in fixed point, as an exact binary64
// integer value.
__device__ __forceinline__ double fx_charge(float w) { return rint_d((double)w * kFxScale); }
// Right-node share rint(theta q) in binary64 (one rounded product, then ties-to-even).
__device__ __forceinline__ double fx_share(float theta, double q) {
  return rint_d((double)theta * q);
}
// Fixed-point value of an FP32 partial sum.
__device__ __forceinline__ long long fx_of(float x) { return rint_i64((double)x * kFxScale); }

__device__ __forceinline__ int find_replica(const int64_t* prefix, int n, int64_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct Window {
  long long* lds;
  int base;
  int size;
  long long* glob;
};

__device__ __forceinline__ void add_to(const Window& w, int idx, long long val) {
  if (val == 0) return;
  int k = idx - w.base;
  if (k >= 0 && k < w.size)
    atomicAdd(reinterpret_cast<unsigned long long*>(&w.lds[k]), (unsigned long long)val);
  else
    gatomic_add(&w.glob[idx], val);
}

// Each lane holds kBatch ions.  Every distinct target of the wave is merged:
// the lowest active lane's target is taken, every lane sums its own ions with
// that target, the sums are reduced across the wave and the result is added to
// a per-lane slot register (lane s owns target base + s).  A target outside the
// 64-slot window is added to the LDS window, else to global memory.  Per-lane
// 64-bit LDS atomics are slow on this hardware, so the merge is never skipped.
//
// Charge deposit: ion j adds a[j] to node key[j] and b[j] to node key[j] + 1
// (wrapping to 0 at `wrap`, or no wrap when wrap = -1).  Exact int64 sums.
__device__ __forceinline__ void merge_charge(int (&key)[kBatch], const double (&a)[kBatch],
                                             const double (&b)[kBatch], int wrap, int base,
                                             long long& acc, const Window& win) {
  const int lane = __lane_id();
  while (true) {
    int mine = key[0];  // any remaining key of the lane (-1 when none is left)
#pragma unroll
    for (int j = 1; j < kBatch; ++j) mine = max(mine, key[j]);
    const unsigned long long act = __ballot(mine >= 0);
    if (act == 0ull) break;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int lk = __builtin_amdgcn_readlane(mine, leader);
    // integer-valued binary64 lane sums: exact, since every lane sum stays below 2^49
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const bool m = key[j] == lk;
      const double one = m ? 1.0 : 0.0;
      sa = fma(one, a[j], sa);
      sb = fma(one, b[j], sb);
      key[j] = m ? -1 : key[j];
    }
    const long long ta = wave_sum_i64(rint_i64(sa));
    const long long tb = wave_sum_i64(rint_i64(sb));
    int r = lk + 1;
    if (r == wrap) r = 0;
    const int sl = lk - base;
    const int sr = r - base;
    acc += lane == sl ? ta : 0ll;
    acc += lane == sr ? tb : 0ll;
    if ((unsigned)sl >= (unsigned)kWave && lane == 0) add_to(win, lk, ta);
    if ((unsigned)sr >= (unsigned)kWave && lane == 0) add_to(win, r, tb);
  }
}

// Restriction snapshot: ion j adds (a0, a1)[j] to block key[j] and (b0, b1)[j]
// to block key[j] + 1 for the (density, momentum) moments.  Every distinct
// block of the wave is merged (FP32 partial sums in a fixed order, converted to
// fixed point); the merged values go to per-lane slot registers, lane s of the
// wave owning block base + s, so that no LDS atomics are needed.  Blocks outside
// the 64-block slot window go to global atomics.
__device__ __forceinline__ void merge_moments(int (&key)[kBatch], const float (&a0)[kBatch],
                                              const float (&a1)[kBatch],
                                              const float (&b0)[kBatch],
                                              const float (&b1)[kBatch], int wrap, int base,
                                              long long& acc0, long long& acc1,
                                              long long* g0, long long* g1) {
  const int lane = __lane_id();
  while (true) {
    int mine = key[0];  // any remaining key of the lane (-1 when none is left)
#pragma unroll
    for (int j = 1; j < kBatch; ++j) mine = max(mine, key[j]);
    const unsigned long long act = __ballot(mine >= 0);
    if (act == 0ull) break;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int lk = __builtin_amdgcn_readlane(mine, leader);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const bool m = key[j] == lk;
      const float one = m ? 1.f : 0.f;  // 1 * x + s and 0 * x + s round as the plain sums
      s0 = fmaf(one, a0[j], s0);
      s1 = fmaf(one, a1[j], s1);
      s2 = fmaf(one, b0[j], s2);
      s3 = fmaf(one, b1[j], s3);
      key[j] = m ? -1 : key[j];
    }
    const long long f0 = fx_of(wave_sum_f32(s0));
    const long long f1 = fx_of(wave_sum_f32(s1));
    const long long f2 = fx_of(wave_sum_f32(s2));
    const long long f3 = fx_of(wave_sum_f32(s3));
    int r = lk + 1;
    if (r == wrap) r = 0;
    const int sl = lk - base;
    const int sr = r - base;
    acc0 += lane == sl ? f0 : 0ll;
    acc1 += lane == sl ? f1 : 0ll;
    acc0 += lane == sr ? f2 : 0ll;
    acc1 += lane == sr ? f3 : 0ll;
    if ((unsigned)sl >= (unsigned)kWave && lane == 0) {
      gatomic_add(g0 + lk, f0);
      gatomic_add(g1 + lk, f1);
    }
    if ((unsigned)sr >= (unsigned)kWave && (f2 | f3) != 0 && lane == 0) {
      gatomic_add(g0 + r, f2);
      gatomic_add(g1 + r, f3);
    }
  }
}

// MODE (compile time): kRestrict | kPush for a burst step, kPush for plain PIC,
// kRestrict for the last snapshot of a burst, kDepositOnly for a charge deposit.
// Four waves per SIMD: the register budget is held at 128 (the pass is bound by
// vector instruction issue, so it needs the occupancy to keep every SIMD busy).
template <int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_particles(const RepDev* __restrict__ reps, const int64_t* __restrict__ item_prefix,
                 int n_reps, int64_t total_items, int tile, int p, double pd, int fresh_flag,
                 int qsel) {
  __shared__ long long lds_q[kQWin];
  __shared__ long long lds_qs[kWaves][kWave];
  __shared__ long long lds_r[kWaves][2][kRWin];
  __shared__ float lds_e[kEWin + 1];
  __shared__ float lds_en[kEWin + 1];
  const int tid = threadIdx.x;
  // a batch is kThreads * kBatch consecutive ions; wave w takes the w-th run of
  // kWave * kBatch of them, lane l its ions l, l + 64, ... (coalesced loads, and
  // each wave's ions span as few cells as possible)
  const unsigned toff = (unsigned)(tid / kWave) * (kWave * kBatch) + (unsigned)(tid % kWave);
  const bool fresh = fresh_flag != 0;
  constexpr bool restrict_ = (MODE & kRestrict) != 0;
  constexpr bool push = (MODE & kPush) != 0;
  constexpr bool deposit = push || (MODE & kDepositOnly) != 0;

  for (int64_t item = blockIdx.x; item < total_items; item += gridDim.x) {
    const int r = find_replica(item_prefix, n_reps, item);
    const RepDev& R = reps[r];
    const int64_t np = uniform_i64(*gmem(R.np));
    const int64_t i0 = (item - R.item_begin) * (int64_t)tile;
    if (i0 >= np) continue;
    const unsigned cnt = (unsigned)min((int64_t)tile, np - i0);
    const int n = R.n_cells;
    // the tile body, compiled once for periodic grids and once for walls
    auto tile_pass = [&](auto bc_tag) {
      constexpr bool periodic = decltype(bc_tag)::value;
      const int nmask = n - 1;
      const float dt = (float)R.dt;
      const float inv_h = (float)R.inv_h;
      const int levels = R.levels;
      const int nc = R.n_coarse;
      // p < 0: plain restriction of the current state (tau = 0, snapshot slot 0)
      // (pd = p as binary64, a kernel argument: converting p here would give a
      // value the compiler keeps in a vector register across the whole kernel)
      const float tau = p < 0 ? 0.f : (float)(R.macro_dt - pd * R.dt);
      const bool coev = R.coevolving != 0 && p >= 0;
      const EFPI_GLOBAL float* __restrict__ e = gmem(R.e);
      const EFPI_GLOBAL float* __restrict__ en = gmem(R.en);
      EFPI_GLOBAL int16_t* __restrict__ cellp = gmem(R.cell + i0);
      EFPI_GLOBAL float* __restrict__ fracp = gmem(R.frac + i0);
      EFPI_GLOBAL float* __restrict__ vp_ = gmem(R.v + i0);
      const EFPI_GLOBAL float* __restrict__ wp = gmem(R.w + i0);
      const float half_dt = 0.5f * dt;
      const float half_dt_r = fresh ? 0.f : half_dt;  // snapshot velocity v + half_dt_r E
      const float dt_push = fresh ? half_dt : dt;     // push: v + dt_push E
      const int lmask = (1 << levels) - 1;
      const float dt_inv_h = dt * inv_h;
      const float tau_inv_h = coev ? tau * inv_h : 0.f;
      const float tau_e = coev ? tau : 0.f;

      const int c_first = __builtin_amdgcn_readfirstlane((int)cellp[0]);
      Window wq{lds_q, c_first - kQMargin, kQWin, reinterpret_cast<long long*>(R.q[qsel])};
      long long* rb = reinterpret_cast<long long*>(R.rbins) + (int64_t)(p < 0 ? 0 : p) * 2 * nc;
      const int rbase = (c_first >> levels) - kRMargin;
      long long racc0 = 0, racc1 = 0;
      const int qbase = c_first - kQSlotMargin;
      long long qacc = 0;

      for (int k = tid; k < kQWin; k += kThreads) lds_q[k] = 0;
      // Field window: nodes ebase .. ebase + kEWin (wrapped, or clamped to the wall
      // nodes), so that a cell c in [ebase, ebase + kEWin) finds E_c and E_{c+1}.
      const int ebase = c_first - kEMargin;
      if (restrict_ || push) {
        for (int k = tid; k <= kEWin; k += kThreads) {
          const int g = periodic ? ((ebase + k) & nmask) : min(max(ebase + k, 0), n);
          lds_e[k] = e[g];
          if (restrict_) lds_en[k] = coev ? en[g] : 0.f;
        }
      }
      __syncthreads();

      for (unsigned b0 = 0; b0 < cnt; b0 += kThreads * kBatch) {
        // loads use a clamped index so that they are unconditional; slots past the
        // end of the tile are marked dead and never stored
        int cl[kBatch];
        float fr[kBatch], vv[kBatch], ww[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          const unsigned idx = b0 + j * kWave + toff;
          const unsigned ci = min(idx, cnt - 1u);
          __builtin_assume(ci < 65536u);  // tiles hold at most 65536 ions
          const int c = *at(cellp, ci);
          cl[j] = idx < cnt ? c : -1;
          fr[j] = *at(fracp, ci);
          vv[j] = *at(vp_, ci);
          ww[j] = *at(wp, ci);
        }
        // Node fields at both ends of each ion's cell, from the LDS window; ions
        // outside it (rare: unsorted or far-drifted stores) read global memory.
        float e0[kBatch], e1[kBatch], n0[kBatch], n1[kBatch];
        bool outside = false;
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          const int c = cl[j];
          const bool alive = c >= 0 && c < n;
          const int k = alive ? c - ebase : 0;
          const bool inw = (unsigned)k < (unsigned)kEWin;
          const int kk = inw ? k : 0;
          outside |= !inw;
          e0[j] = e1[j] = n0[j] = n1[j] = 0.f;
          if (restrict_ || push) {
            e0[j] = lds_e[kk];
            e1[j] = lds_e[kk + 1];
          }
          if (restrict_) {
            n0[j] = lds_en[kk];
            n1[j] = lds_en[kk + 1];
          }
        }
        if ((restrict_ || push) && __ballot(outside) != 0ull) {
#pragma unroll
          for (int j = 0; j < kBatch; ++j) {
            const int c = cl[j];
            const bool alive = c >= 0 && c < n;
            if (alive && (unsigned)(c - ebase) >= (unsigned)kEWin) {
              const int cr = periodic ? ((c + 1) & nmask) : c + 1;
              e0[j] = e[c];
              e1[j] = e[cr];
              if (restrict_ && coev) {
                n0[j] = en[c];
                n1[j] = en[cr];
              }
            }
          }
        }
        // E^p at the ions; then the snapshot values are computed and merged, and only
        // after that the push and the new charge (the two phases' value arrays are
        // never live together, which keeps the kernel at 4 waves per SIMD)
        float epa[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          const float f = fr[j];
          epa[j] = (restrict_ || push) ? (1.f - f) * e0[j] + f * e1[j] : 0.f;
        }
        if (restrict_) {
          int rkey[kBatch];
          float ra0[kBatch], ra1[kBatch], rb0[kBatch], rb1[kBatch];
#pragma unroll
          for (int j = 0; j < kBatch; ++j) {
            const int c = cl[j];
            const float f = fr[j];
            const float v = vv[j];
            const float w = ww[j];
            const bool alive = c >= 0 && c < n;  // cells outside [0, N) are treated as absorbed
            const int cs = alive ? c : 0;         // safe cell index
            const float ep = epa[j];
            // Snapshot p: time-centred velocity, then the approximate characteristic
            // over tau = Delta t - p dt (eq. B.4) and CIC at the moved position (eq. B.5).
            const float vpc = v + half_dt_r * ep;  // half_dt_r = 0 on a fresh state
            const float enx = (1.f - f) * n0[j] + f * n1[j];
            const float xt = f + tau_inv_h * vpc;
            const float vt = vpc + tau_e * enx;
            const float fl = floorf(xt);
            const float fx = xt - fl;
            const bool wrap_up = fx >= 1.f;
            const int ct0 = cs + (int)fl + (wrap_up ? 1 : 0);
            const int ct = periodic ? (ct0 & nmask) : ct0;
            const bool in = alive && (periodic || (ct >= 0 && ct < n));
            const int bl = ct >> levels;
            // both nodes of cell ct in block bl: ct is not the block's last cell, or
            // (walls) the block is the last one, which also owns wall node N, or
            // (periodic) there is a single block
            const bool last = (ct & lmask) == lmask;
            const bool same = !last || (periodic ? nc == 1 : bl == nc - 1);
            // right-node share theta, zero when both nodes are in the same block
            const float th = (wrap_up || same) ? 0.f : fx;
            const float wv = w * vt;
            rkey[j] = in ? bl : -1;
            ra0[j] = w - w * th;
            ra1[j] = wv - wv * th;
            rb0[j] = w * th;
            rb1[j] = wv * th;
          }
          merge_moments(rkey, ra0, ra1, rb0, rb1, periodic ? nc : -1, rbase, racc0, racc1, rb,
                        rb + nc);
        }
        if (deposit) {
          int dkey[kBatch];
          double da[kBatch], db[kBatch];
#pragma unroll
          for (int j = 0; j < kBatch; ++j) {
            const unsigned idx = b0 + j * kWave + toff;
            __builtin_assume(idx < 65536u + kThreads * kBatch);
            const int c = cl[j];
            const float f = fr[j];
            const float v = vv[j];
            const float w = ww[j];
            const bool alive = c >= 0 && c < n;
            const int cs = alive ? c : 0;
            const float ep = epa[j];
            int cn = cs;
            float fn = f, vn = v;
            if (push) {
              vn = v + dt_push * ep;
              const float xn = f + dt_inv_h * vn;
              const float fl = floorf(xn);
              const bool wrap_up = (xn - fl) >= 1.f;
              fn = wrap_up ? 0.f : xn - fl;
              cn = cs + (int)fl + (wrap_up ? 1 : 0);
              cn = periodic ? (cn & nmask) : ((cn < 0 || cn >= n) ? -1 : cn);  // walls absorb
              if (alive && idx < cnt) {
                *at(cellp, idx) = (int16_t)cn;
                *at(fracp, idx) = fn;
                *at(vp_, idx) = vn;
              }
            }
            const bool dep = alive && cn >= 0;
            const double q = fx_charge(w);
            const double qr = fx_share(fn, q);
            dkey[j] = dep ? cn : -1;
            da[j] = q - qr;
            db[j] = qr;
          }
          merge_charge(dkey, da, db, periodic ? n : -1, qbase, qacc, wq);
        }
      }
      if (deposit) lds_qs[tid / kWave][tid % kWave] = qacc;
      if (restrict_) {
        lds_r[tid / kWave][0][tid % kWave] = racc0;
        lds_r[tid / kWave][1][tid % kWave] = racc1;
      }
      __syncthreads();
      if (deposit) {
        long long* gq = reinterpret_cast<long long*>(R.q[qsel]);
        for (int k = tid; k < kQWin; k += kThreads) {
          long long val = lds_q[k];
          const int s = k - (kQMargin - kQSlotMargin);  // slot of node wq.base + k
          if (s >= 0 && s < kWave) {
#pragma unroll
            for (int w = 0; w < kWaves; ++w) val += lds_qs[w][s];
          }
          if (val != 0) gatomic_add(&gq[wq.base + k], val);
        }
      }
      if (restrict_) {
        for (int k = tid; k < 2 * kRWin; k += kThreads) {
          const int m = k / kRWin;
          const int kk = k - m * kRWin;
          long long val = 0;
#pragma unroll
          for (int w = 0; w < kWaves; ++w) val += lds_r[w][m][kk];
          if (val != 0) gatomic_add(&rb[(int64_t)m * nc + rbase + kk], val);
        }
      }
      __syncthreads();
    };
    if (R.bc == 0) tile_pass(std::true_type{});
    else tile_pass(std::false_type{});
  }
}

__global__ void k_fill_u8(uint8_t* p, size_t bytes) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t n16 = bytes / 16;
  uint4* p16 = reinterpret_cast<uint4*>(p);
  for (size_t k = i; k < n16; k += stride) p16[k] = make_uint4(0, 0, 0, 0);
  for (size_t k = n16 * 16 + i; k < bytes; k += stride) p[k] = 0;
}

// Copy particles between a caller's arrays and a replica's store; the count
// is written to the device counter when copying into the store.
__global__ void k_copy_particles(const RepDev* reps, int rep, const int16_t* cell,
                                 const float* frac, const float* v, const float* w, int64_t n,
                                 int to_store, int16_t* ocell, float* ofrac, float* ov,
                                 float* ow) {
  const RepDev& R = reps[rep];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (to_store) {
    if (i == 0) *R.np = n;
    if (i < n) {
      R.cell[i] = cell[i];
      R.frac[i] = frac[i];
      R.v[i] = v[i];
      R.w[i] = w[i];
    }
  } else {
    const int64_t m = *R.np;
    if (i < m) {
      if (ocell) ocell[i] = R.cell[i];
      if (ofrac) ofrac[i] = R.frac[i];
      if (ov) ov[i] = R.v[i];
      if (ow) ow[i] = R.w[i];
    }
  }
}

}  // namespace

namespace {
// With both events given, the launch is bracketed by them (extended launch).
template <int MODE>
void launch_mode(dim3 grid, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1,
                 const RepDev* d_reps, const int64_t* d_item_prefix, int n_reps,
                 int64_t total_items, int tile, int p, int fresh, int qsel) {
  if (ev0 && ev1)
    hipExtLaunchKernelGGL(k_particles<MODE>, grid, dim3(kThreads), 0, stream, ev0, ev1, 0, d_reps,
                          d_item_prefix, n_reps, total_items, tile, p, (double)p, fresh, qsel);
  else
    hipLaunchKernelGGL(k_particles<MODE>, grid, dim3(kThreads), 0, stream, d_reps, d_item_prefix,
                       n_reps, total_items, tile, p, (double)p, fresh, qsel);
}
}  // namespace

void launch_particles(const RepDev* d_reps, const int64_t* d_item_prefix, int n_reps,
                      int64_t total_items, int tile, int grid_blocks, int p, int flags,
                      int qsel, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
  if (total_items <= 0) return;
  const int64_t g = grid_blocks > 0 ? min((int64_t)grid_blocks, total_items) : total_items;
  const int fresh = (flags & kFresh) ? 1 : 0;
  const int mode = flags & (kRestrict | kPush | kDepositOnly);
  const dim3 grid((unsigned)g);
  switch (mode) {
    case kRestrict | kPush:
      launch_mode<kRestrict | kPush>(grid, stream, ev0, ev1, d_reps, d_item_prefix, n_reps,
                                     total_items, tile, p, fresh, qsel);
      break;
    case kPush:
      launch_mode<kPush>(grid, stream, ev0, ev1, d_reps, d_item_prefix, n_reps, total_items, tile,
                         p, fresh, qsel);
      break;
    case kRestrict:
      launch_mode<kRestrict>(grid, stream, ev0, ev1, d_reps, d_item_prefix, n_reps, total_items,
                             tile, p, fresh, qsel);
      break;
    default:
      launch_mode<kDepositOnly>(grid, stream, ev0, ev1, d_reps, d_item_prefix, n_reps,
                                total_items, tile, p, fresh, qsel);
      break;
  }
}

void launch_fill_u8(void* d_ptr, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return;
  size_t blocks = (bytes / 16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)blocks), dim3(256), 0, stream,
                     static_cast<uint8_t*>(d_ptr), bytes);
}

void launch_copy_particles(const RepDev* d_reps, int rep, const int16_t* cell, const float* frac,
                           const float* v, const float* w, int64_t n, int to_store,
                           int16_t* ocell, float* ofrac, float* ov, float* ow,
                           hipStream_t stream) {
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_copy_particles, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0,
                     stream, d_reps, rep, cell, frac, v, w, n, to_store, ocell, ofrac, ov, ow);
}

}  // namespace efpi
