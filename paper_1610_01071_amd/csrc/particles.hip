// Particle pass of the fine burst: field gather, leapfrog push, boundaries,
// fixed-point CIC charge deposit (Sec. 2.2) and the co-evolving restriction
// snapshot of the density and momentum moments (and, for the EFREE variables of
// Sec. 3.2, the second velocity moment) (App. B, eqs. B.4-B.5), fused in
// one streaming pass over the structure-of-arrays ion store.
//
// Work decomposition: every replica's particle slots are cut into tiles of
// `tile` consecutive ions; a persistent grid of 256-thread workgroups walks the
// (replica, tile) items, and wave w of a workgroup takes the w-th quarter of the
// tile.  Waves never wait for each other: each has its own field window and
// accumulators in LDS.  A wave reads its ions in batches of 512, lane l holding
// the groups of four consecutive ions 4l .. 4l + 3 and 256 + 4l .. 256 + 4l + 3,
// so that every load and store is a 16-byte (8-byte for the cells) access and
// the wave's accesses cover contiguous memory.
//
// Accumulation without merges: a cell-sorted store keeps a wave's ions within a
// few cells and coarse blocks of one another over a burst.  Each wave owns a
// window of 16 nodes and of 16 coarse blocks around the cells of its range;
// every lane adds its ions' shares into bins of its own in that window with
// LDS atomics that return nothing (ds_add_f64), so no lane waits and no
// cross-lane merge runs per ion.  Every share is first put in fixed point (unit
// 2^-40: the charge and the snapshot mass split as rint(theta q), q - rint(theta
// q); the momentum likewise) and held as an integer-valued binary64, so every
// bin sum is exact and independent of order; lanes l, l + 16, l + 32 and l + 48
// share a bin.  The particle streams are read and written with nontemporal
// accesses (each ion is touched once per pass).
// At the end of the wave's range the bins are summed across lanes and added to
// global memory with 64-bit integer atomics, so the grid charge and the
// snapshots do not depend on scheduling.  Ions whose target lies outside the
// window add their fixed-point shares with global atomics directly.
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

// Accumulation into a lane's LDS bin (no value returned: ds_add_f64).  The FP32
// form of this atomic is two orders of magnitude slower on this hardware, so all
// bins hold fixed-point values as integer-valued binary64.
__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Orders a wave's LDS accesses around a hand-over between its lanes (the LDS
// executes one wave's instructions in issue order; this keeps the compiler's
// order too).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kGroup = 4;                      // consecutive ions per vector access
constexpr int kHalves = 2;                     // vector groups per lane per batch
constexpr int kPer = kHalves * kGroup;         // ions per lane per batch
constexpr int kBatch = kPer * kWave;           // ions per wave per batch
constexpr int kQBins = 16;                     // node bins of a wave's charge window
// LDS slots per bin (lanes equal modulo kQSlots share one).  With 16 slots a
// workgroup's windows take 26 KB of LDS, and the VGPR budget, not the LDS, sets
// the occupancy (4 waves per SIMD against 3 with 32 slots: 607 against 666 us
// per burst step of 148M ions).
#ifndef EFPI_PASS_SLOTS
#define EFPI_PASS_SLOTS 16
#endif
constexpr int kQSlots = EFPI_PASS_SLOTS;
constexpr int kQBelow = 7;                     // window starts below the reference cell
#ifndef EFPI_PASS_RBINS
#define EFPI_PASS_RBINS 16
#endif
constexpr int kRBins = EFPI_PASS_RBINS;        // coarse-block bins of a wave's window
constexpr int kRBelow = 7;
constexpr int kENodes = 64;                    // field window: cells (64 + 1 nodes)
constexpr int kEBelow = 32;
// Weights (and momenta w V) above this bound could carry a binary64 bin past 2^53
// (at most 16384 / 4 / kQSlots ions share a slot at the largest tile, each below
// kQSlots 2^40): flagged.
constexpr float kWeightBound = (float)kQSlots;

// NM: restricted moments (2: density and momentum; 3: and the second moment).
template <int NM>
struct WaveLds {
  float2 e[kENodes + 2];          // (E^p, E_n) at the window's nodes (one spare entry)
  double q[kQBins][kQSlots];      // fixed-point charge shares (integer-valued binary64)
  double r[NM][kRBins][kQSlots];  // fixed-point moment shares per coarse block
};
template <int MODE>
constexpr int kMoments = (MODE & kMoment3) != 0 ? 3 : 2;


__device__ __forceinline__ int find_replica(const int64_t* prefix, int n, int64_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// 8- and 16-byte accesses at a byte offset from a uniform base (native vector
// types, so that the global address space carries through the copy).  Every ion
// is read and written once per pass, so the particle streams are marked
// nontemporal (EFPI_PASS_NT bit 0: loads, bit 1: stores).
#ifndef EFPI_PASS_NT
#define EFPI_PASS_NT 3
#endif
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ T ldv(const EFPI_GLOBAL void* base, unsigned byte_off) {
  const EFPI_GLOBAL T* a = (const EFPI_GLOBAL T*)((const EFPI_GLOBAL char*)base + byte_off);
  if constexpr ((EFPI_PASS_NT & 1) != 0) return __builtin_nontemporal_load(a);
  else return *a;
}
template <class T>
__device__ __forceinline__ void stv(EFPI_GLOBAL void* base, unsigned byte_off, T v) {
  EFPI_GLOBAL T* a = (EFPI_GLOBAL T*)((EFPI_GLOBAL char*)base + byte_off);
  if constexpr ((EFPI_PASS_NT & 2) != 0) __builtin_nontemporal_store(v, a);
  else *a = v;
}

// The ions of one wave: `cnt` slots from `t0` of replica R.  MODE as in k_particles.
template <int MODE, bool kPeriodic>
__device__ __forceinline__ void wave_range(const RepDev& R, WaveLds<kMoments<MODE>>& L,
                                           int64_t t0, unsigned cnt, int p, double pd, bool fresh, int qsel,
                                           bool& big) {
  constexpr bool restrict_ = (MODE & kRestrict) != 0;
  constexpr bool push = (MODE & kPush) != 0;
  constexpr bool deposit = push || (MODE & kDepositOnly) != 0;
  constexpr bool field = restrict_ || push;
  constexpr int NM = kMoments<MODE>;
  const int lane = __lane_id();
  const int n = R.n_cells;
  const int nmask = n - 1;
  const float dt = (float)R.dt;
  const float inv_h = (float)R.inv_h;
  const int levels = R.levels;
  const int nc = R.n_coarse;
  const int ncmask = nc - 1;
  // p < 0: plain restriction of the current state (tau = 0, snapshot slot 0)
  // (pd = p as binary64, a kernel argument, so no conversion is kept live)
  const float tau = p < 0 ? 0.f : (float)(R.macro_dt - pd * R.dt);
  const bool coev = R.coevolving != 0 && p >= 0;
  const EFPI_GLOBAL float* __restrict__ e = gmem(R.e);
  const EFPI_GLOBAL float* __restrict__ en = gmem(R.en);
  EFPI_GLOBAL int16_t* __restrict__ cellp = gmem(R.cell + t0);
  EFPI_GLOBAL float* __restrict__ fracp = gmem(R.frac + t0);
  EFPI_GLOBAL float* __restrict__ velp = gmem(R.v + t0);
  const EFPI_GLOBAL float* __restrict__ wp = gmem(R.w + t0);
  long long* qg = reinterpret_cast<long long*>(R.q[qsel]);
  long long* rb = reinterpret_cast<long long*>(R.rbins) + (int64_t)(p < 0 ? 0 : p) * NM * nc;
  const float half_dt = 0.5f * dt;
  const float half_dt_r = fresh ? 0.f : half_dt;  // snapshot velocity v + half_dt_r E
  const float dt_push = fresh ? half_dt : dt;     // push: v + dt_push E
  const int lmask = (1 << levels) - 1;
  const float dt_inv_h = dt * inv_h;
  const float tau_inv_h = coev ? tau * inv_h : 0.f;
  const float tau_e = coev ? tau : 0.f;

  // Reference cell of the range: midway between its first and last cells (a
  // cell-sorted store), or whichever of them is live.  Ions drift after a sort,
  // so the last ion may sit a cell or two below the first: on a periodic grid
  // the midpoint is taken along the shorter way round.
  const int c_lo = __builtin_amdgcn_readfirstlane((int)*at(cellp, 0u));
  const int c_hi = __builtin_amdgcn_readfirstlane((int)*at(cellp, cnt - 1u));
  const bool lo_ok = (unsigned)c_lo < (unsigned)n, hi_ok = (unsigned)c_hi < (unsigned)n;
  int cref;
  if (lo_ok && hi_ok) {
    if (kPeriodic) {
      int d = (c_hi - c_lo) & nmask;
      if (d > (n >> 1)) d -= n;
      cref = (c_lo + (d >> 1)) & nmask;
    } else {
      cref = (c_lo + c_hi) >> 1;
    }
  } else {
    cref = lo_ok ? c_lo : (hi_ok ? c_hi : 0);
  }
  const int ebase = cref - kEBelow;
  const int qbase = cref - kQBelow;
  const int rbase = (cref >> levels) - kRBelow;

  // field window: node ebase + k (wrapped, or clamped to the wall nodes) at k, so
  // that a cell c with k = c - ebase in [0, kENodes) finds both of its nodes
  if (field) {
    for (int k = lane; k <= kENodes; k += kWave) {
      const int g = kPeriodic ? ((ebase + k) & nmask) : min(max(ebase + k, 0), n);
      L.e[k] = make_float2(e[g], (restrict_ && coev) ? en[g] : 0.f);
    }
  }
  if (deposit) {
    uint4* z = reinterpret_cast<uint4*>(&L.q[0][0]);
    for (int k = lane; k < (int)(sizeof L.q / sizeof(uint4)); k += kWave) z[k] = make_uint4(0, 0, 0, 0);
  }
  if (restrict_) {
    uint4* z = reinterpret_cast<uint4*>(&L.r[0][0][0]);
    for (int k = lane; k < (int)(sizeof L.r / sizeof(uint4)); k += kWave) z[k] = make_uint4(0, 0, 0, 0);
  }
  wave_lds_sync();

  double* const qbin = &L.q[0][lane & (kQSlots - 1)];
  double* const rbin0 = &L.r[0][0][lane & (kQSlots - 1)];
  double* const rbin1 = &L.r[1][0][lane & (kQSlots - 1)];
  double* const rbin2 = &L.r[NM - 1][0][lane & (kQSlots - 1)];  // NM = 3 only

  // one batch's raw vectors: kHalves x (4 cells, 4 offsets, 4 velocities, 4 weights)
  struct Raw {
    u32x2 c[kHalves];
    f32x4 f[kHalves], v[kHalves], w[kHalves];
  };
  // a group that starts inside the range is read whole: slots past the range lie
  // inside the store's allocation (rounded up to 64 slots) and are treated as
  // absorbed and written back unchanged
  auto load = [&](unsigned b0, Raw& x) {
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      const unsigned g = b0 + (unsigned)h * (kGroup * kWave) + (unsigned)lane * kGroup;
      x.c[h] = u32x2{0xFFFFFFFFu, 0xFFFFFFFFu};
      x.f[h] = f32x4{0.f, 0.f, 0.f, 0.f};
      x.v[h] = x.f[h];
      x.w[h] = x.f[h];
      if (g < cnt) {
        x.c[h] = ldv<u32x2>(cellp, g * 2u);
        x.f[h] = ldv<f32x4>(fracp, g * 4u);
        x.v[h] = ldv<f32x4>(velp, g * 4u);
        x.w[h] = ldv<f32x4>(wp, g * 4u);
      }
    }
  };
  Raw cur;
  load(0u, cur);
  for (unsigned b0 = 0; b0 < cnt; b0 += kBatch) {
    const bool more = b0 + kBatch < cnt;  // uniform over the wave
    int cl[kPer];
    float fr[kPer], vv[kPer], ww[kPer];
    unsigned gi[kHalves];
    bool gvalid[kHalves];
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      const unsigned g = b0 + (unsigned)h * (kGroup * kWave) + (unsigned)lane * kGroup;
      gi[h] = g;
      gvalid[h] = g < cnt;
      u32x2 c2 = cur.c[h];
      const f32x4 f4 = cur.f[h], v4 = cur.v[h], w4 = cur.w[h];
      // slots of a group past the end of the range count as absorbed
      if (__builtin_expect(g + kGroup > cnt, 0)) {
        const unsigned left = cnt - g;  // 1 .. 3 when the group is valid
        if (!gvalid[h] || left < 2) c2.x |= 0xFFFF0000u;
        if (!gvalid[h] || left < 3) c2.y |= 0x0000FFFFu;
        if (!gvalid[h] || left < 4) c2.y |= 0xFFFF0000u;
      }
      const int base = h * kGroup;
      cl[base + 0] = (int)(short)(c2.x & 0xFFFFu);
      cl[base + 1] = (int)(short)(c2.x >> 16);
      cl[base + 2] = (int)(short)(c2.y & 0xFFFFu);
      cl[base + 3] = (int)(short)(c2.y >> 16);
      fr[base + 0] = f4.x; fr[base + 1] = f4.y; fr[base + 2] = f4.z; fr[base + 3] = f4.w;
      vv[base + 0] = v4.x; vv[base + 1] = v4.y; vv[base + 2] = v4.z; vv[base + 3] = v4.w;
      ww[base + 0] = w4.x; ww[base + 1] = w4.y; ww[base + 2] = w4.z; ww[base + 3] = w4.w;
    }
    // live ions: a cell inside [0, N)
    bool alive[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) alive[j] = (unsigned)cl[j] < (unsigned)n;
    // node fields at both ends of each ion's cell, from the window; ions outside
    // it (unsorted or far-drifted stores) read global memory
    float e0[kPer], e1[kPer], n0[kPer], n1[kPer];
    if (field) {
      bool outside = false;
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int c = cl[j];
        const int k = kPeriodic ? ((c - ebase) & nmask) : (c - ebase);
        const bool inw = (unsigned)k < (unsigned)kENodes;
        const int kk = inw ? k : 0;
        outside |= alive[j] && !inw;
        const float2 a = L.e[kk];
        const float2 b = L.e[kk + 1];
        e0[j] = a.x;
        n0[j] = a.y;
        e1[j] = b.x;
        n1[j] = b.y;
      }
      if (__builtin_expect(__ballot(outside) != 0ull, 0)) {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
          const int c = cl[j];
          const int k = kPeriodic ? ((c - ebase) & nmask) : (c - ebase);
          if (alive[j] && (unsigned)k >= (unsigned)kENodes) {
            const int cr = kPeriodic ? ((c + 1) & nmask) : c + 1;
            e0[j] = e[c];
            e1[j] = e[cr];
            n0[j] = (restrict_ && coev) ? en[c] : 0.f;
            n1[j] = (restrict_ && coev) ? en[cr] : 0.f;
          }
        }
      }
    }
    float epa[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) epa[j] = field ? fmaf(fr[j], e1[j] - e0[j], e0[j]) : 0.f;

    if (restrict_) {
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const float f = fr[j];
        const float w = ww[j];
        const int cs = alive[j] ? cl[j] : 0;
        // Snapshot p: time-centred velocity, then the approximate characteristic
        // over tau = Delta t - p dt (eq. B.4) and CIC at the moved position (eq. B.5).
        const float vpc = fmaf(half_dt_r, epa[j], vv[j]);  // half_dt_r = 0 on a fresh state
        const float enx = fmaf(f, n1[j] - n0[j], n0[j]);
        const float xt = fmaf(tau_inv_h, vpc, f);
        const float vt = fmaf(tau_e, enx, vpc);
        const float fl = floorf(xt);
        const float fx = xt - fl;
        const bool wrap_up = fx >= 1.f;
        const int ct0 = cs + (int)fl + (wrap_up ? 1 : 0);
        const int ct = kPeriodic ? (ct0 & nmask) : ct0;
        // walls: positions moved outside [0, L) are in flight to a wall, not counted
        const bool in = alive[j] && (kPeriodic || (unsigned)ct < (unsigned)n);
        const int bl = ct >> levels;
        // both nodes of cell ct in block bl: ct is not the block's last cell, or
        // (walls) the block is the last one, which also owns wall node N, or
        // (periodic) there is a single block
        const bool last = (ct & lmask) == lmask;
        const bool same = !last || (kPeriodic ? nc == 1 : bl == nc - 1);
        // right-node share theta, zero when both nodes are in the same block
        const float th = (wrap_up || same) ? 0.f : fx;
        // fixed-point mass and momentum with their CIC split, as the charge
        // deposit splits the charge: right share rint(theta q), left q - right
        const float wv = w * vt;
        const float wvv = NM == 3 ? wv * vt : 0.f;
        big |= in && !(fabsf(wv) < kWeightBound && fabsf(wvv) < kWeightBound);
        const double qm = fx_charge(w);
        const double qv = fx_charge(wv);
        const double qs = NM == 3 ? fx_charge(wvv) : 0.0;
        const double thd = (double)th;
        const double qm_r = __builtin_rint(thd * qm), qv_r = __builtin_rint(thd * qv);
        const double qm_l = qm - qm_r, qv_l = qv - qv_r;
        const double qs_r = NM == 3 ? __builtin_rint(thd * qs) : 0.0, qs_l = qs - qs_r;
        const int d = kPeriodic ? ((bl - rbase) & ncmask) : (bl - rbase);
        const bool inr = (unsigned)d < (unsigned)(kRBins - 1);
        if (in && inr) {
          lds_add(rbin0 + d * kQSlots, qm_l);
          lds_add(rbin1 + d * kQSlots, qv_l);
          if (NM == 3) lds_add(rbin2 + d * kQSlots, qs_l);
          if (th != 0.f) {
            lds_add(rbin0 + (d + 1) * kQSlots, qm_r);
            lds_add(rbin1 + (d + 1) * kQSlots, qv_r);
            if (NM == 3) lds_add(rbin2 + (d + 1) * kQSlots, qs_r);
          }
        } else if (in) {
          gatomic_add(rb + bl, rint_i64(qm_l));
          gatomic_add(rb + nc + bl, rint_i64(qv_l));
          if (NM == 3) gatomic_add(rb + 2 * nc + bl, rint_i64(qs_l));
          if (th != 0.f) {
            const int br = kPeriodic ? ((bl + 1) & ncmask) : bl + 1;
            gatomic_add(rb + br, rint_i64(qm_r));
            gatomic_add(rb + nc + br, rint_i64(qv_r));
            if (NM == 3) gatomic_add(rb + 2 * nc + br, rint_i64(qs_r));
          }
        }
      }
    }
    if (deposit) {
      int cn_st[kPer];
      float fn_st[kPer], vn_st[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const float f = fr[j];
        const float v = vv[j];
        const float w = ww[j];
        const int cs = alive[j] ? cl[j] : 0;
        int cn = cs;
        float fn = f, vn = v;
        if (push) {
          vn = fmaf(dt_push, epa[j], v);
          const float xn = fmaf(dt_inv_h, vn, f);
          const float fl = floorf(xn);
          const bool wrap_up = (xn - fl) >= 1.f;
          fn = wrap_up ? 0.f : xn - fl;
          cn = cs + (int)fl + (wrap_up ? 1 : 0);
          cn = kPeriodic ? (cn & nmask) : ((unsigned)cn < (unsigned)n ? cn : -1);  // walls absorb
        }
        // stored state: live ions pushed, the rest written back as read
        cn_st[j] = alive[j] ? cn : cl[j];
        fn_st[j] = alive[j] ? fn : f;
        vn_st[j] = alive[j] ? vn : v;
        const bool dep = alive[j] && cn >= 0;
        big |= dep && !(fabsf(w) < kWeightBound);
        const double q = fx_charge(w);
        const double qr = fx_share(fn, q);
        const double ql = q - qr;
        const int d = kPeriodic ? ((cn - qbase) & nmask) : (cn - qbase);
        const bool inq = (unsigned)d < (unsigned)(kQBins - 1);
        if (dep && inq) {
          lds_add(qbin + d * kQSlots, ql);
          lds_add(qbin + (d + 1) * kQSlots, qr);
        } else if (dep) {
          const int cr = kPeriodic ? ((cn + 1) & nmask) : cn + 1;
          gatomic_add(qg + cn, rint_i64(ql));
          gatomic_add(qg + cr, rint_i64(qr));
        }
      }
      if (push) {
#pragma unroll
        for (int h = 0; h < kHalves; ++h) {
          if (gvalid[h]) {
            const int b = h * kGroup;
            const u32x2 c2 = {
                ((unsigned)cn_st[b + 0] & 0xFFFFu) | ((unsigned)cn_st[b + 1] << 16),
                ((unsigned)cn_st[b + 2] & 0xFFFFu) | ((unsigned)cn_st[b + 3] << 16)};
            stv<u32x2>(cellp, gi[h] * 2u, c2);
            const f32x4 f4 = {fn_st[b], fn_st[b + 1], fn_st[b + 2], fn_st[b + 3]};
            const f32x4 v4 = {vn_st[b], vn_st[b + 1], vn_st[b + 2], vn_st[b + 3]};
            stv<f32x4>(fracp, gi[h] * 4u, f4);
            stv<f32x4>(velp, gi[h] * 4u, v4);
          }
        }
      }
    }
    if (more) load(b0 + kBatch, cur);
  }

  wave_lds_sync();
  if (deposit) {
    // bin d's total: lane l sums kQSlots / 4 of the slots of bin l & 15 (rotated by d so
    // that the reads of one pass fall in different banks), then the four partial
    // sums of every bin are added across lanes; the sums are exact
    constexpr int per = kQSlots * kQBins / kWave;  // slots summed per lane
    const int d = lane & (kQBins - 1);
    const int g = lane / kQBins;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < per; ++i) s += L.q[d][g * per + ((i + d) & (per - 1))];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (g == 0 && s != 0.0) {
      const int node = kPeriodic ? ((qbase + d) & nmask) : (qbase + d);
      gatomic_add(qg + node, rint_i64(s));
    }
  }
  if (restrict_) {
    // (moment, block) bin b = lane % nb: the lanes b, b + nb, ... each sum a run
    // of its slots (rotated by b across the banks), then add their partial sums;
    // the sums are exact
    constexpr int nb = 2 * kRBins;
    constexpr int ns = kQSlots * nb / kWave;  // slots summed per lane
    const int b = lane & (nb - 1);
    const int m = b / kRBins;
    const int d = b % kRBins;
    const int g = lane / nb;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < ns; ++i) t += L.r[m][d][g * ns + ((i + b) & (ns - 1))];
#pragma unroll
    for (int o = nb; o < kWave; o <<= 1) t += __shfl_xor(t, o);
    if (g == 0 && t != 0.0) {
      const int blk = kPeriodic ? ((rbase + d) & ncmask) : (rbase + d);
      gatomic_add(rb + (int64_t)m * nc + blk, rint_i64(t));
    }
    if (NM == 3) {
      // the second-moment plane alone: bin b = lane % kRBins, the same way
      constexpr int ns3 = kQSlots * kRBins / kWave;
      const int b3 = lane & (kRBins - 1);
      const int g3 = lane / kRBins;
      double t3 = 0.0;
#pragma unroll
      for (int i = 0; i < ns3; ++i) t3 += L.r[NM - 1][b3][g3 * ns3 + ((i + b3) & (ns3 - 1))];
#pragma unroll
      for (int o = kRBins; o < kWave; o <<= 1) t3 += __shfl_xor(t3, o);
      if (g3 == 0 && t3 != 0.0) {
        const int blk = kPeriodic ? ((rbase + b3) & ncmask) : (rbase + b3);
        gatomic_add(rb + 2 * (int64_t)nc + blk, rint_i64(t3));
      }
    }
  }
  wave_lds_sync();
}

// MODE (compile time): kRestrict | kPush for a burst step, kPush for plain PIC,
// kRestrict for the last snapshot of a burst, kDepositOnly for a charge deposit.
template <int MODE>
__device__ __forceinline__ void particles_body(WaveLds<kMoments<MODE>>* lds,
                                               const RepDev* __restrict__ reps,
                                               const int64_t* __restrict__ item_prefix,
                                               int n_reps, int64_t total_items, int tile, int p,
                                               double pd, int fresh_flag, int qsel,
                                               uint32_t* __restrict__ status) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  WaveLds<kMoments<MODE>>& L = lds[wave];
  const bool fresh = fresh_flag != 0;
  const int64_t quarter = tile / kWaves;
  bool big = false;
  for (int64_t item = blockIdx.x; item < total_items; item += gridDim.x) {
    const int r = find_replica(item_prefix, n_reps, item);
    const RepDev& R = reps[r];
    const int64_t np = uniform_i64(*gmem(R.np));
    const int64_t t0 = (item - R.item_begin) * (int64_t)tile + wave * quarter;
    if (t0 >= np) continue;
    const unsigned cnt = (unsigned)min(quarter, np - t0);
    if (R.bc == 0)
      wave_range<MODE, true>(R, L, t0, cnt, p, pd, fresh, qsel, big);
    else
      wave_range<MODE, false>(R, L, t0, cnt, p, pd, fresh, qsel, big);
  }
  if (__ballot(big) != 0ull && __lane_id() == 0)
    __hip_atomic_fetch_or(status, (uint32_t)EFPI_DEV_WEIGHT, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
}

template <int MODE>
__global__ __launch_bounds__(kThreads)
void k_particles(const RepDev* __restrict__ reps, const int64_t* __restrict__ item_prefix,
                 int n_reps, int64_t total_items, int tile, int p, double pd, int fresh_flag,
                 int qsel, uint32_t* __restrict__ status) {
  __shared__ WaveLds<2> lds[kWaves];
  particles_body<MODE>(lds, reps, item_prefix, n_reps, total_items, tile, p, pd, fresh_flag,
                       qsel, status);
}

// The three-moment restriction (kMoment3 in MODE) held to 4 waves per SIMD: its
// extra share per ion would otherwise take the kernel past 128 VGPRs (3 waves).
template <int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_particles3(const RepDev* __restrict__ reps, const int64_t* __restrict__ item_prefix,
                  int n_reps, int64_t total_items, int tile, int p, double pd, int fresh_flag,
                  int qsel, uint32_t* __restrict__ status) {
  __shared__ WaveLds<3> lds[kWaves];
  particles_body<MODE>(lds, reps, item_prefix, n_reps, total_items, tile, p, pd, fresh_flag,
                       qsel, status);
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
                 int64_t total_items, int tile, int p, int fresh, int qsel, uint32_t* d_status) {
  auto go = [&](auto kernel) {
    if (ev0 && ev1)
      hipExtLaunchKernelGGL(kernel, grid, dim3(kThreads), 0, stream, ev0, ev1, 0, d_reps,
                            d_item_prefix, n_reps, total_items, tile, p, (double)p, fresh, qsel,
                            d_status);
    else
      hipLaunchKernelGGL(kernel, grid, dim3(kThreads), 0, stream, d_reps, d_item_prefix, n_reps,
                         total_items, tile, p, (double)p, fresh, qsel, d_status);
  };
  if constexpr (kMoments<MODE> == 3) go(k_particles3<MODE>);
  else go(k_particles<MODE>);
}
}  // namespace

void launch_particles(const RepDev* d_reps, const int64_t* d_item_prefix, int n_reps,
                      int64_t total_items, int tile, int grid_blocks, int p, int flags,
                      int qsel, uint32_t* d_status, hipStream_t stream, hipEvent_t ev0,
                      hipEvent_t ev1) {
  if (total_items <= 0) return;
  const int64_t g = grid_blocks > 0 ? min((int64_t)grid_blocks, total_items) : total_items;
  const int fresh = (flags & kFresh) ? 1 : 0;
  int mode = flags & (kRestrict | kPush | kDepositOnly | kMoment3);
  if ((mode & kRestrict) == 0) mode &= ~kMoment3;  // the second moment rides on a restriction
  const dim3 grid((unsigned)g);
  switch (mode) {
    case kRestrict | kPush | kMoment3:
      launch_mode<kRestrict | kPush | kMoment3>(grid, stream, ev0, ev1, d_reps, d_item_prefix,
                                                n_reps, total_items, tile, p, fresh, qsel,
                                                d_status);
      break;
    case kRestrict | kMoment3:
      launch_mode<kRestrict | kMoment3>(grid, stream, ev0, ev1, d_reps, d_item_prefix, n_reps,
                                        total_items, tile, p, fresh, qsel, d_status);
      break;
    case kRestrict | kPush:
      launch_mode<kRestrict | kPush>(grid, stream, ev0, ev1, d_reps, d_item_prefix, n_reps,
                                     total_items, tile, p, fresh, qsel, d_status);
      break;
    case kPush:
      launch_mode<kPush>(grid, stream, ev0, ev1, d_reps, d_item_prefix, n_reps, total_items, tile,
                         p, fresh, qsel, d_status);
      break;
    case kRestrict:
      launch_mode<kRestrict>(grid, stream, ev0, ev1, d_reps, d_item_prefix, n_reps, total_items,
                             tile, p, fresh, qsel, d_status);
      break;
    default:
      launch_mode<kDepositOnly>(grid, stream, ev0, ev1, d_reps, d_item_prefix, n_reps,
                                total_items, tile, p, fresh, qsel, d_status);
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
