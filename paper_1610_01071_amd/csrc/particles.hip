// Particle pass of the fine burst: field gather, leapfrog push, boundaries,
// fixed-point CIC charge deposit (Sec. 2.2) and the co-evolving restriction
// snapshot of the density and momentum moments (App. B, eqs. B.4-B.5), fused in
// one streaming pass over the structure-of-arrays ion store.
//
// Work decomposition: every replica's particle slots are cut into tiles of
// `tile` consecutive particles; a persistent grid walks the (replica, tile)
// items.  Inside a tile, 64-lane waves first merge lanes that hit the same node
// or coarse block (wave-wide integer sums), then one lane adds the merged value
// into int64 bins held in LDS for a window of nodes/blocks around the tile; the
// window is flushed to global memory with 64-bit integer atomics at the end of
// the tile.  Targets outside the window go straight to global atomics.  All
// sums are of integers, so the result is independent of scheduling order.
#include "efpi_internal.h"

namespace efpi {
namespace {

constexpr int kThreads = 256;
constexpr int kBatch = 4;       // particles per thread loaded ahead of use
constexpr int kQWin = 256;      // node window (int64 bins)
constexpr int kQMargin = 16;
constexpr int kRWin = 64;       // coarse block window per moment
constexpr int kRMargin = 8;

// Wave-wide sums with a fixed DPP pattern (inclusive scan by row shifts 1, 2, 3
// of the input, then 4 and 8 inside each 16-lane row, then row broadcasts 15 and
// 31 across rows; lane 63 holds the total).  The pattern, and therefore the
// order of every addition, does not depend on scheduling, so FP32 sums are
// reproducible bit for bit.  All 64 lanes must be active.
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, ROW_MASK, BANK_MASK, BOUND);
}

__device__ __forceinline__ int wave_sum_i32(int x) {
  int t = x + dpp_i<0x111, 0xf, 0xf, true>(x);
  t += dpp_i<0x112, 0xf, 0xf, true>(x);
  t += dpp_i<0x113, 0xf, 0xf, true>(x);
  t += dpp_i<0x114, 0xf, 0xe, false>(t);
  t += dpp_i<0x118, 0xf, 0xc, false>(t);
  t += dpp_i<0x142, 0xa, 0xf, false>(t);
  t += dpp_i<0x143, 0xc, 0xf, false>(t);
  return __builtin_amdgcn_readlane(t, 63);
}

__device__ __forceinline__ float wave_sum_f32(float x) {
  float t = x + __int_as_float(dpp_i<0x111, 0xf, 0xf, true>(__float_as_int(x)));
  t += __int_as_float(dpp_i<0x112, 0xf, 0xf, true>(__float_as_int(x)));
  t += __int_as_float(dpp_i<0x113, 0xf, 0xf, true>(__float_as_int(x)));
  t += __int_as_float(dpp_i<0x114, 0xf, 0xe, false>(__float_as_int(t)));
  t += __int_as_float(dpp_i<0x118, 0xf, 0xc, false>(__float_as_int(t)));
  t += __int_as_float(dpp_i<0x142, 0xa, 0xf, false>(__float_as_int(t)));
  t += __int_as_float(dpp_i<0x143, 0xc, 0xf, false>(__float_as_int(t)));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 63));
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

// q = rint(w 2^40): the particle's charge in fixed point.
__device__ __forceinline__ long long fx_charge(float w) { return rint_i64((double)w * kFxScale); }
// Right-node share rint(theta q) in binary64 (one rounded product, then ties-to-even).
__device__ __forceinline__ long long fx_share(float theta, long long q) {
  return rint_i64((double)theta * (double)q);
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
    atomicAdd(reinterpret_cast<unsigned long long*>(&w.glob[idx]), (unsigned long long)val);
}

// Each lane holds kBatch ions.  Targets shared by many lanes are merged: the
// lowest active lane's target is taken, every lane sums its own ions with that
// target, the sums are reduced across the wave and one lane adds the result to
// the bins.  When fewer than kMinMerge lanes hold the target (scattered ions),
// every lane adds all of its remaining ions directly instead, so a scattered
// wave costs one atomic per ion rather than one merge round per distinct target.
constexpr int kMinMerge = 8;

// Charge deposit: ion j adds a[j] to node key[j] and b[j] to node key[j] + 1
// (wrapping to 0 at `wrap`, or no wrap when wrap = -1).  Exact int64 sums.
__device__ __forceinline__ void merge_charge(int (&key)[kBatch], const long long (&a)[kBatch],
                                             const long long (&b)[kBatch], int wrap,
                                             const Window& win) {
  const int lane = __lane_id();
  while (true) {
    int mine = -1;
#pragma unroll
    for (int j = kBatch - 1; j >= 0; --j)
      if (key[j] >= 0) mine = key[j];
    const unsigned long long act = __ballot(mine >= 0);
    if (act == 0ull) break;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int lk = __builtin_amdgcn_readlane(mine, leader);
    long long sa = 0, sb = 0;
    bool has = false;
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (key[j] == lk) {
        sa += a[j];
        sb += b[j];
        has = true;
        key[j] = -1;
      }
    if (__popcll(__ballot(has)) < kMinMerge) {
      int r = lk + 1;
      if (r == wrap) r = 0;
      if (has) {
        add_to(win, lk, sa);
        add_to(win, r, sb);
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
        if (key[j] >= 0) {
          int rr = key[j] + 1;
          if (rr == wrap) rr = 0;
          add_to(win, key[j], a[j]);
          add_to(win, rr, b[j]);
          key[j] = -1;
        }
      break;
    }
    const long long ta = wave_sum_i64(sa);
    const long long tb = wave_sum_i64(sb);
    if (lane == leader) {
      int r = lk + 1;
      if (r == wrap) r = 0;
      add_to(win, lk, ta);
      add_to(win, r, tb);
    }
  }
}

// Restriction snapshot: ion j adds (a0, a1)[j] to block key[j] and (b0, b1)[j]
// to block key[j] + 1 for the (density, momentum) moments.  FP32 partial sums
// in a fixed order, converted to fixed point before the integer atomics.
__device__ __forceinline__ void merge_moments(int (&key)[kBatch], const float (&a0)[kBatch],
                                              const float (&a1)[kBatch],
                                              const float (&b0)[kBatch],
                                              const float (&b1)[kBatch], int wrap,
                                              const Window& w0, const Window& w1) {
  const int lane = __lane_id();
  while (true) {
    int mine = -1;
#pragma unroll
    for (int j = kBatch - 1; j >= 0; --j)
      if (key[j] >= 0) mine = key[j];
    const unsigned long long act = __ballot(mine >= 0);
    if (act == 0ull) break;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int lk = __builtin_amdgcn_readlane(mine, leader);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    bool has = false;
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (key[j] == lk) {
        s0 += a0[j];
        s1 += a1[j];
        s2 += b0[j];
        s3 += b1[j];
        has = true;
        key[j] = -1;
      }
    if (__popcll(__ballot(has)) < kMinMerge) {
      int r = lk + 1;
      if (r == wrap) r = 0;
      if (has) {
        add_to(w0, lk, fx_of(s0));
        add_to(w1, lk, fx_of(s1));
        add_to(w0, r, fx_of(s2));
        add_to(w1, r, fx_of(s3));
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
        if (key[j] >= 0) {
          int rr = key[j] + 1;
          if (rr == wrap) rr = 0;
          add_to(w0, key[j], fx_of(a0[j]));
          add_to(w1, key[j], fx_of(a1[j]));
          add_to(w0, rr, fx_of(b0[j]));
          add_to(w1, rr, fx_of(b1[j]));
          key[j] = -1;
        }
      break;
    }
    const float t0 = wave_sum_f32(s0);
    const float t1 = wave_sum_f32(s1);
    const float t2 = wave_sum_f32(s2);
    const float t3 = wave_sum_f32(s3);
    if (lane == leader) {
      int r = lk + 1;
      if (r == wrap) r = 0;
      add_to(w0, lk, fx_of(t0));
      add_to(w1, lk, fx_of(t1));
      add_to(w0, r, fx_of(t2));
      add_to(w1, r, fx_of(t3));
    }
  }
}

// MODE (compile time): kRestrict | kPush for a burst step, kPush for plain PIC,
// kRestrict for the last snapshot of a burst, kDepositOnly for a charge deposit.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_particles(const RepDev* __restrict__ reps,
                                                         const int64_t* __restrict__ item_prefix,
                                                         int n_reps, int64_t total_items,
                                                         int tile, int p, int fresh_flag,
                                                         int qsel) {
  __shared__ long long lds_q[kQWin];
  __shared__ long long lds_r[2][kRWin];
  const int tid = threadIdx.x;
  const bool fresh = fresh_flag != 0;
  constexpr bool restrict_ = (MODE & kRestrict) != 0;
  constexpr bool push = (MODE & kPush) != 0;
  constexpr bool deposit = push || (MODE & kDepositOnly) != 0;

  for (int64_t item = blockIdx.x; item < total_items; item += gridDim.x) {
    const int r = find_replica(item_prefix, n_reps, item);
    const RepDev& R = reps[r];
    const int64_t np = *R.np;
    const int64_t i0 = (item - R.item_begin) * (int64_t)tile;
    if (i0 >= np) continue;
    const int64_t i1 = min(i0 + (int64_t)tile, np);
    const int n = R.n_cells;
    const bool periodic = (R.bc == 0);
    const int nmask = n - 1;
    const float dt = (float)R.dt;
    const float inv_h = (float)R.inv_h;
    const int levels = R.levels;
    const int nc = R.n_coarse;
    // p < 0: plain restriction of the current state (tau = 0, snapshot slot 0)
    const float tau = p < 0 ? 0.f : (float)(R.macro_dt - (double)p * R.dt);
    const bool coev = R.coevolving != 0 && p >= 0;
    const float* __restrict__ e = R.e;
    const float* __restrict__ en = R.en;
    int16_t* __restrict__ cellp = R.cell;
    float* __restrict__ fracp = R.frac;
    float* __restrict__ vp_ = R.v;
    const float* __restrict__ wp = R.w;

    const int c_first = cellp[i0];
    Window wq{lds_q, c_first - kQMargin, kQWin, reinterpret_cast<long long*>(R.q[qsel])};
    long long* rb = reinterpret_cast<long long*>(R.rbins) + (int64_t)(p < 0 ? 0 : p) * 2 * nc;
    const int rbase = (c_first >> levels) - kRMargin;
    Window wr0{lds_r[0], rbase, kRWin, rb};
    Window wr1{lds_r[1], rbase, kRWin, rb + nc};

    for (int k = tid; k < kQWin; k += kThreads) lds_q[k] = 0;
    for (int k = tid; k < 2 * kRWin; k += kThreads) (&lds_r[0][0])[k] = 0;
    __syncthreads();

    for (int64_t b0 = i0; b0 < i1; b0 += (int64_t)kThreads * kBatch) {
      int cl[kBatch];
      float fr[kBatch], vv[kBatch], ww[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int64_t idx = b0 + (int64_t)j * kThreads + tid;
        if (idx < i1) {
          cl[j] = cellp[idx];
          fr[j] = fracp[idx];
          vv[j] = vp_[idx];
          ww[j] = wp[idx];
        } else {
          cl[j] = -1;
          fr[j] = 0.f;
          vv[j] = 0.f;
          ww[j] = 0.f;
        }
      }
      int rkey[kBatch], dkey[kBatch];
      float ra0[kBatch], ra1[kBatch], rb0[kBatch], rb1[kBatch];
      long long da[kBatch], db[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int64_t idx = b0 + (int64_t)j * kThreads + tid;
        int c = cl[j];
        float f = fr[j];
        float v = vv[j];
        const float w = ww[j];
        const bool alive = c >= 0 && c < n;  // cells outside [0, N) are treated as absorbed
        float ep = 0.f;
        if (alive && (restrict_ || push)) {
          const int cr = periodic ? ((c + 1) & nmask) : c + 1;
          ep = (1.f - f) * e[c] + f * e[cr];
        }
        rkey[j] = -1;
        ra0[j] = ra1[j] = rb0[j] = rb1[j] = 0.f;
        if (restrict_ && alive) {
          // Snapshot p: time-centred velocity, then the approximate characteristic
          // over tau = Delta t - p dt (eq. B.4) and CIC at the moved position (eq. B.5).
          const float vp = fresh ? v : v + 0.5f * dt * ep;
          float xt = f;
          float vt = vp;
          if (coev) {
            const int cr = periodic ? ((c + 1) & nmask) : c + 1;
            const float enx = (1.f - f) * en[c] + f * en[cr];
            xt = f + tau * vp * inv_h;
            vt = vp + tau * enx;
          }
          const float fl = floorf(xt);
          int ct = c + (int)fl;
          float th = xt - fl;
          if (th >= 1.f) { th = 0.f; ct += 1; }
          bool in = true;
          if (periodic) ct &= nmask;
          else in = (ct >= 0 && ct < n);
          if (in) {
            const float wv = w * vt;
            const int bl = ct >> levels;
            int nr = ct + 1;
            if (periodic) nr &= nmask;
            int br = nr >> levels;
            if (br >= nc) br = nc - 1;  // wall node N joins the last block
            rkey[j] = bl;
            if (br == bl) {
              ra0[j] = w;
              ra1[j] = wv;
            } else {
              ra0[j] = w - w * th;
              ra1[j] = wv - wv * th;
              rb0[j] = w * th;
              rb1[j] = wv * th;
            }
          }
        }
        dkey[j] = -1;
        da[j] = db[j] = 0;
        if (deposit && alive) {
          if (push) {
            v = fresh ? v + 0.5f * dt * ep : v + dt * ep;
            const float xn = f + dt * v * inv_h;
            const float fl = floorf(xn);
            c += (int)fl;
            f = xn - fl;
            if (f >= 1.f) { f = 0.f; c += 1; }
            if (periodic) c &= nmask;
            else if (c < 0 || c >= n) c = -1;  // absorbed by a wall
          }
          if (c >= 0) {
            const long long q = fx_charge(w);
            const long long qr = fx_share(f, q);
            dkey[j] = c;
            da[j] = q - qr;
            db[j] = qr;
          }
        }
        if (push && alive && idx < i1) {
          cellp[idx] = (int16_t)c;
          fracp[idx] = f;
          vp_[idx] = v;
        }
      }
      if (restrict_) merge_moments(rkey, ra0, ra1, rb0, rb1, periodic ? nc : -1, wr0, wr1);
      if (deposit) merge_charge(dkey, da, db, periodic ? n : -1, wq);
    }
    __syncthreads();
    if (deposit) {
      long long* gq = reinterpret_cast<long long*>(R.q[qsel]);
      for (int k = tid; k < kQWin; k += kThreads) {
        const long long val = lds_q[k];
        if (val != 0)
          atomicAdd(reinterpret_cast<unsigned long long*>(&gq[wq.base + k]), (unsigned long long)val);
      }
    }
    if (restrict_) {
      for (int k = tid; k < 2 * kRWin; k += kThreads) {
        const int m = k / kRWin;
        const int kk = k - m * kRWin;
        const long long val = lds_r[m][kk];
        if (val != 0)
          atomicAdd(reinterpret_cast<unsigned long long*>(&rb[(int64_t)m * nc + rbase + kk]),
                    (unsigned long long)val);
      }
    }
    __syncthreads();
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

void launch_particles(const RepDev* d_reps, const int64_t* d_item_prefix, int n_reps,
                      int64_t total_items, int tile, int grid_blocks, int p, int flags,
                      int qsel, hipStream_t stream) {
  if (total_items <= 0) return;
  const int64_t g = grid_blocks > 0 ? min((int64_t)grid_blocks, total_items) : total_items;
  const int fresh = (flags & kFresh) ? 1 : 0;
  const int mode = flags & (kRestrict | kPush | kDepositOnly);
  const dim3 grid((unsigned)g), block(kThreads);
  switch (mode) {
    case kRestrict | kPush:
      hipLaunchKernelGGL(k_particles<kRestrict | kPush>, grid, block, 0, stream, d_reps,
                         d_item_prefix, n_reps, total_items, tile, p, fresh, qsel);
      break;
    case kPush:
      hipLaunchKernelGGL(k_particles<kPush>, grid, block, 0, stream, d_reps, d_item_prefix, n_reps,
                         total_items, tile, p, fresh, qsel);
      break;
    case kRestrict:
      hipLaunchKernelGGL(k_particles<kRestrict>, grid, block, 0, stream, d_reps, d_item_prefix,
                         n_reps, total_items, tile, p, fresh, qsel);
      break;
    default:
      hipLaunchKernelGGL(k_particles<kDepositOnly>, grid, block, 0, stream, d_reps, d_item_prefix,
                         n_reps, total_items, tile, p, fresh, qsel);
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
