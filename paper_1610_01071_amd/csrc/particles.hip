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
constexpr int kQWin = 1024;     // node window (int64 bins)
constexpr int kQMargin = 16;
constexpr int kRWin = 64;       // coarse block window per moment
constexpr int kRMargin = 8;

__device__ __forceinline__ long long wave_sum(long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// q = rint(w 2^40): the particle's charge in fixed point.
__device__ __forceinline__ long long fx_charge(float w) {
  return (long long)rint((double)w * kFxScale);
}
// Right-node share rint(theta q) in binary64 (one rounded product, then ties-to-even).
__device__ __forceinline__ long long fx_share(float theta, long long q) {
  return (long long)rint((double)theta * (double)q);
}

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

// Merge lanes with equal `key` (>= 0) and add their (a -> key, b -> key + 1) sums.
// `wrap` is the index that key + 1 wraps to zero at (periodic), or 0 for none.
__device__ __forceinline__ void peel2(int key, long long a, long long b, int wrap,
                                      const Window& win) {
  const int lane = __lane_id();
  while (true) {
    unsigned long long act = __ballot(key >= 0);
    if (act == 0ull) break;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int lk = __shfl(key, leader, 64);
    const bool mine = (key == lk);
    const long long sa = wave_sum(mine ? a : 0ll);
    const long long sb = wave_sum(mine ? b : 0ll);
    if (lane == leader) {
      add_to(win, lk, sa);
      int r = lk + 1;
      if (r == wrap) r = 0;
      add_to(win, r, sb);
    }
    if (mine) key = -1;
  }
}

// Same with two moments (density, momentum) per target.
__device__ __forceinline__ void peel4(int key, long long a0, long long a1, long long b0,
                                      long long b1, int wrap, const Window& w0,
                                      const Window& w1) {
  const int lane = __lane_id();
  while (true) {
    unsigned long long act = __ballot(key >= 0);
    if (act == 0ull) break;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int lk = __shfl(key, leader, 64);
    const bool mine = (key == lk);
    const long long s0 = wave_sum(mine ? a0 : 0ll);
    const long long s1 = wave_sum(mine ? a1 : 0ll);
    const long long s2 = wave_sum(mine ? b0 : 0ll);
    const long long s3 = wave_sum(mine ? b1 : 0ll);
    if (lane == leader) {
      add_to(w0, lk, s0);
      add_to(w1, lk, s1);
      int r = lk + 1;
      if (r == wrap) r = 0;
      add_to(w0, r, s2);
      add_to(w1, r, s3);
    }
    if (mine) key = -1;
  }
}

__global__ __launch_bounds__(kThreads) void k_particles(const RepDev* __restrict__ reps,
                                                         const int64_t* __restrict__ item_prefix,
                                                         int n_reps, int64_t total_items,
                                                         int tile, int p, int flags, int qsel) {
  __shared__ long long lds_q[kQWin];
  __shared__ long long lds_r[2][kRWin];
  const int tid = threadIdx.x;
  const bool fresh = flags & kFresh;
  const bool restrict_ = flags & kRestrict;
  const bool push = flags & kPush;
  const bool deposit = push || (flags & kDepositOnly);

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
    const float tau = (float)(R.macro_dt - (double)p * R.dt);
    const bool coev = R.coevolving != 0;
    const float* __restrict__ e = R.e;
    const float* __restrict__ en = R.en;

    const int c_first = R.cell[i0];
    Window wq{lds_q, c_first - kQMargin, kQWin, reinterpret_cast<long long*>(R.q[qsel])};
    long long* rb = reinterpret_cast<long long*>(R.rbins) + (int64_t)p * 2 * nc;
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
          cl[j] = R.cell[idx];
          fr[j] = R.frac[idx];
          vv[j] = R.v[idx];
          ww[j] = R.w[idx];
        } else {
          cl[j] = -1;
          fr[j] = 0.f;
          vv[j] = 0.f;
          ww[j] = 0.f;
        }
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int64_t idx = b0 + (int64_t)j * kThreads + tid;
        int c = cl[j];
        float f = fr[j];
        float v = vv[j];
        const float w = ww[j];
        const bool alive = c >= 0 && c < n;  // cells outside [0, N) are treated as absorbed
        const long long q = alive ? fx_charge(w) : 0ll;
        float ep = 0.f;
        if (alive && (restrict_ || push)) {
          const int cr = periodic ? ((c + 1) & nmask) : c + 1;
          ep = (1.f - f) * e[c] + f * e[cr];
        }
        if (restrict_) {
          // Snapshot p: time-centred velocity, then the approximate characteristic
          // over tau = Delta t - p dt (eq. B.4) and CIC at the moved position (eq. B.5).
          int key = -1;
          long long a0 = 0, a1 = 0, bb0 = 0, bb1 = 0;
          if (alive) {
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
              const long long qj = fx_charge(w * vt);
              const long long qr = fx_share(th, q);
              const long long qjr = fx_share(th, qj);
              const int bl = ct >> levels;
              int nr = ct + 1;
              if (periodic) nr &= nmask;
              int br = nr >> levels;
              if (br >= nc) br = nc - 1;  // wall node N joins the last block
              key = bl;
              if (br == bl) {
                a0 = q;
                a1 = qj;
              } else {
                a0 = q - qr;
                a1 = qj - qjr;
                bb0 = qr;
                bb1 = qjr;
              }
            }
          }
          peel4(key, a0, a1, bb0, bb1, periodic ? nc : -1, wr0, wr1);
        }
        if (deposit) {
          int key = -1;
          long long qa = 0, qb = 0;
          if (alive) {
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
              const long long qr = fx_share(f, q);
              key = c;
              qa = q - qr;
              qb = qr;
            }
          }
          if (push && idx < i1) {
            R.cell[idx] = (int16_t)c;
            R.frac[idx] = f;
            R.v[idx] = v;
          }
          peel2(key, qa, qb, periodic ? n : -1, wq);
        }
      }
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
  hipLaunchKernelGGL(k_particles, dim3((unsigned)g), dim3(kThreads), 0, stream, d_reps,
                     d_item_prefix, n_reps, total_items, tile, p, flags, qsel);
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
