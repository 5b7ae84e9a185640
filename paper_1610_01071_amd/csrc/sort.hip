// Stable counting sort of the ion store by cell index.
//
// Two least-significant-digit passes over 8-bit digits of the key
// (cell, or 0xFFFF for an absorbed ion, which therefore sorts last and is
// dropped).  Each pass: (1) per-tile digit histograms, (2) per replica and
// digit a parallel scan over tiles, then a scan over digits, giving every
// (tile, digit) its first destination,
// (3) a scatter in which each wave walks its quarter of the tile in index
// order and ranks lanes of equal digit by ballot masks, so the order is stable
// and the result deterministic.  Pass 0 moves the store into the sort copy,
// pass 1 moves it back.
#include "efpi_internal.h"

namespace efpi {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kDigits = 256;

__device__ __forceinline__ int find_replica(const int64_t* prefix, int n, int64_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ unsigned key_of(int16_t c) {
  return c < 0 ? 0xFFFFu : (unsigned)(uint16_t)c;
}

#define EFPI_G __attribute__((address_space(1)))
struct Store {
  const EFPI_G int16_t* cell;
  const EFPI_G float* frac;
  const EFPI_G float* v;
  const EFPI_G float* w;
  EFPI_G int16_t* ocell;
  EFPI_G float* ofrac;
  EFPI_G float* ov;
  EFPI_G float* ow;
};
#undef EFPI_G

__device__ __forceinline__ Store store_of(const RepDev& R, int pass) {
  if (pass == 0)
    return Store{gmem(R.cell), gmem(R.frac), gmem(R.v), gmem(R.w),
                 gmem(R.cell2), gmem(R.frac2), gmem(R.v2), gmem(R.w2)};
  return Store{gmem(R.cell2), gmem(R.frac2), gmem(R.v2), gmem(R.w2),
               gmem(R.cell), gmem(R.frac), gmem(R.v), gmem(R.w)};
}

// Per-wave digit counts of the tile into LDS rows, summed into hist[item][digit].
__global__ __launch_bounds__(kThreads) void k_hist(const RepDev* __restrict__ reps,
                                                    const int64_t* __restrict__ item_prefix,
                                                    int n_reps, int64_t total, int tile, int pass,
                                                    int32_t* __restrict__ hist) {
  __shared__ int s_cnt[kWaves][kDigits];
  const int shift = 8 * pass;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int r = find_replica(item_prefix, n_reps, item);
    const RepDev& R = reps[r];
    const Store S = store_of(R, pass);
    const int64_t np = *gmem(R.np);
    const int64_t i0 = (item - R.item_begin) * (int64_t)tile;
    for (int k = threadIdx.x; k < kWaves * kDigits; k += kThreads) (&s_cnt[0][0])[k] = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t chunk = tile / kWaves;
    const int64_t a = i0 + wave * chunk;
    for (int64_t j = a + lane; j < a + chunk; j += 64) {
      if (j < np) atomicAdd(&s_cnt[wave][(key_of(S.cell[j]) >> shift) & 0xFF], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kDigits; d += kThreads) {
      int s = 0;
      for (int q = 0; q < kWaves; ++q) s += s_cnt[q][d];
      hist[item * kDigits + d] = s;
    }
    __syncthreads();
  }
}

// Per (digit d, replica r): hist[item][d] <- number of ions with digit d in the
// replica's earlier tiles (exclusive scan over tiles), and tot[r][d] <- the
// digit's total.  Each thread scans a contiguous run of tiles; the run totals
// are combined by a scan in LDS.
__global__ __launch_bounds__(kDigits) void k_scan_items(const int64_t* __restrict__ item_prefix,
                                                         int32_t* __restrict__ hist,
                                                         int64_t* __restrict__ tot) {
  __shared__ int64_t s_run[kDigits];
  const int d = blockIdx.x;
  const int r = blockIdx.y;
  const int t = threadIdx.x;
  const int64_t b = item_prefix[r], e = item_prefix[r + 1];
  const int64_t per = (e - b + kDigits - 1) / kDigits;
  const int64_t lo = min(b + t * per, e), hi = min(lo + per, e);
  int64_t sum = 0;
  for (int64_t it = lo; it < hi; ++it) sum += hist[it * kDigits + d];
  s_run[t] = sum;
  __syncthreads();
  // inclusive scan of the run totals (Hillis-Steele)
  for (int off = 1; off < kDigits; off <<= 1) {
    const int64_t add = t >= off ? s_run[t - off] : 0;
    __syncthreads();
    s_run[t] += add;
    __syncthreads();
  }
  int64_t run = s_run[t] - sum;
  for (int64_t it = lo; it < hi; ++it) {
    const int32_t c = hist[it * kDigits + d];
    hist[it * kDigits + d] = (int32_t)run;
    run += c;
  }
  if (t == kDigits - 1) tot[(int64_t)r * kDigits + d] = s_run[t];
}

// Per replica: base[r][d] <- first destination of digit d (exclusive scan of
// the digit totals in digit order).  On the last pass the count of absorbed
// ions (digit 0xFF of the key 0xFFFF, sorted last) is kept in aux[0].
__global__ __launch_bounds__(kDigits) void k_scan_digits(const RepDev* __restrict__ reps, int pass,
                                                          int64_t* __restrict__ tot) {
  __shared__ int64_t s_tot[kDigits];
  const int r = blockIdx.x;
  const int d = threadIdx.x;
  s_tot[d] = tot[(int64_t)r * kDigits + d];
  __syncthreads();
  int64_t base = 0;
  for (int k = 0; k < d; ++k) base += s_tot[k];
  tot[(int64_t)r * kDigits + d] = base;
  if (pass == 1 && d == 0) gmem(reps[r].aux)[0] = s_tot[kDigits - 1];
}

__global__ void k_drop_absorbed(const RepDev* __restrict__ reps) {
  const RepDev& R = reps[blockIdx.x];
  if (threadIdx.x == 0) *gmem(R.np) = *gmem(R.np) - *gmem(R.aux);
}

__global__ __launch_bounds__(kThreads) void k_scatter(const RepDev* __restrict__ reps,
                                                       const int64_t* __restrict__ item_prefix,
                                                       int n_reps, int64_t total, int tile,
                                                       int pass, const int32_t* __restrict__ hist,
                                                       const int64_t* __restrict__ base) {
  __shared__ int s_off[kWaves][kDigits];
  const int shift = 8 * pass;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int r = find_replica(item_prefix, n_reps, item);
    const RepDev& R = reps[r];
    const Store S = store_of(R, pass);
    const int64_t np = *gmem(R.np);
    const int64_t i0 = (item - R.item_begin) * (int64_t)tile;
    const int64_t chunk = tile / kWaves;
    const int64_t a = i0 + wave * chunk;
    for (int k = threadIdx.x; k < kWaves * kDigits; k += kThreads) (&s_off[0][0])[k] = 0;
    __syncthreads();
    for (int64_t j = a + lane; j < a + chunk; j += 64)
      if (j < np) atomicAdd(&s_off[wave][(key_of(S.cell[j]) >> shift) & 0xFF], 1);
    __syncthreads();
    // exclusive prefix over waves, plus the tile's first destination per digit
    for (int d = threadIdx.x; d < kDigits; d += kThreads) {
      int run = hist[item * kDigits + d] + (int)base[(int64_t)r * kDigits + d];
      for (int q = 0; q < kWaves; ++q) {
        const int c = s_off[q][d];
        s_off[q][d] = run;
        run += c;
      }
    }
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t j0 = a; j0 < a + chunk; j0 += 64) {
      const int64_t j = j0 + lane;
      const bool ok = j < np;
      int dig = -1;
      int16_t c = 0;
      float f = 0.f, v = 0.f, w = 0.f;
      if (ok) {
        c = S.cell[j];
        f = S.frac[j];
        v = S.v[j];
        w = S.w[j];
        dig = (int)((key_of(c) >> shift) & 0xFF);
      }
      int dest = -1;
      int key = dig;
      while (true) {
        const unsigned long long act = __ballot(key >= 0);
        if (act == 0ull) break;
        const int leader = __ffsll((unsigned long long)act) - 1;
        const int lk = __shfl(key, leader, 64);
        const unsigned long long m = __ballot(key == lk);
        if (key == lk) {
          dest = s_off[wave][lk] + __popcll(m & lt);
          key = -1;
        }
        if (lane == leader) s_off[wave][lk] += __popcll(m);
      }
      if (ok) {
        S.ocell[dest] = c;
        S.ofrac[dest] = f;
        S.ov[dest] = v;
        S.ow[dest] = w;
      }
    }
    __syncthreads();
  }
}

}  // namespace

void launch_sort(const RepDev* d_reps, const int64_t* d_item_prefix, int n_reps,
                 int64_t total_items, int tile, int32_t* d_hist, int64_t* d_base,
                 int grid_blocks, hipStream_t stream) {
  if (total_items <= 0) return;
  const int64_t g = grid_blocks > 0 ? min((int64_t)grid_blocks, total_items) : total_items;
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_hist, dim3((unsigned)g), dim3(kThreads), 0, stream, d_reps, d_item_prefix,
                       n_reps, total_items, tile, pass, d_hist);
    hipLaunchKernelGGL(k_scan_items, dim3(kDigits, n_reps), dim3(kDigits), 0, stream,
                       d_item_prefix, d_hist, d_base);
    hipLaunchKernelGGL(k_scan_digits, dim3(n_reps), dim3(kDigits), 0, stream, d_reps, pass, d_base);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)g), dim3(kThreads), 0, stream, d_reps,
                       d_item_prefix, n_reps, total_items, tile, pass, d_hist, d_base);
  }
  hipLaunchKernelGGL(k_drop_absorbed, dim3(n_reps), dim3(64), 0, stream, d_reps);
}

}  // namespace efpi
