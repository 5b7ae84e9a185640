// Learned projection: a 1D-convolution network over the coarse index that maps
// the last three coarse states to the increment of a projective step (it stands
// in for the least-squares slope of eq. 3.18 in the projection of eq. 3.17).
//
// Network: conv(6->64) SiLU conv(64->64) SiLU conv(64->64) SiLU conv(64->2),
// kernel width 3, "same" padding (circular on periodic domains, zero on walled
// ones).  Parameters are one FP32 vector: per layer W[c_out][c_in][3], b[c_out].
//
// Every convolution is an implicit GEMM on the matrix cores with bfloat16
// operands and FP32 accumulation (v_mfma_f32_16x16x32_bf16):
//   forward   z[o][i]  = b[o] + sum_{k,c} Wf[o][k*CP + c] * x[c][i + k - 1]
//   adjoint   da[c][j] = sum_{k',o} Wt[c][k'*OP + o] * dz[o][j + k' - 1],
//             Wt[c][k'*OP + o] = W[o][c][2 - k']   (the same kernel, flipped taps)
//   weights   dW[o][k*CP + c] = sum_{s,i} dz[s][o][i] * x[s][c][i + k - 1]
// A workgroup of four waves owns 64 positions of one sample.  Operand tiles are
// staged in LDS as bfloat16 so that every MFMA operand is one 16-byte read:
// the input tile position-major (channels contiguous) for the forward, and the
// im2col rows (positions contiguous) for the weight gradient.  Weight-gradient
// partials are written per workgroup and summed in a fixed order, so training is
// deterministic.
#include "efpi_internal.h"

namespace efpi {
namespace nn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kTile = 64;  // positions per workgroup
constexpr int kSupportRadius = 2;  // blocks: reach of the learned step's support rule

// f32 -> bf16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float sigmoid(float z) { return 1.f / (1.f + __expf(-z)); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

enum Epi : int { kFwdHidden = 0, kFwdLast = 1, kBwdHidden = 2 };

// One convolution (forward or adjoint) for a tile of 64 positions of sample s.
//   CP: input channels padded to a multiple of 8; CIN real input channels
//   ROWS: output rows computed (64 or 16); n_out real output rows
//   KP = 3 CP rounded up to a multiple of 32 (weight pack row length)
// Lane layout of the 16x16x32 MFMA: A[i][k] in lane i + 16 (k / 8), element k % 8;
// B[k][j] in lane j + 16 (k / 8); D[i][j] in lane j + 16 (i / 4), element i % 4.
template <int CP, int ROWS, int EPI>
__global__ __launch_bounds__(kThreads) void k_conv(const float* __restrict__ in, int cin,
                                                   const uint16_t* __restrict__ wpack,
                                                   const float* __restrict__ bias,
                                                   const float* __restrict__ zprev,
                                                   float* __restrict__ out0,
                                                   float* __restrict__ out1, int n_out, int L,
                                                   int periodic) {
  constexpr int KP = (3 * CP + 31) / 32 * 32;
  constexpr int PITCH = CP + 8;  // bf16 elements per LDS row (16-byte aligned rows)
  __shared__ __attribute__((aligned(16))) uint16_t xs[(kTile + 2) * PITCH];
  const int s = blockIdx.y;
  const int p0 = blockIdx.x * kTile;
  const int tid = threadIdx.x;
  const float* src = in + (size_t)s * cin * L;

  // stage x[c][p0 - 1 .. p0 + 64] as bf16, position-major; padding channels = 0
  for (int idx = tid; idx < CP * (kTile + 2); idx += kThreads) {
    const int c = idx / (kTile + 2);
    const int j = idx - c * (kTile + 2);
    int p = p0 - 1 + j;
    float val = 0.f;
    if (c < cin) {
      if (p == -1 && periodic) p = L - 1;
      if (p == L && periodic) p = 0;
      if (p >= 0 && p < L) val = src[(size_t)c * L + p];
    }
    xs[j * PITCH + c] = to_bf16(val);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int lk = lane >> 4;
  constexpr int RT = ROWS / 16;        // row tiles
  constexpr int CT = RT == 4 ? 4 : 1;  // column tiles per wave
  const int rt = RT == 4 ? wave : 0;
  const int ct0 = RT == 4 ? 0 : wave;
  f32x4 acc[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int ks = 0; ks < KP / 32; ++ks) {
    const int kk0 = ks * 32 + 8 * lk;
    const bf16x8 a = load8(wpack + (size_t)(rt * 16 + li) * KP + kk0);
    const int k = kk0 / CP;
    const int c0 = kk0 - k * CP;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      bf16x8 b;
      if (k < 3) {
        b = load8(xs + ((ct0 + c) * 16 + li + k) * PITCH + c0);
      } else {
        b = bf16x8{};  // padding of the reduction dimension
      }
      acc[c] = mfma(a, b, acc[c]);
    }
  }

  // epilogue
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int p = p0 + (ct0 + c) * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = rt * 16 + 4 * lk + r;
      if (o < n_out && p < L) {
        const size_t at = ((size_t)s * n_out + o) * L + p;
        const float v = acc[c][r];
        if (EPI == kFwdHidden) {
          const float z = v + bias[o];
          out0[at] = z;
          out1[at] = z * sigmoid(z);
        } else if (EPI == kFwdLast) {
          out0[at] = v + bias[o];
        } else {
          const float z = zprev[at];
          const float sg = sigmoid(z);
          out0[at] = v * (sg * (1.f + z * (1.f - sg)));
        }
      }
    }
  }
}

// Weight-gradient partial of one tile: part_w[blk][ROWS][KP], part_b[blk][ROWS].
template <int CP, int ROWS>
__global__ __launch_bounds__(kThreads) void k_wgrad(const float* __restrict__ dz, int n_out,
                                                    const float* __restrict__ x, int cin, int L,
                                                    int periodic, float* __restrict__ part_w,
                                                    float* __restrict__ part_b) {
  constexpr int KP = (3 * CP + 31) / 32 * 32;
  constexpr int PP = kTile + 8;  // bf16 per LDS row
  __shared__ __attribute__((aligned(16))) uint16_t ds_[ROWS * PP];
  __shared__ __attribute__((aligned(16))) uint16_t xc[KP * PP];
  const int s = blockIdx.y;
  const int p0 = blockIdx.x * kTile;
  const int blk = blockIdx.y * gridDim.x + blockIdx.x;
  const int tid = threadIdx.x;
  const float* dsrc = dz + (size_t)s * n_out * L;
  const float* xsrc = x + (size_t)s * cin * L;

  for (int idx = tid; idx < ROWS * kTile; idx += kThreads) {
    const int o = idx / kTile;
    const int j = idx - o * kTile;
    const int p = p0 + j;
    const float v = (o < n_out && p < L) ? dsrc[(size_t)o * L + p] : 0.f;
    ds_[o * PP + j] = to_bf16(v);
  }
  // im2col rows kk = k CP + c: x[c][p0 + j + k - 1]
  for (int idx = tid; idx < KP * kTile; idx += kThreads) {
    const int kk = idx / kTile;
    const int j = idx - kk * kTile;
    const int k = kk / CP;
    const int c = kk - k * CP;
    float v = 0.f;
    if (k < 3 && c < cin) {
      int p = p0 + j + k - 1;
      if (p == -1 && periodic) p = L - 1;
      if (p == L && periodic) p = 0;
      if (p >= 0 && p < L) v = xsrc[(size_t)c * L + p];
    }
    xc[kk * PP + j] = to_bf16(v);
  }
  __syncthreads();

  // bias partial: FP32 sum over the tile's valid positions, fixed order
  if (tid < ROWS) {
    float sb = 0.f;
    if (tid < n_out)
      for (int j = 0; j < kTile && p0 + j < L; ++j) sb += dsrc[(size_t)tid * L + p0 + j];
    part_b[(size_t)blk * ROWS + tid] = sb;
  }

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15;
  const int lk = lane >> 4;
  constexpr int RT = ROWS / 16;
  constexpr int NT = KP / 16;                     // column tiles (over kk)
  constexpr int WT = RT == 4 ? NT : NT / 4;       // column tiles per wave
  static_assert(RT == 4 || NT % 4 == 0, "column tiles must split over four waves");
  const int rt = RT == 4 ? wave : 0;
  const int nt0 = RT == 4 ? 0 : wave * WT;
  f32x4 acc[WT];
#pragma unroll
  for (int t = 0; t < WT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < kTile / 32; ++ks) {
    const int j0 = ks * 32 + 8 * lk;
    const bf16x8 a = load8(ds_ + (rt * 16 + li) * PP + j0);
#pragma unroll
    for (int t = 0; t < WT; ++t) {
      const bf16x8 b = load8(xc + ((nt0 + t) * 16 + li) * PP + j0);
      acc[t] = mfma(a, b, acc[t]);
    }
  }
  float* pw = part_w + (size_t)blk * ROWS * KP;
#pragma unroll
  for (int t = 0; t < WT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) pw[(size_t)(rt * 16 + 4 * lk + r) * KP + (nt0 + t) * 16 + li] = acc[t][r];
}

// Parameter and pack layout of layer l (0..3).
struct LayerDims {
  int cin, cout, cp, rows, kp, op, kpt;  // op: cout padded to 8 (adjoint), kpt: its pack row
  int w_off, b_off;                      // offsets into the flat FP32 parameters
  int f_off, t_off;                      // offsets (bf16 elements) of the forward/adjoint packs
};

constexpr LayerDims make_dims(int l) {
  LayerDims d{};
  int w = 0, f = 0, t = 0;
  for (int i = 0; i <= l; ++i) {
    d.cin = i == 0 ? kNnCin : kNnHidden;
    d.cout = i == 3 ? kNnCout : kNnHidden;
    d.cp = (d.cin + 7) / 8 * 8;
    d.rows = d.cout == kNnHidden ? 64 : 16;
    d.kp = (3 * d.cp + 31) / 32 * 32;
    d.op = (d.cout + 7) / 8 * 8;
    d.kpt = (3 * d.op + 31) / 32 * 32;
    d.w_off = w;
    d.b_off = w + d.cout * d.cin * 3;
    d.f_off = f;
    d.t_off = t;
    w += d.cout * d.cin * 3 + d.cout;
    f += d.rows * d.kp;
    t += i == 0 ? 0 : d.cin * d.kpt;
  }
  return d;
}

__host__ __device__ inline LayerDims layer_dims(int l) {
  constexpr LayerDims d0 = make_dims(0), d1 = make_dims(1), d2 = make_dims(2), d3 = make_dims(3);
  return l == 0 ? d0 : (l == 1 ? d1 : (l == 2 ? d2 : d3));
}

static_assert(make_dims(3).b_off + kNnCout == kNnParams, "parameter count");
static_assert(make_dims(3).f_off + make_dims(3).rows * make_dims(3).kp == kNnPackForward,
              "forward pack size");
static_assert(kNnPackForward + make_dims(3).t_off + make_dims(3).cin * make_dims(3).kpt ==
                  kNnPackElems,
              "pack size");

// Write the bfloat16 packs of parameter i (weights only; biases stay FP32).
__device__ inline void pack_one(int i, float val, uint16_t* pack) {
  const int l = i >= layer_dims(3).w_off ? 3 : (i >= layer_dims(2).w_off ? 2 : (i >= layer_dims(1).w_off ? 1 : 0));
  const LayerDims d = layer_dims(l);
  const int r = i - d.w_off;
  if (r >= d.cout * d.cin * 3) return;  // bias
  const int o = r / (d.cin * 3);
  const int c = (r / 3) % d.cin;
  const int k = r % 3;
  const uint16_t b = to_bf16(val);
  pack[d.f_off + o * d.kp + k * d.cp + c] = b;
  if (l > 0) {
    const int tbase = kNnPackForward + d.t_off;
    pack[tbase + c * d.kpt + (2 - k) * d.op + o] = b;
  }
}

__global__ void k_pack(const float* __restrict__ params, uint16_t* __restrict__ pack) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kNnParams) pack_one(i, params[i], pack);
}

__global__ void k_zero_u16(uint16_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// grad[i] = sum over workgroups, in workgroup order, of the partials.
__global__ void k_reduce(const float* __restrict__ part_w, const float* __restrict__ part_b,
                         int n_blk, int layer, float* __restrict__ grad) {
  const LayerDims d = layer_dims(layer);
  const int nw = d.cout * d.cin * 3;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw + d.cout) return;
  float sum = 0.f;
  if (i < nw) {
    const int o = i / (d.cin * 3);
    const int c = (i / 3) % d.cin;
    const int k = i % 3;
    const size_t at = (size_t)o * d.kp + k * d.cp + c;
    for (int b = 0; b < n_blk; ++b) sum += part_w[(size_t)b * d.rows * d.kp + at];
  } else {
    const int o = i - nw;
    for (int b = 0; b < n_blk; ++b) sum += part_b[(size_t)b * d.rows + o];
  }
  grad[d.w_off + i] = sum;
}

__global__ void k_adam(float* __restrict__ params, const float* __restrict__ grad,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t* __restrict__ pack) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNnParams) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float th = params[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  params[i] = th;
  pack_one(i, th, pack);
}

// Mean squared error and its gradient: one workgroup, fixed-order reduction.
__global__ __launch_bounds__(1024) void k_mse(const float* __restrict__ y,
                                              const float* __restrict__ t,
                                              float* __restrict__ dy, float* __restrict__ loss,
                                              int64_t count) {
  __shared__ double red[1024];
  double acc = 0.0;
  const float scale = 2.f / (float)count;
  for (int64_t i = threadIdx.x; i < count; i += 1024) {
    const float d = y[i] - t[i];
    dy[i] = scale * d;
    acc += (double)d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] / (double)count);
}

// x[b][6][N_c] (and optionally t[b][2][N_c]) from states[n-2], states[n-1],
// states[n] (and states[n+1]) with n = index[b], clamped to [2, n_states - 2].
// Uniform variate with mean 0 and variance 1 from a counter (the "lowbias32"
// integer hash of C. Wellons' hash prospector, then scaled to [-sqrt 3, sqrt 3)).
__device__ __forceinline__ float unit_noise(uint32_t seed, uint32_t counter) {
  uint32_t x = seed ^ (counter * 0x9E3779B1u);
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return ((float)x * 2.3283064365386963e-10f - 0.5f) * 3.4641016151377544f;
}

__global__ void k_features(const double* __restrict__ states, int n_states,
                           const int32_t* __restrict__ index, int batch, int nc, efpi_nn_norm nm,
                           float noise, uint32_t seed, float* __restrict__ x,
                           float* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)batch * 2 * nc) return;
  const int b = (int)(i / (2 * nc));
  const int r = (int)(i - (int64_t)b * 2 * nc);
  const int m = r / nc;
  const int k = r - m * nc;
  const int hi = t ? n_states - 2 : n_states - 1;
  const int n = index ? min(max(index[b], 2), hi) : 2;
  const size_t st = 2 * (size_t)nc;
  double cn = states[n * st + r];
  double c1 = states[(n - 1) * st + r];
  double c2 = states[(n - 2) * st + r];
  if (noise > 0.f) {
    // training noise on the input states, in units of the increment scale
    const uint32_t base = 3u * (uint32_t)i;
    const double a = (double)noise * nm.delta[m];
    cn += a * unit_noise(seed, base);
    c1 += a * unit_noise(seed, base + 1u);
    c2 += a * unit_noise(seed, base + 2u);
  }
  float* xb = x + (size_t)b * 6 * nc;
  xb[m * nc + k] = (float)((cn - nm.mu[m]) / nm.sigma[m]);
  xb[(2 + m) * nc + k] = (float)((cn - c1) / nm.delta[m]);
  xb[(4 + m) * nc + k] = (float)((c1 - c2) / nm.delta[m]);
  if (t) t[(size_t)b * 2 * nc + r] = (float)((states[(n + 1) * st + r] - cn) / nm.delta[m]);
}

// c_next = c_n + delta * y
__global__ void k_step(const double* __restrict__ cn, const float* __restrict__ y, int64_t count,
                       int nc, efpi_nn_norm nm, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int m = (int)((i / nc) & 1);
  out[i] = cn[i] + (double)nm.delta[m] * (double)y[i];
}

// eps(a, b) = sqrt(sum (a - b)^2 / sum (a^2 + b^2)) (eq. 4.2), FP64, fixed order.
__global__ __launch_bounds__(1024) void k_rel_l2(const double* __restrict__ a,
                                                 const double* __restrict__ b, int64_t n,
                                                 double* __restrict__ out) {
  __shared__ double num[1024], den[1024];
  double sn = 0.0, sd = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double d = a[i] - b[i];
    sn += d * d;
    sd += a[i] * a[i] + b[i] * b[i];
  }
  num[threadIdx.x] = sn;
  den[threadIdx.x] = sd;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      num[threadIdx.x] += num[threadIdx.x + w];
      den[threadIdx.x] += den[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = den[0] > 0.0 ? sqrt(num[0] / den[0]) : 0.0;
}

}  // namespace

void launch_rel_l2(const double* a, const double* b, int64_t n, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_rel_l2, dim3(1), dim3(1024), 0, stream, a, b, n, out);
}

size_t workspace_floats(int batch, int nc) {
  const size_t act = (size_t)batch * kNnHidden * nc;
  const size_t nblk = (size_t)batch * ((nc + kTile - 1) / kTile);
  return 8 * act + nblk * (64 * 192 + 64) + (size_t)batch * 8 * nc;
}

namespace {
struct Ws {
  float *z0, *a0, *z1, *a1, *z2, *a2, *dza, *dzb, *pw, *pb, *x, *y;
};
Ws carve(float* ws, int batch, int nc) {
  const size_t act = (size_t)batch * kNnHidden * nc;
  Ws w;
  w.z0 = ws;
  w.a0 = w.z0 + act;
  w.z1 = w.a0 + act;
  w.a1 = w.z1 + act;
  w.z2 = w.a1 + act;
  w.a2 = w.z2 + act;
  w.dza = w.a2 + act;
  w.dzb = w.dza + act;
  w.pw = w.dzb + act;
  w.pb = w.pw + (size_t)batch * ((nc + kTile - 1) / kTile) * 64 * 192;
  w.x = w.pb + (size_t)batch * ((nc + kTile - 1) / kTile) * 64;
  w.y = w.x + (size_t)batch * kNnCin * nc;
  return w;
}
}  // namespace

void launch_pack(const float* params, uint16_t* pack, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_u16, dim3((kNnPackElems + 255) / 256), dim3(256), 0, stream, pack,
                     kNnPackElems);
  hipLaunchKernelGGL(k_pack, dim3((kNnParams + 255) / 256), dim3(256), 0, stream, params, pack);
}

void launch_forward(const float* params, const uint16_t* pack, const float* x, float* y,
                    int batch, int nc, int periodic, float* ws, hipStream_t stream) {
  const Ws w = carve(ws, batch, nc);
  const dim3 grid((nc + kTile - 1) / kTile, batch), block(kThreads);
  const LayerDims d0 = layer_dims(0), d1 = layer_dims(1), d2 = layer_dims(2), d3 = layer_dims(3);
  hipLaunchKernelGGL((k_conv<8, 64, kFwdHidden>), grid, block, 0, stream, x, kNnCin,
                     pack + d0.f_off, params + d0.b_off, nullptr, w.z0, w.a0, kNnHidden, nc,
                     periodic);
  hipLaunchKernelGGL((k_conv<64, 64, kFwdHidden>), grid, block, 0, stream, w.a0, kNnHidden,
                     pack + d1.f_off, params + d1.b_off, nullptr, w.z1, w.a1, kNnHidden, nc,
                     periodic);
  hipLaunchKernelGGL((k_conv<64, 64, kFwdHidden>), grid, block, 0, stream, w.a1, kNnHidden,
                     pack + d2.f_off, params + d2.b_off, nullptr, w.z2, w.a2, kNnHidden, nc,
                     periodic);
  hipLaunchKernelGGL((k_conv<64, 16, kFwdLast>), grid, block, 0, stream, w.a2, kNnHidden,
                     pack + d3.f_off, params + d3.b_off, nullptr, y, nullptr, kNnCout, nc,
                     periodic);
}

void launch_backward(const uint16_t* pack, const float* x, const float* dy, float* grad,
                     int batch, int nc, int periodic, float* ws, hipStream_t stream) {
  const Ws w = carve(ws, batch, nc);
  const int tiles = (nc + kTile - 1) / kTile;
  const int nblk = batch * tiles;
  const dim3 grid(tiles, batch), block(kThreads);
  const uint16_t* tp = pack + kNnPackForward;
  auto reduce = [&](int l) {
    const LayerDims d = layer_dims(l);
    const int n = d.cout * d.cin * 3 + d.cout;
    hipLaunchKernelGGL(k_reduce, dim3((n + 255) / 256), dim3(256), 0, stream, w.pw, w.pb, nblk,
                       l, grad);
  };
  // layer 3: input a2, output gradient dy (2 channels)
  hipLaunchKernelGGL((k_wgrad<64, 16>), grid, block, 0, stream, dy, kNnCout, w.a2, kNnHidden,
                     nc, periodic, w.pw, w.pb);
  reduce(3);
  hipLaunchKernelGGL((k_conv<8, 64, kBwdHidden>), grid, block, 0, stream, dy, kNnCout,
                     tp + layer_dims(3).t_off, nullptr, w.z2, w.dza, nullptr, kNnHidden, nc,
                     periodic);
  // layer 2
  hipLaunchKernelGGL((k_wgrad<64, 64>), grid, block, 0, stream, w.dza, kNnHidden, w.a1,
                     kNnHidden, nc, periodic, w.pw, w.pb);
  reduce(2);
  hipLaunchKernelGGL((k_conv<64, 64, kBwdHidden>), grid, block, 0, stream, w.dza, kNnHidden,
                     tp + layer_dims(2).t_off, nullptr, w.z1, w.dzb, nullptr, kNnHidden, nc,
                     periodic);
  // layer 1
  hipLaunchKernelGGL((k_wgrad<64, 64>), grid, block, 0, stream, w.dzb, kNnHidden, w.a0,
                     kNnHidden, nc, periodic, w.pw, w.pb);
  reduce(1);
  hipLaunchKernelGGL((k_conv<64, 64, kBwdHidden>), grid, block, 0, stream, w.dzb, kNnHidden,
                     tp + layer_dims(1).t_off, nullptr, w.z0, w.dza, nullptr, kNnHidden, nc,
                     periodic);
  // layer 0: input x (6 channels)
  hipLaunchKernelGGL((k_wgrad<8, 64>), grid, block, 0, stream, w.dza, kNnHidden, x, kNnCin, nc,
                     periodic, w.pw, w.pb);
  reduce(0);
}

void launch_mse(const float* y, const float* t, float* dy, float* loss, int64_t count,
                hipStream_t stream) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, stream, y, t, dy, loss, count);
}

void launch_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                 float b1, float b2, float eps, uint16_t* pack, hipStream_t stream) {
  const float c1 = 1.f - powf(b1, (float)step);
  const float c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((kNnParams + 255) / 256), dim3(256), 0, stream, params, grad,
                     m, v, lr, b1, b2, eps, c1, c2, pack);
}

void launch_features(const double* states, int n_states, const int32_t* index, int batch, int nc,
                     const efpi_nn_norm& nm, float noise, uint32_t seed, float* x, float* t,
                     hipStream_t stream) {
  const int64_t n = (int64_t)batch * 2 * nc;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, states,
                     n_states, index, batch, nc, nm, noise, seed, x, t);
}

void launch_step(const double* cn, const float* y, int batch, int nc, const efpi_nn_norm& nm,
                 double* out, hipStream_t stream) {
  const int64_t n = (int64_t)batch * 2 * nc;
  hipLaunchKernelGGL(k_step, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, cn, y, n,
                     nc, nm, out);
}

// One learned step of a single window with the support rule: a coarse block whose
// density is exactly zero in c_n at every block within kSupportRadius (periodic
// wrap, or the blocks inside the walls) keeps its values (no increment); else
// c_next = c_n + delta * y.
__global__ void k_step_support(const double* __restrict__ cn, const float* __restrict__ y, int nc,
                               int periodic, efpi_nn_norm nm, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * nc) return;
  const int m = i >= nc ? 1 : 0;
  const int k = i - m * nc;
  bool empty = true;
  for (int d = -kSupportRadius; d <= kSupportRadius; ++d) {
    int j = k + d;
    if (periodic) j = ((j % nc) + nc) % nc;
    else if (j < 0 || j >= nc) continue;
    empty = empty && cn[j] == 0.0;
  }
  out[i] = empty ? cn[i] : cn[i] + (double)nm.delta[m] * (double)y[i];
}

void launch_predict_step(const float* params, const uint16_t* pack, const double* states, int nc,
                         int periodic, const efpi_nn_norm& nm, double* out, float* ws,
                         hipStream_t stream) {
  const Ws w = carve(ws, 1, nc);
  const int64_t n = 2 * (int64_t)nc;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, states,
                     3, nullptr, 1, nc, nm, 0.f, 0u, w.x, nullptr);
  launch_forward(params, pack, w.x, w.y, 1, nc, periodic, ws, stream);
  // states[2] is c_n of the single sample window
  hipLaunchKernelGGL(k_step_support, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                     states + 2 * (size_t)2 * nc, w.y, nc, periodic, nm, out);
}

}  // namespace nn
}  // namespace efpi
