// Kinetic electrons of the two-species fine solver (the paper's XES1 setting,
// Sec. 2, eq. 2.5): field gather, leapfrog push with q/m = qm_e, periodic wrap
// and the fixed-point CIC deposit of the (negative) electron charge; and the
// electron loading profile of the Boltzmann equilibrium at lift (eqs. 3.15-3.16).
//
// Electrons are not kept in cell order: at dt ~ 0.25 / omega_pe a thermal
// electron crosses a quarter cell per step, so a lifted store loses its order
// within a burst.  Every workgroup therefore deposits into a whole-grid LDS
// histogram of int64 fixed-point charge (LDS atomics are exact and
// order-independent) and adds its non-zero entries to the global charge once.
#include <hip/hip_ext.h>

#include "efpi_internal.h"

namespace efpi {
namespace {

constexpr int kEThreads = 256;
constexpr int kEPer = 16;                          // electrons per thread per chunk
constexpr int kEChunk = kEThreads * kEPer;
constexpr int kEMaxNodes = 8192;                   // 64 KB of int64 LDS


template <bool PUSH>
__global__ __launch_bounds__(kEThreads) void k_electrons(const RepDev* __restrict__ ereps,
                                                         int fresh, int qsel) {
  extern __shared__ long long s_q[];
  const RepDev& R = ereps[blockIdx.y];
  const int n = R.n_cells;  // periodic: n nodes
  const int nmask = n - 1;
  const int64_t np = *gmem(R.np);
  const int64_t chunks = (np + kEChunk - 1) / kEChunk;
  if ((int64_t)blockIdx.x >= chunks) return;  // the whole workgroup leaves together
  for (int k = threadIdx.x; k < n; k += kEThreads) s_q[k] = 0;
  __syncthreads();
  const EFPI_GLOBAL float* __restrict__ e = gmem(R.e);
  EFPI_GLOBAL int16_t* __restrict__ cellp = gmem(R.cell);
  EFPI_GLOBAL float* __restrict__ fracp = gmem(R.frac);
  EFPI_GLOBAL float* __restrict__ velp = gmem(R.v);
  const EFPI_GLOBAL float* __restrict__ wp = gmem(R.w);
  const float dt_inv_h = (float)R.dt * (float)R.inv_h;
  // v + (q/m) dt E; the first push after a load is the half step that starts
  // the leapfrog from integer-time velocities
  const float kick = (float)(R.qm * (fresh ? 0.5 * R.dt : R.dt));
  for (int64_t c0 = (int64_t)blockIdx.x * kEChunk; c0 < np; c0 += (int64_t)gridDim.x * kEChunk) {
#pragma unroll 4
    for (int j = 0; j < kEPer; ++j) {
      const int64_t i = c0 + j * kEThreads + threadIdx.x;
      if (i >= np) break;
      const int c = cellp[i];
      if (c < 0 || c >= n) continue;
      float f = fracp[i];
      const float w = wp[i];
      int cn = c;
      if constexpr (PUSH) {
        const float e0 = e[c];
        const float e1 = e[(c + 1) & nmask];
        const float ep = (1.f - f) * e0 + f * e1;
        const float vn = velp[i] + kick * ep;
        const float xn = f + dt_inv_h * vn;
        const float fl = floorf(xn);
        const bool wrap_up = (xn - fl) >= 1.f;
        f = wrap_up ? 0.f : xn - fl;
        cn = (c + (int)fl + (wrap_up ? 1 : 0)) & nmask;
        cellp[i] = (int16_t)cn;
        fracp[i] = f;
        velp[i] = vn;
      }
      const double q = fx_charge(w);
      const double qr = fx_share(f, q);
      atomicAdd(reinterpret_cast<unsigned long long*>(&s_q[cn]),
                (unsigned long long)(-(long long)(q - qr)));
      atomicAdd(reinterpret_cast<unsigned long long*>(&s_q[(cn + 1) & nmask]),
                (unsigned long long)(-(long long)qr));
    }
  }
  __syncthreads();
  unsigned long long* __restrict__ gq = reinterpret_cast<unsigned long long*>(R.q[qsel]);
  for (int k = threadIdx.x; k < n; k += kEThreads) {
    const long long v = s_q[k];
    if (v != 0) atomicAdd(&gq[k], (unsigned long long)v);
  }
}

// Fixed-point CIC momentum of the ions (the electron reset's mean velocity):
// p = rint(w v_c 2^40) split as the charge, with v_c = v + half_kick dt/2 E(x).
__global__ __launch_bounds__(kEThreads) void k_ion_momentum(const RepDev* __restrict__ reps,
                                                            int half_kick) {
  extern __shared__ long long s_q[];
  const RepDev& R = reps[blockIdx.y];
  const int n = R.n_cells;
  const int nmask = n - 1;
  const int64_t np = *gmem(R.np);
  const int64_t chunks = (np + kEChunk - 1) / kEChunk;
  if ((int64_t)blockIdx.x >= chunks) return;
  for (int k = threadIdx.x; k < n; k += kEThreads) s_q[k] = 0;
  __syncthreads();
  const EFPI_GLOBAL float* __restrict__ e = gmem(R.e);
  const EFPI_GLOBAL int16_t* __restrict__ cellp = gmem(R.cell);
  const EFPI_GLOBAL float* __restrict__ fracp = gmem(R.frac);
  const EFPI_GLOBAL float* __restrict__ velp = gmem(R.v);
  const EFPI_GLOBAL float* __restrict__ wp = gmem(R.w);
  const float kick = half_kick ? (float)(R.qm * 0.5 * R.dt) : 0.f;
  for (int64_t c0 = (int64_t)blockIdx.x * kEChunk; c0 < np; c0 += (int64_t)gridDim.x * kEChunk) {
#pragma unroll 4
    for (int j = 0; j < kEPer; ++j) {
      const int64_t i = c0 + j * kEThreads + threadIdx.x;
      if (i >= np) break;
      const int c = cellp[i];
      if (c < 0 || c >= n) continue;
      const float f = fracp[i];
      const float ep = (1.f - f) * e[c] + f * e[(c + 1) & nmask];
      const float vc = velp[i] + kick * ep;
      const double p = __builtin_rint((double)wp[i] * (double)vc * kFxScale);
      const double pr = fx_share(f, p);
      atomicAdd(reinterpret_cast<unsigned long long*>(&s_q[c]),
                (unsigned long long)(long long)(p - pr));
      atomicAdd(reinterpret_cast<unsigned long long*>(&s_q[(c + 1) & nmask]),
                (unsigned long long)(long long)pr);
    }
  }
  __syncthreads();
  unsigned long long* __restrict__ gj = reinterpret_cast<unsigned long long*>(R.jfx);
  for (int k = threadIdx.x; k < n; k += kEThreads) {
    const long long v = s_q[k];
    if (v != 0) atomicAdd(&gj[k], (unsigned long long)v);
  }
}

__global__ void k_electron_profile(const RepDev* __restrict__ reps,
                                   const RepDev* __restrict__ ereps, int from_moments,
                                   int qsel) {
  const RepDev& R = reps[blockIdx.x];
  const RepDev& E = ereps[blockIdx.x];
  const auto phi = gmem(R.phi);
  const auto u = gmem(R.prof_u);
  const auto qi = gmem(reinterpret_cast<const long long*>(R.q[qsel]));
  const auto ji = gmem(reinterpret_cast<const long long*>(R.jfx));
  const auto pn = gmem(E.prof_n);
  const auto pu = gmem(E.prof_u);
  // node density q 2^-40 / h against n_floor, i.e. q against n_floor h 2^40
  const double qfloor = R.n_floor * R.h * kFxScale;
  for (int k = threadIdx.x; k < R.n_nodes; k += blockDim.x) {
    pn[k] = exp(phi[phi_slot(k, R.n_cells, R.field_m)]);
    if (from_moments) {
      const double q = (double)qi[k];
      pu[k] = q > qfloor ? (double)ji[k] / q : 0.0;
    } else {
      pu[k] = u[k];
    }
  }
  if (threadIdx.x == 0)
    gmem(E.aux)[1] = (int64_t)(uint32_t)((uint32_t)gmem(R.aux)[1] ^ kElectronShiftXor);
}

}  // namespace

void launch_electrons(const RepDev* d_ereps, int n_reps, int push, int fresh, int qsel,
                      int max_nodes, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
  if (n_reps <= 0 || max_nodes > kEMaxNodes) return;
  // enough workgroups for every chunk of the largest store the host allows;
  // the surplus of a smaller store leaves at once
  const dim3 grid(1024, (unsigned)n_reps);
  const size_t lds = sizeof(long long) * (size_t)max_nodes;
  if (push && ev0 && ev1)  // bracketed by the timing events (extended launch)
    hipExtLaunchKernelGGL(k_electrons<true>, grid, dim3(kEThreads), lds, stream, ev0, ev1, 0,
                          d_ereps, fresh, qsel);
  else if (push)
    hipLaunchKernelGGL(k_electrons<true>, grid, dim3(kEThreads), lds, stream, d_ereps, fresh, qsel);
  else
    hipLaunchKernelGGL(k_electrons<false>, grid, dim3(kEThreads), lds, stream, d_ereps, fresh,
                       qsel);
}

void launch_electron_profile(const RepDev* d_reps, const RepDev* d_ereps, int n_reps,
                             int from_moments, int qsel, hipStream_t stream) {
  hipLaunchKernelGGL(k_electron_profile, dim3(n_reps), dim3(256), 0, stream, d_reps, d_ereps,
                     from_moments, qsel);
}

void launch_ion_momentum(const RepDev* d_reps, int n_reps, int half_kick, int max_nodes,
                         hipStream_t stream) {
  if (n_reps <= 0 || max_nodes > kEMaxNodes) return;
  const dim3 grid(1024, (unsigned)n_reps);
  const size_t lds = sizeof(long long) * (size_t)max_nodes;
  hipLaunchKernelGGL(k_ion_momentum, grid, dim3(kEThreads), lds, stream, d_reps, half_kick);
}

}  // namespace efpi
