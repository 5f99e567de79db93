// k_util.hip -- state conversion, a-priori speed and conserved totals.
#include "dev_common.h"
#include "phys.h"

namespace claw {

// FP64 device array -> working precision state (compensation cleared).
template <typename R>
__global__ void k_load_state(R* __restrict__ q, R* __restrict__ c, const double* __restrict__ in,
                             size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    q[t] = (R)in[t];
    if (c) c[t] = R(0);
  }
}

// Working state -> FP64 (value minus compensation, formed in FP64).
template <typename R>
__global__ void k_store_state(double* __restrict__ out, const R* __restrict__ q,
                              const R* __restrict__ c, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x)
    out[t] = c ? (double)q[t] - (double)c[t] : (double)q[t];
}

template <typename R>
__global__ void k_convert(R* __restrict__ dst, const double* __restrict__ src, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x)
    dst[t] = (R)src[t];
}

// Largest characteristic speed / spacing over the cells (first step size).
template <typename R, class P>
__global__ void k_cell_speed(const GridDesc* __restrict__ grids, int src,
                             unsigned long long* __restrict__ out) {
  const GridDesc& G = grids[0];
  const size_t n = (size_t)G.nx * G.ny;
  const R* __restrict__ q = (const R*)G.q[src];
  const R* __restrict__ aux = (const R*)G.aux;
  const P phys(G);
  const double rdx = 1.0 / G.dx, rdy = 1.0 / G.dy;
  double best = 0.0;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    R v[P::M], a[kMaxAux];
#pragma unroll
    for (int k = 0; k < P::M; ++k) v[k] = q[k * n + t];
    for (int k = 0; k < P::NA; ++k) a[k] = aux[k * n + t];
    best = fmax(best, phys.cell_speed(v, a, rdx, rdy));
  }
  best = wave_max(best);
  if ((threadIdx.x & (kLanes - 1)) == 0) atomicMax(out, dbits(best));
}

// Conserved totals, deterministic: block b sums a fixed contiguous range in
// a fixed order (tree inside the block), then one block sums the partials.
constexpr int kTotBlocks = 256, kTotThreads = 256;

template <typename R>
__global__ __launch_bounds__(kTotThreads) void k_totals_partial(const R* __restrict__ q,
                                                                const R* __restrict__ c, int m,
                                                                size_t n,
                                                                double* __restrict__ part) {
  __shared__ double red[kTotThreads];
  const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const size_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  for (int k = 0; k < m; ++k) {
    double s = 0.0;
    for (size_t t = lo + threadIdx.x; t < hi; t += blockDim.x)
      s += c ? (double)q[k * n + t] - (double)c[k * n + t] : (double)q[k * n + t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[k * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ void k_totals_final(const double* __restrict__ part, int m, int nb, double cell,
                               double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k < m) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[k * nb + b];
    out[k] = s * cell;
  }
}

// Head of a step in a scratch buffer that keeps the previous call's
// contents: the grid descriptor (passed by value), a zeroed controller
// record and zeroed Courant-reduction slots.  A fill kernel rather than
// memset and copy nodes, so a captured sequence replays it as it is.
__global__ void k_static_setup(GridDesc g, GridDesc* __restrict__ dst, Ctrl* __restrict__ ctrl,
                               SpeedSlot* __restrict__ slots) {
  if (threadIdx.x == 0) *dst = g;
  unsigned int* c = (unsigned int*)ctrl;
  for (unsigned t = threadIdx.x; t < sizeof(Ctrl) / sizeof(unsigned int); t += blockDim.x) c[t] = 0u;
  unsigned int* sl = (unsigned int*)slots;
  for (unsigned t = threadIdx.x; t < kSpeedSlots * sizeof(SpeedSlot) / sizeof(unsigned int);
       t += blockDim.x)
    sl[t] = 0u;
}

// Courant number of the step just taken: dt times the launch-end maximum of
// |speed| / spacing that the step kernels left in the controller record.
__global__ void k_static_courant(const Ctrl* __restrict__ ctrl, double dt, double* __restrict__ out) {
  if (threadIdx.x == 0) *out = dt * ctrl->last_speed;
}

// ---------------------------------------------------------------------------
static dim3 grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

hipError_t launch_load_state(int fp32, void* q, void* c, const double* in, size_t n,
                             hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_load_state<float>, grid_for(n), dim3(256), 0, st, (float*)q, (float*)c, in, n);
  else
    hipLaunchKernelGGL(k_load_state<double>, grid_for(n), dim3(256), 0, st, (double*)q, (double*)c, in, n);
  return hipGetLastError();
}

hipError_t launch_store_state(int fp32, double* out, const void* q, const void* c, size_t n,
                              hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_store_state<float>, grid_for(n), dim3(256), 0, st, out, (const float*)q,
                       (const float*)c, n);
  else
    hipLaunchKernelGGL(k_store_state<double>, grid_for(n), dim3(256), 0, st, out, (const double*)q,
                       (const double*)c, n);
  return hipGetLastError();
}

hipError_t launch_convert(int fp32, void* dst, const double* src, size_t n, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_convert<float>, grid_for(n), dim3(256), 0, st, (float*)dst, src, n);
  else
    hipLaunchKernelGGL(k_convert<double>, grid_for(n), dim3(256), 0, st, (double*)dst, src, n);
  return hipGetLastError();
}

template <typename R>
static hipError_t cell_speed_t(int ndim, int riemann, const GridDesc* g, int src, size_t n,
                               unsigned long long* out, hipStream_t st) {
  const dim3 grid = grid_for(n), blk(256);
  if (ndim == 2) {
    switch (riemann) {
      case 1: hipLaunchKernelGGL((k_cell_speed<R, Advection<R, 2>>), grid, blk, 0, st, g, src, out); break;
      case 2: hipLaunchKernelGGL((k_cell_speed<R, ShallowWater<R, 2>>), grid, blk, 0, st, g, src, out); break;
      case 3: hipLaunchKernelGGL((k_cell_speed<R, EulerHLLE<R, 2>>), grid, blk, 0, st, g, src, out); break;
      case 4: hipLaunchKernelGGL((k_cell_speed<R, Elastic<R>>), grid, blk, 0, st, g, src, out); break;
      case 5: hipLaunchKernelGGL((k_cell_speed<R, EulerRoe<R, 2, false>>), grid, blk, 0, st, g, src, out); break;
      case 6: hipLaunchKernelGGL((k_cell_speed<R, EulerRoe<R, 2, true>>), grid, blk, 0, st, g, src, out); break;
      case 7: hipLaunchKernelGGL((k_cell_speed<R, PSystem<R, 2>>), grid, blk, 0, st, g, src, out); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (riemann) {
      case 1: hipLaunchKernelGGL((k_cell_speed<R, Advection<R, 1>>), grid, blk, 0, st, g, src, out); break;
      case 2: hipLaunchKernelGGL((k_cell_speed<R, ShallowWater<R, 1>>), grid, blk, 0, st, g, src, out); break;
      case 3: hipLaunchKernelGGL((k_cell_speed<R, EulerHLLE<R, 1>>), grid, blk, 0, st, g, src, out); break;
      case 5: hipLaunchKernelGGL((k_cell_speed<R, EulerRoe<R, 1, false>>), grid, blk, 0, st, g, src, out); break;
      case 6: hipLaunchKernelGGL((k_cell_speed<R, EulerRoe<R, 1, true>>), grid, blk, 0, st, g, src, out); break;
      case 7: hipLaunchKernelGGL((k_cell_speed<R, PSystem<R, 1>>), grid, blk, 0, st, g, src, out); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_cell_speed(int ndim, int riemann, int fp32, const GridDesc* g, int src, size_t n,
                             unsigned long long* out, hipStream_t st) {
  return fp32 ? cell_speed_t<float>(ndim, riemann, g, src, n, out, st)
              : cell_speed_t<double>(ndim, riemann, g, src, n, out, st);
}

hipError_t launch_static_setup(const GridDesc& g, GridDesc* d_grid, Ctrl* d_ctrl,
                               SpeedSlot* d_slots, hipStream_t st) {
  hipLaunchKernelGGL(k_static_setup, dim3(1), dim3(256), 0, st, g, d_grid, d_ctrl, d_slots);
  return hipGetLastError();
}

hipError_t launch_static_courant(const Ctrl* d_ctrl, double dt, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_static_courant, dim3(1), dim3(64), 0, st, d_ctrl, dt, out);
  return hipGetLastError();
}

int totals_blocks() { return kTotBlocks; }

hipError_t launch_totals(int fp32, const void* q, const void* c, int m, size_t n, double cell,
                         double* part, double* out, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_totals_partial<float>, dim3(kTotBlocks), dim3(kTotThreads), 0, st,
                       (const float*)q, (const float*)c, m, n, part);
  else
    hipLaunchKernelGGL(k_totals_partial<double>, dim3(kTotBlocks), dim3(kTotThreads), 0, st,
                       (const double*)q, (const double*)c, m, n, part);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, st, part, m, kTotBlocks, cell, out);
  return hipGetLastError();
}

}  // namespace claw
