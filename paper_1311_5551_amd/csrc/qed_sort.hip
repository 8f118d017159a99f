// Spatial reordering of the particles of an instance with a grid field, by 8 x 8-cell tile of
// their position: a counting sort (histogram of tile keys, exclusive scan, scatter of
// destination slots) followed by a permutation of every array of the species.  Particles that
// share a tile then sit next to each other, so the lanes of a wave gather from the same grid
// cache lines.  The order within a tile follows the atomics; per-particle results of later steps
// do not depend on the order (random streams are keyed by uid).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "qed_device.h"
#include "qed_kernels.h"

namespace qedk {

constexpr int kTile = 8;

template <bool MIXED>
__global__ __launch_bounds__(256) void k_sort_key(const qed_instance* __restrict__ inst, int ii, int s,
                                                  const Glob* __restrict__ glob, double dt, int32_t* __restrict__ key,
                                                  uint32_t* __restrict__ hist, int tiles_x) {
  using Real = typename std::conditional<MIXED, float, double>::type;
  const qed_instance& I = inst[ii];
  const qed_species& S = I.s[s];
  const qed_field& F = I.field;
  int64_t n = *S.count_dev;
  if (n > S.capacity) n = S.capacity;
  const int64_t step = glob->step_next;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double x, y;
    if (s < 2) {
      x = ((const Real*)S.x_dev)[k];
      y = ((const Real*)S.y_dev)[k];
      if (MIXED) {
        x += S.x_lo_dev[k];
        y += S.y_lo_dev[k];
      }
    } else {  // photon position at the start of the next step
      const double kx = ((const Real*)S.ux_dev)[k], ky = ((const Real*)S.uy_dev)[k], kz = ((const Real*)S.uz_dev)[k];
      const double e = sqrt(kx * kx + ky * ky + kz * kz);
      const double age = (double)(step - (int64_t)S.birth_step_dev[k]) * dt;
      x = (double)((const Real*)S.x_dev)[k] + (e > 0.0 ? age * kx / e : 0.0);
      y = (double)((const Real*)S.y_dev)[k] + (e > 0.0 ? age * ky / e : 0.0);
    }
    double gx = floor((x - F.x0) / F.dx), gy = floor((y - F.y0) / F.dy);
    if (!(fabs(gx) < 1e15)) gx = 0.0;  // non-finite positions go to tile 0
    if (!(fabs(gy) < 1e15)) gy = 0.0;
    const int64_t i = wrap_index((int64_t)gx, F.nx), j = wrap_index((int64_t)gy, F.ny);
    const int32_t kk = (int32_t)((j / kTile) * tiles_x + i / kTile);
    key[k] = kk;
    atomicAdd(&hist[kk], 1u);
  }
}

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t* __restrict__ a, int m) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) a[i] = 0u;
}

// exclusive scan of hist[0, m) in place, one block of 1024 threads
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* __restrict__ hist, int m) {
  __shared__ uint32_t part[1024];
  const int per = (m + 1023) / 1024;
  const int b = threadIdx.x * per, e = min(m, b + per);
  uint32_t sum = 0;
  for (int i = b; i < e; ++i) sum += hist[i];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan of the partial sums
    const uint32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
  for (int i = b; i < e; ++i) {
    const uint32_t h = hist[i];
    hist[i] = run;
    run += h;
  }
}

__global__ __launch_bounds__(256) void k_sort_dst(const qed_species* __restrict__ sp, const int32_t* __restrict__ key,
                                                  uint32_t* __restrict__ offs, uint32_t* __restrict__ dst) {
  int64_t n = *sp->count_dev;
  if (n > sp->capacity) n = sp->capacity;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = atomicAdd(&offs[key[k]], 1u);
}

// stage[dst[k]] = a[k], then a[k] = stage[k] (two kernels)
template <class T>
__global__ __launch_bounds__(256) void k_scatter(const qed_species* __restrict__ sp, const T* __restrict__ a,
                                                 T* __restrict__ stage, const uint32_t* __restrict__ dst) {
  int64_t n = *sp->count_dev;
  if (n > sp->capacity) n = sp->capacity;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    stage[dst[k]] = a[k];
}
template <class T>
__global__ __launch_bounds__(256) void k_copy_back(const qed_species* __restrict__ sp, T* __restrict__ a,
                                                   const T* __restrict__ stage) {
  int64_t n = *sp->count_dev;
  if (n > sp->capacity) n = sp->capacity;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    a[k] = stage[k];
}

template <class T>
static void permute(const qed_species* sp_dev, void* a, void* stage, const uint32_t* dst, int grid, hipStream_t s) {
  if (!a) return;
  hipLaunchKernelGGL(k_scatter<T>, dim3(grid), dim3(256), 0, s, sp_dev, (const T*)a, (T*)stage, dst);
  hipLaunchKernelGGL(k_copy_back<T>, dim3(grid), dim3(256), 0, s, sp_dev, (T*)a, (const T*)stage);
}

hipError_t launch_sort_species(const qed_instance* inst_dev, const qed_instance& inst_host, int ii, int s,
                               const Glob* glob, double dt, bool mixed, const SortScratch& w, int grid, hipStream_t st) {
  const qed_field& F = inst_host.field;
  const int tiles_x = (F.nx + kTile - 1) / kTile, tiles_y = (F.ny + kTile - 1) / kTile;
  const int n_tiles = tiles_x * tiles_y;
  if (n_tiles > w.hist_len) return hipErrorInvalidValue;
  const qed_species* sp_dev = &inst_dev[ii].s[s];
  const qed_species& S = inst_host.s[s];
  hipLaunchKernelGGL(k_fill_zero, dim3(256), dim3(256), 0, st, w.hist, n_tiles);
  if (mixed)
    hipLaunchKernelGGL(k_sort_key<true>, dim3(grid), dim3(256), 0, st, inst_dev, ii, s, glob, dt, w.key, w.hist,
                       tiles_x);
  else
    hipLaunchKernelGGL(k_sort_key<false>, dim3(grid), dim3(256), 0, st, inst_dev, ii, s, glob, dt, w.key, w.hist,
                       tiles_x);
  hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, st, w.hist, n_tiles);
  hipLaunchKernelGGL(k_sort_dst, dim3(grid), dim3(256), 0, st, sp_dev, w.key, w.hist, w.dst);
  const bool d3 = inst_host.dims == 3;
  if (mixed) {
    permute<float>(sp_dev, S.x_dev, w.stage, w.dst, grid, st);
    permute<float>(sp_dev, S.y_dev, w.stage, w.dst, grid, st);
    if (d3) permute<float>(sp_dev, S.z_dev, w.stage, w.dst, grid, st);
    permute<float>(sp_dev, S.ux_dev, w.stage, w.dst, grid, st);
    permute<float>(sp_dev, S.uy_dev, w.stage, w.dst, grid, st);
    permute<float>(sp_dev, S.uz_dev, w.stage, w.dst, grid, st);
    if (s < 2) {
      permute<float>(sp_dev, S.x_lo_dev, w.stage, w.dst, grid, st);
      permute<float>(sp_dev, S.y_lo_dev, w.stage, w.dst, grid, st);
      if (d3) permute<float>(sp_dev, S.z_lo_dev, w.stage, w.dst, grid, st);
      permute<float>(sp_dev, S.ux_lo_dev, w.stage, w.dst, grid, st);
      permute<float>(sp_dev, S.uy_lo_dev, w.stage, w.dst, grid, st);
      permute<float>(sp_dev, S.uz_lo_dev, w.stage, w.dst, grid, st);
    }
  } else {
    permute<double>(sp_dev, S.x_dev, w.stage, w.dst, grid, st);
    permute<double>(sp_dev, S.y_dev, w.stage, w.dst, grid, st);
    if (d3) permute<double>(sp_dev, S.z_dev, w.stage, w.dst, grid, st);
    permute<double>(sp_dev, S.ux_dev, w.stage, w.dst, grid, st);
    permute<double>(sp_dev, S.uy_dev, w.stage, w.dst, grid, st);
    permute<double>(sp_dev, S.uz_dev, w.stage, w.dst, grid, st);
  }
  permute<double>(sp_dev, S.tau_dev, w.stage, w.dst, grid, st);
  permute<uint64_t>(sp_dev, S.uid_dev, w.stage, w.dst, grid, st);
  if (s == 2) permute<int32_t>(sp_dev, S.birth_step_dev, w.stage, w.dst, grid, st);
  return hipGetLastError();
}

// Scratch of qed_sort_static: a fixed array in device memory (each GPU holds its own copy from
// the load of the library to the end of the process), laid out as the staging words (8 B per
// slot), the tile keys and destination slots (4 B per slot each), then the tile histogram.  In
// host code its name is not a device address: the address comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[kStaticSortBytes];

hipError_t static_sort_scratch(SortScratch* out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      addr[dev] = p;
    }
  }
  char* base = (char*)addr[dev];
  out->stage = base;
  out->key = (int32_t*)(base + kStaticSortSlots * 8);
  out->dst = (uint32_t*)(base + kStaticSortSlots * 12);
  out->hist = (uint32_t*)(base + kStaticSortSlots * 16);
  out->hist_len = kStaticSortTiles;
  return hipSuccess;
}

}  // namespace qedk
