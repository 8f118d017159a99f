// Maxwell's equations on the 2-D Yee grid of the field-feedback kind (QED_FIELD_GRID_FDTD), the
// field half of the coupling to a particle-in-cell code (Sec. 3.2): after the particles of a step
// have deposited their current, E and B advance one step in code units (dE/dt = curl B - J,
// dB/dt = -curl E), periodic.  B advances half a step with E^n, E a full step with that B and
// J^{n+1/2}, B the second half step with E^{n+1}, so that the next step gathers E and B at the
// same time level.  Each component sits at its own staggered node (i, j) (Yee offsets Ex(i+1/2, j),
// Ey(i, j+1/2), Ez(i, j), Bx(i, j+1/2), By(i+1/2, j), Bz(i+1/2, j+1/2)):
//   Bx(i,j) -= (dt/2) (Ez(i,j+1) - Ez(i,j))/dy
//   By(i,j) += (dt/2) (Ez(i+1,j) - Ez(i,j))/dx
//   Bz(i,j) -= (dt/2) ((Ey(i+1,j) - Ey(i,j))/dx - (Ex(i,j+1) - Ex(i,j))/dy)
//   Ex(i,j) += dt ((Bz(i,j) - Bz(i,j-1))/dy - Jx(i,j))
//   Ey(i,j) += dt (-(Bz(i,j) - Bz(i-1,j))/dx - Jy(i,j))
//   Ez(i,j) += dt ((By(i,j) - By(i-1,j))/dx - (Bx(i,j) - Bx(i,j-1))/dy - Jz(i,j))
// A B update reads only E and its own node, an E update only B, J and its own node, so each
// pass updates in place.  The E pass clears the current it has used (the next step deposits
// into zeroed planes).  HBM-bound stencils: one thread per node, consecutive threads along x.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "qed_device.h"
#include "qed_kernels.h"

namespace qedk {

constexpr int kFdtdBlock = 256;

__global__ __launch_bounds__(kFdtdBlock) void k_fdtd_half_b(const qed_instance* __restrict__ inst, double dt) {
  const qed_field& F = inst[blockIdx.y].field;
  if (F.kind != QED_FIELD_GRID_FDTD) return;
  const int64_t P = (int64_t)F.nx * F.ny;
  double* const G = F.fdtd_dev;
  gptr<const double> Ex = as_global((const double*)G), Ey = Ex + P, Ez = Ey + P;
  gptr<double> Bx = as_global(G + 3 * P), By = Bx + P, Bz = By + P;
  const double h = 0.5 * dt, dx = F.dx, dy = F.dy;
  // the nodes dealt as (row, run of kFdtdBlock columns) pairs, consecutive threads along x
  const int nx = F.nx, ny = F.ny, runs = (nx + kFdtdBlock - 1) / kFdtdBlock;
  for (int64_t q = blockIdx.x; q < (int64_t)ny * runs; q += gridDim.x) {
    const int j = (int)(q / runs), i = (int)(q % runs) * kFdtdBlock + threadIdx.x;
    if (i >= nx) continue;
    const int ip = i + 1 == nx ? 0 : i + 1, jp = j + 1 == ny ? 0 : j + 1;
    const int64_t k = (int64_t)j * nx + i, kx = (int64_t)j * nx + ip, ky = (int64_t)jp * nx + i;
    const double ez = Ez[k], ey = Ey[k], ex = Ex[k];
    Bx[k] = Bx[k] - h * ((Ez[ky] - ez) / dy);
    By[k] = By[k] + h * ((Ez[kx] - ez) / dx);
    Bz[k] = Bz[k] - h * ((Ey[kx] - ey) / dx - (Ex[ky] - ex) / dy);
  }
}

__global__ __launch_bounds__(kFdtdBlock) void k_fdtd_e(const qed_instance* __restrict__ inst, double dt) {
  const qed_field& F = inst[blockIdx.y].field;
  if (F.kind != QED_FIELD_GRID_FDTD) return;
  const int64_t P = (int64_t)F.nx * F.ny;
  double* const G = F.fdtd_dev;
  gptr<double> Ex = as_global(G), Ey = Ex + P, Ez = Ey + P;
  gptr<const double> Bx = as_global((const double*)G + 3 * P), By = Bx + P, Bz = By + P;
  gptr<double> Jx = as_global(G + 6 * P), Jy = Jx + P, Jz = Jy + P;
  const double dx = F.dx, dy = F.dy;
  const int nx = F.nx, ny = F.ny, runs = (nx + kFdtdBlock - 1) / kFdtdBlock;
  for (int64_t q = blockIdx.x; q < (int64_t)ny * runs; q += gridDim.x) {
    const int j = (int)(q / runs), i = (int)(q % runs) * kFdtdBlock + threadIdx.x;
    if (i >= nx) continue;
    const int im = i == 0 ? nx - 1 : i - 1, jm = j == 0 ? ny - 1 : j - 1;
    const int64_t k = (int64_t)j * nx + i, kx = (int64_t)j * nx + im, ky = (int64_t)jm * nx + i;
    const double bz = Bz[k];
    Ex[k] = Ex[k] + dt * ((bz - Bz[ky]) / dy - Jx[k]);
    Ey[k] = Ey[k] + dt * (-(bz - Bz[kx]) / dx - Jy[k]);
    Ez[k] = Ez[k] + dt * ((By[k] - By[kx]) / dx - (Bx[k] - Bx[ky]) / dy - Jz[k]);
    Jx[k] = 0.0;
    Jy[k] = 0.0;
    Jz[k] = 0.0;
  }
}

void launch_fdtd(const qed_instance* inst, int n_inst, int max_nodes_rows, double dt, hipStream_t s) {
  // enough blocks to stream the largest grid at full bandwidth; blocks past a smaller grid's
  // rows leave at once
  const int blocks = std::max(1, std::min(max_nodes_rows, 8192));
  const dim3 g(blocks, n_inst);
  hipLaunchKernelGGL(k_fdtd_half_b, g, dim3(kFdtdBlock), 0, s, inst, dt);
  hipLaunchKernelGGL(k_fdtd_e, g, dim3(kFdtdBlock), 0, s, inst, dt);
  hipLaunchKernelGGL(k_fdtd_half_b, g, dim3(kFdtdBlock), 0, s, inst, dt);
}

}  // namespace qedk
