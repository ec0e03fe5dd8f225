// Plane transforms of the 3D plane Couette problem (see cou.hip): host interface.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>

namespace sps {

// Geometry of the (x, z) planes: Kx = Nx/2 half-spectrum x modes, Nz z modes (FFT order, mode
// index k = m Nz + n), padded grids Ngx x Ngz, Ngy y nodes; lx, lz the periods of the frame the
// kernels work in; unode[Ngy] the base-flow velocity at the y nodes and dunode its derivative.
struct CouetteGeom {
  int Kx, Nz, Ngx, Ngz, Ngy;
  double lx, lz;
  const double* unode;   // host array, copied
  double dunode;
};

class CouettePlanes {
 public:
  CouettePlanes(const CouetteGeom& g, hipStream_t s);
  ~CouettePlanes();
  // nl[3][Ngy][K]: explicit-term densities of the z-grid fields zg[6][Ngy][K] (u_par, v, u_perp
  // and their y-derivatives per mode), rotated back to (par, v, perp), spectral in (x, z) with
  // 1/(Ngx Ngz) normalization.  Uses its own scratch (may overlap a vjp on another stream).
  void forward(const double2* zg, double2* nl, hipStream_t s);
  // zbar[6][Ngy][K] = (d nl / d zg)^H nlbar at zg.
  void vjp(const double2* nlbar, const double2* zg, double2* zbar, hipStream_t s);

 private:
  struct Impl;
  std::unique_ptr<Impl> p_;
};

}  // namespace sps
