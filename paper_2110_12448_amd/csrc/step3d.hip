// step3d.hip -- fused psi/U explicit step on the 3D cubic lattice (gfx950).
#include "pf_device.hpp"

namespace pf {

Geom3D geom3d(int nx, int ny, int nz, int seg, int ztile) {
  Geom3D g;
  g.nstrips = (nx + 59) / 60;
  g.wout = (nx + g.nstrips - 1) / g.nstrips;
  g.ztile = ztile < 1 ? 1 : ztile;
  g.nzt = (nz + g.ztile - 1) / g.ztile;
  g.seg = seg < 1 ? 1 : seg;
  g.nsegs = (ny + g.seg - 1) / g.seg;
  g.threads = 64 * (g.ztile + 2);
  g.blocks = g.nstrips * g.nzt * g.nsegs;
  return g;
}

template <typename T>
hipError_t launch_step3d(const Step3DArgs<T> &, const Geom3D &, bool, bool, bool, hipStream_t) {
  return hipErrorNotSupported;
}

template hipError_t launch_step3d<float>(const Step3DArgs<float> &, const Geom3D &, bool, bool,
                                         bool, hipStream_t);
template hipError_t launch_step3d<double>(const Step3DArgs<double> &, const Geom3D &, bool, bool,
                                          bool, hipStream_t);

}  // namespace pf
