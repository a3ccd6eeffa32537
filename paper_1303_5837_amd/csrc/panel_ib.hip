// Panel kernels with inner blocks (panel_body.hpp, InnerBlock): binary trees
// whose leaves and stacked eliminations are factored in blocks of 16 or 32
// columns (the block size of the level below, paper Section 3.1 item 1(a)).
#include "panel_body.hpp"
#include "panel_launch.hpp"

namespace caqr {

namespace {

template <int RPT, int NB, int IBS>
hipError_t launch_panel_t(const PanelParams &p, bool device_tree, hipStream_t s) {
  const int grid = (p.L + p.lpw - 1) / p.lpw;
  if (device_tree)
    hipLaunchKernelGGL((tsqr_panel_kernel<RPT, NB, true, IBS, 2>), dim3(grid), dim3(kPanelThreads), 0, s, p);
  else
    hipLaunchKernelGGL((tsqr_panel_kernel<RPT, NB, false, IBS, 2>), dim3(grid), dim3(kPanelThreads), 0, s, p);
  return hipGetLastError();
}

// inner blocks of ibs slots, narrower than the panel (checked by the caller)
template <int RPT>
hipError_t launch_panel_nq(const PanelParams &p, bool device_tree, int ibs, hipStream_t s) {
  switch ((p.b + 15) / 16) {
    case 2: return launch_panel_t<RPT, 2, 1>(p, device_tree, s);
    case 3: return ibs == 1 ? launch_panel_t<RPT, 3, 1>(p, device_tree, s) : launch_panel_t<RPT, 3, 2>(p, device_tree, s);
    case 4: return ibs == 1 ? launch_panel_t<RPT, 4, 1>(p, device_tree, s) : launch_panel_t<RPT, 4, 2>(p, device_tree, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NB, int IBS>
hipError_t launch_level_t(const PanelParams &p, int s, int h, hipStream_t st) {
  const int groups = (p.L - s + 2 * s - 1) / (2 * s);
  hipLaunchKernelGGL((tsqr_level_kernel<NB, IBS, 2>), dim3(groups), dim3(kPanelThreads), 0, st, p, s, h);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tsqr_panel_ib(const PanelParams &p, int leaf_rows, hipStream_t s, bool device_tree, int ibs) {
  switch (leaf_rows) {
    case 64: return launch_panel_nq<4>(p, device_tree, ibs, s);
    case 128: return launch_panel_nq<8>(p, device_tree, ibs, s);
    case 256: return launch_panel_nq<16>(p, device_tree, ibs, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tsqr_level_ib(const PanelParams &p, int s, int leaf_rows, hipStream_t st, int ibs) {
  switch ((p.b + 15) / 16) {
    case 2: return launch_level_t<2, 1>(p, s, leaf_rows, st);
    case 3: return ibs == 1 ? launch_level_t<3, 1>(p, s, leaf_rows, st) : launch_level_t<3, 2>(p, s, leaf_rows, st);
    case 4: return ibs == 1 ? launch_level_t<4, 1>(p, s, leaf_rows, st) : launch_level_t<4, 2>(p, s, leaf_rows, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace caqr
