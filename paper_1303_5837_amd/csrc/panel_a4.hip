// Panel kernels with trees of arity 4 (panel_body.hpp): every node eliminates
// up to three stacked R factors against a survivor, so a panel of L leaves
// has ceil(log4 L) levels of stacked eliminations on its critical path.
#include "panel_body.hpp"
#include "panel_launch.hpp"

namespace caqr {

namespace {

template <int RPT, int NB>
hipError_t launch_panel_t(const PanelParams &p, bool device_tree, hipStream_t s) {
  const int grid = (p.L + p.lpw - 1) / p.lpw;
  if (device_tree)
    hipLaunchKernelGGL((tsqr_panel_kernel<RPT, NB, true, 0, 4>), dim3(grid), dim3(kPanelThreads), 0, s, p);
  else
    hipLaunchKernelGGL((tsqr_panel_kernel<RPT, NB, false, 0, 4>), dim3(grid), dim3(kPanelThreads), 0, s, p);
  return hipGetLastError();
}

template <int RPT>
hipError_t launch_panel_nq(const PanelParams &p, bool device_tree, hipStream_t s) {
  switch ((p.b + 15) / 16) {
    case 1: return launch_panel_t<RPT, 1>(p, device_tree, s);
    case 2: return launch_panel_t<RPT, 2>(p, device_tree, s);
    case 3: return launch_panel_t<RPT, 3>(p, device_tree, s);
    case 4: return launch_panel_t<RPT, 4>(p, device_tree, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NB>
hipError_t launch_level_t(const PanelParams &p, int s, int h, hipStream_t st) {
  const int groups = (p.L - s + 4 * s - 1) / (4 * s);  // groups with two or more members
  hipLaunchKernelGGL((tsqr_level_kernel<NB, 0, 4>), dim3(groups), dim3(kPanelThreads), 0, st, p, s, h);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tsqr_panel_a4(const PanelParams &p, int leaf_rows, hipStream_t s, bool device_tree) {
  switch (leaf_rows) {
    case 64: return launch_panel_nq<4>(p, device_tree, s);
    case 128: return launch_panel_nq<8>(p, device_tree, s);
    case 256: return launch_panel_nq<16>(p, device_tree, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tsqr_level_a4(const PanelParams &p, int s, int leaf_rows, hipStream_t st) {
  switch ((p.b + 15) / 16) {
    case 1: return launch_level_t<1>(p, s, leaf_rows, st);
    case 2: return launch_level_t<2>(p, s, leaf_rows, st);
    case 3: return launch_level_t<3>(p, s, leaf_rows, st);
    case 4: return launch_level_t<4>(p, s, leaf_rows, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace caqr
