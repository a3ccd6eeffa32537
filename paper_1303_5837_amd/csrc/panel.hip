// Launchers of the panel factorization (panel_body.hpp): the binary-tree
// kernels without inner blocks are instantiated here; arity-4 trees and inner
// blocks live in panel_a4.hip and panel_ib.hip.
#include "panel_body.hpp"
#include "panel_launch.hpp"

namespace caqr {

namespace {

template <int RPT, int NB>
hipError_t launch_panel_t(const PanelParams &p, bool device_tree, hipStream_t s) {
  const int grid = (p.L + p.lpw - 1) / p.lpw;
  if (device_tree)
    hipLaunchKernelGGL((tsqr_panel_kernel<RPT, NB, true, 0, 2>), dim3(grid), dim3(kPanelThreads), 0, s, p);
  else
    hipLaunchKernelGGL((tsqr_panel_kernel<RPT, NB, false, 0, 2>), dim3(grid), dim3(kPanelThreads), 0, s, p);
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
  const int groups = (p.L - s + 2 * s - 1) / (2 * s);  // groups with two members
  hipLaunchKernelGGL((tsqr_level_kernel<NB, 0, 2>), dim3(groups), dim3(kPanelThreads), 0, st, p, s, h);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tsqr_panel(const PanelParams &p, int leaf_rows, hipStream_t s, bool device_tree, int inner_block) {
  if (p.b < 1 || p.b > kMaxB || p.L < 1 || p.lpw < 1) return hipErrorInvalidValue;
  if (p.arity != 2 && p.arity != 4) return hipErrorInvalidValue;
  if (device_tree && !p.tickets) return hipErrorInvalidValue;
  if (inner_block % 16 || inner_block < 0) return hipErrorInvalidValue;
  const int ibs = inner_block / 16;  // 16-column slots per inner block (four waves)
  const int nq = (p.b + 15) / 16;
  if ((ibs == 1 && nq > 1) || (ibs == 2 && nq > 2)) {
    if (p.arity != 2) return hipErrorInvalidValue;
    return launch_tsqr_panel_ib(p, leaf_rows, s, device_tree, ibs);
  }
  if (p.arity == 4) return launch_tsqr_panel_a4(p, leaf_rows, s, device_tree);
  switch (leaf_rows) {
    case 64: return launch_panel_nq<4>(p, device_tree, s);
    case 128: return launch_panel_nq<8>(p, device_tree, s);
    case 256: return launch_panel_nq<16>(p, device_tree, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tsqr_level(const PanelParams &p, int s, int leaf_rows, hipStream_t st, int inner_block) {
  if (p.b < 1 || p.b > kMaxB || s < 1 || s >= p.L) return hipErrorInvalidValue;
  if (p.arity != 2 && p.arity != 4) return hipErrorInvalidValue;
  if (inner_block % 16 || inner_block < 0) return hipErrorInvalidValue;
  const int ibs = inner_block / 16;
  const int nq = (p.b + 15) / 16;
  if ((ibs == 1 && nq > 1) || (ibs == 2 && nq > 2)) {
    if (p.arity != 2) return hipErrorInvalidValue;
    return launch_tsqr_level_ib(p, s, leaf_rows, st, ibs);
  }
  if (p.arity == 4) return launch_tsqr_level_a4(p, s, leaf_rows, st);
  switch (nq) {
    case 1: return launch_level_t<1>(p, s, leaf_rows, st);
    case 2: return launch_level_t<2>(p, s, leaf_rows, st);
    case 3: return launch_level_t<3>(p, s, leaf_rows, st);
    case 4: return launch_level_t<4>(p, s, leaf_rows, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace caqr
