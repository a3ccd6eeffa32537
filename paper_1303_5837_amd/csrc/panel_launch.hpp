// Launchers of the panel kernels split over several translation units (so
// that their many template instances compile in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace caqr {

// Arity-4 trees (panel_a4.hip).
hipError_t launch_tsqr_panel_a4(const PanelParams &p, int leaf_rows, hipStream_t s, bool device_tree);
hipError_t launch_tsqr_level_a4(const PanelParams &p, int s, int leaf_rows, hipStream_t st);
// Binary trees with inner blocks of ibs 16-column slots, ibs = 1 or 2 (panel_ib.hip).
hipError_t launch_tsqr_panel_ib(const PanelParams &p, int leaf_rows, hipStream_t s, bool device_tree, int ibs);
hipError_t launch_tsqr_level_ib(const PanelParams &p, int s, int leaf_rows, hipStream_t st, int ibs);

}  // namespace caqr
