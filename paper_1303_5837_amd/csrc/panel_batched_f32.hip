// Batched panel kernels (panel_body.hpp) on float elements: many independent
// uneven panels in one launch per (leaf height, ceil(n/16), arity), and one
// launch per device tree level for all of them.
#include "panel_body.hpp"

namespace caqr {

namespace {

using Elem = float;

template <int RPT, int NB, int K>
hipError_t launch_batched_t(const PanelParamsT<Elem> *probs, const int2 *items, int nitems, hipStream_t s) {
  hipLaunchKernelGGL((tsqr_panel_batched_kernel<Elem, RPT, NB, K>), dim3(nitems), dim3(kPanelThreads), 0, s, probs,
                     items);
  return hipGetLastError();
}

template <int RPT, int K>
hipError_t launch_batched_nq(int nq, const PanelParamsT<Elem> *probs, const int2 *items, int nitems, hipStream_t s) {
  switch (nq) {
    case 1: return launch_batched_t<RPT, 1, K>(probs, items, nitems, s);
    case 2: return launch_batched_t<RPT, 2, K>(probs, items, nitems, s);
    case 3: return launch_batched_t<RPT, 3, K>(probs, items, nitems, s);
    case 4: return launch_batched_t<RPT, 4, K>(probs, items, nitems, s);
    default: return hipErrorInvalidValue;
  }
}

template <int K>
hipError_t launch_batched_k(const PanelParamsT<Elem> *probs, const int2 *items, int nitems, int leaf_rows, int nq,
                            hipStream_t s) {
  switch (leaf_rows) {
    case 64: return launch_batched_nq<4, K>(nq, probs, items, nitems, s);
    case 128: return launch_batched_nq<8, K>(nq, probs, items, nitems, s);
    case 256: return launch_batched_nq<16, K>(nq, probs, items, nitems, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NB, int K>
hipError_t launch_level_t(const PanelParamsT<Elem> *probs, const int4 *nodes, int nnodes, hipStream_t s) {
  hipLaunchKernelGGL((tsqr_tree_level_kernel<Elem, NB, K>), dim3(nnodes), dim3(kPanelThreads), 0, s, probs, nodes);
  return hipGetLastError();
}

template <int K>
hipError_t launch_level_k(const PanelParamsT<Elem> *probs, const int4 *nodes, int nnodes, int nq, hipStream_t s) {
  switch (nq) {
    case 1: return launch_level_t<1, K>(probs, nodes, nnodes, s);
    case 2: return launch_level_t<2, K>(probs, nodes, nnodes, s);
    case 3: return launch_level_t<3, K>(probs, nodes, nnodes, s);
    case 4: return launch_level_t<4, K>(probs, nodes, nnodes, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_tsqr_panel_batched(const PanelParamsT<Elem> *probs, const int2 *items, int nitems, int leaf_rows,
                                     int nq, int arity, hipStream_t s) {
  if (nitems < 1 || nq < 1 || nq > 4) return hipErrorInvalidValue;
  if (arity == 2) return launch_batched_k<2>(probs, items, nitems, leaf_rows, nq, s);
  if (arity == 4) return launch_batched_k<4>(probs, items, nitems, leaf_rows, nq, s);
  return hipErrorInvalidValue;
}

hipError_t launch_tsqr_tree_level(const PanelParamsT<Elem> *probs, const int4 *nodes, int nnodes, int nq, int arity,
                                  hipStream_t s) {
  if (nnodes < 1) return hipErrorInvalidValue;
  if (arity == 2) return launch_level_k<2>(probs, nodes, nnodes, nq, s);
  if (arity == 4) return launch_level_k<4>(probs, nodes, nnodes, nq, s);
  return hipErrorInvalidValue;
}

}  // namespace caqr
