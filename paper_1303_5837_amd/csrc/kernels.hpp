// Kernel parameter blocks and launchers (host and device side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace caqr {

// Columns of C per workgroup of the update kernels.
constexpr int kUpdTile = 32;
// Updates of at most this many tiles climb the tree inside one launch (with
// tickets, L per tile); wider ones run one launch per tree level.
constexpr int kTreeTiles = 4;

// One panel of the factorization: rows [0, m) x columns [0, b) at A (lda),
// elements of type T (double, or float for the single-precision batched TSQR).
template <class T>
struct PanelParamsT {
  T *A;
  int64_t lda;
  int64_t m;
  int b;          // panel width, 1..64
  int L;          // number of leaves (row blocks of leaf_rows rows)
  int lpw;        // leaves per workgroup (1, 2, 4; a power of arity)
  int arity;      // tree arity K: 2 or 4
  T *tau_leaf;    // [L][64]
  T *tau_node;    // [L][64], node id = first eliminated member g + s (1..L-1)
  T *d;           // [64] signs of the root R
  unsigned *tickets;  // [L], zero on entry and on exit
};
using PanelParams = PanelParamsT<double>;
using PanelParams32 = PanelParamsT<float>;

// Application of one panel's Q (or Q^T) to C (m rows x k columns at C, ldc).
// Leaves, nodes and their reflectors as produced by the panel kernel.
struct UpdateParams {
  const double *Y;    // panel origin (reflectors live here), ldy
  int64_t ldy;
  double *C;          // rows aligned with the panel's rows
  int64_t ldc;
  int64_t m;          // panel rows
  int64_t k;          // columns of C
  int b;              // panel width
  int L;              // leaves
  int h;              // leaf rows
  const double *T_leaf;
  const double *T_node;
  const double *d;    // signs
  int tiles;          // column tiles of kUpdTile
  int arity;          // tree arity K: 2 or 4
  int stride;         // node kernels: tree level processed, as its stride s = K^j
  int f32;            // 1: the leaf products Y^T C and Y W on FP32 MFMA (mixed-precision factorization)
  unsigned *tickets;  // [kTreeTiles * L] zero on entry and exit, or null; with
                      // tickets, a Q^T of at most kTreeTiles tiles runs the
                      // whole tree in one launch
};

// Leaves and tree (arity p.arity) of one panel.  With device_tree (tickets
// required), the workgroups climb the whole tree; without, each stops at its
// own subtree and launch_tsqr_level finishes the tree, one launch per level.
// inner_block (0, 16 or 32; no effect unless narrower than the panel; binary
// trees only): every leaf and stacked elimination is factored in inner blocks
// of that many columns, each block applied to the columns right of it at once.
hipError_t launch_tsqr_panel(const PanelParams &p, int leaf_rows, hipStream_t s, bool device_tree = true,
                             int inner_block = 0);
// Level s (groups of survivor g = K s i, members g + t s) of one panel's
// tree; the top level also normalizes the root.
hipError_t launch_tsqr_level(const PanelParams &p, int s, int leaf_rows, hipStream_t st, int inner_block = 0);

// Independent panels of equal ceil(b/16) = nq, leaf height and tree arity in
// one launch: probs (device) holds one PanelParams per problem, items
// (device) one (problem, first leaf) pair per workgroup; each workgroup stops
// at the tree levels that join its leaves with another workgroup's.
hipError_t launch_tsqr_panel_batched(const PanelParams *probs, const int2 *items, int nitems, int leaf_rows, int nq,
                                     int arity, hipStream_t s);
hipError_t launch_tsqr_panel_batched(const PanelParams32 *probs, const int2 *items, int nitems, int leaf_rows, int nq,
                                     int arity, hipStream_t s);
// One device-level tree step of many panels of equal ceil(b/16) = nq and
// arity: node (problem, survivor slot g, stride s, leaf rows | root << 12 |
// members << 16) per workgroup.
hipError_t launch_tsqr_tree_level(const PanelParams *probs, const int4 *nodes, int nnodes, int nq, int arity,
                                  hipStream_t s);
hipError_t launch_tsqr_tree_level(const PanelParams32 *probs, const int4 *nodes, int nnodes, int nq, int arity,
                                  hipStream_t s);

// C <- Q^T C for one panel: leaf updates and the tree bottom-up, then rows
// 0..b-1 scaled by D.  One workgroup per (leaf, tile), then one launch per
// tree level; with tickets and at most kTreeTiles tiles, one launch in which
// each (leaf, tile) workgroup climbs its tile's tree.
hipError_t launch_apply_qt(const UpdateParams &u, hipStream_t s);

// Bind the next launch_apply_qt on this thread to two events: start takes its
// first kernel's start time, stop its last kernel's end time (no packets of
// their own on the stream).  (nullptr, nullptr) unbinds.
void set_launch_trace(hipEvent_t start, hipEvent_t stop);

// C <- Q C for one panel: rows 0..b-1 scaled by D, the tree top-down (one
// launch per level), then the leaves.
hipError_t launch_apply_qn(const UpdateParams &u, hipStream_t s);

// T factors (column-major 64x64, ld 64) of every leaf and node of a factored
// panel; h must be a multiple of 16.
struct FormTParams {
  const double *Y;  // panel origin
  int64_t ldy;
  int64_t m;
  int b, L, h;
  int arity;        // tree arity K: 2 or 4
  const double *tau_leaf, *tau_node;
  double *T_leaf, *T_node;
};
hipError_t launch_form_t(const FormTParams &f, hipStream_t s);

// Least squares helpers.
// Back substitution R X = B (R n-by-n upper, B n-by-nrhs), in place.
hipError_t launch_trsm_upper(const double *R, int64_t ldr, int64_t n, double *B, int64_t ldb, int64_t nrhs,
                             hipStream_t s);
// status[0] <- 0, or 1 + (first j with R_jj == 0); status[1] <- 1 if some R_jj or
// some entry of X(0:n, :) is not finite.
hipError_t launch_check_solution(const double *R, int64_t ldr, int64_t n, const double *X, int64_t ldx,
                                 int64_t nrhs, int64_t *status, hipStream_t s);

}  // namespace caqr
