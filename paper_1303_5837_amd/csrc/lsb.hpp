// Batched least squares after a batched TSQR (problems with n <= 64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace caqr {

// One problem of a batched least-squares solve, after its factorization:
// A holds R on top, the leaf reflectors below each leaf's diagonal and the
// tree nodes' V over the eliminated slots; tau_leaf / tau_node ([L][64]) and
// the signs d as the batched TSQR wrote them.
struct LsbProb {
  const double *A;
  int64_t lda, m;
  int b, L, h;  // n, leaves, leaf rows (64, 128 or 256)
  int arity;    // tree arity K: 2 or 4
  const double *tau_leaf, *tau_node, *d;
  double *B;  // m x nrhs, ldb; rows 0..n-1 receive the solution
  int64_t ldb;
  int nrhs;
  int status0;  // first of this problem's status pairs (one pair per right-hand side)
};

// Q^T applied to B by the leaf reflectors: one wave per (problem, leaf, rhs)
// item {problem, leaf, rhs, 0}.
hipError_t launch_lsb_leaves(const LsbProb *probs, const int4 *items, int nitems, hipStream_t s);
// By the node reflectors of one tree level: item {problem, survivor slot g,
// stride s, rhs} (members g + t s, t < K, present below L); levels must run
// bottom-up, after the leaves.
hipError_t launch_lsb_nodes(const LsbProb *probs, const int4 *items, int nitems, hipStream_t s);
// x = R^-1 D (Q_impl^T b)(0:n) in place, and the status pair of each item
// {problem, rhs}: status[2 (status0 + rhs) + 0] = 1 + first j with R_jj == 0
// (else 0), [+1] = 1 if some R_jj or x_i is not finite.
hipError_t launch_lsb_solve(const LsbProb *probs, const int2 *items, int nitems, int64_t *status, hipStream_t s);

}  // namespace caqr
