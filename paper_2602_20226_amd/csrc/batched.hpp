// Instance descriptor of the batched persistent kernel (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include "wg_gemm.hpp"

namespace qtt {

constexpr int QTT_BATCH_MAXN = 32;        // cores per instance
constexpr int QTT_BSTATUS_OK = 0, QTT_BSTATUS_NONFINITE = 1, QTT_BSTATUS_NOCONV = 2;

struct BInst {
  const double* a[QTT_BATCH_MAXN];
  const double* b[QTT_BATCH_MAXN];
  double* out[QTT_BATCH_MAXN];
  double* ws;  // this instance's workspace (offsets below are in doubles)
  long offM[QTT_BATCH_MAXN], offT[QTT_BATCH_MAXN];
  long offCenter, offR, offY, offZ, offX, offXc, offYn, offTB, offSig, offPerm, offTmp, offOne;
  int ra[QTT_BATCH_MAXN + 1], rb[QTT_BATCH_MAXN + 1];
  int rho[QTT_BATCH_MAXN + 1];
  int m[QTT_BATCH_MAXN];
  int d[QTT_BATCH_MAXN], dj[QTT_BATCH_MAXN];
  int n;
  int mpo;
};

// Reset the work queue and launch the persistent kernel (variant bit 0:
// Jacobi blocks of 4 rows instead of 8).  max_L bounds the Jacobi row length;
// max_sweeps caps each Jacobi iteration (status NOCONV when reached).
hipError_t batched_launch(hipStream_t s, int variant, int grid, const BInst* insts, const int* order, int count,
                          unsigned* queue, const TileMap& tm, double rel_tol, long max_rank, int max_sweeps,
                          long* ranks_out, double* tails_out, int* status, int max_L);
// One launch of the tuner probe: grid workgroups each computing C = A B
// (row-major M x K times K x N) with tile variant `variant` (wg_gemm.hpp).
hipError_t tile_probe_launch(hipStream_t s, int variant, int grid, int M, int N, int K, const double* A,
                             const double* B, double* C);

}  // namespace qtt
