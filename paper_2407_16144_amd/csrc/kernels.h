// Argument block of the two per-step kernels.
#pragma once
#include <stdint.h>

#include "halp_types.h"

namespace halp {

template <class T>
struct IterArgs {
  // K (rows = constraints) and the explicit K^T (rows = variables), scaled
  const int32_t* K_rp;
  const int32_t* K_ci;
  const T* K_v;
  const int32_t* KT_rp;
  const int32_t* KT_ci;
  const T* KT_v;
  const int32_t* brpK;   // row pointers of sliced blocks of K / K^T
  const int32_t* brpKT;
  // n-space
  const T* c;
  const T* l;
  const T* u;
  const double* Dc;
  T* x;      // iterate z^{n,k}, x part
  T* x0;     // anchor z^{n,0}
  T* xbar;   // 2 x+ - x, gathered by the dual SpMV
  T* xT;     // T(z) at the last check
  T* ktyp;   // K^T y+ at the last eval
  T* cx1;    // dual-infeasibility ray candidates (recession-projected)
  T* cx2;
  T* xs;     // average PDHG: sum of the epoch's iterates x^{n,0..k}
  uint8_t* actx;  // activity of x+ at the last check: 1 at l, 2 at u, 0 inside, 255 none yet
  // m-space
  const T* q;
  const double* Dr;
  T* y;
  T* y0;
  T* yT;
  T* dy;     // y - y+ at the last check
  T* kxbar;  // K xbar at the last check
  T* kxp;    // K x+ at the last eval
  T* cy1;    // primal-infeasibility ray candidates (clamped)
  T* cy2;
  T* ys;     // average PDHG: sum of the epoch's iterates y^{n,0..k}
  uint8_t* acty;  // activity of y+ at the last check: 1 at zero (inequality rows), 0 else
  // slice partial row sums of sliced row groups: [3][kSlices][space]
  T* spartD;   // m-space (dual step)
  T* spartP;   // n-space (primal step)
  // eval-step products of column-sorted blocks with the ray candidates:
  // K^T cy1, K^T cy2 (n-space) and K cx1, K cx2 (m-space)
  T* kt1;
  T* kt2;
  T* kx1;
  T* kx2;
  int64_t MS, NS;
  // control
  InstState* st;
  const int64_t* gbase;
  int* cnt;
  int* status_out;
  double* partP;
  double* partD;
  const Blk* schedP;   // one block per row group (primal / dual step kernels)
  const Blk* schedD;
  const Blk* schedPS;  // slice blocks of sliced row groups (slice kernel)
  const Blk* schedDS;
};

}  // namespace halp
