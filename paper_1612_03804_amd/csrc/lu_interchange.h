// Row interchanges of one panel of the blocked LU factorisation with partial
// pivoting (the determinant of the final step of a weight evaluation), as one
// permutation of the rows they touch.
//
// The panel covers columns j0 .. j0+nbw-1; column j0+c swapped row j0+c with
// row ipiv[j0+c] (applied in order c = 0, 1, ...).  Partial pivoting only ever
// picks a row at or below the diagonal, so a valid pivot lies in
// [j0 + c, N).  On return rows srow[0..ns) receive the entries of rows
// ssrc[0..ns): the panel's own rows come first (srow[k] = j0 + k for k < nbw),
// then every row below the panel that an interchange touched, at most nbw of
// them, so srow and ssrc need 2*nbw entries.
//
// A pivot outside [j0 + c, N) (never produced by the factorisation; it would
// index memory outside the matrix) is replaced by j0 + c (no interchange),
// written back to ipiv so that later users of the pivots see the same rows,
// and reported by a return value of 1.  Every row index in srow and ssrc is
// then in [j0, N).
//
// Plain integer code with no HIP intrinsics: the same function runs on the
// device inside the LU kernel and on the host in a CPU check of the guard.
#pragma once

#include <cstdint>

namespace slq {

__host__ __device__ inline int lu_panel_permutation(int N, int j0, int nbw, uint16_t* ipiv, int* srow, int* ssrc,
                                                    int* ns_out) {
  int bad = 0;
  int ns = nbw;
  for (int k = 0; k < nbw; ++k) srow[k] = ssrc[k] = j0 + k;
  for (int c = 0; c < nbw; ++c) {
    int pr = ipiv[j0 + c];
    if (pr < j0 + c || pr >= N) {
      pr = j0 + c;
      ipiv[j0 + c] = (uint16_t)pr;
      bad = 1;
    }
    int k2 = -1;
    if (pr < j0 + nbw) {
      k2 = pr - j0;
    } else {
      for (int k = nbw; k < ns; ++k)
        if (srow[k] == pr) k2 = k;
      if (k2 < 0) {
        k2 = ns++;
        srow[k2] = ssrc[k2] = pr;
      }
    }
    const int t = ssrc[c];
    ssrc[c] = ssrc[k2];
    ssrc[k2] = t;
  }
  *ns_out = ns;
  return bad;
}

}  // namespace slq
