/*
 * Oracle (test infrastructure only): the FP64 acoustic recurrence of oracle/fd.py
 * written as plain C loops, for Green functions at full grid size.
 *
 *   a u^{n+1} = 2 u^n - b u^{n-1} + kappa (L4 u^n + f^n),   u^0 = u^{-1} = 0,
 *   L4 = [-1/12, 4/3, -5/2, 4/3, -1/12] / h^2 per axis, zero beyond the grid,
 *   f^n = delta_{n,0} at the receiver cell (Green function of the block Hessian
 *   equation of the paper).
 *
 * Coefficient arrays (kappa, a, b on the padded grid) come from oracle/fd.py's
 * Medium, so the set-up is shared with the NumPy oracle, not with the GPU
 * library.  Pinned against the NumPy recurrence in tests/test_oracle_fd.py.
 */
#include <stdlib.h>
#include <string.h>

#define W0 (-5.0 / 2.0)
#define W1 (4.0 / 3.0)
#define W2 (-1.0 / 12.0)

/* out: [nrec][nt][nzs][nxs] samples u^n (n = 1..nt) at padded rows zs[], cols xs[] */
int fd_green(int Z, int X, const double* kappa, const double* a, const double* b, double h,
             int nt, int nrec, const int* src_z, const int* src_x, int nzs, const int* zs, int nxs,
             const int* xs, double* out) {
  const int P = X + 4; /* row pitch with a zero ring of 2 cells */
  const size_t cells = (size_t)(Z + 4) * P;
  const double hh = h * h;
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int r = 0; r < nrec; ++r) {
    double* up = (double*)calloc(cells, sizeof(double));
    double* uc = (double*)calloc(cells, sizeof(double));
    double* un = (double*)calloc(cells, sizeof(double));
    if (!up || !uc || !un) {
      fail = 1;
      free(up);
      free(uc);
      free(un);
      continue;
    }
    for (int n = 0; n < nt; ++n) {
      for (int iz = 0; iz < Z; ++iz) {
        const double* c = uc + (size_t)(iz + 2) * P + 2;
        const double* p = up + (size_t)(iz + 2) * P + 2;
        double* o = un + (size_t)(iz + 2) * P + 2;
        const double* kz = kappa + (size_t)iz * X;
        const double* az = a + (size_t)iz * X;
        const double* bz = b + (size_t)iz * X;
        for (int ix = 0; ix < X; ++ix) {
          double lap = 2.0 * W0 * c[ix];
          lap += W1 * (c[ix - P] + c[ix + P] + c[ix - 1] + c[ix + 1]);
          lap += W2 * (c[ix - 2 * P] + c[ix + 2 * P] + c[ix - 2] + c[ix + 2]);
          lap /= hh;
          double rhs = lap;
          if (n == 0 && iz == src_z[r] && ix == src_x[r]) rhs += 1.0;
          o[ix] = (2.0 * c[ix] - bz[ix] * p[ix] + kz[ix] * rhs) / az[ix];
        }
      }
      double* t = up;
      up = uc;
      uc = un;
      un = t;
      double* dst = out + ((size_t)r * nt + n) * (size_t)nzs * nxs;
      for (int i = 0; i < nzs; ++i)
        for (int j = 0; j < nxs; ++j) dst[(size_t)i * nxs + j] = uc[(size_t)(zs[i] + 2) * P + xs[j] + 2];
    }
    free(up);
    free(uc);
    free(un);
  }
  return fail;
}
