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
 *
 * Two entry points:
 *   fd_green    all nt samples of every receiver at once (small records);
 *   fd_advance  a given number of steps from a caller-held state, so that the
 *               caller can take the DFT window by window and never hold the
 *               whole time history (full-size surveys).
 * OpenMP runs over receivers; each receiver's recurrence is sequential.
 */
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define W0 (-5.0 / 2.0)
#define W1 (4.0 / 3.0)
#define W2 (-1.0 / 12.0)

/* Rows [z0, z1) of one step n -> n+1 of one field on a plane with a zero ring
 * of 2 cells (row pitch P = X + 4).  c holds u^n; p holds u^{n-1} on entry and
 * u^{n+1} on return (each cell of p is read before it is written, and only by
 * itself). */
__attribute__((target_clones("avx512f", "avx2", "default")))
static void step_rows(int z0, int z1, int X, const double* kappa, const double* a, const double* b, double hh,
                      int n, int sz, int sx, const double* c0, double* p0) {
  const int P = X + 4;
  for (int iz = z0; iz < z1; ++iz) {
    const double* c = c0 + (size_t)(iz + 2) * P + 2;
    double* p = p0 + (size_t)(iz + 2) * P + 2;
    const double* kz = kappa + (size_t)iz * X;
    const double* az = a + (size_t)iz * X;
    const double* bz = b + (size_t)iz * X;
    const int src = (n == 0 && iz == sz) ? sx : -1;  /* column of the impulse in this row */
    for (int ix = 0; ix < X; ++ix) {
      double lap = 2.0 * W0 * c[ix];
      lap += W1 * (c[ix - P] + c[ix + P] + c[ix - 1] + c[ix + 1]);
      lap += W2 * (c[ix - 2 * P] + c[ix + 2 * P] + c[ix - 2] + c[ix + 2]);
      lap /= hh;
      const double rhs = lap + (ix == src ? 1.0 : 0.0);
      p[ix] = (2.0 * c[ix] - bz[ix] * p[ix] + kz[ix] * rhs) / az[ix];
    }
  }
}

static void record(int X, const double* u, int nzs, const int* zs, int nxs, const int* xs, double* dst) {
  const int P = X + 4;
  for (int i = 0; i < nzs; ++i)
    for (int j = 0; j < nxs; ++j) dst[(size_t)i * nxs + j] = u[(size_t)(zs[i] + 2) * P + xs[j] + 2];
}

/* out: [nrec][nt][nzs][nxs] samples u^n (n = 1..nt) at padded rows zs[], cols xs[] */
int fd_green(int Z, int X, const double* kappa, const double* a, const double* b, double h,
             int nt, int nrec, const int* src_z, const int* src_x, int nzs, const int* zs, int nxs,
             const int* xs, double* out) {
  const size_t cells = (size_t)(Z + 4) * (X + 4);
  const double hh = h * h;
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int r = 0; r < nrec; ++r) {
    double* buf = (double*)calloc(2 * cells, sizeof(double));
    if (!buf) {
      fail = 1;
      continue;
    }
    for (int n = 0; n < nt; ++n) {
      double* cur = buf + (size_t)(n & 1) * cells;        /* u^n */
      double* nxt = buf + (size_t)((n + 1) & 1) * cells;  /* u^{n-1} -> u^{n+1} */
      step_rows(0, Z, X, kappa, a, b, hh, n, src_z[r], src_x[r], cur, nxt);
      record(X, nxt, nzs, zs, nxs, xs, out + ((size_t)r * nt + n) * (size_t)nzs * nxs);
    }
    free(buf);
  }
  return fail;
}

/* Advance every receiver's field from step n0 (state holds u^{n0} in buffer
 * n0 % 2 and u^{n0-1} in the other) by nsteps steps, writing the samples
 * u^{n0+1} .. u^{n0+nsteps} to out [nsteps][nrec][nzs][nxs] (step-major, so that
 * the window's transform is one matrix product over all receivers).
 * state: [nrec][2][(Z+4)(X+4)], zero-initialised by the caller for n0 = 0;
 * its ring of 2 cells around the grid stays zero.
 * Within a step the rows are shared out over the threads and every receiver's
 * row is updated in turn (each row of every field depends only on the
 * previous two levels), so the coefficient rows are read once per step. */
void fd_advance(int Z, int X, const double* kappa, const double* a, const double* b, double h,
                int n0, int nsteps, int nrec, const int* src_z, const int* src_x, double* state,
                int nzs, const int* zs, int nxs, const int* xs, double* out) {
  const size_t cells = (size_t)(Z + 4) * (X + 4);
  const double hh = h * h;
  for (int k = 0; k < nsteps; ++k) {
    const int n = n0 + k;
#pragma omp parallel for schedule(static)
    for (int iz = 0; iz < Z; ++iz)
      for (int r = 0; r < nrec; ++r) {
        double* buf = state + (size_t)r * 2 * cells;
        step_rows(iz, iz + 1, X, kappa, a, b, hh, n, src_z[r], src_x[r], buf + (size_t)(n & 1) * cells,
                  buf + (size_t)((n + 1) & 1) * cells);
      }
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nrec; ++r)
      record(X, state + (size_t)r * 2 * cells + (size_t)((n + 1) & 1) * cells, nzs, zs, nxs, xs,
             out + ((size_t)k * nrec + r) * (size_t)nzs * nxs);
  }
}

/* Threads an OpenMP loop of this library runs on (for reporting). */
int fd_threads(void) { return omp_get_max_threads(); }
