/*
 * sps_host.h — host-only introspection of the library's operator assembly.
 *
 * Needs no GPU.  It exposes the real banded systems the library factors for the 2D
 * Rayleigh-Benard problem, so the assembly of M and L (paper, Supplementary: Initial
 * value problems; Sparse spectral methods: banded operators and tau rows) can be
 * checked on the CPU.  For wavenumber k the library factors
 *     B_k = a * BM_k + b * BL_k,   BM_k = D_r M_k R D_c,   BL_k = D_r L_k R D_c,
 * permuted to the interleaved order rowmap/colmap, where D_r multiplies the rows whose
 * slot has rowph = 1 by -i, D_c the columns with colph = 1 by +i, and R recombines
 * coefficients: X[s] = y[s] + rho[s] * y[s + 2].
 */
#ifndef SPS_HOST_H
#define SPS_HOST_H

#include "sps.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Fills kl, ku (band widths) and, when the pointers are non-NULL, the row bands
 * BM, BL of shape [K][S][kl + ku + 1] (entry (i, j) of solver order at
 * [k][i][j - i + kl]), rowmap[S] (solver row i <- equation slot), colmap[S] (solver
 * column i -> unknown slot), rowph[S], colph[S] and rho[S].  Call first with NULL
 * arrays to learn kl and ku.  K = nx / 2, S = 4 nz + 7.  Returns SPS_OK or an error. */
int sps_rbc_host_bands(const sps_desc *desc, int *kl, int *ku, double *BM, double *BL, int *rowmap,
                       int *colmap, signed char *rowph, signed char *colph, double *rho);

#ifdef __cplusplus
}
#endif

#endif /* SPS_HOST_H */
