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

/* The complex banded matrix the plane Poiseuille stability solver factors (sps_poiseuille_solve)
 * for streamwise wavenumber alpha, Reynolds number re and shift sigma = sig_re + i sig_im:
 *     B = P_r (sigma M + L) R P_c,
 * the operators of the Orr-Sommerfeld problem in primitive variables (paper, Results:
 * Parametric sensitivity and numerical continuation; the discretization is that of the 2D
 * problem), rows permuted to the interleaved order rowmap (band row i <- equation slot), columns
 * to colmap (band column j -> unknown slot), R recombining X[s] = y[s] + rho[s] * y[s + 2].
 * Fills S = 3 nz + 5, kl, ku and, when non-NULL, band[S][kl + ku + 1] complex (entry (i, j) at
 * [i][j - i + kl], (re, im) pairs), rowmap[S], colmap[S], rho[S].  Call first with NULL arrays to
 * learn S, kl and ku.  8 <= nz <= 256.  Returns SPS_OK or an error. */
int sps_poiseuille_host_band(int nz, double alpha, double re, double sig_re, double sig_im, int *S, int *kl,
                             int *ku, double *band, int *rowmap, int *colmap, double *rho);

#ifdef __cplusplus
}
#endif

#endif /* SPS_HOST_H */
