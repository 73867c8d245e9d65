/*
 * fld_chem.h -- C-ABI of the isothermal hydrogen chemistry that couples to
 * the FLD radiation step by operator splitting (Norman et al.,
 * arXiv:1306.0645, Sec. 3.3 and Sec. 3.4; Test 1 of Sec. 4.1.1).
 *
 * The operation (the loosely coupled chemistry solver of Sec. 3.3, for pure
 * hydrogen at fixed temperature): with x = n_HII / n_H the ionized fraction,
 * the species equation of eq. "heat_chem" reduces to
 *
 *     dx/dt = Gamma (1 - x) - alpha_B n_H x^2,   Gamma = c sigma E / (h nu),
 *
 * Gamma being the photo-ionization rate of monochromatic radiation at the
 * ionization threshold with energy density E.  One linearly implicit
 * backward-Euler update per sub-step of length h takes x at the new time
 * where it enters linearly and the electron density of the recombination
 * term at the old time:
 *
 *     x <- (x + h Gamma) / (1 + h (Gamma + alpha_B n_H x)),
 *
 * after which the opacity for the next radiation step is kappa = sigma n_H
 * (1 - x).  E is the field at the end of the radiation step and is held
 * fixed over the chemistry step (Sec. 3.4 forms the rates from the new E
 * before the chemistry runs).
 *
 * Conventions (as in fld.h): field pointers are DEVICE pointers to FP64
 * arrays of nx*ny*nz cells in C order, owned by the caller; work is enqueued
 * on the given hipStream_t (NULL = the default stream) and no call
 * synchronises it or allocates device memory.  Arguments are checked before
 * any launch: FLD_EINVAL for a bad argument (nothing is written),
 * FLD_EDEVICE for a HIP launch error.  The status values are those of
 * fld.h.
 */
#ifndef FLD_CHEM_H_
#define FLD_CHEM_H_

#include <stdint.h>

#include "fld.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fld_chem_params {
  double c;          /* speed of light, > 0, in the units of the grid       */
  double sigma;      /* HI photo-ionization cross-section at h nu, >= 0      */
  double hnu;        /* photon energy, > 0, in the energy unit of E          */
  double alpha_b;    /* case-B recombination coefficient, >= 0               */
  int32_t substeps;  /* equal sub-steps per call, 1 .. 1000000               */
  int32_t reserved;  /* must be 0                                            */
} fld_chem_params;

/* Test-1 constants in CGS (Sec. 4.1.1): sigma = 6.3e-18 cm^2 at 13.6 eV,
 * h nu = 13.6 eV, alpha_B = 2.59e-13 cm^3/s (case B at 1e4 K), c in cm/s,
 * one sub-step. */
void fld_chem_default_params(fld_chem_params *p);

/* One chemistry step of length dt >= 0 over every cell of the grid (only
 * its extents are used; each must be >= 1, the product < 2^31):
 *   E      in : comoving radiation energy density after the radiation step
 *   n_h    in : comoving hydrogen number density
 *   x      in/out : ionized fraction, in [0, 1]
 *   kappa  out : proper opacity sigma n_H (1 - x) / a^3 with the new x
 *   a      : expansion factor, > 0 (comoving = proper * a^3, Sec. 2); the
 *            rates use E / a^3 and n_h / a^3; a = 1 for a static problem
 * dt = 0 leaves x unchanged and only recomputes kappa.  x and kappa must
 * not overlap each other or the inputs. */
fld_status fld_chem_h_update(const fld_grid *grid, const fld_chem_params *p,
                             void *hip_stream, const double *E,
                             const double *n_h, double *x, double *kappa,
                             double dt, double a);

/* sum_out[0] = sum of x over all cells (device pointer, one double), summed
 * in a fixed order so that the result is reproducible.  With V_cell the
 * cell volume, sum * V_cell is the ionized volume and
 * (3 sum V_cell / (4 pi))^(1/3) the ionization-front radius of a single
 * spherical region. */
fld_status fld_chem_ionized_sum(const fld_grid *grid, void *hip_stream,
                                const double *x, double *sum_out);

#ifdef __cplusplus
}
#endif

#endif /* FLD_CHEM_H_ */
