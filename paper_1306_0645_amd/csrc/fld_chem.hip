// Isothermal hydrogen chemistry coupled to the radiation step by operator
// splitting: the loosely coupled per-cell update of Sec. 3.3 for the
// hydrogen-only gas of Test 1 (Sec. 4.1.1).  Entry points in
// include/fld_chem.h.
//
// Both kernels are streaming: k_chem_h reads E, n_H and x and writes x and
// kappa (40 bytes per cell, no reuse), so it is bound by HBM bandwidth and
// runs one cell per lane with a grid-stride loop.  k_ion_sum is a
// diagnostic reduction run once per output time; it uses a single block so
// that the summation order, and hence the result, is fixed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fld.h"
#include "fld_chem.h"
#include "fld_internal.h"

namespace fld {
namespace {

constexpr int kChemBlock = 256;
constexpr int kChemMaxBlocks = 16384;
constexpr int kSumBlock = 1024;

__global__ __launch_bounds__(kChemBlock) void k_chem_h(
    const double *__restrict__ E, const double *__restrict__ nh,
    double *__restrict__ x, double *__restrict__ kappa, int64_t n, double h,
    int substeps, double c, double sigma, double hnu, double alpha,
    double inv_a3) {
  const double c_sigma = c * sigma;
  for (int64_t i = (int64_t)blockIdx.x * kChemBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kChemBlock) {
    // proper densities from the comoving fields
    const double np = nh[i] * inv_a3;
    const double gamma = c_sigma * (E[i] * inv_a3) / hnu;  // photo-ionization
    const double an = alpha * np;
    double xv = x[i];
    for (int s = 0; s < substeps; ++s)
      xv = (xv + h * gamma) / (1.0 + h * (gamma + an * xv));
    x[i] = xv;
    kappa[i] = sigma * np * (1.0 - xv);
  }
}

__global__ __launch_bounds__(kSumBlock) void k_ion_sum(const double *__restrict__ x,
                                                      int64_t n,
                                                      double *__restrict__ out) {
  __shared__ double part[kSumBlock];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kSumBlock) acc += x[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kSumBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

bool extents_ok(const fld_grid *g, int64_t *n) {
  if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return false;
  const int64_t m = (int64_t)g->nx * g->ny * g->nz;
  if (m >= (int64_t(1) << 31)) return false;
  *n = m;
  return true;
}

bool disjoint(const void *a, int64_t na, const void *b, int64_t nb) {
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa + na <= pb || pb + nb <= pa;
}

}  // namespace
}  // namespace fld

extern "C" {

void fld_chem_default_params(fld_chem_params *p) {
  if (!p) return;
  p->c = 2.99792458e10;
  p->sigma = 6.3e-18;
  p->hnu = 13.6 * 1.602176634e-12;
  p->alpha_b = 2.59e-13;
  p->substeps = 1;
  p->reserved = 0;
}

fld_status fld_chem_h_update(const fld_grid *grid, const fld_chem_params *p,
                             void *hip_stream, const double *E,
                             const double *n_h, double *x, double *kappa,
                             double dt, double a) {
  using namespace fld;
  int64_t n = 0;
  if (!extents_ok(grid, &n) || !p || !E || !n_h || !x || !kappa)
    return FLD_EINVAL;
  if (!(std::isfinite(p->c) && p->c > 0.0) ||
      !(std::isfinite(p->sigma) && p->sigma >= 0.0) ||
      !(std::isfinite(p->hnu) && p->hnu > 0.0) ||
      !(std::isfinite(p->alpha_b) && p->alpha_b >= 0.0) || p->substeps < 1 ||
      p->substeps > 1000000 || p->reserved != 0)
    return FLD_EINVAL;
  if (!(std::isfinite(dt) && dt >= 0.0)) return FLD_EINVAL;
  if (!(std::isfinite(a) && a > 0.0)) return FLD_EINVAL;
  const int64_t bytes = n * (int64_t)sizeof(double);
  if (!disjoint(x, bytes, kappa, bytes) || !disjoint(x, bytes, E, bytes) ||
      !disjoint(x, bytes, n_h, bytes) || !disjoint(kappa, bytes, E, bytes) ||
      !disjoint(kappa, bytes, n_h, bytes))
    return FLD_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t want = (n + kChemBlock - 1) / kChemBlock;
  const int blocks = (int)(want < kChemMaxBlocks ? want : kChemMaxBlocks);
  FLD_LAUNCH(K_CHEM_H, k_chem_h, blocks, kChemBlock, s, E, n_h, x, kappa, n,
             dt / (double)p->substeps, p->substeps, p->c, p->sigma, p->hnu,
             p->alpha_b, 1.0 / (a * a * a));
  return hipGetLastError() == hipSuccess ? FLD_OK : FLD_EDEVICE;
}

fld_status fld_chem_ionized_sum(const fld_grid *grid, void *hip_stream,
                                const double *x, double *sum_out) {
  using namespace fld;
  int64_t n = 0;
  if (!extents_ok(grid, &n) || !x || !sum_out) return FLD_EINVAL;
  if (!disjoint(x, n * (int64_t)sizeof(double), sum_out, sizeof(double)))
    return FLD_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  FLD_LAUNCH(K_ION_SUM, k_ion_sum, 1, kSumBlock, s, x, n, sum_out);
  return hipGetLastError() == hipSuccess ? FLD_OK : FLD_EDEVICE;
}

}  // extern "C"
