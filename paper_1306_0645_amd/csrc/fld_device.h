// Device-side helpers shared by the HIP kernel files: tile addressing
// (XCD-aware block renumbering, range lists), periodic neighbour indices,
// deterministic block reductions, typed coefficient access and the V-cycle
// right-hand-side source.
#pragma once

#include <math.h>

#include "fld_internal.h"

namespace fld {

// ---------------------------------------------------------------------------
// tile addressing
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs.  Renumber them so
// that XCD x processes the contiguous block range [start_x, start_x + cnt_x).
__device__ __forceinline__ int xcd_block(int nb) {
  const int b = blockIdx.x;
  const int x = b & 7, q = nb >> 3, rem = nb & 7;
  return x * q + (x < rem ? x : rem) + (b >> 3);
}

__device__ __forceinline__ Tile get_tile(const TileList &L) {
  const int b = xcd_block(L.nblocks);
  int lo = 0;
  if (L.nranges > 1) {
    int hi = L.nranges - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L.ranges[2 * mid] <= b) lo = mid; else hi = mid - 1;
    }
  }
  return L.base[L.ranges[2 * lo + 1] + (b - L.ranges[2 * lo])];
}

// index of the tile inside the full table (for per-tile partial sums)
__device__ __forceinline__ int get_tile_index(const TileList &L) {
  const int b = xcd_block(L.nblocks);
  int lo = 0;
  if (L.nranges > 1) {
    int hi = L.nranges - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L.ranges[2 * mid] <= b) lo = mid; else hi = mid - 1;
    }
  }
  return L.ranges[2 * lo + 1] + (b - L.ranges[2 * lo]);
}

// Thread -> cells: a thread owns the column (i, j) of the tile and walks its
// planes (the tables give every tile cpt = 1 cell per thread along x).
struct Col {
  int i, j;
  bool on;
};

__device__ __forceinline__ Col tile_col(const Tile &t) {
  Col c;
  const int tpr = t.tx / t.cpt;
  const int lx = threadIdx.x % tpr, ly = threadIdx.x / tpr;
  c.i = t.x0 + lx * t.cpt;
  c.j = t.y0 + ly;
  c.on = ly < t.ty;
  return c;
}

// linear indices of a cell and its 6 periodic neighbours
struct Nb {
  int c, xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ Nb nbrs(int i, int j, int k, int nx, int ny, int nz) {
  Nb n;
  const int plane = nx * ny;
  const int row = k * plane + j * nx;
  n.c = row + i;
  n.xm = row + (i == 0 ? nx - 1 : i - 1);
  n.xp = row + (i == nx - 1 ? 0 : i + 1);
  n.ym = (j == 0) ? n.c + (ny - 1) * nx : n.c - nx;
  n.yp = (j == ny - 1) ? n.c - (ny - 1) * nx : n.c + nx;
  n.zm = (k == 0) ? n.c + (nz - 1) * plane : n.c - plane;
  n.zp = (k == nz - 1) ? n.c - (nz - 1) * plane : n.c + plane;
  return n;
}

// ---------------------------------------------------------------------------
// reductions (deterministic)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block; the result is valid in every thread.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += sh[i];
  return s;
}

// N sums of a tile into out[N * tile + i] (one LDS round for all of them)
template <int N>
__device__ __forceinline__ void write_sums(double *out, int tile, const double (&v)[N]) {
  constexpr int NW = kBlock / 64;
  __shared__ double sh[N][NW];
  double w[N];
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = wave_sum(v[i]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) sh[i][threadIdx.x >> 6] = w[i];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += sh[threadIdx.x][k];
    out[N * tile + threadIdx.x] = s;
  }
}

__device__ __forceinline__ void write_partials(const Tables &T, int tile,
                                               double a0, double a1) {
  __shared__ double sh[kBlock / 64];
  const double s0 = block_sum<kBlock / 64>(a0, sh);
  const double s1 = block_sum<kBlock / 64>(a1, sh);
  if (threadIdx.x == 0) {
    T.part[2 * tile] = s0;
    T.part[2 * tile + 1] = s1;
  }
}

// ---------------------------------------------------------------------------
// typed access to a level's coefficients
// ---------------------------------------------------------------------------

template <typename R>
struct Coef {
  const R *tx, *ty, *tz, *d;
};

template <typename R>
__device__ __forceinline__ Coef<R> coefs(const LevelDev &L);

template <>
__device__ __forceinline__ Coef<double> coefs<double>(const LevelDev &L) {
  return {L.Tx, L.Ty, L.Tz, L.diag};
}

template <>
__device__ __forceinline__ Coef<float> coefs<float>(const LevelDev &L) {
  return {L.Tx32, L.Ty32, L.Tz32, L.diag32};
}

// sum over the 6 neighbours of T_face * u_neighbour
template <typename R, typename U>
__device__ __forceinline__ R offsum(const Coef<R> &C, const Nb &n, const U &u) {
  return C.tx[n.c] * u(n.xp) + C.tx[n.xm] * u(n.xm) + C.ty[n.c] * u(n.yp) +
         C.ty[n.ym] * u(n.ym) + C.tz[n.c] * u(n.zp) + C.tz[n.zm] * u(n.zm);
}

__device__ __forceinline__ double recip(double d) { return 1.0 / d; }
__device__ __forceinline__ float recip(float d) {
  return __builtin_amdgcn_rcpf(d);  // ~1 ulp: ample for a preconditioner
}

// ---------------------------------------------------------------------------
// V-cycle right-hand side.  R = level precision, L0 = finest level (the
// right-hand side is the FP64 Krylov residual scaled by 1/s).
// ---------------------------------------------------------------------------

template <typename R, bool L0>
struct FSrc {
  const R *f;
  const double *r;
  double inv_s;
  __device__ __forceinline__ R operator()(int c) const {
    if constexpr (L0) return (R)(r[c] * inv_s);
    else return f[c];
  }
};

// Assembly and warm start of a problem are due: for the host-driven step
// whenever the problem takes part (the host launches them when due); for
// device-controlled stepping when its controller asked for them.
__device__ __forceinline__ bool asm_due(const Scal &sc) {
  return sc.live && (!sc.ctl || sc.stage == 1);
}
__device__ __forceinline__ bool warm_due(const Scal &sc) {
  return sc.live && (!sc.ctl || sc.stage == 2);
}

// the current residual buffer, and the other one
__device__ __forceinline__ double *rcur(const ProbDev &P, const Scal &sc) {
  return sc.rbuf ? P.r2 : P.r;
}
__device__ __forceinline__ double *rnext(const ProbDev &P, const Scal &sc) {
  return sc.rbuf ? P.r : P.r2;
}

template <typename R, bool L0>
__device__ __forceinline__ FSrc<R, L0> fsrc(const LevelDev &L, const ProbDev &P,
                                             const Scal &sc) {
  FSrc<R, L0> s;
  s.f = (const R *)L.f;
  s.r = rcur(P, sc);
  s.inv_s = sc.inv_s;
  return s;
}

// Coarse-grid correction at fine cell (gx, gy, gz) of a level whose coarse
// level has extents (cnx, cny, cnz) = half the fine ones.
//  trilinear = false: piecewise constant, e(parent)
//  trilinear = true:  cell-centred trilinear interpolation from the 8 nearest
//                     coarse cells, weights 3/4 (own parent) and 1/4 (the
//                     neighbour on the fine cell's side) per direction
template <typename R>
__device__ __forceinline__ R coarse_corr(const R *e, int gx, int gy, int gz,
                                         int cnx, int cny, int cnz,
                                         bool trilinear) {
  const int I = gx >> 1, J = gy >> 1, K = gz >> 1;
  if (!trilinear) return e[(K * cny + J) * cnx + I];
  const int I2 = (gx & 1) ? (I + 1 == cnx ? 0 : I + 1) : (I == 0 ? cnx - 1 : I - 1);
  const int J2 = (gy & 1) ? (J + 1 == cny ? 0 : J + 1) : (J == 0 ? cny - 1 : J - 1);
  const int K2 = (gz & 1) ? (K + 1 == cnz ? 0 : K + 1) : (K == 0 ? cnz - 1 : K - 1);
  const R a = (R)0.75, b = (R)0.25;
  const int r00 = (K * cny + J) * cnx, r01 = (K * cny + J2) * cnx;
  const int r10 = (K2 * cny + J) * cnx, r11 = (K2 * cny + J2) * cnx;
  const R zK = a * (a * e[r00 + I] + b * e[r00 + I2]) +
               b * (a * e[r01 + I] + b * e[r01 + I2]);
  const R zK2 = a * (a * e[r10 + I] + b * e[r10 + I2]) +
                b * (a * e[r11 + I] + b * e[r11 + I2]);
  return a * zK + b * zK2;
}

}  // namespace fld
