// HIP kernels (gfx950 / CDNA4) of the implicit grey FLD step.
//
// What is computed (Norman et al., arXiv:1306.0645):
//  - assembly: the flux limiter on every face from E^n (Sec. 2) and the
//    theta-method system (I - theta dt L) dE = dt (L E^n + eta) in
//    residual-correction form (Sec. 3.3);
//  - the multigrid V-cycle preconditioner with red/black Gauss-Seidel
//    smoothing (Table 1);
//  - the preconditioned conjugate-gradient recurrences (Table 1).
//
// All of this is memory-bound stencil and vector work (well under 1 flop per
// byte), so no kernel uses MFMA.  Every kernel processes a list of tiles;
// one 256-thread block (4 wave64) handles one tile: each thread owns one
// (x, y) column of the tile and walks its tz planes, so x-consecutive lanes
// read x-consecutive cells (coalesced).  Blocks are remapped so that each of
// the 8 XCDs gets a contiguous run of tiles and neighbouring tiles share an L2.
// Reductions are deterministic: a fixed wave64 butterfly, a fixed LDS order,
// one partial per tile, then a per-problem finalize kernel that sums the
// partials in tile order.

#include "fld_device.h"
#include "fld_profile.h"

#include <math.h>

#include <type_traits>
#include <vector>

namespace fld {

// ---------------------------------------------------------------------------
// assembly (Sec. 2 limiter, Sec. 3.3 theta-method)
// ---------------------------------------------------------------------------

// D on the face between cells 1 and 2: arithmetic-mean E, harmonic-mean
// kappa, R from the face-normal difference (floored at R_min, and R_min when
// the face mean is not positive), capped at D_max.  Comparisons are written
// so that NaN inputs propagate.
__device__ __forceinline__ double face_D(double e1, double e2, double k1,
                                         double k2, double ih, double c,
                                         double dmax, double rmin) {
  const double ebar = 0.5 * (e1 + e2);
  const double ks = k1 + k2;
  const double kb = (ks != 0.0) ? 2.0 * k1 * k2 / ks : 0.0;
  double R = (ebar > 0.0) ? fabs(e2 - e1) * ih / ebar : rmin;
  R = (R < rmin) ? rmin : R;
  const double D = c / sqrt(9.0 * kb * kb + R * R);
  return (D > dmax) ? dmax : D;
}

// One thread per (x, y) column of the tile, walking z: E and kappa of the
// column at k-1, k, k+1 stay in registers and the -z face of plane k is the +z
// face computed at plane k-1, so each cell evaluates 5 limiters, not 6.
__global__ __launch_bounds__(kBlock) void k_assemble(Tables T, TileList L0,
                                                     double c, double theta,
                                                     double dmax, double rmin,
                                                     int mixed) {
  const int tid = get_tile_index(L0);
  const Tile t = L0.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!asm_due(sc)) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const StepDev S = T.sd[t.prob];
  const Col col = tile_col(t);
  const double tdt = theta * S.dt;
  const double ix2 = S.idx * S.idx, iy2 = S.idy * S.idy, iz2 = S.idz * S.idz;
  const double *__restrict__ E = S.E;
  const double *__restrict__ K = S.kappa;
  const double *__restrict__ eta = S.eta;
  double *__restrict__ Tx = L.Tx;
  double *__restrict__ Ty = L.Ty;
  double *__restrict__ Tz = L.Tz;
  double *__restrict__ Dg = L.diag;
  double *__restrict__ bv = P.b;
  double *__restrict__ rv = rcur(P, sc);
  double *__restrict__ xv = P.x;
  // warm start from two history buffers that nothing writes here, so their
  // values at a neighbour are read on the fly (the thread holds all 6 faces):
  // extrapolated guess x0 = w1 dE(n) + w2 dE(n-1): r = b - A x0 comes out of
  // this pass; Galerkin guess: this pass sums (h_i, A h_j) and (h_i, b) for
  // the new operator, and k_warm_x forms x0 and r once c is known
  const bool warm = S.warm > 0.0, gal = S.warm > 1.0;
  const double w1 = S.w1, w2 = S.w2;
  const double *__restrict__ h1 = S.h1;
  const double *__restrict__ h2 = S.h2;
  auto guess = [&](int g) { return h2 ? w1 * h1[g] + w2 * h2[g] : w1 * h1[g]; };
  double bb = 0.0, rr = 0.0, g11 = 0.0, g12 = 0.0, g22 = 0.0, gb1 = 0.0,
         gb2 = 0.0;
  if (col.on) {
    const int nx = L.nx, ny = L.ny, nz = L.nz, plane = nx * ny;
    const int i = col.i, j = col.j;
    const int dxm = (i == 0) ? nx - 1 : -1, dxp = (i == nx - 1) ? 1 - nx : 1;
    const int dym = (j == 0) ? (ny - 1) * nx : -nx;
    const int dyp = (j == ny - 1) ? -(ny - 1) * nx : nx;
    int cc = t.z0 * plane + j * nx + i;
    const int cm = (t.z0 == 0) ? cc + (nz - 1) * plane : cc - plane;
    double Em = E[cm], Km = K[cm];
    double Ec = E[cc], Kc = K[cc];
    double Dzm = face_D(Em, Ec, Km, Kc, S.idz, c, dmax, rmin);
    double gm = 0.0, gc = 0.0;  // guess (Galerkin: dE(n)) at planes k - 1, k
    double um = 0.0, uc = 0.0;  // Galerkin: dE(n-1) at planes k - 1, k
    if (gal) {
      gm = h1[cm];
      gc = h1[cc];
      if (h2) {
        um = h2[cm];
        uc = h2[cc];
      }
    } else if (warm) {
      gm = guess(cm);
      gc = guess(cc);
    }
    for (int k = t.z0; k < t.z0 + t.tz; ++k) {
      const int cp = (k == nz - 1) ? cc - (nz - 1) * plane : cc + plane;
      const double Ep = E[cp], Kp = K[cp];
      const double Exp = E[cc + dxp], Exm = E[cc + dxm];
      const double Eyp = E[cc + dyp], Eym = E[cc + dym];
      const double Dxp = face_D(Ec, Exp, Kc, K[cc + dxp], S.idx, c, dmax, rmin);
      const double Dxm = face_D(Exm, Ec, K[cc + dxm], Kc, S.idx, c, dmax, rmin);
      const double Dyp = face_D(Ec, Eyp, Kc, K[cc + dyp], S.idy, c, dmax, rmin);
      const double Dym = face_D(Eym, Ec, K[cc + dym], Kc, S.idy, c, dmax, rmin);
      const double Dzp = face_D(Ec, Ep, Kc, Kp, S.idz, c, dmax, rmin);
      const double mu = S.adot_a + c * Kc;
      const double faces =
          (Dxp + Dxm) * ix2 + (Dyp + Dym) * iy2 + (Dzp + Dzm) * iz2;
      const double diag = 1.0 + tdt * (mu + faces);
      const double LE = (Dxp * (Exp - Ec) - Dxm * (Ec - Exm)) * ix2 +
                        (Dyp * (Eyp - Ec) - Dym * (Ec - Eym)) * iy2 +
                        (Dzp * (Ep - Ec) - Dzm * (Ec - Em)) * iz2 - mu * Ec;
      const double b = S.dt * (LE + eta[cc]);
      const double tx = tdt * Dxp * ix2, ty = tdt * Dyp * iy2, tz = tdt * Dzp * iz2;
      Tx[cc] = tx;
      Ty[cc] = ty;
      Tz[cc] = tz;
      Dg[cc] = diag;
      if (mixed) {
        L.Tx32[cc] = (float)tx;
        L.Ty32[cc] = (float)ty;
        L.Tz32[cc] = (float)tz;
        L.diag32[cc] = (float)diag;
      }
      bv[cc] = b;
      bb += b * b;
      if (gal) {
        // A h at the cell for h = dE(n) and dE(n-1); x and r are k_warm_x's
        const double txm = tdt * Dxm * ix2, tym = tdt * Dym * iy2,
                     tzm = tdt * Dzm * iz2;
        const double gp = h1[cp];
        const double a1 = diag * gc - (tx * h1[cc + dxp] + txm * h1[cc + dxm] +
                                       ty * h1[cc + dyp] + tym * h1[cc + dym] +
                                       tz * gp + tzm * gm);
        g11 += gc * a1;
        gb1 += gc * b;
        gm = gc;
        gc = gp;
        if (h2) {
          const double up = h2[cp];
          const double a2 = diag * uc - (tx * h2[cc + dxp] + txm * h2[cc + dxm] +
                                         ty * h2[cc + dyp] + tym * h2[cc + dym] +
                                         tz * up + tzm * um);
          g12 += uc * a1;  // (dE(n-1), A dE(n)): A is symmetric
          g22 += uc * a2;
          gb2 += uc * b;
          um = uc;
          uc = up;
        }
      } else if (warm) {
        const double gp = guess(cp);
        const double txm = tdt * Dxm * ix2, tym = tdt * Dym * iy2,
                     tzm = tdt * Dzm * iz2;
        const double off = tx * guess(cc + dxp) + txm * guess(cc + dxm) +
                           ty * guess(cc + dyp) + tym * guess(cc + dym) +
                           tz * gp + tzm * gm;
        const double r = b - (diag * gc - off);
        xv[cc] = gc;
        rv[cc] = r;
        rr += r * r;
        gm = gc;
        gc = gp;
      } else {
        xv[cc] = 0.0;
        rv[cc] = b;
      }
      Em = Ec;
      Km = Kc;
      Ec = Ep;
      Kc = Kp;
      Dzm = Dzp;
      cc = cp;
    }
  }
  const double sums[kAsmSums] = {bb, rr, g11, g12, g22, gb1, gb2};
  write_sums(T.gpart, tid, sums);
}

// Coarse operator of level lc from level lc-1 (one thread per coarse cell).
// The coarse "mass" (diagonal minus faces) is the sum of the 8 children's.
// Coarse faces, op = 0: coarse_scale times the sum of the 4 fine faces they
// cover.  op = 1: each of the 4 fine rows that cross the coarse face joins
// the two coarse centres through three fine faces in series, half of the
// inner face of each coarse cell and the whole face between them, so the row
// conducts 1 / (0.5 / T_in + 1 / T_mid + 0.5 / T_in'); the coarse face is
// 2 coarse_scale times the sum over the rows (for a uniform medium both rules
// give coarse_scale times the 4 fine faces).  Either way a coarse face is the
// same sum of the same terms for both cells it joins, so the coarse operator
// is exactly symmetric.
__device__ __forceinline__ double series3(double a, double b, double c) {
  return 1.0 / (0.5 / a + 1.0 / b + 0.5 / c);
}

__global__ __launch_bounds__(kBlock) void k_coarsen(Tables T, TileList LC,
                                                    int lc, double scale,
                                                    int mixed, int op) {
  const Tile t = get_tile(LC);
  const Scal &sc = T.sc[t.prob];
  if (!asm_due(sc)) return;
  const LevelDev F = T.lv[(lc - 1) * T.nprob + t.prob];
  const LevelDev C = T.lv[lc * T.nprob + t.prob];
  const Col col = tile_col(t);
  if (!col.on) return;
  const int fx = F.nx, fy = F.ny, fz = F.nz;
  for (int K = t.z0; K < t.z0 + t.tz; ++K) {
    for (int e = 0; e < t.cpt; ++e) {
      const int I = col.i + e, J = col.j;
      double mass = 0.0, txp = 0.0, txm = 0.0, typ = 0.0, tym = 0.0,
             tzp = 0.0, tzm = 0.0;
#pragma unroll
      for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            const Nb n = nbrs(2 * I + cx, 2 * J + cy, 2 * K + cz, fx, fy, fz);
            const double fxp = F.Tx[n.c], fxm = F.Tx[n.xm];
            const double fyp = F.Ty[n.c], fym = F.Ty[n.ym];
            const double fzp = F.Tz[n.c], fzm = F.Tz[n.zm];
            mass += F.diag[n.c] - (fxp + fxm + fyp + fym + fzp + fzm);
            if (op == 0) {
              if (cx == 1) txp += fxp; else txm += fxm;
              if (cy == 1) typ += fyp; else tym += fym;
              if (cz == 1) tzp += fzp; else tzm += fzm;
            } else {
              // a child on the + side: its -face (inner), its +face (the
              // coarse face) and the neighbour's +face; on the - side: the
              // -face of the cell two below, its own -face and +face
              if (cx == 1) {
                txp += series3(fxm, fxp, F.Tx[n.xp]);
              } else {
                const int i2 = 2 * I >= 2 ? 2 * I - 2 : 2 * I - 2 + fx;
                txm += series3(F.Tx[n.c - 2 * I + i2], fxm, fxp);
              }
              if (cy == 1) {
                typ += series3(fym, fyp, F.Ty[n.yp]);
              } else {
                const int j2 = 2 * J >= 2 ? 2 * J - 2 : 2 * J - 2 + fy;
                tym += series3(F.Ty[n.c + (j2 - 2 * J) * fx], fym, fyp);
              }
              if (cz == 1) {
                tzp += series3(fzm, fzp, F.Tz[n.zp]);
              } else {
                const int k2 = 2 * K >= 2 ? 2 * K - 2 : 2 * K - 2 + fz;
                tzm += series3(F.Tz[n.c + (long long)(k2 - 2 * K) * fx * fy], fzm, fzp);
              }
            }
          }
      const double s2 = op == 0 ? scale : 2.0 * scale;
      txp *= s2; txm *= s2; typ *= s2; tym *= s2; tzp *= s2; tzm *= s2;
      const double diag = mass + txp + txm + typ + tym + tzp + tzm;
      const int o = (K * C.ny + J) * C.nx + I;
      C.Tx[o] = txp;
      C.Ty[o] = typ;
      C.Tz[o] = tzp;
      C.diag[o] = diag;
      if (mixed) {
        C.Tx32[o] = (float)txp;
        C.Ty32[o] = (float)typ;
        C.Tz32[o] = (float)tzp;
        C.diag32[o] = (float)diag;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// V-cycle kernels (any sweep count; one cell per lane, colour test per cell)
// ---------------------------------------------------------------------------

// First pre-smoothing sweep from x = 0: red cells x = f/d, then black cells
// from those red values (computed on the fly, so one pass suffices).
template <typename R, bool L0>
__global__ __launch_bounds__(kBlock) void k_pre0(Tables T, TileList TL, int l) {
  const Tile t = get_tile(TL);
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[l * T.nprob + t.prob];
  const ProbDev P = T.pd[t.prob];
  const Coef<R> C = coefs<R>(L);
  const auto f = fsrc<R, L0>(L, P, sc);
  R *x = (R *)L.x;
  const Col col = tile_col(t);
  if (!col.on) return;
  for (int k = t.z0; k < t.z0 + t.tz; ++k) {
    const Nb n = nbrs(col.i, col.j, k, L.nx, L.ny, L.nz);
    R v;
    if (((col.i + col.j + k) & 1) == 0) {
      v = f(n.c) * recip(C.d[n.c]);
    } else {
      auto red = [&](int q) { return f(q) * recip(C.d[q]); };
      v = (f(n.c) + offsum(C, n, red)) * recip(C.d[n.c]);
    }
    x[n.c] = v;
  }
}

// One half-sweep of red/black Gauss-Seidel on the cells of one colour
// (colour 0 = red = even i+j+k), in place.
template <typename R, bool L0>
__global__ __launch_bounds__(kBlock) void k_half(Tables T, TileList TL, int l,
                                                 int colour) {
  const Tile t = get_tile(TL);
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[l * T.nprob + t.prob];
  const ProbDev P = T.pd[t.prob];
  const Coef<R> C = coefs<R>(L);
  const auto f = fsrc<R, L0>(L, P, sc);
  R *x = (R *)L.x;
  const Col col = tile_col(t);
  if (!col.on) return;
  auto xv = [&](int q) { return x[q]; };
  for (int k = t.z0; k < t.z0 + t.tz; ++k) {
    if (((col.i + col.j + k) & 1) != colour) continue;
    const Nb n = nbrs(col.i, col.j, k, L.nx, L.ny, L.nz);
    x[n.c] = (f(n.c) + offsum(C, n, xv)) * recip(C.d[n.c]);
  }
}

// Black half-sweep fused with the coarse-grid correction: the red
// neighbours are read as x + e(parent).  (The black cells' own corrected
// value is overwritten by the sweep, so it is never formed.)
template <typename R, bool L0>
__global__ __launch_bounds__(kBlock) void k_prolong_black(Tables T, TileList TL,
                                                          int l, int trilinear) {
  const Tile t = get_tile(TL);
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[l * T.nprob + t.prob];
  const ProbDev P = T.pd[t.prob];
  const bool has_coarse = l + 1 < P.levels;
  const LevelDev Cl = T.lv[(has_coarse ? l + 1 : l) * T.nprob + t.prob];
  const Coef<R> C = coefs<R>(L);
  const auto f = fsrc<R, L0>(L, P, sc);
  R *x = (R *)L.x;
  const R *e = (const R *)Cl.x;
  const int cnx = Cl.nx, cny = Cl.ny, cnz = Cl.nz;
  const bool tri = trilinear != 0;
  const Col col = tile_col(t);
  if (!col.on) return;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  for (int k = t.z0; k < t.z0 + t.tz; ++k) {
    if (((col.i + col.j + k) & 1) != 1) continue;
    const int i = col.i, j = col.j;
    const Nb n = nbrs(i, j, k, nx, ny, nz);
    R s;
    if (has_coarse) {
      const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
      const int jm = j == 0 ? ny - 1 : j - 1, jp = j == ny - 1 ? 0 : j + 1;
      const int km = k == 0 ? nz - 1 : k - 1, kp = k == nz - 1 ? 0 : k + 1;
      auto par = [&](int a, int b2, int c2) {
        return coarse_corr(e, a, b2, c2, cnx, cny, cnz, tri);
      };
      s = C.tx[n.c] * (x[n.xp] + par(ip, j, k)) +
          C.tx[n.xm] * (x[n.xm] + par(im, j, k)) +
          C.ty[n.c] * (x[n.yp] + par(i, jp, k)) +
          C.ty[n.ym] * (x[n.ym] + par(i, jm, k)) +
          C.tz[n.c] * (x[n.zp] + par(i, j, kp)) +
          C.tz[n.zm] * (x[n.zm] + par(i, j, km));
    } else {
      auto xv = [&](int q) { return x[q]; };
      s = offsum(C, n, xv);
    }
    x[n.c] = (f(n.c) + s) * recip(C.d[n.c]);
  }
}

// Last red half-sweep on the finest level, producing z = s * x (FP64 form: in
// place; mixed form: x itself as z32, z = zscale z32) and the partial sums r.z
// and (flexible PCG, except at a (re)start) r.z_old.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_half_out(Tables T, TileList TL,
                                                     int flexible) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const Coef<R> C = coefs<R>(L);
  const auto f = fsrc<R, true>(L, P, sc);
  R *x = (R *)L.x;
  const double s = sc.s, zs_old = sc.zscale;
  const bool rd_old = flexible && !sc.restart;
  const Col col = tile_col(t);
  double rz = 0.0, rzo = 0.0;
  if (col.on) {
    auto xv = [&](int q) { return x[q]; };
    for (int k = t.z0; k < t.z0 + t.tz; ++k) {
      const Nb n = nbrs(col.i, col.j, k, L.nx, L.ny, L.nz);
      R v;
      const bool red = ((col.i + col.j + k) & 1) == 0;
      if (red) v = (f(n.c) + offsum(C, n, xv)) * recip(C.d[n.c]);
      else v = x[n.c];
      const double rv = f.r[n.c];
      const double zv = (double)v * s;
      if constexpr (sizeof(R) == 8) {
        // FP64: the finest iterate is z itself
        if (red) x[n.c] = (R)zv;
      } else {
        if (rd_old) rzo += rv * ((double)P.z32[n.c] * zs_old);
        P.z32[n.c] = v;
      }
      rz += rv * zv;
    }
  }
  write_partials(T, tid, rz, rzo);
}

// Residual f - A x on the fine level summed over the 8 children of each
// coarse cell: the coarse right-hand side (restriction = transpose of the
// piecewise-constant prolongation).  One thread per coarse cell (cpt of them
// along x).
template <typename R, bool L0>
__global__ __launch_bounds__(kBlock) void k_resid_restrict(Tables T,
                                                           TileList LC, int lc) {
  const Tile t = get_tile(LC);
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev F = T.lv[(lc - 1) * T.nprob + t.prob];
  const LevelDev Cv = T.lv[lc * T.nprob + t.prob];
  const ProbDev P = T.pd[t.prob];
  const Coef<R> C = coefs<R>(F);
  const auto f = fsrc<R, L0>(F, P, sc);
  const R *x = (const R *)F.x;
  R *fc = (R *)Cv.f;
  const Col col = tile_col(t);
  if (!col.on) return;
  auto xv = [&](int q) { return x[q]; };
  for (int K = t.z0; K < t.z0 + t.tz; ++K) {
    for (int e = 0; e < t.cpt; ++e) {
      const int I = col.i + e;
      R acc = 0;
#pragma unroll
      for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            const Nb n = nbrs(2 * I + cx, 2 * col.j + cy, 2 * K + cz, F.nx,
                              F.ny, F.nz);
            acc += f(n.c) - (C.d[n.c] * x[n.c] - offsum(C, n, xv));
          }
      fc[(K * Cv.ny + col.j) * Cv.nx + I] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Weighted Jacobi smoother (the alternative to red/black Gauss-Seidel):
//   x_new = x + w (f - A x) / d,  w = 6/7,
// which updates every cell from the old iterate, so it ping-pongs between
// LevelDev::x and LevelDev::x2.  Symmetric in both sweeps, so the FP64
// V-cycle stays a symmetric preconditioner.
// ---------------------------------------------------------------------------

constexpr double kJacobiW = 6.0 / 7.0;

template <typename R, bool L0>
__global__ __launch_bounds__(kBlock) void k_jacobi(Tables T, TileList TL, int l,
                                                   int mode, int in_x2,
                                                   int flexible) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[l * T.nprob + t.prob];
  const ProbDev P = T.pd[t.prob];
  const Coef<R> C = coefs<R>(L);
  const auto f = fsrc<R, L0>(L, P, sc);
  const R w = (R)kJacobiW;
  const R *xin = (const R *)(in_x2 ? L.x2 : L.x);
  R *xout = (R *)(in_x2 ? L.x : L.x2);
  const Col col = tile_col(t);
  double rz = 0.0, rzo = 0.0;
  if (col.on) {
    auto xv = [&](int q) { return xin[q]; };
    for (int k = t.z0; k < t.z0 + t.tz; ++k) {
      const Nb n = nbrs(col.i, col.j, k, L.nx, L.ny, L.nz);
      R v;
      if (mode == 0) {
        v = w * f(n.c) * recip(C.d[n.c]);
      } else {
        const R xc = xin[n.c];
        v = xc + w * (f(n.c) - (C.d[n.c] * xc - offsum(C, n, xv))) * recip(C.d[n.c]);
      }
      if constexpr (L0) {
        if (mode == 2) {
          // z = s x (FP64 form: into z; mixed form: x itself into z32)
          const double zv = (double)v * sc.s;
          const double rv = f.r[n.c];
          if constexpr (sizeof(R) == 8) {
            if (flexible) rzo += rv * P.z[n.c];
            P.z[n.c] = zv;
          } else {
            if (flexible && !sc.restart) rzo += rv * ((double)P.z32[n.c] * sc.zscale);
            P.z32[n.c] = v;
          }
          rz += rv * zv;
          continue;
        }
      }
      xout[n.c] = v;
    }
  }
  if constexpr (L0) {
    if (mode == 2) write_partials(T, tid, rz, rzo);
  }
}

// out = x + P e over every cell of level l (P from coarse_corr); out is x
// itself or x2
template <typename R>
__global__ __launch_bounds__(kBlock) void k_prolong_add(Tables T, TileList TL,
                                                        int l, int trilinear,
                                                        int to_x2) {
  const Tile t = get_tile(TL);
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[l * T.nprob + t.prob];
  const ProbDev P = T.pd[t.prob];
  const bool has_coarse = l + 1 < P.levels;  // one-level problem: a copy
  const LevelDev Cl = T.lv[(has_coarse ? l + 1 : l) * T.nprob + t.prob];
  const R *e = (const R *)Cl.x;
  const R *x = (const R *)L.x;
  R *out = (R *)(to_x2 ? L.x2 : L.x);
  const Col col = tile_col(t);
  if (!col.on) return;
  for (int k = t.z0; k < t.z0 + t.tz; ++k) {
    const int c = (k * L.ny + col.j) * L.nx + col.i;
    const R ec = has_coarse ? coarse_corr(e, col.i, col.j, k, Cl.nx, Cl.ny,
                                          Cl.nz, trilinear != 0)
                            : (R)0;
    out[c] = x[c] + ec;
  }
}

// ---------------------------------------------------------------------------
// Tail of the V-cycle, one workgroup per problem: the coarsest level's
// Jacobi-CG solve and, above it, the levels from P.tail down (each small):
// pre-smoothing and restriction down to the coarsest level, the solve, then
// prolongation and post-smoothing back up to P.tail, in the order of the
// per-level path (red/black, red = even i+j+k), separated by workgroup
// barriers on data that stays in the L2.  (By default P.tail is the
// coarsest level: on gfx950 one workgroup sweeping 16^3 or 32^3 levels is
// no faster than the per-level launches it replaces.)
// ---------------------------------------------------------------------------

template <typename R>
struct LvlView {
  int nx, ny, nz, n;
  Coef<R> C;
  R *x, *f;
  __device__ __forceinline__ void ijk(int c, int &i, int &j, int &k) const {
    i = c % nx;
    j = (c / nx) % ny;
    k = c / (nx * ny);
  }
};

template <typename R>
__device__ __forceinline__ LvlView<R> lvl_view(const Tables &T, int l, int p) {
  const LevelDev L = T.lv[l * T.nprob + p];
  LvlView<R> v;
  v.nx = L.nx;
  v.ny = L.ny;
  v.nz = L.nz;
  v.n = L.n;
  v.C = coefs<R>(L);
  v.x = (R *)L.x;
  v.f = (R *)L.f;
  return v;
}

// first pre-sweep from x = 0 (red x = f/d, black from those red values)
template <typename R>
__device__ void tail_pre0(const LvlView<R> &V) {
  for (int c = threadIdx.x; c < V.n; c += kTailBlock) {
    int i, j, k;
    V.ijk(c, i, j, k);
    const Nb n = nbrs(i, j, k, V.nx, V.ny, V.nz);
    R v;
    if (((i + j + k) & 1) == 0) {
      v = V.f[c] * recip(V.C.d[c]);
    } else {
      auto red = [&](int q) { return V.f[q] * recip(V.C.d[q]); };
      v = (V.f[c] + offsum(V.C, n, red)) * recip(V.C.d[c]);
    }
    V.x[c] = v;
  }
}

template <typename R>
__device__ void tail_half(const LvlView<R> &V, int colour) {
  auto xv = [&](int q) { return V.x[q]; };
  for (int c = threadIdx.x; c < V.n; c += kTailBlock) {
    int i, j, k;
    V.ijk(c, i, j, k);
    if (((i + j + k) & 1) != colour) continue;
    const Nb n = nbrs(i, j, k, V.nx, V.ny, V.nz);
    V.x[c] = (V.f[c] + offsum(V.C, n, xv)) * recip(V.C.d[c]);
  }
}

// coarse right-hand side: fine residual summed over the 8 children
template <typename R>
__device__ void tail_restrict(const LvlView<R> &F, const LvlView<R> &Cv) {
  auto xv = [&](int q) { return F.x[q]; };
  for (int c = threadIdx.x; c < Cv.n; c += kTailBlock) {
    int I, J, K;
    Cv.ijk(c, I, J, K);
    R acc = 0;
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          const Nb n = nbrs(2 * I + cx, 2 * J + cy, 2 * K + cz, F.nx, F.ny, F.nz);
          acc += F.f[n.c] - (F.C.d[n.c] * F.x[n.c] - offsum(F.C, n, xv));
        }
    Cv.f[c] = acc;
  }
}

// black half-sweep with the coarse-grid correction folded in (red
// neighbours read as x + e(parent))
template <typename R>
__device__ void tail_prolong_black(const LvlView<R> &V, const LvlView<R> &Cv,
                                   bool tri) {
  for (int c = threadIdx.x; c < V.n; c += kTailBlock) {
    int i, j, k;
    V.ijk(c, i, j, k);
    if (((i + j + k) & 1) != 1) continue;
    const Nb n = nbrs(i, j, k, V.nx, V.ny, V.nz);
    const int im = i == 0 ? V.nx - 1 : i - 1, ip = i == V.nx - 1 ? 0 : i + 1;
    const int jm = j == 0 ? V.ny - 1 : j - 1, jp = j == V.ny - 1 ? 0 : j + 1;
    const int km = k == 0 ? V.nz - 1 : k - 1, kp = k == V.nz - 1 ? 0 : k + 1;
    auto par = [&](int a, int b2, int c2) {
      return coarse_corr(Cv.x, a, b2, c2, Cv.nx, Cv.ny, Cv.nz, tri);
    };
    const R s = V.C.tx[c] * (V.x[n.xp] + par(ip, j, k)) +
                V.C.tx[n.xm] * (V.x[n.xm] + par(im, j, k)) +
                V.C.ty[c] * (V.x[n.yp] + par(i, jp, k)) +
                V.C.ty[n.ym] * (V.x[n.ym] + par(i, jm, k)) +
                V.C.tz[c] * (V.x[n.zp] + par(i, j, kp)) +
                V.C.tz[n.zm] * (V.x[n.zm] + par(i, j, km));
    V.x[c] = (V.f[c] + s) * recip(V.C.d[c]);
  }
}

// coarsest level: Jacobi-preconditioned CG in FP64 to a relative residual of
// 1e-12 (an effectively exact solve), scratch in P.cs
template <typename R>
__device__ void tail_coarse_solve(const Tables &T, const ProbDev &P, int p,
                                  double *sh) {
  const int lc = P.levels - 1;
  const LevelDev L = T.lv[lc * T.nprob + p];
  const int n = L.n, nx = L.nx, ny = L.ny, nz = L.nz;
  double *xs = P.cs, *rs = P.cs + n, *ps = P.cs + 2 * n, *qs = P.cs + 3 * n;
  const R *f = (const R *)L.f;
  R *xo = (R *)L.x;
  double acc = 0.0;
  for (int c = threadIdx.x; c < n; c += kTailBlock) {
    const double v = (double)f[c];
    rs[c] = v;
    xs[c] = 0.0;
    acc += v * v;
  }
  const double bb = block_sum<kTailBlock / 64>(acc, sh);
  double rz_old = 1.0;
  if (bb > 0.0) {
    for (int it = 0; it < 1000; ++it) {
      acc = 0.0;
      for (int c = threadIdx.x; c < n; c += kTailBlock) acc += rs[c] * rs[c] / L.diag[c];
      const double rz = block_sum<kTailBlock / 64>(acc, sh);
      const double beta = it == 0 ? 0.0 : rz / rz_old;
      rz_old = rz;
      for (int c = threadIdx.x; c < n; c += kTailBlock)
        ps[c] = rs[c] / L.diag[c] + (it == 0 ? 0.0 : beta * ps[c]);
      __syncthreads();
      acc = 0.0;
      for (int c = threadIdx.x; c < n; c += kTailBlock) {
        const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        const Nb nb = nbrs(i, j, k, nx, ny, nz);
        const double q = L.diag[c] * ps[c] -
                         (L.Tx[c] * ps[nb.xp] + L.Tx[nb.xm] * ps[nb.xm] +
                          L.Ty[c] * ps[nb.yp] + L.Ty[nb.ym] * ps[nb.ym] +
                          L.Tz[c] * ps[nb.zp] + L.Tz[nb.zm] * ps[nb.zm]);
        qs[c] = q;
        acc += ps[c] * q;
      }
      const double pq = block_sum<kTailBlock / 64>(acc, sh);
      const double alpha = rz / pq;
      acc = 0.0;
      for (int c = threadIdx.x; c < n; c += kTailBlock) {
        xs[c] += alpha * ps[c];
        const double r = rs[c] - alpha * qs[c];
        rs[c] = r;
        acc += r * r;
      }
      const double rr = block_sum<kTailBlock / 64>(acc, sh);
      if (!(rr > 1e-24 * bb)) break;  // converged (or NaN: stop)
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += kTailBlock) xo[c] = (R)xs[c];
}

template <typename R>
__global__ __launch_bounds__(kTailBlock) void k_vtail(Tables T, int nu_pre,
                                                     int nu_post, int trilinear) {
  const int p = blockIdx.x;
  const Scal &sc = T.sc[p];
  const ProbDev P = T.pd[p];
  if (!sc.active || P.levels < 2) return;
  __shared__ double sh[kTailBlock / 64];
  const int lt = P.tail, lc = P.levels - 1;
  const bool tri = trilinear != 0;
  for (int l = lt; l < lc; ++l) {
    const LvlView<R> V = lvl_view<R>(T, l, p);
    tail_pre0(V);
    __syncthreads();
    for (int s2 = 1; s2 < nu_pre; ++s2) {
      tail_half(V, 0);
      __syncthreads();
      tail_half(V, 1);
      __syncthreads();
    }
    tail_restrict(V, lvl_view<R>(T, l + 1, p));
    __syncthreads();
  }
  tail_coarse_solve<R>(T, P, p, sh);
  __syncthreads();
  for (int l = lc - 1; l >= lt; --l) {
    const LvlView<R> V = lvl_view<R>(T, l, p);
    tail_prolong_black(V, lvl_view<R>(T, l + 1, p), tri);
    __syncthreads();
    tail_half(V, 0);
    __syncthreads();
    for (int s2 = 1; s2 < nu_post; ++s2) {
      tail_half(V, 1);
      __syncthreads();
      tail_half(V, 0);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Krylov kernels (FP64, finest level; two x-consecutive cells per thread)
// ---------------------------------------------------------------------------

// p_new = z + beta p_old (formed at the cell and its neighbours on the fly),
// q = A p_new, partial p_new . q.  p is double-buffered so neighbours read
// the old direction while the new one is written.  Each thread walks its
// column in z keeping p_new at planes k-1, k, k+1 and the -z face in
// registers.
// LAZY: also x += alpha_old p_old at the cell (the fused iteration defers
// that update of the previous iteration to here, where p_old is read anyway).
// Krylov storage modes (KM): KM_FP64: z and p FP64.  KM_MIX32 (mixed form):
// z, p_old and p_new FP32 at a scale each (zs for z and p_new, ps for
// p_old); p_new is rounded to FP32 before it is used, so q, the dot and the
// later x update all see the direction that is stored.  KM_MIX64 (mixed form
// with an FP64 direction): z FP32 at the scale zs (the V-cycle's output as
// it is), p_old and p_new FP64.
enum : int { KM_FP64 = 0, KM_MIX32 = 1, KM_MIX64 = 2 };

template <int KM>
using ZT = std::conditional_t<KM == KM_FP64, double, float>;
template <int KM>
using DirT = std::conditional_t<KM == KM_MIX32, float, double>;

template <bool BETA, bool LAZY, int KM>
__device__ __forceinline__ double spmv_column(
    const Tile &t, const Col &col, int nx, int ny, int nz, double beta,
    const ZT<KM> *__restrict__ z, double zs, const DirT<KM> *__restrict__ po,
    double ps, DirT<KM> *__restrict__ pn, double *__restrict__ q,
    const double *__restrict__ Tx, const double *__restrict__ Ty,
    const double *__restrict__ Tz, const double *__restrict__ Dg,
    double alpha_old, double *__restrict__ x) {
  using D = DirT<KM>;
  const double cb = KM == KM_MIX32 ? beta * ps / zs : beta;  // p_old's share, in z's scale
  auto raw = [&](int g) -> D {  // p_new as stored
    if constexpr (KM == KM_MIX32)
      return BETA ? (float)((double)z[g] + cb * (double)po[g]) : z[g];
    else if constexpr (KM == KM_MIX64)
      return BETA ? zs * (double)z[g] + beta * po[g] : zs * (double)z[g];
    else return BETA ? z[g] + beta * po[g] : z[g];
  };
  auto val = [&](D v) -> double {  // its value
    if constexpr (KM == KM_MIX32) return zs * (double)v;
    else return v;
  };
  const int plane = nx * ny, i = col.i, j = col.j;
  const int dxm = (i == 0) ? nx - 1 : -1, dxp = (i == nx - 1) ? 1 - nx : 1;
  const int dym = (j == 0) ? (ny - 1) * nx : -nx;
  const int dyp = (j == ny - 1) ? -(ny - 1) * nx : nx;
  int c = t.z0 * plane + j * nx + i;
  const int cm0 = (t.z0 == 0) ? c + (nz - 1) * plane : c - plane;
  D r_m = raw(cm0), r_c = raw(c);
  double tz_m = Tz[cm0];
  double acc = 0.0;
  for (int k = t.z0; k < t.z0 + t.tz; ++k) {
    const int cp = (k == nz - 1) ? c - (nz - 1) * plane : c + plane;
    const D r_p = raw(cp);
    const double s = Tx[c] * val(raw(c + dxp)) + Tx[c + dxm] * val(raw(c + dxm)) +
                     Ty[c] * val(raw(c + dyp)) + Ty[c + dym] * val(raw(c + dym)) +
                     Tz[c] * val(r_p) + tz_m * val(r_m);
    const double p_c = val(r_c);
    const double qq = Dg[c] * p_c - s;
    if constexpr (LAZY) {
      if constexpr (KM == KM_MIX32) x[c] = x[c] + alpha_old * (ps * (double)po[c]);
      else x[c] = x[c] + alpha_old * po[c];
    }
    pn[c] = r_c;
    q[c] = qq;
    acc += p_c * qq;
    tz_m = Tz[c];
    r_m = r_c;
    r_c = r_p;
    c = cp;
  }
  return acc;
}

template <bool LAZY, int KM>
__global__ __launch_bounds__(kBlock) void k_spmv_p(Tables T, TileList TL) {
  using D = DirT<KM>;
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const double beta = sc.beta, alpha = sc.alpha, zs = sc.zscale, ps = sc.pscale;
  const ZT<KM> *z;
  const D *po;
  D *pn;
  if constexpr (KM == KM_FP64) z = P.z;
  else z = P.z32;
  if constexpr (KM == KM_MIX32) {
    po = sc.pbuf ? P.pf1 : P.pf0;
    pn = sc.pbuf ? P.pf0 : P.pf1;
  } else {
    po = sc.pbuf ? P.p1 : P.p0;
    pn = sc.pbuf ? P.p0 : P.p1;
  }
  const Col col = tile_col(t);
  double pq = 0.0;
  if (col.on) {
    if (LAZY && sc.xlag)
      pq = spmv_column<true, true, KM>(t, col, L.nx, L.ny, L.nz, beta, z, zs, po, ps,
                                       pn, P.q, L.Tx, L.Ty, L.Tz, L.diag, alpha, P.x);
    else if (beta != 0.0)
      pq = spmv_column<true, false, KM>(t, col, L.nx, L.ny, L.nz, beta, z, zs, po, ps,
                                        pn, P.q, L.Tx, L.Ty, L.Tz, L.diag, 0.0, P.x);
    else
      pq = spmv_column<false, false, KM>(t, col, L.nx, L.ny, L.nz, beta, z, zs, po,
                                         ps, pn, P.q, L.Tx, L.Ty, L.Tz, L.diag, 0.0, P.x);
  }
  write_partials(T, tid, pq, 0.0);
}

// The fused iteration's SpMV on the fused tiles (64 x 16 cells, tz planes):
// each thread takes kSpRows consecutive rows of one column and walks z, so
// the y neighbours inside its rows come from registers and only the rows
// just below and above are loaded (2 of 16 rows, against 2 of 4 for the
// 64 x 4 tiles), as are the z neighbours (2 planes per tile).  The x
// neighbours come from the adjacent lanes (a wave is one 64-cell row
// segment); only the lanes at the tile's x edges load theirs.  Nothing is
// read twice: a plane's direction and z were loaded one plane earlier and
// are held, where reading them again a plane later would miss the L2, which
// holds less than one plane of all the resident tiles.  Per cell the
// arithmetic is spmv_column's, term by term, so q and p are the same.
constexpr int kSpRows = 4;

template <bool BETA, bool LAZY, int KM>
__device__ __forceinline__ double spmv_rows(
    const Tile &t, int lx, int i, int j0, int nr, int nx, int ny, int nz, double beta,
    const ZT<KM> *__restrict__ z, double zs, const DirT<KM> *__restrict__ po,
    double ps, DirT<KM> *__restrict__ pn, double *__restrict__ q,
    const double *__restrict__ Tx, const double *__restrict__ Ty,
    const double *__restrict__ Tz, const double *__restrict__ Dg, double alpha_old,
    double *__restrict__ x) {
  using D = DirT<KM>;
  const double cb = KM == KM_MIX32 ? beta * ps / zs : beta;
  // p_new as stored, from z and p_old at a cell
  auto mk = [&](ZT<KM> zv, D pv) -> D {
    if constexpr (KM == KM_MIX32)
      return BETA ? (float)((double)zv + cb * (double)pv) : zv;
    else if constexpr (KM == KM_MIX64)
      return BETA ? zs * (double)zv + beta * pv : zs * (double)zv;
    else return BETA ? zv + beta * pv : zv;
  };
  auto raw = [&](int g) -> D { return mk(z[g], BETA ? po[g] : (D)0); };
  auto val = [&](D v) -> double {
    if constexpr (KM == KM_MIX32) return zs * (double)v;
    else return v;
  };
  const int plane = nx * ny;
  const int dxm = (i == 0) ? nx - 1 : -1, dxp = (i == nx - 1) ? 1 - nx : 1;
  const bool ledge = lx == 0, redge = lx == t.tx - 1;
  const int rlo = (j0 == 0 ? ny - 1 : j0 - 1) * nx;        // the row below
  const int rhi = (j0 + nr == ny ? 0 : j0 + nr) * nx;      // the row above
  const int km0 = t.z0 == 0 ? nz - 1 : t.z0 - 1;
  D pm[kSpRows], pc[kSpRows], oc[kSpRows];  // p_new at k - 1, k; p_old at k
  double tzm[kSpRows];
#pragma unroll
  for (int r = 0; r < kSpRows; ++r) {
    if (r < nr) {
      const int o = (j0 + r) * nx + i, c = t.z0 * plane + o;
      pm[r] = raw(km0 * plane + o);
      oc[r] = BETA ? po[c] : (D)0;
      pc[r] = mk(z[c], oc[r]);
      tzm[r] = Tz[km0 * plane + o];
    }
  }
  double acc = 0.0;
  for (int k = t.z0; k < t.z0 + t.tz; ++k) {
    const int kp = (k == nz - 1) ? 0 : k + 1;
    const int b = k * plane + i;
    D pp[kSpRows], op[kSpRows];
#pragma unroll
    for (int r = 0; r < kSpRows; ++r) {
      if (r < nr) {
        const int g = kp * plane + (j0 + r) * nx + i;
        op[r] = BETA ? po[g] : (D)0;
        pp[r] = mk(z[g], op[r]);
      }
    }
    const D plo = raw(b + rlo), phi = raw(b + rhi);
    double tyd = Ty[b + rlo];  // the -y face of the next row
#pragma unroll
    for (int r = 0; r < kSpRows; ++r) {
      if (r < nr) {
        const int c = b + (j0 + r) * nx;
        D xl = __shfl_up(pc[r], 1, 64), xr = __shfl_down(pc[r], 1, 64);
        if (ledge) xl = raw(c + dxm);
        if (redge) xr = raw(c + dxp);
        const D dn = r == 0 ? plo : pc[r > 0 ? r - 1 : 0];
        const D up = r + 1 == nr ? phi : pc[r + 1 < kSpRows ? r + 1 : r];
        const double tyc = Ty[c];
        const double sm = Tx[c] * val(xr) + Tx[c + dxm] * val(xl) + tyc * val(up) +
                          tyd * val(dn) + Tz[c] * val(pp[r]) + tzm[r] * val(pm[r]);
        const double p_c = val(pc[r]);
        const double qq = Dg[c] * p_c - sm;
        if constexpr (LAZY) {
          if constexpr (KM == KM_MIX32) x[c] = x[c] + alpha_old * (ps * (double)oc[r]);
          else x[c] = x[c] + alpha_old * oc[r];
        }
        pn[c] = pc[r];
        q[c] = qq;
        acc += p_c * qq;
        tzm[r] = Tz[c];
        tyd = tyc;
      }
    }
#pragma unroll
    for (int r = 0; r < kSpRows; ++r) {
      if (r < nr) {
        pm[r] = pc[r];
        pc[r] = pp[r];
        oc[r] = op[r];
      }
    }
  }
  return acc;
}

template <bool LAZY, int KM>
__global__ __launch_bounds__(kBlock) void k_spmv_f(Tables T, TileList TL) {
  using D = DirT<KM>;
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const double beta = sc.beta, alpha = sc.alpha, zs = sc.zscale, ps = sc.pscale;
  const ZT<KM> *z;
  const D *po;
  D *pn;
  if constexpr (KM == KM_FP64) z = P.z;
  else z = P.z32;
  if constexpr (KM == KM_MIX32) {
    po = sc.pbuf ? P.pf1 : P.pf0;
    pn = sc.pbuf ? P.pf0 : P.pf1;
  } else {
    po = sc.pbuf ? P.p1 : P.p0;
    pn = sc.pbuf ? P.p0 : P.p1;
  }
  const int lx = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int nr = min(kSpRows, t.ty - kSpRows * g);
  double pq = 0.0;
  if (lx < t.tx && nr > 0) {
    const int i = t.x0 + lx, j0 = t.y0 + kSpRows * g;
    if (LAZY && sc.xlag)
      pq = spmv_rows<true, true, KM>(t, lx, i, j0, nr, L.nx, L.ny, L.nz, beta, z, zs, po,
                                     ps, pn, P.q, L.Tx, L.Ty, L.Tz, L.diag, alpha, P.x);
    else if (beta != 0.0)
      pq = spmv_rows<true, false, KM>(t, lx, i, j0, nr, L.nx, L.ny, L.nz, beta, z, zs, po,
                                      ps, pn, P.q, L.Tx, L.Ty, L.Tz, L.diag, 0.0, P.x);
    else
      pq = spmv_rows<false, false, KM>(t, lx, i, j0, nr, L.nx, L.ny, L.nz, beta, z, zs,
                                       po, ps, pn, P.q, L.Tx, L.Ty, L.Tz, L.diag, 0.0, P.x);
  }
  write_partials(T, tid, pq, 0.0);
}

// out = s z32 right after a mixed-form cycle (s: the scale it ran at)
__global__ __launch_bounds__(kBlock) void k_z_out(Tables T, TileList TL,
                                                  double *__restrict__ out) {
  const Tile t = get_tile(TL);
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const double zs = T.sc[t.prob].s;
  const Col col = tile_col(t);
  if (!col.on) return;
  const int plane = L.nx * L.ny;
  int c = t.z0 * plane + col.j * L.nx + col.i;
  for (int k = 0; k < t.tz; ++k, c += plane) out[c] = (double)P.z32[c] * zs;
}

// the newest direction p at cell c (after FIN_PQ has swapped the buffers)
template <int KM>
__device__ __forceinline__ double newest_p(const ProbDev &P, const Scal &sc, int c) {
  if constexpr (KM == KM_MIX32) return sc.pscale * (double)(sc.pbuf ? P.pf1 : P.pf0)[c];
  else return (sc.pbuf ? P.p1 : P.p0)[c];
}

// x += alpha p (the newest direction) for problems that stopped iterating
// while the fused iteration's x update was still pending
template <int KM>
__global__ __launch_bounds__(kBlock) void k_xfix(Tables T, TileList TL) {
  const Tile t = get_tile(TL);
  const Scal &sc = T.sc[t.prob];
  if (!sc.xlag || sc.phase == PH_ITER) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const double alpha = sc.alpha;
  const Col col = tile_col(t);
  if (!col.on) return;
  const int plane = L.nx * L.ny;
  int c = t.z0 * plane + col.j * L.nx + col.i;
  for (int k = 0; k < t.tz; ++k, c += plane)
    P.x[c] = P.x[c] + alpha * newest_p<KM>(P, sc, c);
}

// x += alpha p, r -= alpha q, partial ||r||^2
template <int KM>
__global__ __launch_bounds__(kBlock) void k_update(Tables T, TileList TL) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const double alpha = sc.alpha;
  const double *__restrict__ q = P.q;
  double *__restrict__ x = P.x;
  double *__restrict__ r = rcur(P, sc);
  const Col col = tile_col(t);
  double rr = 0.0;
  if (col.on) {
    const int plane = L.nx * L.ny;
    int c = t.z0 * plane + col.j * L.nx + col.i;
    for (int k = 0; k < t.tz; ++k, c += plane) {
      const double pc = newest_p<KM>(P, sc, c), qc = q[c], xc = x[c], rc = r[c];
      x[c] = xc + alpha * pc;
      const double rn = rc - alpha * qc;
      r[c] = rn;
      rr += rn * rn;
    }
  }
  write_partials(T, tid, rr, 0.0);
}

// true residual r = b - A x in FP64 (problems whose recursive residual met
// the tolerance), partial ||r||^2
__global__ __launch_bounds__(kBlock) void k_true_resid(Tables T, TileList TL) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (sc.phase != PH_VERIFY) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const Coef<double> C = coefs<double>(L);
  const Col col = tile_col(t);
  double rr = 0.0;
  if (col.on) {
    auto xv = [&](int q) { return P.x[q]; };
    for (int k = t.z0; k < t.z0 + t.tz; ++k) {
      for (int e = 0; e < t.cpt; ++e) {
        const Nb n = nbrs(col.i + e, col.j, k, L.nx, L.ny, L.nz);
        const double r = P.b[n.c] - (C.d[n.c] * P.x[n.c] - offsum(C, n, xv));
        rcur(P, sc)[n.c] = r;
        rr += r * r;
      }
    }
  }
  write_partials(T, tid, rr, 0.0);
}

// Galerkin warm guess, once FIN_BB has solved for c: x0 = c1 dE(n) + c2
// dE(n-1), formed at the cell and its neighbours on the fly, and r = b - A x0
// with the assembled FP64 operator; partial ||r||^2 for FIN_WARM.
__global__ __launch_bounds__(kBlock) void k_warm_x(Tables T, TileList TL) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  const StepDev S = T.sd[t.prob];
  if (!warm_due(sc) || !(S.warm > 1.0) || sc.phase != PH_ITER || sc.cold) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const double c1 = sc.c1, c2 = sc.c2;
  const double *__restrict__ h1 = S.h1;
  const double *__restrict__ h2 = S.h2;
  auto g = [&](int q) { return h2 ? c1 * h1[q] + c2 * h2[q] : c1 * h1[q]; };
  const double *__restrict__ Tx = L.Tx;
  const double *__restrict__ Ty = L.Ty;
  const double *__restrict__ Tz = L.Tz;
  double *__restrict__ rv = rcur(P, sc);
  const Col col = tile_col(t);
  double rr = 0.0;
  if (col.on) {
    const int nx = L.nx, ny = L.ny, nz = L.nz, plane = nx * ny;
    const int i = col.i, j = col.j;
    const int dxm = (i == 0) ? nx - 1 : -1, dxp = (i == nx - 1) ? 1 - nx : 1;
    const int dym = (j == 0) ? (ny - 1) * nx : -nx;
    const int dyp = (j == ny - 1) ? -(ny - 1) * nx : nx;
    int c = t.z0 * plane + j * nx + i;
    const int cm0 = (t.z0 == 0) ? c + (nz - 1) * plane : c - plane;
    double x_m = g(cm0), x_c = g(c), tz_m = Tz[cm0];
    for (int k = t.z0; k < t.z0 + t.tz; ++k) {
      const int cp = (k == nz - 1) ? c - (nz - 1) * plane : c + plane;
      const double x_p = g(cp);
      const double off = Tx[c] * g(c + dxp) + Tx[c + dxm] * g(c + dxm) +
                         Ty[c] * g(c + dyp) + Ty[c + dym] * g(c + dym) +
                         Tz[c] * x_p + tz_m * x_m;
      const double r = P.b[c] - (L.diag[c] * x_c - off);
      P.x[c] = x_c;
      rv[c] = r;
      rr += r * r;
      tz_m = Tz[c];
      x_m = x_c;
      x_c = x_p;
      c = cp;
    }
  }
  write_partials(T, tid, rr, 0.0);
}

// Local smoothing.  Where a cell's coupling to its neighbours dominates its
// diagonal (an ionized bubble: little absorption, D near D_max, so the cell
// is almost a pure diffusion cell), one red/black sweep leaves the error that
// is smooth inside the bubble nearly untouched and the coarse levels, whose
// cells mix bubble and neutral children, do not represent it; extra sweeps
// restricted to those cells act on it at a small fraction of a full sweep's
// cost.  k_lmask marks them once per assembly from the FP64 finest operator
// and lists them per tile and colour; k_local runs one half-sweep of colour
// `colour` over a tile's listed cells, in place in the cycle's FP32 output
// z32, with the cycle's scaled right-hand side and FP32 coefficients, and
// records the change of r.z that the update makes (r the FP64 residual the
// cycle ran on, z = s z32).
//
// The list of a tile lives in llist at the tile's own cells: entry q (the
// colour-0 cells first, then the colour-1 cells, each in thread and plane
// order) is stored at the q-th cell of the tile's box in x, y, z order, so
// tiles never overlap and one wave reads 64 consecutive entries.  lcnt[2u],
// lcnt[2u + 1]: the counts per colour of the problem's finest tile u (held
// with the problem: a server rebuilds its tables between the assembly and
// the sweeps).  Within one colour the updates are independent (a cell of
// that colour reads only cells of the other), so k_local gives every listed
// cell a thread of its own.

// exclusive prefix sums of a and b over the block's threads (thread order)
// and their totals
__device__ __forceinline__ void block_scan2(int a, int b, int *sh, int &ea, int &eb,
                                            int &ta, int &tb) {
  constexpr int NW = kBlock / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int ia = a, ib = b;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int ua = __shfl_up(ia, d, 64), ub = __shfl_up(ib, d, 64);
    if (lane >= d) {
      ia += ua;
      ib += ub;
    }
  }
  if (lane == 63) {
    sh[w] = ia;
    sh[NW + w] = ib;
  }
  __syncthreads();
  int oa = 0, ob = 0;
  ta = 0;
  tb = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if (i < w) {
      oa += sh[i];
      ob += sh[NW + i];
    }
    ta += sh[i];
    tb += sh[NW + i];
  }
  ea = oa + ia - a;
  eb = ob + ib - b;
}

// index of the q-th cell of tile t's box (x fastest)
__device__ __forceinline__ int box_cell(const Tile &t, int q, int nx, int ny) {
  const int txy = t.tx * t.ty, lz = q / txy, rm = q - lz * txy, ly = rm / t.tx;
  return ((t.z0 + lz) * ny + t.y0 + ly) * nx + t.x0 + (rm - ly * t.tx);
}

__global__ __launch_bounds__(kBlock) void k_lmask(Tables T, TileList TL,
                                                  double coupling) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!asm_due(sc)) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const Col col = tile_col(t);
  unsigned long long bits = 0;  // marked planes of the column: bit k - z0
  int m0 = 0, m1 = 0;           // marked cells of colour 0, 1
  if (col.on) {
    for (int k = t.z0; k < t.z0 + t.tz; ++k) {
      const Nb n = nbrs(col.i, col.j, k, L.nx, L.ny, L.nz);
      const double faces = L.Tx[n.c] + L.Tx[n.xm] + L.Ty[n.c] + L.Ty[n.ym] +
                           L.Tz[n.c] + L.Tz[n.zm];
      if (faces > coupling * L.diag[n.c]) {
        bits |= 1ull << (k - t.z0);
        if ((col.i + col.j + k) & 1) ++m1;
        else ++m0;
      }
    }
  }
  __shared__ int sh[2 * (kBlock / 64)];
  int e0, e1, n0, n1;
  block_scan2(m0, m1, sh, e0, e1, n0, n1);
  while (bits) {
    const int b = __ffsll((long long)bits) - 1;
    bits &= bits - 1;
    const int k = t.z0 + b;
    const int q = ((col.i + col.j + k) & 1) ? n0 + e1++ : e0++;
    P.llist[box_cell(t, q, L.nx, L.ny)] = (k * L.ny + col.j) * L.nx + col.i;
  }
  if (threadIdx.x == 0) {
    P.lcnt[2 * (tid - P.t0)] = n0;
    P.lcnt[2 * (tid - P.t0) + 1] = n1;
  }
}

__global__ __launch_bounds__(kBlock) void k_local(Tables T, TileList TL, int colour) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const ProbDev P = T.pd[t.prob];
  // the counts come from k_lmask; bounded by the tile's box all the same, so
  // that no read of the list can leave the tile's own cells
  const int u = tid - P.t0, box = t.tx * t.ty * t.tz;
  const int first = colour ? min(max(P.lcnt[2 * u], 0), box) : 0;
  const int cnt = min(max(P.lcnt[2 * u + colour], 0), box - first);
  if (cnt == 0) {
    if (threadIdx.x == 0) T.lpart[2 * tid + colour] = 0.0;
    return;
  }
  const LevelDev L = T.lv[t.prob];
  const Coef<float> C = coefs<float>(L);
  const double *r = rcur(P, sc);
  const double inv_s = sc.inv_s, s = sc.s;
  float *z = P.z32;
  const int plane = L.nx * L.ny;
  double dz = 0.0;
  for (int q = threadIdx.x; q < cnt; q += kBlock) {
    const int c = P.llist[box_cell(t, first + q, L.nx, L.ny)];
    if ((unsigned)c >= (unsigned)(plane * L.nz)) continue;  // not a cell
    const int k = c / plane, rm = c - k * plane, j = rm / L.nx;
    const Nb n = nbrs(rm - j * L.nx, j, k, L.nx, L.ny, L.nz);
    const float f = (float)(r[n.c] * inv_s);
    const float sum = C.tx[n.c] * z[n.xp] + C.tx[n.xm] * z[n.xm] +
                      C.ty[n.c] * z[n.yp] + C.ty[n.ym] * z[n.ym] +
                      C.tz[n.c] * z[n.zp] + C.tz[n.zm] * z[n.zm];
    const float xn = (f + sum) * recip(C.d[n.c]);
    const float xo = z[n.c];
    z[n.c] = xn;
    dz += r[n.c] * (s * ((double)xn - (double)xo));
  }
  __shared__ double sh[kBlock / 64];
  const double v = block_sum<kBlock / 64>(dz, sh);
  if (threadIdx.x == 0) T.lpart[2 * tid + colour] = v;
}

// Warm-started problems whose guess was dropped (by FIN_BB or FIN_WARM: it
// did not reduce the residual): x = 0, r = b.  And b = 0: the solution is 0
// whatever the guess.
__global__ __launch_bounds__(kBlock) void k_warm_revert(Tables T, TileList TL) {
  const Tile t = get_tile(TL);
  const Scal &sc = T.sc[t.prob];
  if (!warm_due(sc) || !(T.sd[t.prob].warm > 0.0)) return;
  const bool zero_b = sc.phase == PH_DONE && sc.status == ST_OK;
  if (!zero_b && !(sc.phase == PH_ITER && sc.cold)) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  double *rv = rcur(P, sc);
  const Col col = tile_col(t);
  if (!col.on) return;
  for (int k = t.z0; k < t.z0 + t.tz; ++k) {
    const int c0 = (k * L.ny + col.j) * L.nx + col.i;
    for (int e = 0; e < t.cpt; ++e) {
      P.x[c0 + e] = 0.0;
      rv[c0 + e] = P.b[c0 + e];
    }
  }
}

// out = A u (single problem, inspection entry point)
__global__ __launch_bounds__(kBlock) void k_apply(Tables T, TileList TL,
                                                  const double *u, double *out) {
  const Tile t = get_tile(TL);
  const LevelDev L = T.lv[t.prob];
  const Coef<double> C = coefs<double>(L);
  const Col col = tile_col(t);
  if (!col.on) return;
  auto uv = [&](int q) { return u[q]; };
  for (int k = t.z0; k < t.z0 + t.tz; ++k) {
    for (int e = 0; e < t.cpt; ++e) {
      const Nb n = nbrs(col.i + e, col.j, k, L.nx, L.ny, L.nz);
      out[n.c] = C.d[n.c] * u[n.c] - offsum(C, n, uv);
    }
  }
}

// load an external residual (preconditioner entry point): r = given, ||r||^2
__global__ __launch_bounds__(kBlock) void k_set_r(Tables T, TileList TL,
                                                  const double *rin) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  double *rv = rcur(P, sc);
  const Col col = tile_col(t);
  double rr = 0.0;
  if (col.on) {
    for (int k = t.z0; k < t.z0 + t.tz; ++k) {
      const int c0 = (k * L.ny + col.j) * L.nx + col.i;
      for (int e = 0; e < t.cpt; ++e) {
        const double r = rin[c0 + e];
        rv[c0 + e] = r;
        rr += r * r;
      }
    }
  }
  write_partials(T, tid, rr, 0.0);
}

// E_out = E + dE with the relative-change sum (dE / max(|E_out|, floor))^2
// and ||dE||^2; copy_only: E_out = dE (solve entry point).
// in_solve: launched right after the verification; acts only on problems it
// just decided (done, ok, not yet committed)
__device__ __forceinline__ bool commit_now(const Scal &sc) {
  return sc.live && sc.phase == PH_DONE && sc.status == ST_OK && !sc.committed;
}

__global__ __launch_bounds__(kBlock) void k_update_E(Tables T, TileList TL,
                                                     double floor,
                                                     int copy_only, int in_solve) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (in_solve ? !commit_now(sc) : !sc.live) return;
  const LevelDev L = T.lv[t.prob];
  const ProbDev P = T.pd[t.prob];
  const StepDev S = T.sd[t.prob];
  const Col col = tile_col(t);
  double ch = 0.0, dd = 0.0;
  if (col.on) {
    for (int k = t.z0; k < t.z0 + t.tz; ++k) {
      const int c0 = (k * L.ny + col.j) * L.nx + col.i;
      for (int e = 0; e < t.cpt; ++e) {
        const int c = c0 + e;
        const double d = P.x[c];
        dd += d * d;
        if (copy_only) {
          S.Eout[c] = d;
        } else {
          const double en = S.E[c] + d;
          S.Eout[c] = en;
          double w = fabs(en);
          w = (w < floor) ? floor : w;
          if (w > 0.0) {
            const double q = d / w;
            ch += q * q;
          }
        }
      }
    }
  }
  write_partials(T, tid, ch, dd);
}

// ---------------------------------------------------------------------------
// per-problem finalize: sum the tile partials in tile order, update scalars
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

__device__ __forceinline__ void set_scale(Scal &sc, int n, int mixed) {
  double s = 1.0;
  if (mixed) {
    s = sqrt(sc.rr / (double)n);
    if (!(s > 0.0) || !finite(s)) s = 1.0;
  }
  sc.s = s;
  sc.inv_s = 1.0 / s;
}

__device__ __forceinline__ void fail(Scal &sc, int status) {
  sc.status = status;
  sc.phase = PH_DONE;
  sc.active = 0;
}

// FIN_BB: the assembly's sums (in tile order), the start of the solve and,
// for a warm start, the guess: the extrapolated one is kept if it reduces
// the residual; the Galerkin one gets its coefficients here (k_warm_x then
// forms it and FIN_WARM applies the same test)
__global__ __launch_bounds__(kFinBlock) void k_fin_bb(Tables T, int mixed) {
  const int p = blockIdx.x;
  Scal &sc = T.sc[p];
  if (!asm_due(sc)) return;
  const ProbDev &P = T.pd[p];
  double a[kAsmSums];
#pragma unroll
  for (int i = 0; i < kAsmSums; ++i) a[i] = 0.0;
  for (int t = P.t0 + (int)threadIdx.x; t < P.t1; t += kFinBlock) {
#pragma unroll
    for (int i = 0; i < kAsmSums; ++i) a[i] += T.gpart[kAsmSums * t + i];
  }
  constexpr int NW = kFinBlock / 64;
  __shared__ double sh[kAsmSums][NW];
#pragma unroll
  for (int i = 0; i < kAsmSums; ++i) {
    const double w = wave_sum(a[i]);
    if ((threadIdx.x & 63) == 0) sh[i][threadIdx.x >> 6] = w;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = 0; i < kAsmSums; ++i) {
    double v = 0.0;
    for (int k = 0; k < NW; ++k) v += sh[i][k];
    a[i] = v;
  }
  const double bb = a[AS_BB];
  sc.bb = bb;
  sc.rr = bb;
  sc.rr_true = bb;
  sc.iter = 0;
  sc.restart = 1;
  sc.restarts = 0;
  sc.pbuf = 0;
  sc.has_dir = sc.xlag = sc.snew = 0;
  sc.fresh = 1;
  sc.committed = 0;
  sc.status = ST_OK;
  sc.phase = PH_ITER;
  sc.active = 1;
  sc.cold = 0;
  const double warm = T.sd[p].warm;
  if (!finite(bb)) {
    fail(sc, ST_ENONFINITE);
  } else if (bb == 0.0) {
    sc.phase = PH_DONE;
    sc.active = 0;
  } else if (warm > 1.0) {
    // (h_i, A h_j) c = (h_i, b): the A-norm-closest point of span{h} to the
    // solution; one vector when the pair is (nearly) dependent or absent
    const double g11 = a[AS_G11], g12 = a[AS_G12], g22 = a[AS_G22];
    const double b1 = a[AS_B1], b2 = a[AS_B2];
    const double det = g11 * g22 - g12 * g12;
    double c1 = 0.0, c2 = 0.0;
    bool ok = g11 > 0.0 && finite(g11) && finite(b1);
    if (ok && T.sd[p].h2 && g22 > 0.0 && det > 1e-10 * g11 * g22 &&
        finite(g12) && finite(g22) && finite(b2)) {
      c1 = (b1 * g22 - b2 * g12) / det;
      c2 = (b2 * g11 - b1 * g12) / det;
    } else if (ok) {
      c1 = b1 / g11;
    }
    ok = ok && finite(c1) && finite(c2);
    sc.c1 = c1;
    sc.c2 = c2;
    sc.cold = !ok;
  } else if (warm > 0.0) {
    // PCG from the warm guess (same ||b||), or from 0 (k_warm_revert)
    // if the guess does not reduce the residual
    const double rr = a[AS_RR];
    sc.cold = !(rr < bb);
    if (!sc.cold) sc.rr = rr;
    if (!finite(rr)) fail(sc, ST_ENONFINITE);
  }
  set_scale(sc, P.n, mixed);
  if (sc.ctl) sc.stage = 2;  // device-controlled: the warm start is next
}

__global__ __launch_bounds__(kFinBlock) void k_fin(Tables T, int which, int mixed,
                                                  int alt) {
  const int p = blockIdx.x;
  Scal &sc = T.sc[p];
  const ProbDev P = T.pd[p];
  // partials of the fused tiles: the fused cycle's r.z, the down pass's
  // ||r||^2 and the fused iteration's SpMV
  const bool fz = (alt && which == FIN_RZ) || (alt && which == FIN_PQ && P.spf) ||
                  which == FIN_RR2;
  const int t0 = fz ? P.f0 : P.t0;
  const int t1 = (which == FIN_XFIX || which == FIN_FRESH) ? t0 : (fz ? P.f1 : P.t1);
  bool part;
  switch (which) {
    case FIN_STEP: part = alt ? commit_now(sc) : sc.live != 0; break;
    case FIN_TRUE: part = sc.phase == PH_VERIFY; break;
    case FIN_SETR: part = true; break;
    case FIN_RR2: part = sc.active && sc.has_dir; break;
    case FIN_XFIX: part = sc.xlag && sc.phase != PH_ITER; break;
    case FIN_FRESH: part = sc.active && sc.fresh; break;
    case FIN_WARM:
      part = warm_due(sc) && T.sd[p].warm > 1.0 && sc.phase == PH_ITER && !sc.cold;
      break;
    case FIN_STAGE:
      if (threadIdx.x == 0 && sc.ctl && sc.stage == 2) sc.stage = 0;
      return;
    default: part = sc.active != 0; break;
  }
  if (!part) return;
  // independent loads in flight: 4 per thread per round, summed in order
  double a0 = 0.0, a1 = 0.0;
  if (which == FIN_RZ && alt == 2) {
    // r.z changes of the local sweeps (black, red), per finest tile
    for (int t = P.t0 + (int)threadIdx.x; t < P.t1; t += kFinBlock)
      a0 += T.lpart[2 * t] + T.lpart[2 * t + 1];
  }
  int t = t0 + (int)threadIdx.x;
  for (; t + 3 * kFinBlock < t1; t += 4 * kFinBlock) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v[2 * u] = T.part[2 * (t + u * kFinBlock)];
      v[2 * u + 1] = T.part[2 * (t + u * kFinBlock) + 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a0 += v[2 * u];
      a1 += v[2 * u + 1];
    }
  }
  for (; t < t1; t += kFinBlock) {
    a0 += T.part[2 * t];
    a1 += T.part[2 * t + 1];
  }
  __shared__ double sh[kFinBlock / 64];
  a0 = block_sum<kFinBlock / 64>(a0, sh);
  a1 = block_sum<kFinBlock / 64>(a1, sh);
  if (threadIdx.x != 0) return;
  switch (which) {
    case FIN_RZ: {
      sc.zscale = sc.s;  // the scale z was just formed with
      sc.rho = a0;
      sc.rzo = a1;
      if (!finite(a0) || !finite(a1)) { fail(sc, ST_ENONFINITE); break; }
      if (!(a0 > 0.0)) { fail(sc, ST_ENOCONV); break; }
      double beta = 0.0;
      if (!sc.restart) beta = mixed ? (a0 - a1) / sc.rho_old : a0 / sc.rho_old;
      sc.beta = beta;
      sc.restart = 0;
      sc.rho_old = a0;
      break;
    }
    case FIN_PQ:
      sc.pscale = sc.zscale;  // the direction just formed has z's scale
      sc.pq = a0;
      if (!finite(a0)) { fail(sc, ST_ENONFINITE); break; }
      if (!(a0 > 0.0)) { fail(sc, ST_ENOCONV); break; }
      sc.alpha = sc.rho / a0;
      sc.pbuf ^= 1;
      if (alt) {
        // fused iteration: r -= alpha q happens in the next down pass, x +=
        // alpha p in the next SpMV; the V-cycle scale changes between cycles
        sc.has_dir = 1;
        sc.xlag = 1;
        if (sc.snew) {
          sc.s = sc.s_next;
          sc.inv_s = 1.0 / sc.s_next;
          sc.snew = 0;
        }
      }
      break;
    case FIN_RR2:
      sc.rr = a0;
      sc.iter += 1;
      sc.rbuf ^= 1;  // the down pass wrote r - alpha q to the other buffer
      if (!finite(a0)) { fail(sc, ST_ENONFINITE); break; }
      if (a0 <= sc.tol2 * sc.bb) {
        sc.phase = PH_VERIFY;
        sc.active = 0;
      } else if (sc.iter >= sc.max_iter) {
        fail(sc, ST_ENOCONV);
      }
      {
        // scale of the next V-cycle (this one already uses the current s)
        const double s0 = sc.s, i0 = sc.inv_s;
        set_scale(sc, P.n, mixed);
        sc.s_next = sc.s;
        sc.s = s0;
        sc.inv_s = i0;
        sc.snew = 1;
      }
      break;
    case FIN_XFIX:
      sc.xlag = 0;
      break;
    case FIN_FRESH:
      sc.fresh = 0;
      break;
    case FIN_WARM:
      // keep the projected guess only if it reduces the residual (else
      // k_warm_revert starts from 0)
      sc.cold = !(a0 < sc.bb);
      if (!finite(a0)) { fail(sc, ST_ENONFINITE); break; }
      if (!sc.cold) {
        sc.rr = a0;
        set_scale(sc, P.n, mixed);
      }
      break;
    case FIN_RR:
      sc.rr = a0;
      sc.iter += 1;
      if (!finite(a0)) { fail(sc, ST_ENONFINITE); break; }
      if (a0 <= sc.tol2 * sc.bb) {
        sc.phase = PH_VERIFY;
        sc.active = 0;
      } else if (sc.iter >= sc.max_iter) {
        fail(sc, ST_ENOCONV);
      }
      set_scale(sc, P.n, mixed);
      break;
    case FIN_TRUE:
      sc.rr_true = a0;
      sc.rr = a0;
      if (!finite(a0)) { fail(sc, ST_ENONFINITE); break; }
      if (a0 <= sc.tol2 * sc.bb) {
        sc.status = ST_OK;
        sc.phase = PH_DONE;
        sc.active = 0;
      } else if (sc.iter < sc.max_iter) {
        sc.phase = PH_ITER;
        sc.active = 1;
        sc.restart = 1;
        sc.restarts += 1;
        sc.has_dir = sc.snew = 0;
        sc.fresh = 1;
        set_scale(sc, P.n, mixed);
      } else {
        fail(sc, ST_ENOCONV);
      }
      break;
    case FIN_STEP:
      sc.change2 = a0;
      sc.dEdE = a1;
      sc.committed = 1;
      break;
    case FIN_SETR:
      sc.rr = a0;
      sc.active = 1;
      sc.phase = PH_ITER;
      sc.has_dir = sc.xlag = sc.snew = sc.fresh = 0;
      set_scale(sc, P.n, mixed);
      break;
  }
}

// ---------------------------------------------------------------------------
// per-kernel timing hook (include/fld_profile.h)
// ---------------------------------------------------------------------------

static const char *kKernelNames[K_NUM] = {
    "assemble", "coarsen", "fin", "pre0_fine", "pre0_coarse", "half_fine",
    "half_coarse", "half_out", "resid_restrict_fine", "resid_restrict_coarse",
    "prolong_black_fine", "prolong_black_coarse", "coarse_solve", "spmv_p",
    "update", "true_resid", "apply", "set_r", "update_E", "vdown_fine",
    "vdown_coarse", "vup_fine", "vup_coarse", "chem_h", "ionized_sum",
    "warm_revert", "jacobi0_fine", "jacobi_fine", "jacobi_out",
    "jacobi_coarse", "prolong_add_fine", "prolong_add_coarse", "spmv_px",
    "xfix", "warm_x", "lmask", "local", "control", "copy_E"};

namespace prof {
struct Rec {
  hipEvent_t a, b;
  int k;
};
static int sel = -1;
static std::vector<Rec> recs;
static std::vector<hipEvent_t> pool;

static hipEvent_t get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static bool on(int k, hipStream_t s) {
  if (!(sel == k || sel == -2)) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return false;
  return true;
}

}  // namespace prof

ProfScope::ProfScope(int k_, hipStream_t s_) : k(k_), s(s_), a(nullptr) {
  if (prof::on(k, s)) {
    a = prof::get();
    if (a) hipEventRecord(a, s);
  }
}

ProfScope::~ProfScope() {
  if (!a) return;
  hipEvent_t b = prof::get();
  if (!b) return;
  hipEventRecord(b, s);
  prof::recs.push_back({a, b, k});
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define LAUNCH FLD_LAUNCH

void launch_assemble(const Tables &T, TileList L0, double c, double theta,
                     double dmax, double rmin, int mixed, hipStream_t s) {
  if (L0.nblocks) LAUNCH(K_ASSEMBLE, k_assemble, L0.nblocks, kBlock, s, T, L0, c, theta, dmax, rmin, mixed);
}

void launch_coarsen(const Tables &T, TileList LC, int lc, double scale,
                    int mixed, int op, hipStream_t s) {
  if (LC.nblocks) LAUNCH(K_COARSEN, k_coarsen, LC.nblocks, kBlock, s, T, LC, lc, scale, mixed, op);
}

void launch_fin(const Tables &T, int which, int mixed, hipStream_t s, int alt) {
  if (!T.nprob) return;
  if (which == FIN_BB) LAUNCH(K_FIN, k_fin_bb, T.nprob, kFinBlock, s, T, mixed);
  else LAUNCH(K_FIN, k_fin, T.nprob, kFinBlock, s, T, which, mixed, alt);
}

void launch_pre0(const Tables &T, TileList L, int l, int prec, hipStream_t s) {
  if (!L.nblocks) return;
  const int id = l == 0 ? K_PRE0_F : K_PRE0_C;
  if (prec) {
    if (l == 0) LAUNCH(id, (k_pre0<float, true>), L.nblocks, kBlock, s, T, L, l);
    else LAUNCH(id, (k_pre0<float, false>), L.nblocks, kBlock, s, T, L, l);
  } else {
    if (l == 0) LAUNCH(id, (k_pre0<double, true>), L.nblocks, kBlock, s, T, L, l);
    else LAUNCH(id, (k_pre0<double, false>), L.nblocks, kBlock, s, T, L, l);
  }
}

void launch_half(const Tables &T, TileList L, int l, int colour, int prec,
                 hipStream_t s) {
  if (!L.nblocks) return;
  const int id = l == 0 ? K_HALF_F : K_HALF_C;
  if (prec) {
    if (l == 0) LAUNCH(id, (k_half<float, true>), L.nblocks, kBlock, s, T, L, l, colour);
    else LAUNCH(id, (k_half<float, false>), L.nblocks, kBlock, s, T, L, l, colour);
  } else {
    if (l == 0) LAUNCH(id, (k_half<double, true>), L.nblocks, kBlock, s, T, L, l, colour);
    else LAUNCH(id, (k_half<double, false>), L.nblocks, kBlock, s, T, L, l, colour);
  }
}

void launch_half_out(const Tables &T, TileList L0, int prec, int flexible,
                     hipStream_t s) {
  if (!L0.nblocks) return;
  if (prec) LAUNCH(K_HALF_OUT, (k_half_out<float>), L0.nblocks, kBlock, s, T, L0, flexible);
  else LAUNCH(K_HALF_OUT, (k_half_out<double>), L0.nblocks, kBlock, s, T, L0, flexible);
}

void launch_resid_restrict(const Tables &T, TileList LC, int lc, int prec,
                           hipStream_t s) {
  if (!LC.nblocks) return;
  const int id = lc == 1 ? K_RESTRICT_F : K_RESTRICT_C;
  if (prec) {
    if (lc == 1) LAUNCH(id, (k_resid_restrict<float, true>), LC.nblocks, kBlock, s, T, LC, lc);
    else LAUNCH(id, (k_resid_restrict<float, false>), LC.nblocks, kBlock, s, T, LC, lc);
  } else {
    if (lc == 1) LAUNCH(id, (k_resid_restrict<double, true>), LC.nblocks, kBlock, s, T, LC, lc);
    else LAUNCH(id, (k_resid_restrict<double, false>), LC.nblocks, kBlock, s, T, LC, lc);
  }
}

void launch_prolong_black(const Tables &T, TileList L, int l, int prec,
                          int trilinear, hipStream_t s) {
  if (!L.nblocks) return;
  const int id = l == 0 ? K_PROLONG_F : K_PROLONG_C;
  if (prec) {
    if (l == 0) LAUNCH(id, (k_prolong_black<float, true>), L.nblocks, kBlock, s, T, L, l, trilinear);
    else LAUNCH(id, (k_prolong_black<float, false>), L.nblocks, kBlock, s, T, L, l, trilinear);
  } else {
    if (l == 0) LAUNCH(id, (k_prolong_black<double, true>), L.nblocks, kBlock, s, T, L, l, trilinear);
    else LAUNCH(id, (k_prolong_black<double, false>), L.nblocks, kBlock, s, T, L, l, trilinear);
  }
}

void launch_vtail(const Tables &T, int prec, int nu_pre, int nu_post,
                  int trilinear, hipStream_t s) {
  if (!T.nprob) return;
  if (prec)
    LAUNCH(K_COARSE_SOLVE, (k_vtail<float>), T.nprob, kTailBlock, s, T, nu_pre, nu_post, trilinear);
  else
    LAUNCH(K_COARSE_SOLVE, (k_vtail<double>), T.nprob, kTailBlock, s, T, nu_pre, nu_post, trilinear);
}


void launch_spmv_f(const Tables &T, TileList F0, int km, hipStream_t s) {
  if (!F0.nblocks) return;
  if (km == KM_MIX64) LAUNCH(K_SPMV_PX, (k_spmv_f<true, KM_MIX64>), F0.nblocks, kBlock, s, T, F0);
  else LAUNCH(K_SPMV_PX, (k_spmv_f<true, KM_MIX32>), F0.nblocks, kBlock, s, T, F0);
}

void launch_spmv_p(const Tables &T, TileList L0, int lazy, int km, hipStream_t s) {
  if (!L0.nblocks) return;
  if (lazy && km == KM_MIX64) LAUNCH(K_SPMV_PX, (k_spmv_p<true, KM_MIX64>), L0.nblocks, kBlock, s, T, L0);
  else if (lazy) LAUNCH(K_SPMV_PX, (k_spmv_p<true, KM_MIX32>), L0.nblocks, kBlock, s, T, L0);
  else if (km == KM_MIX64) LAUNCH(K_SPMV_P, (k_spmv_p<false, KM_MIX64>), L0.nblocks, kBlock, s, T, L0);
  else if (km == KM_MIX32) LAUNCH(K_SPMV_P, (k_spmv_p<false, KM_MIX32>), L0.nblocks, kBlock, s, T, L0);
  else LAUNCH(K_SPMV_P, (k_spmv_p<false, KM_FP64>), L0.nblocks, kBlock, s, T, L0);
}

void launch_z_out(const Tables &T, TileList L0, double *out, hipStream_t s) {
  if (L0.nblocks) LAUNCH(K_APPLY, k_z_out, L0.nblocks, kBlock, s, T, L0, out);
}

void launch_xfix(const Tables &T, TileList L0, int km, hipStream_t s) {
  if (!L0.nblocks) return;
  if (km == KM_MIX32) LAUNCH(K_XFIX, k_xfix<KM_MIX32>, L0.nblocks, kBlock, s, T, L0);
  else if (km == KM_MIX64) LAUNCH(K_XFIX, k_xfix<KM_MIX64>, L0.nblocks, kBlock, s, T, L0);
  else LAUNCH(K_XFIX, k_xfix<KM_FP64>, L0.nblocks, kBlock, s, T, L0);
}

void launch_update(const Tables &T, TileList L0, int km, hipStream_t s) {
  if (!L0.nblocks) return;
  if (km == KM_MIX32) LAUNCH(K_UPDATE, k_update<KM_MIX32>, L0.nblocks, kBlock, s, T, L0);
  else if (km == KM_MIX64) LAUNCH(K_UPDATE, k_update<KM_MIX64>, L0.nblocks, kBlock, s, T, L0);
  else LAUNCH(K_UPDATE, k_update<KM_FP64>, L0.nblocks, kBlock, s, T, L0);
}

void launch_true_resid(const Tables &T, TileList L0, hipStream_t s) {
  if (L0.nblocks) LAUNCH(K_TRUE_RESID, k_true_resid, L0.nblocks, kBlock, s, T, L0);
}


void launch_lmask(const Tables &T, TileList L0, double coupling, hipStream_t s) {
  if (L0.nblocks) LAUNCH(K_LMASK, k_lmask, L0.nblocks, kBlock, s, T, L0, coupling);
}

void launch_local(const Tables &T, TileList L0, int colour, hipStream_t s) {
  if (L0.nblocks) LAUNCH(K_LOCAL, k_local, L0.nblocks, kBlock, s, T, L0, colour);
}

void launch_warm_x(const Tables &T, TileList L0, hipStream_t s) {
  if (L0.nblocks) LAUNCH(K_WARM_X, k_warm_x, L0.nblocks, kBlock, s, T, L0);
}

void launch_apply(const Tables &T, TileList L0, const double *u, double *out,
                  hipStream_t s) {
  if (L0.nblocks) LAUNCH(K_APPLY, k_apply, L0.nblocks, kBlock, s, T, L0, u, out);
}

void launch_set_r(const Tables &T, TileList L0, const double *r, int prec,
                  hipStream_t s) {
  (void)prec;
  if (L0.nblocks) LAUNCH(K_SET_R, k_set_r, L0.nblocks, kBlock, s, T, L0, r);
}


void launch_jacobi(const Tables &T, TileList L, int l, int prec, int mode,
                   int in_x2, int flexible, hipStream_t s) {
  if (!L.nblocks) return;
  const int id = l ? K_JACOBI_C : mode == 0 ? K_JACOBI0_F : mode == 1 ? K_JACOBI_F : K_JACOBI_OUT;
  if (prec) {
    if (l == 0) LAUNCH(id, (k_jacobi<float, true>), L.nblocks, kBlock, s, T, L, l, mode, in_x2, flexible);
    else LAUNCH(id, (k_jacobi<float, false>), L.nblocks, kBlock, s, T, L, l, mode, in_x2, flexible);
  } else {
    if (l == 0) LAUNCH(id, (k_jacobi<double, true>), L.nblocks, kBlock, s, T, L, l, mode, in_x2, flexible);
    else LAUNCH(id, (k_jacobi<double, false>), L.nblocks, kBlock, s, T, L, l, mode, in_x2, flexible);
  }
}

void launch_prolong_add(const Tables &T, TileList L, int l, int prec,
                        int trilinear, int to_x2, hipStream_t s) {
  if (!L.nblocks) return;
  const int id = l ? K_PROLONG_ADD_C : K_PROLONG_ADD_F;
  if (prec) LAUNCH(id, k_prolong_add<float>, L.nblocks, kBlock, s, T, L, l, trilinear, to_x2);
  else LAUNCH(id, k_prolong_add<double>, L.nblocks, kBlock, s, T, L, l, trilinear, to_x2);
}

void launch_warm_revert(const Tables &T, TileList L0, hipStream_t s) {
  if (L0.nblocks) LAUNCH(K_WARM_REVERT, k_warm_revert, L0.nblocks, kBlock, s, T, L0);
}

void launch_update_E(const Tables &T, TileList L0, double floor, int copy_only,
                     hipStream_t s, int in_solve) {
  if (L0.nblocks)
    LAUNCH(K_UPDATE_E, k_update_E, L0.nblocks, kBlock, s, T, L0, floor, copy_only,
           in_solve);
}

}  // namespace fld

extern "C" {

int32_t fld_profile_num_kernels(void) { return fld::K_NUM; }

const char *fld_profile_kernel_name(int32_t k) {
  return (k >= 0 && k < fld::K_NUM) ? fld::kKernelNames[k] : nullptr;
}

int32_t fld_profile_select(int32_t k) {
  if (k < -2 || k >= fld::K_NUM) return -1;
  for (auto &r : fld::prof::recs) {
    hipEventSynchronize(r.b);
    fld::prof::pool.push_back(r.a);
    fld::prof::pool.push_back(r.b);
  }
  fld::prof::recs.clear();
  fld::prof::sel = k;
  return 0;
}

int32_t fld_profile_read(int32_t k, double *total_ms, int64_t *launches) {
  if (k < 0 || k >= fld::K_NUM) return -1;
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto &r : fld::prof::recs) {
    if (r.k != k) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return -1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -1;
    tot += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return 0;
}

}  // extern "C"
