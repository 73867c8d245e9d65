// Fused V-cycle kernels for one red/black Gauss-Seidel sweep before and after
// the coarse-grid correction (Table 1: 1 pre- and 1 post-relaxation sweep).
//
// With x = 0 on entry to a level, the pre-sweep gives
//   red:   x_r = f / d = y
//   black: x_b = (f + sum_nb T y) / d
// so the residual f - A x vanishes at black cells and equals sum_nb T x_b at
// red cells.  The restriction (sum over the 8 children) therefore needs only
// the red residuals, and the pre-smoothed x never has to be stored: the
// post-sweep's black update reads its red neighbours as y + e(parent) and the
// black cells' own pre-smoothed values are overwritten.  Hence two passes per
// level:
//   k_vdown: y and x_b in LDS -> red residuals -> coarse right-hand side
//   k_vup:   y + e and the new x_b in LDS -> new red values -> x (or z)
// Each block owns a 64 x 16 tile of one level and marches in z through tz
// planes: iteration m loads plane z0 - 2 + m (m = 0 .. tz + 3), forms x_b on
// plane z0 - 3 + m (m >= 2) and finishes plane z0 - 4 + m (m >= 4), so the
// y, x_b and output planes run two and one plane behind the loads.
// Three-plane rolling LDS buffers hold y (tile + 2 halo) and x_b (tile + 1
// halo).  HBM traffic per finest cell: the
// right-hand side and 4 coefficients in, 1/8 coarse out (vdown); the same plus
// the 1/8 coarse correction in and z out (vup).
#include <type_traits>

#include "fld_device.h"

namespace fld {

constexpr int kFX = 64, kFY = 16;          // interior tile
constexpr int kE2X = kFX + 4, kE2Y = kFY + 4;
constexpr int kE1X = kFX + 2, kE1Y = kFY + 2;
constexpr int kE2 = kE2X * kE2Y, kE1 = kE1X * kE1Y;

// periodic wrap of an index at most 2 outside [0, n), n >= 2
__device__ __forceinline__ int wrapi(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Per-thread share of one plane of the tile + 2: at most kU cells, whose
// global loads are issued together (and one plane ahead of their use).
constexpr int kU = (kE2 + kBlock - 1) / kBlock;
// black cells of the tile + 1 per thread (each row of the tile + 1 has an
// even number of cells, half of them black)
constexpr int kB = (kE1 / 2 + kBlock - 1) / kBlock;

template <typename R, bool L0>
struct PlaneRegs {
  using FT = typename std::conditional<L0, double, R>::type;
  FT f[kU];
  R d[kU];
  R e[kU];
};

// Issue the loads of plane pz of the tile + 2 (right-hand side, diagonal and,
// for the up pass, the coarse correction at red cells).
template <typename R, bool L0, bool UP>
__device__ __forceinline__ void load_plane(PlaneRegs<R, L0> &pr, const Tile &t,
                                           int pz, int nx, int ny, int nz,
                                           const FSrc<R, L0> &f, const R *d,
                                           const R *e, bool has_coarse, int cnx,
                                           int cny, int cnz = 1,
                                           bool trilinear = false) {
  const int e2x = t.tx + 4, n2 = e2x * (t.ty + 4);
  const int kz = wrapi(pz, nz);
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int c = threadIdx.x + u * kBlock;
    if (c < n2) {
      const int ey = c / e2x, ex = c - ey * e2x;
      const int ux = t.x0 - 2 + ex, uy = t.y0 - 2 + ey;
      const int gx = wrapi(ux, nx), gy = wrapi(uy, ny);
      const int g = (kz * ny + gy) * nx + gx;
      if constexpr (L0) pr.f[u] = f.r[g];
      else pr.f[u] = f.f[g];
      pr.d[u] = d[g];
      if constexpr (UP) {
        pr.e[u] = (has_coarse && ((ux + uy + pz) & 1) == 0)
                      ? coarse_corr(e, gx, gy, kz, cnx, cny, cnz, trilinear)
                      : (R)0;
      }
    }
  }
}

// y = f / d (+ e for the up pass) into the LDS plane
template <typename R, bool L0, bool UP>
__device__ __forceinline__ void store_plane(const PlaneRegs<R, L0> &pr,
                                            const Tile &t, R *out,
                                            double inv_s) {
  const int e2x = t.tx + 4, n2 = e2x * (t.ty + 4);
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int c = threadIdx.x + u * kBlock;
    if (c < n2) {
      const int ey = c / e2x, ex = c - ey * e2x;
      R fv;
      if constexpr (L0) fv = (R)(pr.f[u] * inv_s);
      else fv = pr.f[u];
      R v = fv * recip(pr.d[u]);
      if constexpr (UP) v += pr.e[u];
      out[ey * kE2X + ex] = v;
    }
  }
}

// Black cells of plane pb over the tile + 1:
//   x_b = v_b + (sum_nb T v_nb) / d_b
// from the LDS planes pb - 1, pb, pb + 1 of v (v = y, or y + e at red cells).
template <typename R>
__device__ __forceinline__ void black_plane(const Tile &t, int pb, int nx,
                                            int ny, int nz, const Coef<R> &C,
                                            const R *vm, const R *v0,
                                            const R *vp, R *xo) {
  const int e1x = t.tx + 2, half = e1x >> 1, nb1 = half * (t.ty + 2);
  const int kb = wrapi(pb, nz);
#pragma unroll
  for (int u = 0; u < kB; ++u) {
    const int c = threadIdx.x + u * kBlock;
    if (c < nb1) {
      const int ey = c / half, h = c - ey * half;
      // the black cell of pair h in row ey: (x0-1+ex) + (y0-1+ey) + pb odd,
      // i.e. ex = 1 + x0 + y0 + ey + pb (mod 2)
      const int ex = 2 * h + ((1 + t.x0 + t.y0 + ey + pb) & 1);
      const int gx = t.x0 - 1 + ex, gy = t.y0 - 1 + ey;
      const Nb n = nbrs(wrapi(gx, nx), wrapi(gy, ny), kb, nx, ny, nz);
      const int s = (ey + 1) * kE2X + (ex + 1);
      const R sum = C.tx[n.c] * v0[s + 1] + C.tx[n.xm] * v0[s - 1] +
                    C.ty[n.c] * v0[s + kE2X] + C.ty[n.ym] * v0[s - kE2X] +
                    C.tz[n.c] * vp[s] + C.tz[n.zm] * vm[s];
      xo[ey * kE1X + ex] = v0[s] + sum * recip(C.d[n.c]);
    }
  }
}

template <typename R, bool L0>
__global__ __launch_bounds__(kBlock) void k_vdown(Tables T, TileList TL, int l) {
  const Tile t = get_tile(TL);
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[l * T.nprob + t.prob];
  const LevelDev Cv = T.lv[(l + 1) * T.nprob + t.prob];
  const ProbDev P = T.pd[t.prob];
  const Coef<R> C = coefs<R>(L);
  const auto f = fsrc<R, L0>(L, P, sc);
  const double inv_s = sc.inv_s;
  R *fc = (R *)Cv.f;
  __shared__ R ys[3][kE2];
  __shared__ R xs[3][kE1];
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  // each thread owns one coarse cell (2 x 2 fine columns) of the tile
  const int ci = threadIdx.x & 31, cj = threadIdx.x >> 5;
  const bool cown = 2 * ci < t.tx && 2 * cj < t.ty;
  PlaneRegs<R, L0> pr;
  load_plane<R, L0, false>(pr, t, t.z0 - 2, nx, ny, nz, f, C.d, nullptr, false, 0, 0);
  R acc = 0;
  for (int m = 0; m < t.tz + 4; ++m) {
    const int pz = t.z0 - 2 + m;
    // (1) y = f / d on plane pz (loaded one iteration ahead)
    store_plane<R, L0, false>(pr, t, ys[m % 3], inv_s);
    if (m + 1 < t.tz + 4)
      load_plane<R, L0, false>(pr, t, pz + 1, nx, ny, nz, f, C.d, nullptr, false, 0, 0);
    __syncthreads();
    // coefficients of the red cells of plane pz - 2, loaded before the black
    // pass so their latency overlaps it
    const int pr2 = pz - 2;
    const bool out = m >= 4 && cown;
    R ctx[2], ctxm[2], cty[2], ctym[2], ctz[2], ctzm[2];
    int cs[2];
    if (out) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int a = (b + pr2) & 1;  // the red cell of row b
        const int lx = 2 * ci + a, ly = 2 * cj + b;
        const Nb n = nbrs(t.x0 + lx, t.y0 + ly, pr2, nx, ny, nz);
        cs[b] = (ly + 1) * kE1X + (lx + 1);
        ctx[b] = C.tx[n.c];
        ctxm[b] = C.tx[n.xm];
        cty[b] = C.ty[n.c];
        ctym[b] = C.ty[n.ym];
        ctz[b] = C.tz[n.c];
        ctzm[b] = C.tz[n.zm];
      }
    }
    // (2) black cells of plane pz - 1 over the tile + 1
    if (m >= 2) {
      black_plane<R>(t, pz - 1, nx, ny, nz, C, ys[(m + 1) % 3], ys[(m + 2) % 3],
                     ys[m % 3], xs[m % 3]);
      __syncthreads();
    }
    // (3) red residuals of plane pz - 2, summed into the coarse cell
    if (out) {
      const R *xm = xs[(m + 1) % 3], *x0 = xs[(m + 2) % 3], *xp = xs[m % 3];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int s = cs[b];
        acc += ctx[b] * x0[s + 1] + ctxm[b] * x0[s - 1] + cty[b] * x0[s + kE1X] +
               ctym[b] * x0[s - kE1X] + ctz[b] * xp[s] + ctzm[b] * xm[s];
      }
      if ((pr2 - t.z0) & 1) {
        fc[((pr2 >> 1) * Cv.ny + (t.y0 >> 1) + cj) * Cv.nx + (t.x0 >> 1) + ci] = acc;
        acc = 0;
      }
    }
  }
}

// TRI selects trilinear prolongation of the coarse correction (at compile
// time: the piecewise-constant variant keeps its lower register count).
template <typename R, bool L0, bool TRI>
__global__ __launch_bounds__(kBlock) void k_vup(Tables T, TileList TL, int l,
                                                int flexible) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  const LevelDev L = T.lv[l * T.nprob + t.prob];
  const ProbDev P = T.pd[t.prob];
  const bool has_coarse = l + 1 < P.levels;
  const LevelDev Cl = T.lv[(has_coarse ? l + 1 : l) * T.nprob + t.prob];
  const Coef<R> C = coefs<R>(L);
  const auto f = fsrc<R, L0>(L, P, sc);
  const double inv_s = sc.inv_s;
  const R *e = (const R *)Cl.x;
  R *xout = (R *)L.x;
  const double s_out = sc.s;
  __shared__ R vs[3][kE2];
  __shared__ R xs[3][kE1];
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int cnx = Cl.nx, cny = Cl.ny, cnz = Cl.nz;
  constexpr bool tri = TRI;
  const int ci = threadIdx.x & 31, cj = threadIdx.x >> 5;
  const bool cown = 2 * ci < t.tx && 2 * cj < t.ty;
  PlaneRegs<R, L0> pr;
  load_plane<R, L0, true>(pr, t, t.z0 - 2, nx, ny, nz, f, C.d, e, has_coarse, cnx,
                          cny, cnz, tri);
  double rz = 0.0, rzo = 0.0;
  for (int m = 0; m < t.tz + 4; ++m) {
    const int pz = t.z0 - 2 + m;
    // (1) v = y at black cells, y + e(parent) at red cells (loaded ahead)
    store_plane<R, L0, true>(pr, t, vs[m % 3], inv_s);
    if (m + 1 < t.tz + 4)
      load_plane<R, L0, true>(pr, t, pz + 1, nx, ny, nz, f, C.d, e, has_coarse,
                              cnx, cny, cnz, tri);
    __syncthreads();
    // (2) new black values of plane pz - 1 over the tile + 1
    if (m >= 2) {
      black_plane<R>(t, pz - 1, nx, ny, nz, C, vs[(m + 1) % 3], vs[(m + 2) % 3],
                     vs[m % 3], xs[m % 3]);
      __syncthreads();
    }
    // (3) plane pz - 2 on the tile: new red values from the new black ones;
    //     every cell is written (finest level: z = s x in FP64 plus dots)
    if (m >= 4 && cown) {
      const int pr2 = pz - 2;
      const R *xm = xs[(m + 1) % 3], *x0 = xs[(m + 2) % 3], *xp = xs[m % 3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = u & 1, b = u >> 1;
        const int lx = 2 * ci + a, ly = 2 * cj + b;
        const int s = (ly + 1) * kE1X + (lx + 1);
        const Nb n = nbrs(t.x0 + lx, t.y0 + ly, pr2, nx, ny, nz);
        R v;
        if (((a + b + pr2) & 1) == 0) {
          const R sum = C.tx[n.c] * x0[s + 1] + C.tx[n.xm] * x0[s - 1] +
                        C.ty[n.c] * x0[s + kE1X] + C.ty[n.ym] * x0[s - kE1X] +
                        C.tz[n.c] * xp[s] + C.tz[n.zm] * xm[s];
          v = (f(n.c) + sum) * recip(C.d[n.c]);
        } else {
          v = x0[s];
        }
        if constexpr (L0) {
          const double z = (double)v * s_out;
          const double r = P.r[n.c];
          if (flexible) rzo += r * P.z[n.c];
          P.z[n.c] = z;
          rz += r * z;
        } else {
          xout[n.c] = v;
        }
      }
    }
  }
  if constexpr (L0) write_partials(T, tid, rz, rzo);
}

// launchers ------------------------------------------------------------------

void launch_vdown(const Tables &T, TileList L, int l, int prec, hipStream_t s) {
  if (!L.nblocks) return;
  const int id = l == 0 ? K_VDOWN_F : K_VDOWN_C;
  if (prec) {
    if (l == 0) FLD_LAUNCH(id, (k_vdown<float, true>), L.nblocks, kBlock, s, T, L, l);
    else FLD_LAUNCH(id, (k_vdown<float, false>), L.nblocks, kBlock, s, T, L, l);
  } else {
    if (l == 0) FLD_LAUNCH(id, (k_vdown<double, true>), L.nblocks, kBlock, s, T, L, l);
    else FLD_LAUNCH(id, (k_vdown<double, false>), L.nblocks, kBlock, s, T, L, l);
  }
}

template <typename R, bool L0>
static void launch_vup_t(const Tables &T, TileList L, int l, int id, int flexible,
                         int trilinear, hipStream_t s) {
  if (trilinear)
    FLD_LAUNCH(id, (k_vup<R, L0, true>), L.nblocks, kBlock, s, T, L, l, flexible);
  else
    FLD_LAUNCH(id, (k_vup<R, L0, false>), L.nblocks, kBlock, s, T, L, l, flexible);
}

void launch_vup(const Tables &T, TileList L, int l, int prec, int flexible,
                int trilinear, hipStream_t s) {
  if (!L.nblocks) return;
  const int id = l == 0 ? K_VUP_F : K_VUP_C;
  if (prec) {
    if (l == 0) launch_vup_t<float, true>(T, L, l, id, flexible, trilinear, s);
    else launch_vup_t<float, false>(T, L, l, id, flexible, trilinear, s);
  } else {
    if (l == 0) launch_vup_t<double, true>(T, L, l, id, flexible, trilinear, s);
    else launch_vup_t<double, false>(T, L, l, id, flexible, trilinear, s);
  }
}

}  // namespace fld
