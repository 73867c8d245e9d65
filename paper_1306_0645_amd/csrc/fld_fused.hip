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
// halo).
//
// Every face coefficient joins one red and one black cell, so both
// half-sweeps of a plane read all of them, one z-step apart; between the two
// reads a block streams more than its share of the XCD's L2, so re-reading
// them from memory doubles the coefficient traffic.  Instead thread
// (ci, cj) = (tid & 31, tid >> 5) owns the 2 x 2 columns
// x = x0 + 2ci + a, y = y0 + 2cj + b (a, b in {0, 1}) of the tile: it loads
// their right-hand side, diagonal and faces once per plane with 2-wide vector
// loads (plus the -x faces of its a = 0 cells and the -y faces of its b = 0
// cells, which share cache lines with its neighbours' loads, issued at the
// same time) and keeps them in registers from the black pass of a plane to
// its red pass.  The black cells of the ring just outside the tile, which the
// red cells on the tile's edge need, are done by every third thread from
// loads of their own, and the tile + 2 halo of the y plane by a linear map
// over the halo cells.  HBM traffic per finest cell: the right-hand side and
// 4 coefficients in, 1/8 coarse out (vdown); the same plus the 1/8 coarse
// correction in, the right-hand side read again for the output, and z out
// (vup).
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

template <typename R>
using Vec2 = R __attribute__((ext_vector_type(2)));

template <typename R>
__device__ __forceinline__ void ld2(const R *p, R &u, R &v) {
  const Vec2<R> w = *reinterpret_cast<const Vec2<R> *>(p);
  u = w.x;
  v = w.y;
}

template <typename R>
__device__ __forceinline__ void st2(R *p, R u, R v) {
  Vec2<R> w;
  w.x = u;
  w.y = v;
  *reinterpret_cast<Vec2<R> *>(p) = w;
}

// in-plane faces of one quad: Tx, Ty at (a, b) (the + faces of each cell),
// the -x faces of the a = 0 cells and the -y faces of the b = 0 cells
template <typename R>
struct QFace {
  R x00, x10, x01, x11, xl0, xl1;
  R y00, y10, y01, y11, yb0, yb1;
};

// one plane's Tz, diagonal reciprocal, ... of a quad, cell (a, b) = vab
template <typename R>
struct Q4 {
  R v00, v10, v01, v11;
};

// the 6 faces of cell (a, b) of the quad, a = a1 (run time), b = B
template <typename R>
struct Faces6 {
  R xp, xm, yp, ym, zp, zm;
};

template <int B, typename R>
__device__ __forceinline__ Faces6<R> cell_faces(const QFace<R> &F, const Q4<R> &Zp,
                                               const Q4<R> &Zm, bool a1) {
  Faces6<R> f;
  if constexpr (B == 0) {
    f.xp = a1 ? F.x10 : F.x00;
    f.xm = a1 ? F.x00 : F.xl0;
    f.yp = a1 ? F.y10 : F.y00;
    f.ym = a1 ? F.yb1 : F.yb0;
    f.zp = a1 ? Zp.v10 : Zp.v00;
    f.zm = a1 ? Zm.v10 : Zm.v00;
  } else {
    f.xp = a1 ? F.x11 : F.x01;
    f.xm = a1 ? F.x01 : F.xl1;
    f.yp = a1 ? F.y11 : F.y01;
    f.ym = a1 ? F.y10 : F.y00;
    f.zp = a1 ? Zp.v11 : Zp.v01;
    f.zm = a1 ? Zm.v11 : Zm.v01;
  }
  return f;
}

template <int B, typename R>
__device__ __forceinline__ R pick(const Q4<R> &q, bool a1) {
  if constexpr (B == 0) return a1 ? q.v10 : q.v00;
  else return a1 ? q.v11 : q.v01;
}

template <typename R>
__device__ __forceinline__ void load_faces(QFace<R> &F, Q4<R> &Z, const Coef<R> &C,
                                           int kz, int qx, int qy, int qxl,
                                           int qyb, int nx, int ny, bool inplane) {
  const int r0 = (kz * ny + qy) * nx, r1 = r0 + nx;
  if (inplane) {
    ld2(C.tx + r0 + qx, F.x00, F.x10);
    ld2(C.tx + r1 + qx, F.x01, F.x11);
    F.xl0 = C.tx[r0 + qxl];
    F.xl1 = C.tx[r1 + qxl];
    ld2(C.ty + r0 + qx, F.y00, F.y10);
    ld2(C.ty + r1 + qx, F.y01, F.y11);
    ld2(C.ty + (kz * ny + qyb) * nx + qx, F.yb0, F.yb1);
  }
  ld2(C.tz + r0 + qx, Z.v00, Z.v10);
  ld2(C.tz + r1 + qx, Z.v01, Z.v11);
}

// halo cell q of the tile + 2 frame (the cells outside the tile): LDS
// coordinates (ex, ey)
__device__ __forceinline__ void halo_cell(int q, int tx, int ty, int &ex, int &ey) {
  const int e2x = tx + 4;
  if (q < 2 * e2x) {
    ey = q / e2x;
    ex = q - ey * e2x;
  } else if (q < 4 * e2x) {
    const int r = q - 2 * e2x, ry = r / e2x;
    ey = ty + 2 + ry;
    ex = r - ry * e2x;
  } else {
    const int r = q - 4 * e2x, c = r & 3;
    ey = 2 + (r >> 2);
    ex = c < 2 ? c : tx + c;
  }
}

// black cell q (of tx + ty) of the ring just outside the tile on a plane of
// parity pp, in the tile + 1 frame: rows y0 - 1 and y0 + ty, then columns
// x0 - 1 and x0 + tx (x0, y0 and the extents are even)
__device__ __forceinline__ void ring_black(int q, int tx, int ty, int pp, int &ex,
                                           int &ey) {
  const int hx = tx >> 1, hy = ty >> 1;
  if (q < hx) {
    ey = 0;
    ex = 1 + 2 * q + pp;
  } else if (q < 2 * hx) {
    ey = ty + 1;
    ex = 2 + 2 * (q - hx) - pp;
  } else if (q < 2 * hx + hy) {
    ex = 0;
    ey = 1 + 2 * (q - 2 * hx) + pp;
  } else {
    ex = tx + 1;
    ey = 2 + 2 * (q - 2 * hx - hy) - pp;
  }
}

// the 7 coefficients of one ring black cell
template <typename R>
struct RingCoef {
  R d, xp, xm, yp, ym, zp, zm;
  int ex, ey;
};

template <typename R>
__device__ __forceinline__ void load_ring(RingCoef<R> &rc, const Coef<R> &C,
                                          const Tile &t, int q, int pb, int nx,
                                          int ny, int nz) {
  ring_black(q, t.tx, t.ty, pb & 1, rc.ex, rc.ey);
  const Nb n = nbrs(wrapi(t.x0 - 1 + rc.ex, nx), wrapi(t.y0 - 1 + rc.ey, ny),
                    wrapi(pb, nz), nx, ny, nz);
  rc.d = C.d[n.c];
  rc.xp = C.tx[n.c];
  rc.xm = C.tx[n.xm];
  rc.yp = C.ty[n.c];
  rc.ym = C.ty[n.ym];
  rc.zp = C.tz[n.c];
  rc.zm = C.tz[n.zm];
}

// x_b = v_b + (sum_nb T v_nb) / d_b at LDS offset s of the tile + 2 frame
template <typename R>
__device__ __forceinline__ R black_value(const Faces6<R> &f, R idv, const R *vm,
                                         const R *v0, const R *vp, int s) {
  const R sum = f.xp * v0[s + 1] + f.xm * v0[s - 1] + f.yp * v0[s + kE2X] +
                f.ym * v0[s - kE2X] + f.zp * vp[s] + f.zm * vm[s];
  return v0[s] + sum * idv;
}

// sum_nb T x_nb over the black neighbours at LDS offset s of the tile + 1 frame
template <typename R>
__device__ __forceinline__ R red_sum(const Faces6<R> &f, const R *xm, const R *x0,
                                     const R *xp, int s) {
  return f.xp * x0[s + 1] + f.xm * x0[s - 1] + f.yp * x0[s + kE1X] +
         f.ym * x0[s - kE1X] + f.zp * xp[s] + f.zm * xm[s];
}

constexpr int kHalo = (4 * (kFX + 4) + 4 * kFY + kBlock - 1) / kBlock;

// right-hand side, diagonal (and coarse correction) of one plane: the quad's
// 4 cells and this thread's halo cells
template <typename R, bool L0, bool UP>
struct QPlane {
  using FT = typename std::conditional<L0, double, R>::type;
  FT f00, f10, f01, f11;
  R d00, d10, d01, d11;
  R e0, e1;  // coarse correction at the red cells of rows 0 and 1
  FT hf[kHalo];
  R hd[kHalo], he[kHalo];
};

// Trilinear correction (3/4 own parent, 1/4 the neighbour on the fine cell's
// side, per direction) from coarse planes staged in LDS: slot c % 3 holds
// relative coarse plane c, that is plane z0 / 2 - 2 + c, over the tile's
// coarse columns x0 / 2 - 2 .. (x0 + tx) / 2 + 1 and rows
// y0 / 2 - 2 .. (y0 + ty) / 2 + 1, which covers the parents and the
// interpolation neighbours of the tile and its 2-cell halo.  A fine cell at
// tile-frame offset (ex, ey) of the tile + 2 frame (or a quad cell, offset
// (2 ci + a + 2, 2 cj + b + 2)) has its parent at (ex / 2 + 1, ey / 2 + 1) of
// the staged region, since x0 and y0 are even.  c0, c1: the slots of the
// fine plane's parent plane and of the plane on its side.  The weights are
// combined in the order coarse_corr uses.
constexpr int kCX = kFX / 2 + 4, kCY = kFY / 2 + 4, kC = kCX * kCY;
constexpr int kCR = (kC + kBlock - 1) / kBlock;

template <typename R>
__device__ __forceinline__ R tri_at(const R *c0, const R *c1, int I, int I2, int J,
                                    int J2) {
  const int r0 = J * kCX, r1 = J2 * kCX;
  const R a = (R)0.75, b = (R)0.25;
  const R zK = a * (a * c0[r0 + I] + b * c0[r0 + I2]) + b * (a * c0[r1 + I] + b * c0[r1 + I2]);
  const R zK2 = a * (a * c1[r0 + I] + b * c1[r0 + I2]) + b * (a * c1[r1 + I] + b * c1[r1 + I2]);
  return a * zK + b * zK2;
}

// correction at offset (ex, ey) of the tile + 2 frame
template <typename R>
__device__ __forceinline__ R tri_frame(const R *c0, const R *c1, int ex, int ey) {
  const int I = (ex >> 1) + 1, J = (ey >> 1) + 1;
  return tri_at(c0, c1, I, (ex & 1) ? I + 1 : I - 1, J, (ey & 1) ? J + 1 : J - 1);
}

// Staging of one coarse plane: thread slot u covers entry q = tid + u kBlock
// of the kCX x kCY region (row-major, so q is also its LDS offset); its
// in-plane source offset is the same on every plane and is computed once.
// The global loads go to registers first and to LDS later, so that their
// latency overlaps other work.
template <typename R>
struct CStage {
  int off[kCR];
  R v[kCR];
};

__device__ __forceinline__ int pmod(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

template <typename R>
__device__ __forceinline__ void cstage_init(CStage<R> &cv, const Tile &t, int cnx, int cny) {
  const int I0 = (t.x0 >> 1) - 2, J0 = (t.y0 >> 1) - 2;
#pragma unroll
  for (int u = 0; u < kCR; ++u) {
    const int q = threadIdx.x + u * kBlock, jy = q / kCX, ix = q - jy * kCX;
    cv.off[u] = pmod(J0 + jy, cny) * cnx + pmod(I0 + ix, cnx);
  }
}

template <typename R>
__device__ __forceinline__ void cstage_load(CStage<R> &cv, const R *e, int c, int cnx,
                                            int cny, int cnz) {
  const R *pl = e + (size_t)pmod(c, cnz) * cny * cnx;
#pragma unroll
  for (int u = 0; u < kCR; ++u)
    if (threadIdx.x + u * kBlock < kC) cv.v[u] = pl[cv.off[u]];
}

template <typename R>
__device__ __forceinline__ void cstage_store(const CStage<R> &cv, R *dst) {
#pragma unroll
  for (int u = 0; u < kCR; ++u) {
    const int q = threadIdx.x + u * kBlock;
    if (q < kC) dst[q] = cv.v[u];
  }
}

// the up pass of a trilinear cycle (TRI) takes its coarse correction at the
// store (q_store_plane), from the staged coarse planes
template <typename R, bool L0, bool UP, bool TRI>
__device__ __forceinline__ void q_load_plane(
    QPlane<R, L0, UP> &pl, const Tile &t, int pz, bool qon, int qx, int qy,
    int nx, int ny, int nz, const FSrc<R, L0> &f, const R *d, const R *e,
    bool has_coarse, int cnx, int cny, int cnz) {
  const int kz = wrapi(pz, nz);
  if (qon) {
    const int r0 = (kz * ny + qy) * nx + qx, r1 = r0 + nx;
    if constexpr (L0) {
      ld2(f.r + r0, pl.f00, pl.f10);
      ld2(f.r + r1, pl.f01, pl.f11);
    } else {
      ld2(f.f + r0, pl.f00, pl.f10);
      ld2(f.f + r1, pl.f01, pl.f11);
    }
    ld2(d + r0, pl.d00, pl.d10);
    ld2(d + r1, pl.d01, pl.d11);
    if constexpr (UP && !TRI) {
      pl.e0 = pl.e1 = has_coarse ? coarse_corr(e, qx, qy, kz, cnx, cny, cnz, false) : (R)0;
    }
  }
  const int e2x = t.tx + 4, nh = 4 * e2x + 4 * t.ty;
#pragma unroll
  for (int u = 0; u < kHalo; ++u) {
    const int q = threadIdx.x + u * kBlock;
    if (q < nh) {
      int ex, ey;
      halo_cell(q, t.tx, t.ty, ex, ey);
      const int ux = t.x0 - 2 + ex, uy = t.y0 - 2 + ey;
      const int gx = wrapi(ux, nx), gy = wrapi(uy, ny);
      const int g = (kz * ny + gy) * nx + gx;
      if constexpr (L0) pl.hf[u] = f.r[g];
      else pl.hf[u] = f.f[g];
      pl.hd[u] = d[g];
      if constexpr (UP && !TRI) {
        pl.he[u] = (has_coarse && ((ux + uy + pz) & 1) == 0)
                       ? coarse_corr(e, gx, gy, kz, cnx, cny, cnz, false)
                       : (R)0;
      }
    }
  }
}

// q of plane pz at the quad's cells and this thread's halo cells (same cells
// as q_load_plane)
__device__ __forceinline__ void q_load_q(double (&qq)[4], double (&hq)[kHalo],
                                         const double *q, const Tile &t, int pz,
                                         bool qon, int qx, int qy, int nx, int ny,
                                         int nz) {
  const int kz = wrapi(pz, nz);
  if (qon) {
    const int r0 = (kz * ny + qy) * nx + qx;
    ld2(q + r0, qq[0], qq[1]);
    ld2(q + r0 + nx, qq[2], qq[3]);
  }
  const int e2x = t.tx + 4, nh = 4 * e2x + 4 * t.ty;
#pragma unroll
  for (int u = 0; u < kHalo; ++u) {
    const int c = threadIdx.x + u * kBlock;
    if (c < nh) {
      int ex, ey;
      halo_cell(c, t.tx, t.ty, ex, ey);
      const int gx = wrapi(t.x0 - 2 + ex, nx), gy = wrapi(t.y0 - 2 + ey, ny);
      hq[u] = q[(kz * ny + gy) * nx + gx];
    }
  }
}

template <typename R, bool L0>
__device__ __forceinline__ R scaled(typename QPlane<R, L0, false>::FT v, double inv_s) {
  if constexpr (L0) return (R)(v * inv_s);
  else return v;
}

// y = f / d (+ e at red cells for the up pass) into the LDS plane; returns
// the quad's diagonal reciprocals.  TRI (up pass, has_coarse): e from the
// staged coarse planes cs
template <typename R, bool L0, bool UP, bool TRI = false>
__device__ __forceinline__ Q4<R> q_store_plane(const QPlane<R, L0, UP> &pl,
                                               const Tile &t, int pz, bool qon,
                                               int ci, int cj, R *out,
                                               double inv_s, bool has_coarse = false,
                                               const R (*cs)[kC] = nullptr) {
  const R *c0 = nullptr, *c1 = nullptr;
  if constexpr (TRI) {
    const int K = (pz >> 1) - (t.z0 >> 1) + 2;
    c0 = cs[K % 3];
    c1 = cs[((pz & 1) ? K + 1 : K - 1) % 3];
  }
  Q4<R> id;
  if (qon) {
    id.v00 = recip(pl.d00);
    id.v10 = recip(pl.d10);
    id.v01 = recip(pl.d01);
    id.v11 = recip(pl.d11);
    R y00 = scaled<R, L0>(pl.f00, inv_s) * id.v00;
    R y10 = scaled<R, L0>(pl.f10, inv_s) * id.v10;
    R y01 = scaled<R, L0>(pl.f01, inv_s) * id.v01;
    R y11 = scaled<R, L0>(pl.f11, inv_s) * id.v11;
    if constexpr (UP) {
      R e0 = (R)0, e1 = (R)0;
      if constexpr (TRI) {
        if (has_coarse) {
          // red cells: row 0 at a = pp, row 1 at a = 1 - pp
          const int pp = pz & 1, ex = 2 * ci + 2, ey = 2 * cj + 2;
          e0 = tri_frame(c0, c1, ex + pp, ey);
          e1 = tri_frame(c0, c1, ex + 1 - pp, ey + 1);
        }
      } else {
        e0 = pl.e0;
        e1 = pl.e1;
      }
      if (pz & 1) {  // red: (1, 0) and (0, 1)
        y10 += e0;
        y01 += e1;
      } else {       // red: (0, 0) and (1, 1)
        y00 += e0;
        y11 += e1;
      }
    }
    const int s = (2 * cj + 2) * kE2X + 2 * ci + 2;
    out[s] = y00;
    out[s + 1] = y10;
    out[s + kE2X] = y01;
    out[s + kE2X + 1] = y11;
  }
  const int e2x = t.tx + 4, nh = 4 * e2x + 4 * t.ty;
#pragma unroll
  for (int u = 0; u < kHalo; ++u) {
    const int q = threadIdx.x + u * kBlock;
    if (q < nh) {
      int ex, ey;
      halo_cell(q, t.tx, t.ty, ex, ey);
      R v = scaled<R, L0>(pl.hf[u], inv_s) * recip(pl.hd[u]);
      if constexpr (UP) {
        if constexpr (TRI) {
          if (has_coarse && ((ex + ey + pz) & 1) == 0) v += tri_frame(c0, c1, ex, ey);
        } else {
          v += pl.he[u];
        }
      }
      out[ey * kE2X + ex] = v;
    }
  }
  return id;
}

template <typename R, bool L0>
__global__ __launch_bounds__(kBlock) void k_vdown(Tables T, TileList TL, int l,
                                                  int sel) {
  const int tid = get_tile_index(TL);
  const Tile t = TL.base[tid];
  const Scal &sc = T.sc[t.prob];
  if (!sc.active) return;
  if ((sel == VD_FRESH && !sc.fresh) || (sel == VD_CONT && sc.fresh)) return;
  const LevelDev L = T.lv[l * T.nprob + t.prob];
  const ProbDev P = T.pd[t.prob];
  // a one-level problem runs this pass only for the residual update
  const bool has_coarse = l + 1 < P.levels;
  const LevelDev Cv = T.lv[(has_coarse ? l + 1 : l) * T.nprob + t.prob];
  const Coef<R> C = coefs<R>(L);
  const auto f = fsrc<R, L0>(L, P, sc);
  const double inv_s = sc.inv_s;
  R *fc = (R *)Cv.f;
  __shared__ R ys[3][kE2];
  __shared__ R xs[3][kE1];
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int ci = threadIdx.x & 31, cj = threadIdx.x >> 5;
  const bool qon = 2 * ci < t.tx && 2 * cj < t.ty;
  const int qx = t.x0 + 2 * ci, qy = t.y0 + 2 * cj;
  const int qxl = wrapi(qx - 1, nx), qyb = wrapi(qy - 1, ny);
  const int rq = threadIdx.x / 3;
  const bool ron = threadIdx.x == 3 * rq && rq < t.tx + t.ty;
  // finest level of the fused PCG iteration: this iteration's residual is
  // r - alpha q (alpha, q of the previous iteration), formed on the fly for
  // every y plane, halo included, and written to the other residual buffer
  // for the tile's own cells, with its partial ||.||^2
  // (mixed precision only: the FP64 iteration updates r in a pass of its own)
  constexpr bool kUpd = L0 && sizeof(R) == 4;
  const bool upd = kUpd && sc.has_dir;
  const double alpha = sc.alpha;
  const double *qv = P.q;
  double *rn = rnext(P, sc);
  double qq[4] = {0.0, 0.0, 0.0, 0.0}, hq[kHalo] = {};
  double rr = 0.0;
  QPlane<R, L0, false> pl;
  q_load_plane<R, L0, false, false>(pl, t, t.z0 - 2, qon, qx, qy, nx, ny, nz, f,
                                    C.d, nullptr, false, 0, 0, 0);
  if constexpr (kUpd) {
    if (upd) q_load_q(qq, hq, qv, t, t.z0 - 2, qon, qx, qy, nx, ny, nz);
  }
  QFace<R> Fb{}, Fr{};  // in-plane faces of planes pz - 1 (black), pz - 2 (red)
  Q4<R> Zb{}, Zr{}, Zrm{};  // Tz of planes pz - 1, pz - 2, pz - 3
  Q4<R> I0{}, I1{};  // diagonal reciprocals of planes pz, pz - 1
  RingCoef<R> rc{};
  R acc = 0;
  for (int m = 0; m < t.tz + 4; ++m) {
    const int pz = t.z0 - 2 + m, pb = pz - 1, pr2 = pz - 2;
    Fr = Fb;
    Zrm = Zr;
    Zr = Zb;
    // faces of plane pb (its Tz only at m = 1: the -z face of plane pb + 1)
    if (m >= 1 && qon)
      load_faces(Fb, Zb, C, wrapi(pb, nz), qx, qy, qxl, qyb, nx, ny, m >= 2);
    if (m >= 2 && ron) load_ring(rc, C, t, rq, pb, nx, ny, nz);
    // (1) y = f / d on plane pz (loaded one iteration ahead)
    if constexpr (kUpd) {
      if (upd) {
        pl.f00 = __builtin_fma(-alpha, qq[0], pl.f00);
        pl.f10 = __builtin_fma(-alpha, qq[1], pl.f10);
        pl.f01 = __builtin_fma(-alpha, qq[2], pl.f01);
        pl.f11 = __builtin_fma(-alpha, qq[3], pl.f11);
#pragma unroll
        for (int u = 0; u < kHalo; ++u) pl.hf[u] = __builtin_fma(-alpha, hq[u], pl.hf[u]);
        if (qon && pz >= t.z0 && pz < t.z0 + t.tz) {
          const int r0 = (pz * ny + qy) * nx + qx;
          st2(rn + r0, pl.f00, pl.f10);
          st2(rn + r0 + nx, pl.f01, pl.f11);
          rr += pl.f00 * pl.f00;
          rr += pl.f10 * pl.f10;
          rr += pl.f01 * pl.f01;
          rr += pl.f11 * pl.f11;
        }
      }
    }
    I1 = I0;
    I0 = q_store_plane<R, L0, false>(pl, t, pz, qon, ci, cj, ys[m % 3], inv_s);
    if (m + 1 < t.tz + 4) {
      q_load_plane<R, L0, false, false>(pl, t, pz + 1, qon, qx, qy, nx, ny, nz, f,
                                        C.d, nullptr, false, 0, 0, 0);
      if constexpr (kUpd) {
        if (upd) q_load_q(qq, hq, qv, t, pz + 1, qon, qx, qy, nx, ny, nz);
      }
    }
    __syncthreads();
    // (2) black cells of plane pb over the tile + 1
    if (m >= 2) {
      const R *vm = ys[(m + 1) % 3], *v0 = ys[(m + 2) % 3], *vp = ys[m % 3];
      R *xo = xs[m % 3];
      if (qon) {
        const bool b0 = (pb & 1) == 0, b1 = !b0;  // a of the black cell of rows 0, 1
        const int s = (2 * cj + 2) * kE2X + 2 * ci + 2;
        const int o = (2 * cj + 1) * kE1X + 2 * ci + 1;
        xo[o + b0] = black_value(cell_faces<0>(Fb, Zb, Zr, b0), pick<0>(I1, b0), vm,
                                 v0, vp, s + b0);
        xo[o + kE1X + b1] = black_value(cell_faces<1>(Fb, Zb, Zr, b1),
                                        pick<1>(I1, b1), vm, v0, vp, s + kE2X + b1);
      }
      if (ron) {
        const Faces6<R> fr{rc.xp, rc.xm, rc.yp, rc.ym, rc.zp, rc.zm};
        xo[rc.ey * kE1X + rc.ex] = black_value(fr, recip(rc.d), vm, v0, vp,
                                               (rc.ey + 1) * kE2X + rc.ex + 1);
      }
      __syncthreads();
    }
    // (3) red residuals of plane pr2, summed into the coarse cell
    if (m >= 4 && qon) {
      const R *xm = xs[(m + 1) % 3], *x0 = xs[(m + 2) % 3], *xp = xs[m % 3];
      const bool r0 = (pr2 & 1) != 0, r1 = !r0;  // a of the red cell of rows 0, 1
      const int o = (2 * cj + 1) * kE1X + 2 * ci + 1;
      acc += red_sum(cell_faces<0>(Fr, Zr, Zrm, r0), xm, x0, xp, o + r0);
      acc += red_sum(cell_faces<1>(Fr, Zr, Zrm, r1), xm, x0, xp, o + kE1X + r1);
      if ((pr2 - t.z0) & 1) {
        if (has_coarse)
          fc[((pr2 >> 1) * Cv.ny + (t.y0 >> 1) + cj) * Cv.nx + (t.x0 >> 1) + ci] = acc;
        acc = 0;
      }
    }
  }
  if constexpr (kUpd) write_partials(T, tid, rr, 0.0);
}

// Three blocks per CU: the mixed trilinear finest instance would otherwise
// take more registers than that leaves (measured at 640^3: 2.35 ms a launch
// with three blocks and a few spilled registers, 2.64 ms with two).  The FP64
// instances need more registers than three blocks allow whatever the bound.
template <typename R, bool L0, bool TRI>
__global__ __launch_bounds__(kBlock, 3) void k_vup(Tables T, TileList TL, int l,
                                                int flexible) {
  using FT = typename QPlane<R, L0, true>::FT;
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
  // flexible PCG needs r.z_old, except where the PCG (re)starts (beta = 0);
  // the mixed form keeps z as the cycle's FP32 output, z = zscale z32
  const bool rd_old = flexible && !sc.restart;
  const double zs_old = sc.zscale;
  __shared__ R vs[3][kE2];
  __shared__ R xs[3][kE1];
  // trilinear: the coarse planes under the tile, a ring of 3 (corr_lds); the
  // fine plane loaded in iteration m needs relative coarse planes m / 2 + 1
  // and m / 2 + 2, so plane j + 2 is staged in iteration 2j - 1, after the
  // last read of the slot it replaces (iteration 2j - 3) and a barrier before
  // its first read (iteration 2j)
  __shared__ R cs[TRI ? 3 : 1][kC];
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int cnx = Cl.nx, cny = Cl.ny, cnz = Cl.nz;
  const int ci = threadIdx.x & 31, cj = threadIdx.x >> 5;
  const bool qon = 2 * ci < t.tx && 2 * cj < t.ty;
  const int qx = t.x0 + 2 * ci, qy = t.y0 + 2 * cj;
  const int qxl = wrapi(qx - 1, nx), qyb = wrapi(qy - 1, ny);
  const int rq = threadIdx.x / 3;
  const bool ron = threadIdx.x == 3 * rq && rq < t.tx + t.ty;
  const int cbase = (t.z0 >> 1) - 2;
  CStage<R> cv;
  if constexpr (TRI) {
    if (has_coarse) {
      // the first three planes: all loads in flight before the first store
      cstage_init(cv, t, cnx, cny);
      CStage<R> c1 = cv, c2 = cv;
      cstage_load(cv, e, cbase, cnx, cny, cnz);
      cstage_load(c1, e, cbase + 1, cnx, cny, cnz);
      cstage_load(c2, e, cbase + 2, cnx, cny, cnz);
      cstage_store(cv, cs[0]);
      cstage_store(c1, cs[1]);
      cstage_store(c2, cs[2]);
      __syncthreads();
    }
  }
  QPlane<R, L0, true> pl;
  q_load_plane<R, L0, true, TRI>(pl, t, t.z0 - 2, qon, qx, qy, nx, ny, nz, f, C.d, e,
                                 has_coarse, cnx, cny, cnz);
  QFace<R> Fb{}, Fr{};
  Q4<R> Zb{}, Zr{}, Zrm{};
  Q4<R> I0{}, I1{}, I2{};   // diagonal reciprocals of planes pz, pz - 1, pz - 2
  RingCoef<R> rc{};
  double rz = 0.0, rzo = 0.0;
  for (int m = 0; m < t.tz + 4; ++m) {
    const int pz = t.z0 - 2 + m, pb = pz - 1, pr2 = pz - 2;
    Fr = Fb;
    Zrm = Zr;
    Zr = Zb;
    if (m >= 1 && qon)
      load_faces(Fb, Zb, C, wrapi(pb, nz), qx, qy, qxl, qyb, nx, ny, m >= 2);
    if (m >= 2 && ron) load_ring(rc, C, t, rq, pb, nx, ny, nz);
    const bool out = m >= 4 && qon;
    const int o0 = (pr2 * ny + qy) * nx + qx;  // row 0 of the quad on plane pr2
    // relative coarse plane staged in this iteration (trilinear), 0 if none
    const int cst = (TRI && has_coarse && (m & 1) && m <= t.tz + 1) ? (m + 1) / 2 + 2 : 0;
    if (cst) cstage_load(cv, e, cbase + cst, cnx, cny, cnz);

    // right-hand side of plane pr2 (read again: keeping it for the three
    // iterations since its first load would cost more registers than the
    // read costs bytes) and, for the flexible dot, the old z
    Q4<FT> H{};
    R zo00 = 0, zo10 = 0, zo01 = 0, zo11 = 0;
    if (out) {
      const FT *src;
      if constexpr (L0) src = f.r;
      else src = f.f;
      ld2(src + o0, H.v00, H.v10);
      ld2(src + o0 + nx, H.v01, H.v11);
      if constexpr (L0 && sizeof(R) == 4) {
        if (rd_old) {
          ld2(P.z32 + o0, zo00, zo10);
          ld2(P.z32 + o0 + nx, zo01, zo11);
        }
      }
    }
    // (1) v = y, + e(parent) at red cells, on plane pz
    I2 = I1;
    I1 = I0;
    I0 = q_store_plane<R, L0, true, TRI>(pl, t, pz, qon, ci, cj, vs[m % 3], inv_s,
                                         has_coarse, cs);
    if (m + 1 < t.tz + 4)
      q_load_plane<R, L0, true, TRI>(pl, t, pz + 1, qon, qx, qy, nx, ny, nz, f, C.d, e,
                                     has_coarse, cnx, cny, cnz);
    if (cst) cstage_store(cv, cs[cst % 3]);
    __syncthreads();
    // (2) new black values of plane pb over the tile + 1
    if (m >= 2) {
      const R *vm = vs[(m + 1) % 3], *v0 = vs[(m + 2) % 3], *vp = vs[m % 3];
      R *xo = xs[m % 3];
      if (qon) {
        const bool b0 = (pb & 1) == 0, b1 = !b0;
        const int s = (2 * cj + 2) * kE2X + 2 * ci + 2;
        const int o = (2 * cj + 1) * kE1X + 2 * ci + 1;
        xo[o + b0] = black_value(cell_faces<0>(Fb, Zb, Zr, b0), pick<0>(I1, b0), vm,
                                 v0, vp, s + b0);
        xo[o + kE1X + b1] = black_value(cell_faces<1>(Fb, Zb, Zr, b1),
                                        pick<1>(I1, b1), vm, v0, vp, s + kE2X + b1);
      }
      if (ron) {
        const Faces6<R> fr{rc.xp, rc.xm, rc.yp, rc.ym, rc.zp, rc.zm};
        xo[rc.ey * kE1X + rc.ex] = black_value(fr, recip(rc.d), vm, v0, vp,
                                               (rc.ey + 1) * kE2X + rc.ex + 1);
      }
      __syncthreads();
    }
    // (3) plane pr2 on the tile: new red values from the new black ones, every
    //     cell written (finest level: z = s x and the dots; the mixed form
    //     stores x itself, FP32, as z32)
    if (out) {
      const R *xm = xs[(m + 1) % 3], *x0 = xs[(m + 2) % 3], *xp = xs[m % 3];
      const bool red00 = (pr2 & 1) == 0;  // (0,0), (1,1) red; else (1,0), (0,1)
      const int o = (2 * cj + 1) * kE1X + 2 * ci + 1;
      R v00, v10, v01, v11;
      if (red00) {
        v00 = (scaled<R, L0>(H.v00, inv_s) +
               red_sum(cell_faces<0>(Fr, Zr, Zrm, false), xm, x0, xp, o)) * I2.v00;
        v10 = x0[o + 1];
        v01 = x0[o + kE1X];
        v11 = (scaled<R, L0>(H.v11, inv_s) +
               red_sum(cell_faces<1>(Fr, Zr, Zrm, true), xm, x0, xp, o + kE1X + 1)) *
              I2.v11;
      } else {
        v00 = x0[o];
        v10 = (scaled<R, L0>(H.v10, inv_s) +
               red_sum(cell_faces<0>(Fr, Zr, Zrm, true), xm, x0, xp, o + 1)) * I2.v10;
        v01 = (scaled<R, L0>(H.v01, inv_s) +
               red_sum(cell_faces<1>(Fr, Zr, Zrm, false), xm, x0, xp, o + kE1X)) *
              I2.v01;
        v11 = x0[o + kE1X + 1];
      }
      if constexpr (L0) {
        const double z00 = (double)v00 * s_out, z10 = (double)v10 * s_out;
        const double z01 = (double)v01 * s_out, z11 = (double)v11 * s_out;
        if (rd_old) rzo += H.v00 * ((double)zo00 * zs_old);
        rz += H.v00 * z00;
        if (rd_old) rzo += H.v10 * ((double)zo10 * zs_old);
        rz += H.v10 * z10;
        if (rd_old) rzo += H.v01 * ((double)zo01 * zs_old);
        rz += H.v01 * z01;
        if (rd_old) rzo += H.v11 * ((double)zo11 * zs_old);
        rz += H.v11 * z11;
        if constexpr (sizeof(R) == 4) {
          st2(P.z32 + o0, v00, v10);
          st2(P.z32 + o0 + nx, v01, v11);
        } else {
          st2(P.z + o0, z00, z10);
          st2(P.z + o0 + nx, z01, z11);
        }
      } else {
        st2(xout + o0, v00, v10);
        st2(xout + o0 + nx, v01, v11);
      }
    }
  }
  if constexpr (L0) write_partials(T, tid, rz, rzo);
}

// launchers ------------------------------------------------------------------

void launch_vdown(const Tables &T, TileList L, int l, int prec, int sel,
                  hipStream_t s) {
  if (!L.nblocks) return;
  const int id = l == 0 ? K_VDOWN_F : K_VDOWN_C;
  if (prec) {
    if (l == 0) FLD_LAUNCH(id, (k_vdown<float, true>), L.nblocks, kBlock, s, T, L, l, sel);
    else FLD_LAUNCH(id, (k_vdown<float, false>), L.nblocks, kBlock, s, T, L, l, sel);
  } else {
    if (l == 0) FLD_LAUNCH(id, (k_vdown<double, true>), L.nblocks, kBlock, s, T, L, l, sel);
    else FLD_LAUNCH(id, (k_vdown<double, false>), L.nblocks, kBlock, s, T, L, l, sel);
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
