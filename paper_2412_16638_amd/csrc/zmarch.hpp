// Z-marching tiles for the 7-point stencil kernels.
//
// A workgroup owns R whole x-rows (y0 .. y0 + R - 1) of a run of planes z0 .. z1 - 1 and
// marches through them.  Each thread owns one group of VEC consecutive x-values of one row: it
// keeps the stencil input of its group for planes k - 1, k and k + 1 in registers (the z
// neighbours) while plane k + 2 is in flight, and writes plane k into an LDS tile of R + 2 rows
// (one halo row below and above, spread over the workgroup's threads), double buffered, from which
// the x and y neighbours are read.  Every input value enters the CU once per tile (halo rows add
// 2 / R, served by L2), instead of the seven loads per group of the gather form: the stencil
// then costs the memory system about what a plain stream of the same arrays does.
//
// The stencil input is produced by the caller (`src`): a plain load, or values computed from
// several arrays (the GMRES step forms the preconditioned direction from the basis).  The
// caller's per-group work (`body`) runs on each owned group of each plane with the stencil
// result; its own loads for plane k + 1 are issued during plane k.
#pragma once

#include "device.hpp"

namespace mprk {

constexpr int ZM_LZ_MIN = 2;  // fewest planes per tile the library launches

struct ZLaunch {
  int gx;        // groups per x-row (nx / VEC)
  int R;         // rows per tile
  int LZ;        // planes per tile
  int nty, ntz;  // tiles along y and z
  int G;         // workgroups (a multiple of 8, >= nty * ntz; the rest only join reductions)
};

// Whether a grid can run z-marching tiles with VEC values per group: whole groups per row, a
// row fits one workgroup and its halo slots fit one per thread.
__host__ __device__ inline bool zmarch_fits(const Geo& g, int vec) {
  return vec > 1 && g.nx % vec == 0 && g.nx / vec <= TPB / 2 && g.ny >= 1 && g.nz >= 1;
}

// LDS bytes of a z-marching launch with compute type of `cbytes` bytes.
__host__ __device__ inline size_t zmarch_lds(const Geo& g, const ZLaunch& z, int cbytes) {
  return (size_t)2 * (z.R + 2) * g.nx * cbytes;
}

inline ZLaunch make_zlaunch(const Geo& g, int vec, int LZ) {
  ZLaunch z{};
  z.gx = g.nx / vec;
  z.R = TPB / z.gx;
  z.LZ = LZ < 1 ? 1 : LZ;
  z.nty = (g.ny + z.R - 1) / z.R;
  z.ntz = (g.nz + z.LZ - 1) / z.LZ;
  const long G = (long)z.nty * z.ntz;
  z.G = (int)std::max(8L, (G + 7) / 8 * 8);
  return z;
}

// Plane index pz of the input: wrapped (periodic) or -1 (outside a zero-Dirichlet boundary).
__device__ __forceinline__ int zm_wrap(int p, int n, int per) {
  if (p >= 0 && p < n) return p;
  return per ? (p < 0 ? p + n : p - n) : -1;
}

// src(int e, C (&o)[VEC], bool own): stencil input of the group starting at element e (own:
//   the thread's own group in one of the tile's planes, which src may also store or
//   accumulate, each exactly once; else a halo group or a plane beyond the tile).
// body.pre(int e): issue the loads of the owned group at e (the next plane's) into the body's
//   second register set; body.next() makes that set the current one.
// body.fin(int e, const C (&ctr)[VEC], const C (&out)[VEC]): the group's stencil result, with
//   the current register set.
// lds: 2 (R + 2) nx values of C (dynamic shared memory).
// The 2 gx halo groups are spread evenly over the workgroup's waves (src may be as costly as
// an owned group's), LPB consecutive groups on consecutive lanes (src may exchange values
// within such lane groups by shuffles; gx must then be a multiple of LPB).
template <typename C, int VEC, int LPB = 1, typename Src, typename Body>
__device__ __forceinline__ void zmarch(const Geo& g, const Coef<C>& k, const ZLaunch& zl, int L,
                                       const Src& src, Body& body, C* lds) {
  if (L >= zl.nty * zl.ntz) return;
  const int per = g.bc == 1;
  const int nx = g.nx;
  const int t = threadIdx.x;
  const int ty = L % zl.nty, tz = L / zl.nty;
  const int y0 = ty * zl.R, z0 = tz * zl.LZ;
  const int z1 = min(z0 + zl.LZ, g.nz);
  const int Rv = min(zl.R, g.ny - y0);
  const int r = t / zl.gx, xg = t - r * zl.gx;
  const bool own = r < Rv;
  const int x0 = xg * VEC;
  const int y = y0 + r;
  // halo group h (0 .. 2 gx - 1; below the tile, then above) on thread (h / LPB) hs LPB +
  // h % LPB, hs = TPB / (2 gx)
  const int hstride = (TPB / (2 * zl.gx)) * LPB;
  const int hq = t / hstride, hl = t - hq * hstride;
  const int h = hq * LPB + hl;
  const bool hal = hl < LPB && h < 2 * zl.gx;
  const int hside = h < zl.gx ? 0 : 1;
  const int hx0 = (h - hside * zl.gx) * VEC;
  const int hy = zm_wrap(hside ? y0 + Rv : y0 - 1, g.ny, per);
  const int hrow = hside ? Rv + 1 : 0;
  auto own_at = [&](int pz, C (&o)[VEC]) {
    const int q = zm_wrap(pz, g.nz, per);
    if (q < 0) {
#pragma unroll
      for (int v = 0; v < VEC; ++v) o[v] = C(0);
    } else {
      src(q * g.plane + y * nx + x0, o, pz >= z0 && pz < z1);
    }
  };
  auto halo_at = [&](int pz, C (&o)[VEC]) {
    const int q = zm_wrap(pz, g.nz, per);
    if (q < 0 || hy < 0) {
#pragma unroll
      for (int v = 0; v < VEC; ++v) o[v] = C(0);
    } else {
      src(q * g.plane + hy * nx + hx0, o, false);
    }
  };
  C cm[VEC], cc[VEC], cp[VEC], cn[VEC], hc[VEC], hn[VEC];
  if (own) {
    own_at(z0 - 1, cm);
    own_at(z0, cc);
    own_at(z0 + 1, cp);
    body.pre(z0 * g.plane + y * nx + x0);
    body.next();
  }
  if (hal) halo_at(z0, hc);
  const int pitch = nx;
  for (int kz = z0; kz < z1; ++kz) {
    C* buf = lds + (size_t)((kz - z0) & 1) * (zl.R + 2) * pitch;
    // loads for the next planes go out first and stay in flight across the barrier
    if (own && kz + 2 <= z1) own_at(kz + 2, cn);
    if (hal && kz + 1 < z1) halo_at(kz + 1, hn);
    if (own) {
      Vec<C, VEC> w;
#pragma unroll
      for (int v = 0; v < VEC; ++v) w.v[v] = cc[v];
      *reinterpret_cast<Vec<C, VEC>*>(buf + (r + 1) * pitch + x0) = w;
    }
    if (hal) {
      Vec<C, VEC> w;
#pragma unroll
      for (int v = 0; v < VEC; ++v) w.v[v] = hc[v];
      *reinterpret_cast<Vec<C, VEC>*>(buf + hrow * pitch + hx0) = w;
    }
    __syncthreads();
    if (own) {
      const int e = kz * g.plane + y * nx + x0;
      if (kz + 1 < z1) body.pre(e + g.plane);
      const C* row = buf + (r + 1) * pitch;
      const Vec<C, VEC> ym = *reinterpret_cast<const Vec<C, VEC>*>(row - pitch + x0);
      const Vec<C, VEC> yp = *reinterpret_cast<const Vec<C, VEC>*>(row + pitch + x0);
      C l, rr;
      if (x0 > 0) l = row[x0 - 1];
      else l = per ? row[nx - 1] : C(0);
      if (x0 + VEC < nx) rr = row[x0 + VEC];
      else rr = per ? row[0] : C(0);
      C out[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const C left = v > 0 ? cc[v - 1] : l;
        const C right = v < VEC - 1 ? cc[v + 1] : rr;
        C acc = k.c * cc[v];
        acc += k.xm * left;
        acc += k.xp * right;
        acc += k.ym * ym.v[v];
        acc += k.yp * yp.v[v];
        acc += k.zm * cm[v];
        acc += k.zp * cp[v];
        out[v] = acc;
      }
      body.fin(e, cc, out);
      body.next();
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        cm[v] = cc[v];
        cc[v] = cp[v];
        cp[v] = cn[v];
      }
    }
    if (hal) {
#pragma unroll
      for (int v = 0; v < VEC; ++v) hc[v] = hn[v];
    }
  }
}

}  // namespace mprk
