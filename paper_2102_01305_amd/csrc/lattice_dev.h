// Device-side lattice helpers shared by the collide and marker kernels:
// D3Q19 velocity set and weights, the storage formats, the padded row-major
// slab layout with its x-face ghost records, the pull gather and the
// equilibrium of the open faces.
#pragma once

#include <hip/hip_fp16.h>

#include "internal.h"

namespace ibmk {

// ------------------------------------------------------------------ D3Q19 --
__host__ __device__ constexpr int cxq(int i) {
  constexpr int t[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return t[i];
}
__host__ __device__ constexpr int cyq(int i) {
  constexpr int t[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return t[i];
}
__host__ __device__ constexpr int czq(int i) {
  constexpr int t[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return t[i];
}
__host__ __device__ constexpr int oppq(int i) {
  constexpr int t[kQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  return t[i];
}
__host__ __device__ constexpr float wq(int i) {
  return i == 0 ? 1.0f / 3.0f : (i < 7 ? 1.0f / 18.0f : 1.0f / 36.0f);
}
__host__ __device__ constexpr double wqd(int i) {
  return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---------------------------------------------------------------- storage --
// ld()/st() take and give f~ itself; ldr()/stnr() the stored value, which is
// kS f~ (kS = 2^12 for FP16, else 1), for the collide kernel, which works
// in those units throughout.  stn/stnr are streaming (non-temporal) stores
// for data the current kernel will not read again; stb is stnr through a
// buffer descriptor (byte offsets: vo per lane, so from a scalar register).
constexpr int kRawBufferWord3 = 0x00020000;   // untyped (raw) buffer, 32-bit data format
constexpr int kStreamAux = 2;                 // non-temporal
struct StF32 {
  using T = float;
  static constexpr float kS = 1.0f, kInv = 1.0f;
  __device__ static float ld(const T* p) { return *p; }
  __device__ static void st(T* p, float v) { *p = v; }
  __device__ static void stn(T* p, float v) { __builtin_nontemporal_store(v, p); }
  __device__ static float ldr(const T* p) { return *p; }
  __device__ static void stnr(T* p, float v) { __builtin_nontemporal_store(v, p); }
  __device__ static void stb(__amdgpu_buffer_rsrc_t r, int vo, int so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, vo, so, kStreamAux);
  }
};
struct StF16 {
  using T = __half;
  static constexpr float kS = kF16Scale, kInv = kF16Unscale;
  __device__ static float ldr(const T* p) { return __half2float(*p); }
  __device__ static void stnr(T* p, float v) {
    __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v)), reinterpret_cast<unsigned short*>(p));
  }
  __device__ static float ld(const T* p) { return ldr(p) * kInv; }
  __device__ static void st(T* p, float v) { *p = __float2half_rn(v * kS); }
  __device__ static void stn(T* p, float v) { stnr(p, v * kS); }
  __device__ static void stb(__amdgpu_buffer_rsrc_t r, int vo, int so, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), r, vo, so, kStreamAux);
  }
};
struct StBF16 {
  using T = unsigned short;
  static constexpr float kS = 1.0f, kInv = 1.0f;
  // round to nearest even (the gfx950 conversion instruction)
  __device__ static unsigned short enc(float v) { return __builtin_bit_cast(unsigned short, (__bf16)v); }
  __device__ static float ld(const T* p) { return __uint_as_float(((unsigned)*p) << 16); }
  __device__ static void st(T* p, float v) { *p = enc(v); }
  __device__ static void stn(T* p, float v) { __builtin_nontemporal_store(enc(v), p); }
  __device__ static float ldr(const T* p) { return ld(p); }
  __device__ static void stnr(T* p, float v) { stn(p, v); }
  __device__ static void stb(__amdgpu_buffer_rsrc_t r, int vo, int so, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(enc(v), r, vo, so, kStreamAux);
  }
};

// Row-major slabs: the 19 populations of one lattice row are adjacent, so a
// wave's 19 loads and 19 stores stay within a few DRAM pages.
__device__ __forceinline__ long long rowbase(const Geo& g, int y, int z) {
  return (long long)(z * g.ny + y + 1) * (kQ * g.px);
}

// Slot of population i among the five that cross an x face (c_x = +1:
// 1, 7, 9, 11, 13; c_x = -1: 2, 8, 10, 12, 14).
__host__ __device__ constexpr int xslot(int i) {
  constexpr int t[kQ] = {0, 0, 0, 0, 0, 0, 0, 1, 1, 2, 2, 3, 3, 4, 4, 0, 0, 0, 0};
  return t[i];
}

// Ghost values of a state: what the x = -1 (side 0) and x = nx (side 1)
// cells hold for the populations that enter the box from there, one
// 32-byte record per lattice row and side, after the state's slabs.  A block
// of 4 rows writes one whole 128-byte line per side.
template <class T>
__device__ __forceinline__ T* ghost_ptr(T* state, const Geo& g, int side, int y, int z, int i) {
  constexpr int per = 32 / (int)sizeof(T);
  T* base = reinterpret_cast<T*>(reinterpret_cast<char*>(state) + g.goff);
  return base + ((long long)side * g.ny * g.nz + (long long)z * g.ny + y) * per + xslot(i);
}
template <class T>
__device__ __forceinline__ const T* ghost_ptr(const T* state, const Geo& g, int side, int y, int z, int i) {
  return ghost_ptr(const_cast<T*>(state), g, side, y, z, i);
}

// Pre-collision distributions of cell (x, y, z): pull f~_i from x - c_i of
// the post-collision state S.  y/z: periodic wrap or half-way bounce-back
// (f_i <- S_opp(i) of the cell itself).  x: from the ghost records of S,
// which hold the periodic image, the bounce-back value or the inlet/outlet
// equilibrium.  All 19 source rows are chosen first, without branches, so
// the loads issue back to back; when y and z are wave-uniform the row
// pointers stay in scalar registers.  RAW: values in stored units (ldr).
template <class St, bool RAW = false>
__device__ __forceinline__ void pull19(const typename St::T* __restrict__ S, const Geo& g,
                                       int x, int y, int z, float f[kQ]) {
  using T = typename St::T;
  const T* src[kQ];
  const T* own = S + rowbase(g, y, z);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int cy = cyq(i), cz = czq(i), cx = cxq(i);
    int yy = y - cy, zz = z - cz;
    bool wall = false;
    if (cy != 0) {
      const bool out = yy < 0 || yy >= g.ny;
      wall = wall || (out && !g.yper);
      yy = yy < 0 ? yy + g.ny : (yy >= g.ny ? yy - g.ny : yy);
    }
    if (cz != 0) {
      const bool out = zz < 0 || zz >= g.nz;
      wall = wall || (out && !g.zper);
      zz = zz < 0 ? zz + g.nz : (zz >= g.nz ? zz - g.nz : zz);
    }
    const T* pn = S + (long long)i * g.ps + rowbase(g, yy, zz) - cx + x;
    if (cx == 1) pn = x == 0 ? ghost_ptr(S, g, 0, yy, zz, i) : pn;
    if (cx == -1) pn = x == g.nx - 1 ? ghost_ptr(S, g, 1, yy, zz, i) : pn;
    const T* pb = own + (long long)oppq(i) * g.ps + x;
    src[i] = wall ? pb : pn;
  }
#pragma unroll
  for (int i = 0; i < kQ; ++i) f[i] = RAW ? St::ldr(src[i]) : St::ld(src[i]);
}

// pull19 for a wave-uniform row (y, z) whose sources all lie inside the box
// or across a periodic face (no y or z wall reflects into it; see
// pull_rows_inside): the 9 source rows (y - c_y, z - c_z) are wrapped once
// in scalar registers and each population row is a scalar base plus the
// lane's 32-bit offset, so the wraps and row products cost no per-cell
// instructions; only the c_x = -/+1 rows select the ghost record per lane
// at the x faces.  Same sources as pull19.
__device__ __forceinline__ bool pull_rows_inside(const Geo& g, int y, int z) {
  return (g.yper || (y > 0 && y < g.ny - 1)) && (g.zper || (z > 0 && z < g.nz - 1));
}
template <class St>
__device__ __forceinline__ void pull19_rows(const typename St::T* __restrict__ S, const Geo& g,
                                            int x, int y, int z, float f[kQ]) {
  using T = typename St::T;
  constexpr unsigned es = sizeof(T);
  const char* Sb = reinterpret_cast<const char*>(S);
  const unsigned rowb = (unsigned)kQ * (unsigned)g.px * es, popb = (unsigned)g.px * es;
  const unsigned xo = (unsigned)x * es;
  // source row of direction (c_y, c_z), c in {-1, 0, 1}: index [1 - c]
  const int ys[3] = {y == 0 ? g.ny - 1 : y - 1, y, y == g.ny - 1 ? 0 : y + 1};   // y - c_y
  const int zs[3] = {z == 0 ? g.nz - 1 : z - 1, z, z == g.nz - 1 ? 0 : z + 1};   // z - c_z
  const char* base[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      base[a][b] = Sb + (unsigned long long)(unsigned)(zs[b] * g.ny + ys[a] + 1) * rowb;
  constexpr int per = 32 / (int)sizeof(T);
  const T* gb = reinterpret_cast<const T*>(Sb + g.goff);
  const long long rows = (long long)g.ny * g.nz;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const unsigned q = (unsigned)i * popb - (unsigned)(cxq(i) * (int)es);
    const T* pp = reinterpret_cast<const T*>(base[1 - cyq(i)][1 - czq(i)] + (xo + q));
    const long long gr = (long long)(zs[1 - czq(i)] * g.ny + ys[1 - cyq(i)]);   // source row
    if (cxq(i) == 1) pp = x == 0 ? gb + gr * per + xslot(i) : pp;
    if (cxq(i) == -1) pp = x == g.nx - 1 ? gb + (rows + gr) * per + xslot(i) : pp;
    f[i] = St::ldr(pp);
  }
}

// Global-memory view of a pointer.  Loads through it are global loads, which
// the compiler knows cannot alias LDS; through a generic pointer each load
// of a global-to-LDS copy would wait for the one before it.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// Copy n values from global memory into LDS with four loads in flight per
// thread.
template <class T>
__device__ __forceinline__ void copy_to_lds(T* dst, const T* src, int n) {
  const auto* g = gmem(src);
  const int bd = (int)blockDim.x;
  int e = (int)threadIdx.x;
  for (; e + 3 * bd < n; e += 4 * bd) {
    const T v0 = g[e], v1 = g[e + bd], v2 = g[e + 2 * bd], v3 = g[e + 3 * bd];
    dst[e] = v0;
    dst[e + bd] = v1;
    dst[e + 2 * bd] = v2;
    dst[e + 3 * bd] = v3;
  }
  for (; e < n; e += bd) dst[e] = g[e];
}

// The solve a block of a grouped launch belongs to (binary search over the
// block offsets, all in kernel arguments) and its block index within it.
__device__ __forceinline__ int group_index(const Group& g, int& lb) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = g.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  lb = b - g.start[lo];
  return lo;
}
__device__ __forceinline__ const void* group_find(const Group& g, int& lb) {
  return g.args[group_index(g, lb)];
}

// Block offsets of a grouped launch from per-solve block counts; returns the
// total.
inline int group_fill(Group& g, const void* const* dev, const int* blocks, int n) {
  g.n = n;
  int t = 0;
  for (int k = 0; k < n; ++k) {
    g.start[k] = t;
    g.args[k] = dev[k];
    t += blocks[k];
  }
  g.start[n] = t;
  return t;
}

// Zou-He faces: rebuild the populations entering through an x face at a
// boundary cell from its known ones (non-equilibrium bounce-back of the
// normal population plus a transverse momentum correction, D3Q19), so that
// the cell carries the prescribed velocity (density from the known
// populations) or the prescribed density (transverse velocity zero).
// Cells whose entering links also touch a y or z wall keep the ghost values
// pulled already.  f holds deviations f - w, times s (stored units) if RAW;
// the lattice weights cancel in every difference used here.
template <class St, bool RAW, int IN>
__device__ __forceinline__ void zou_he_face(const Phys& p, int kind, float f[kQ]) {
  // IN: c_x of the entering populations (+1 on the -x face, -1 on the +x face)
  const float s = RAW ? St::kS : 1.0f, inv = RAW ? St::kInv : 1.0f;
  float sz = 0.f, sout = 0.f, ny = 0.f, nz = 0.f;  // sums over c_x = 0 and leaving populations
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    if (cxq(i) == 0) {
      sz += f[i];
      ny += cyq(i) * f[i];
      nz += czq(i) * f[i];
    } else if (cxq(i) == -IN) {
      sout += f[i];
    }
  }
  const float known = 1.0f + (sz + 2.0f * sout) * inv;   // sum_Z f + 2 sum_out f
  float rho, ux, uy, uz;
  if (kind == BC_ZH_VELOCITY) {
    ux = p.u_in[0]; uy = p.u_in[1]; uz = p.u_in[2];
    rho = known / (1.0f - IN * ux);
  } else {
    rho = p.rho_out;
    ux = IN * (1.0f - known / rho);
    uy = 0.f; uz = 0.f;
  }
  const float Ny = 0.5f * ny - s * rho * uy * (1.0f / 3.0f);
  const float Nz = 0.5f * nz - s * rho * uz * (1.0f / 3.0f);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    if (cxq(i) != IN) continue;
    const float cu = cxq(i) * ux + cyq(i) * uy + czq(i) * uz;
    f[i] = f[oppq(i)] + s * 6.0f * wq(i) * rho * cu - cyq(i) * Ny - czq(i) * Nz;
  }
}

template <class St, bool RAW>
__device__ __forceinline__ void zou_he(const Geo& g, const Phys& p, int x, int y, int z, float f[kQ]) {
  const bool lo = x == 0 && g.bclo >= BC_ZH_VELOCITY;
  const bool hi = x == g.nx - 1 && g.bchi >= BC_ZH_VELOCITY;
  if (!lo && !hi) return;
  if (!g.yper && (y == 0 || y == g.ny - 1)) return;
  if (!g.zper && (z == 0 || z == g.nz - 1)) return;
  if (lo)
    zou_he_face<St, RAW, 1>(p, g.bclo, f);
  else
    zou_he_face<St, RAW, -1>(p, g.bchi, f);
}

// c_i . v summed over the nonzero components of c_i in x, y, z order.  A
// product 0 * v is not folded away under IEEE rules (v could be infinite),
// and leaving it out changes no finite result.
__device__ __forceinline__ float cdot(int i, float vx, float vy, float vz) {
  const int c[3] = {cxq(i), cyq(i), czq(i)};
  const float v[3] = {vx, vy, vz};
  float r = 0.f;
  bool any = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (c[d] == 0) continue;
    const float t = c[d] > 0 ? v[d] : -v[d];
    r = any ? r + t : t;
    any = true;
  }
  return r;
}

// Zeroth and first moments of 19 values: sum f_i and sum c_i f_i, in i order
// (zero components of c_i left out, as in cdot).
__device__ __forceinline__ void moments19(const float f[kQ], float& d, float& jx, float& jy, float& jz) {
  d = jx = jy = jz = 0.f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    d += f[i];
    if (cxq(i) != 0) jx = cxq(i) > 0 ? jx + f[i] : jx - f[i];
    if (cyq(i) != 0) jy = cyq(i) > 0 ? jy + f[i] : jy - f[i];
    if (czq(i) != 0) jz = czq(i) > 0 ? jz + f[i] : jz - f[i];
  }
}

// Equilibrium deviation f~eq_i = w_i (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2)).
__device__ __forceinline__ float feq_dev(int i, float drho, float rho, float ux, float uy,
                                         float uz, float usq) {
  const float cu = cdot(i, ux, uy, uz);
  return wq(i) * (drho + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * usq));
}

// feq_dev with every operation rounded on its own (no contraction into
// FMAs), so that it gives the same bits in every kernel it is compiled into.
__device__ __forceinline__ float feq_dev_strict(int i, float drho, float rho, float ux, float uy,
                                                float uz, float usq) {
#pragma clang fp contract(off)
  const float cu = cdot(i, ux, uy, uz);
  return wq(i) * (drho + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * usq));
}

// Ghost records of the state being written, from the post-collision values
// `o` of a boundary cell (x == 0 or x == nx-1).  The ghost at (-1, y', z')
// for population i (c_x = +1) is read only by cell (0, y'+c_y, z'+c_z); the
// +x ghost likewise for c_x = -1.  This runs inside the collide and, after an
// initialisation, in the ghost kernel; a resumed run has to find the same
// ghosts as an uninterrupted one, so the arithmetic is kept free of
// contraction and gives the same bits in both.
template <class St>
__device__ void write_ghosts(typename St::T* __restrict__ D, const Geo& g, const Phys& p,
                             int x, int y, int z, const float o[kQ]) {
#pragma clang fp contract(off)
  float drho, jx, jy, jz;
  moments19(o, drho, jx, jy, jz);
  const float rho = 1.0f + drho;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int dir = side == 0 ? 1 : -1;        // populations leaving the ghost into the box
    const int kind = side == 0 ? g.bclo : g.bchi;
    const int bcell = side == 0 ? 0 : g.nx - 1; // boundary cell feeding this face
    const int pcell = side == 0 ? g.nx - 1 : 0; // periodic image feeding this face
    if (kind == BC_PERIODIC) {
      if (x != pcell) continue;
#pragma unroll
      for (int i = 0; i < kQ; ++i)
        if (cxq(i) == dir) St::st(ghost_ptr(D, g, side, y, z, i), o[i]);
      continue;
    }
    if (x != bcell) continue;
    if (kind == BC_WALL) {
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        if (cxq(i) != dir) continue;
        int yy = y - cyq(i), zz = z - czq(i);
        bool skip = false;
        if (yy < 0) { if (g.yper) yy += g.ny; else skip = true; }
        else if (yy >= g.ny) { if (g.yper) yy -= g.ny; else skip = true; }
        if (zz < 0) { if (g.zper) zz += g.nz; else skip = true; }
        else if (zz >= g.nz) { if (g.zper) zz -= g.nz; else skip = true; }
        if (!skip) St::st(ghost_ptr(D, g, side, yy, zz, i), o[oppq(i)]);
      }
      continue;
    }
    float rg, ux, uy, uz;
    if (kind == BC_VELOCITY || kind == BC_ZH_VELOCITY) {
      rg = rho;
      ux = p.u_in[0]; uy = p.u_in[1]; uz = p.u_in[2];
    } else {  // BC_PRESSURE, BC_ZH_PRESSURE
      rg = p.rho_out;
      const float inv = 1.0f / rho;
      ux = jx * inv; uy = jy * inv; uz = jz * inv;
    }
    const float usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      if (cxq(i) == dir)
        St::st(ghost_ptr(D, g, side, y, z, i), feq_dev_strict(i, rg - 1.0f, rg, ux, uy, uz, usq));
  }
}

}  // namespace ibmk
