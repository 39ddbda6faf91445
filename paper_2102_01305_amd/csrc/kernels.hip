// gfx950 kernels of the D3Q19 BGK + implicit-IBM time step.
//
//  collide   fused pull-streaming, moments, IBM velocity correction, Guo
//            forcing and BGK relaxation over every cell (Eqs. 1-11, 16, 26);
//            also writes the x-face ghost layer of the next state.
//  ghost     the same ghost rule for a freshly initialised state.
//  factor    perimeter block of the no-slip matrix and its inverse (Eq. 18).
//  interp    marker kinematics (Eqs. 20-23) and delta interpolation of rho and
//            u* to the markers, right-hand side B (Eqs. 14, 17, 19).
//  solve     minimum-norm solution of A X = B (Eq. 19) for one span layer of
//            one foil, then the force and moment on it (Eq. 26); the last
//            layer block of a foil writes the coefficients to the history.
//  spread    du(x) = sum_l du_B D dA (Eq. 15) with float atomics, and marks
//            the 8^3 tiles the collide kernel must correct.
//
// Distributions are stored as deviations from the lattice weights,
// f~_i = f_i - w_i, so FP32 (and 16-bit) storage keeps the small velocity
// signal out of the rounding of the O(w_i) rest value.
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
struct StF32 {
  using T = float;
  __device__ static float ld(const T* p) { return *p; }
  __device__ static void st(T* p, float v) { *p = v; }
};
struct StF16 {
  using T = __half;
  __device__ static float ld(const T* p) { return __half2float(*p); }
  __device__ static void st(T* p, float v) { *p = __float2half_rn(v); }
};
struct StBF16 {
  using T = unsigned short;
  __device__ static float ld(const T* p) { return __uint_as_float(((unsigned)*p) << 16); }
  __device__ static void st(T* p, float v) {
    unsigned u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
    *p = (unsigned short)(u >> 16);
  }
};

__device__ __forceinline__ long long rowbase(const Geo& g, int y, int z) {
  return (long long)(z * g.ny + y + 1) * g.px;
}

// Pre-collision distributions of cell (x, y, z): pull f~_i from x - c_i of
// the post-collision state S.  y/z: periodic wrap or half-way bounce-back
// (f_i <- S_opp(i) of the cell itself).  x: through the ghost layer, which
// holds the periodic image, the bounce-back value or the inlet/outlet
// equilibrium.
template <class St>
__device__ __forceinline__ void pull19(const typename St::T* __restrict__ S, const Geo& g,
                                       int x, int y, int z, float f[kQ]) {
  const long long own = rowbase(g, y, z) + x;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int cy = cyq(i), cz = czq(i), cx = cxq(i);
    int yy = y - cy, zz = z - cz;
    bool wall = false;
    if (cy != 0) {
      if (yy < 0) { if (g.yper) yy += g.ny; else wall = true; }
      else if (yy >= g.ny) { if (g.yper) yy -= g.ny; else wall = true; }
    }
    if (cz != 0) {
      if (zz < 0) { if (g.zper) zz += g.nz; else wall = true; }
      else if (zz >= g.nz) { if (g.zper) zz -= g.nz; else wall = true; }
    }
    if (wall)
      f[i] = St::ld(S + (long long)oppq(i) * g.ps + own);
    else
      f[i] = St::ld(S + (long long)i * g.ps + rowbase(g, yy, zz) + x - cx);
  }
}

// Equilibrium deviation f~eq_i = w_i (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2)).
__device__ __forceinline__ float feq_dev(int i, float drho, float rho, float ux, float uy,
                                         float uz, float usq) {
  const float cu = cxq(i) * ux + cyq(i) * uy + czq(i) * uz;
  return wq(i) * (drho + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * usq));
}

// Ghost layer of the state being written, from the post-collision values
// `o` of a boundary cell (x == 0 or x == nx-1).  The ghost at (-1, y', z')
// for population i (c_x = +1) is read only by cell (0, y'+c_y, z'+c_z); the
// +x ghost likewise for c_x = -1.
template <class St>
__device__ void write_ghosts(typename St::T* __restrict__ D, const Geo& g, const Phys& p,
                             int x, int y, int z, const float o[kQ]) {
  const long long rb = rowbase(g, y, z);
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    drho += o[i];
    jx += cxq(i) * o[i];
    jy += cyq(i) * o[i];
    jz += czq(i) * o[i];
  }
  const float rho = 1.0f + drho;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int dir = side == 0 ? 1 : -1;        // populations leaving the ghost into the box
    const int kind = side == 0 ? g.bclo : g.bchi;
    const int bcell = side == 0 ? 0 : g.nx - 1; // boundary cell feeding this face
    const int pcell = side == 0 ? g.nx - 1 : 0; // periodic image feeding this face
    const long long gcol = side == 0 ? -1 : g.nx;
    if (kind == BC_PERIODIC) {
      if (x != pcell) continue;
#pragma unroll
      for (int i = 0; i < kQ; ++i)
        if (cxq(i) == dir) St::st(D + (long long)i * g.ps + rb + gcol, o[i]);
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
        if (!skip) St::st(D + (long long)i * g.ps + rowbase(g, yy, zz) + gcol, o[oppq(i)]);
      }
      continue;
    }
    float rg, ux, uy, uz;
    if (kind == BC_VELOCITY) {
      rg = rho;
      ux = p.u_in[0]; uy = p.u_in[1]; uz = p.u_in[2];
    } else {  // BC_PRESSURE
      rg = p.rho_out;
      const float inv = 1.0f / rho;
      ux = jx * inv; uy = jy * inv; uz = jz * inv;
    }
    const float usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      if (cxq(i) == dir)
        St::st(D + (long long)i * g.ps + rb + gcol, feq_dev(i, rg - 1.0f, rg, ux, uy, uz, usq));
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
// that each XCD streams one contiguous slab and the x-neighbour cache lines
// of a row stay in one L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int xcd = b & 7, local = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// ---------------------------------------------------------------- collide --
template <class St, bool IBM, bool FORCE, bool CHECK>
__global__ void __launch_bounds__(kBlockX * kBlockRows)
k_collide(CollideArgs a) {
  using T = typename St::T;
  const Geo& g = a.g;
  const T* __restrict__ S = static_cast<const T*>(a.src);
  T* __restrict__ D = static_cast<T*>(a.dst);
  const int lb = xcd_remap(blockIdx.x, a.nblocks);
  const int xc = lb % a.nxc;
  const int rg = lb / a.nxc;
  const int x = xc * kBlockX + threadIdx.x;
  const int row = rg * kBlockRows + threadIdx.y;
  const bool active = x < g.nx && row < g.ny * g.nz;
  double dm = 0.0;
  bool bad = false;
  if (active) {
    const int z = row / g.ny;
    const int y = row - z * g.ny;
    float f[kQ];
    pull19<St>(S, g, x, y, z, f);
    float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      drho += f[i];
      jx += cxq(i) * f[i];
      jy += cyq(i) * f[i];
      jz += czq(i) * f[i];
    }
    const float rho = 1.0f + drho;
    const float inv = 1.0f / rho;
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    if (FORCE) {
      Fx = a.p.fb[0]; Fy = a.p.fb[1]; Fz = a.p.fb[2];
      jx += 0.5f * Fx; jy += 0.5f * Fy; jz += 0.5f * Fz;
    }
    float ux = jx * inv, uy = jy * inv, uz = jz * inv;
    bool forced = FORCE;
    if (IBM) {
      const int tile = ((z >> 3) * a.tny + (y >> 3)) * a.tnx + (x >> 3);
      if (a.stamps[tile] == a.stamp) {
        const size_t N = (size_t)g.nx * g.ny * g.nz;
        const size_t cell = ((size_t)z * g.ny + y) * g.nx + x;
        const float dux = a.du[cell], duy = a.du[N + cell], duz = a.du[2 * N + cell];
        a.du[cell] = 0.f;
        a.du[N + cell] = 0.f;
        a.du[2 * N + cell] = 0.f;
        ux += dux; uy += duy; uz += duz;                 // Eq. 16
        Fx += 2.0f * rho * dux;                          // Eq. 11 / Eq. 26
        Fy += 2.0f * rho * duy;
        Fz += 2.0f * rho * duz;
        forced = true;
      }
    }
    const float usq = ux * ux + uy * uy + uz * uz;
    const float om = a.p.omega;
    float o[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) o[i] = f[i] - om * (f[i] - feq_dev(i, drho, rho, ux, uy, uz, usq));
    if (forced) {
      const float k = a.p.guo_k;
      const float uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        const float cu = cxq(i) * ux + cyq(i) * uy + czq(i) * uz;
        const float cF = cxq(i) * Fx + cyq(i) * Fy + czq(i) * Fz;
        o[i] += k * wq(i) * (3.0f * (cF - uF) + 9.0f * cu * cF);   // Eq. 8
      }
    }
    const long long own = rowbase(g, y, z) + x;
#pragma unroll
    for (int i = 0; i < kQ; ++i) St::st(D + (long long)i * g.ps + own, o[i]);
    if (x == 0 || x == g.nx - 1) write_ghosts<St>(D, g, a.p, x, y, z, o);
    if (CHECK) {
      dm = (double)drho;
      bad = !isfinite(drho);
    }
  }
  if (CHECK) {
    // wave reduction, then 4 waves through LDS, fixed order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dm += __shfl_xor(dm, off);
    __shared__ double part[kBlockRows];
    if (threadIdx.x == 0) part[threadIdx.y] = dm;
    if (bad) atomicOr(a.flags, 1);
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
      double s = 0.0;
      for (int r = 0; r < kBlockRows; ++r) s += part[r];
      a.mass_part[lb] = s;
    }
  }
}

template <class St, bool IBM, bool FORCE, bool CHECK>
static hipError_t launch_collide_t(const CollideArgs& a, hipStream_t s) {
  k_collide<St, IBM, FORCE, CHECK><<<a.nblocks, dim3(kBlockX, kBlockRows), 0, s>>>(a);
  return hipGetLastError();
}

template <class St>
static hipError_t launch_collide_s(bool ibm, bool force, bool check, const CollideArgs& a,
                                   hipStream_t s) {
  const int key = (ibm ? 4 : 0) | (force ? 2 : 0) | (check ? 1 : 0);
  switch (key) {
    case 0: return launch_collide_t<St, false, false, false>(a, s);
    case 1: return launch_collide_t<St, false, false, true>(a, s);
    case 2: return launch_collide_t<St, false, true, false>(a, s);
    case 3: return launch_collide_t<St, false, true, true>(a, s);
    case 4: return launch_collide_t<St, true, false, false>(a, s);
    case 5: return launch_collide_t<St, true, false, true>(a, s);
    case 6: return launch_collide_t<St, true, true, false>(a, s);
    default: return launch_collide_t<St, true, true, true>(a, s);
  }
}

hipError_t launch_collide(int storage, bool ibm, bool force, bool check, const CollideArgs& a,
                          hipStream_t s) {
  switch (storage) {
    case ST_F32: return launch_collide_s<StF32>(ibm, force, check, a, s);
    case ST_F16: return launch_collide_s<StF16>(ibm, force, check, a, s);
    default: return launch_collide_s<StBF16>(ibm, force, check, a, s);
  }
}

// ------------------------------------------------------------ ghost, init --
template <class St>
__global__ void k_ghost(Geo g, Phys p, typename St::T* buf) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= g.ny * g.nz) return;
  const int z = row / g.ny, y = row - z * g.ny;
  const long long rb = rowbase(g, y, z);
  float o[kQ];
  for (int side = 0; side < 2; ++side) {
    const int x = side == 0 ? 0 : g.nx - 1;
#pragma unroll
    for (int i = 0; i < kQ; ++i) o[i] = St::ld(buf + (long long)i * g.ps + rb + x);
    write_ghosts<St>(buf, g, p, x, y, z, o);
    if (g.nx == 1) break;
  }
}

hipError_t launch_ghost(int storage, const Geo& g, const Phys& p, void* buf, hipStream_t s) {
  const int rows = g.ny * g.nz;
  const int nb = (rows + 255) / 256;
  switch (storage) {
    case ST_F32: k_ghost<StF32><<<nb, 256, 0, s>>>(g, p, static_cast<float*>(buf)); break;
    case ST_F16: k_ghost<StF16><<<nb, 256, 0, s>>>(g, p, static_cast<__half*>(buf)); break;
    default: k_ghost<StBF16><<<nb, 256, 0, s>>>(g, p, static_cast<unsigned short*>(buf)); break;
  }
  return hipGetLastError();
}

// Equilibrium (Eq. 4) of FP64 rho, u (dense, x fastest; NULL = 1 / 0),
// evaluated in FP64 and rounded once to the storage type.
template <class St>
__global__ void k_init_eq(Geo g, const double* rho, const double* u, typename St::T* D) {
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= N) return;
  const int x = (int)(cell % g.nx);
  const size_t r = cell / g.nx;
  const int y = (int)(r % g.ny), z = (int)(r / g.ny);
  const double rh = rho ? rho[cell] : 1.0;
  const double ux = u ? u[cell] : 0.0, uy = u ? u[N + cell] : 0.0, uz = u ? u[2 * N + cell] : 0.0;
  const double usq = ux * ux + uy * uy + uz * uz;
  const long long own = rowbase(g, y, z) + x;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const double cu = cxq(i) * ux + cyq(i) * uy + czq(i) * uz;
    const double v = wqd(i) * ((rh - 1.0) + rh * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
    St::st(D + (long long)i * g.ps + own, (float)v);
  }
}

hipError_t launch_init_eq(int storage, const Geo& g, const double* rho, const double* u,
                          void* dst, hipStream_t s) {
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const unsigned nb = (unsigned)((N + 255) / 256);
  switch (storage) {
    case ST_F32: k_init_eq<StF32><<<nb, 256, 0, s>>>(g, rho, u, static_cast<float*>(dst)); break;
    case ST_F16: k_init_eq<StF16><<<nb, 256, 0, s>>>(g, rho, u, static_cast<__half*>(dst)); break;
    default: k_init_eq<StBF16><<<nb, 256, 0, s>>>(g, rho, u, static_cast<unsigned short*>(dst)); break;
  }
  return hipGetLastError();
}

// rho and u* = (sum c f + F_body/2)/rho of the pre-collision state, as
// 4 dense float planes (rho, ux, uy, uz).
template <class St>
__global__ void k_moments(Geo g, Phys p, const typename St::T* S, float* out) {
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= N) return;
  const int x = (int)(cell % g.nx);
  const size_t r = cell / g.nx;
  const int y = (int)(r % g.ny), z = (int)(r / g.ny);
  float f[kQ];
  pull19<St>(S, g, x, y, z, f);
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    drho += f[i];
    jx += cxq(i) * f[i];
    jy += cyq(i) * f[i];
    jz += czq(i) * f[i];
  }
  const float rho = 1.0f + drho;
  out[cell] = rho;
  out[N + cell] = (jx + 0.5f * p.fb[0]) / rho;
  out[2 * N + cell] = (jy + 0.5f * p.fb[1]) / rho;
  out[3 * N + cell] = (jz + 0.5f * p.fb[2]) / rho;
}

hipError_t launch_moments(int storage, const Geo& g, const Phys& p, const void* src,
                          float* out, hipStream_t s) {
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const unsigned nb = (unsigned)((N + 255) / 256);
  switch (storage) {
    case ST_F32: k_moments<StF32><<<nb, 256, 0, s>>>(g, p, static_cast<const float*>(src), out); break;
    case ST_F16: k_moments<StF16><<<nb, 256, 0, s>>>(g, p, static_cast<const __half*>(src), out); break;
    default: k_moments<StBF16><<<nb, 256, 0, s>>>(g, p, static_cast<const unsigned short*>(src), out); break;
  }
  return hipGetLastError();
}

__global__ void k_mass_reduce(const double* part, int n, double ncells, double* out, long long step) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ncells + sh[0];
    out[1] = (double)step;
  }
}

hipError_t launch_mass_reduce(const double* part, int n, double ncells, double* out,
                              long long step, hipStream_t s) {
  k_mass_reduce<<<1, 256, 0, s>>>(part, n, ncells, out, step);
  return hipGetLastError();
}

// ---------------------------------------------------------------- markers --

// Eq. 14: (1 + cos(pi |r| / 2)) / 4 for |r| <= 2, else 0.
__device__ __forceinline__ double delta_k(double r) {
  r = fabs(r);
  return r <= 2.0 ? 0.25 * (1.0 + cos(0.5 * M_PI * r)) : 0.0;
}

// Chord angle, its rate, pivot position and velocity at time t
// (Eqs. 20-21, 23; ABS_SIN takes the forward derivative at the kinks, the
// kink located from the half-period phase so that every side agrees).
__device__ void wing_pose(const WingDev& w, double t, double& th, double& thd, double& hx,
                          double& hy, double& vx, double& vy) {
  double al = w.mean, ald = 0.0;
  if (w.shape != 0) {
    const double om = 2.0 * M_PI / w.period;
    if (w.shape == 1) {
      const double arg = om * t + w.phase;
      al = w.mean + w.amp * sin(arg);
      ald = w.amp * om * cos(arg);
    } else {
      const double psi = t / w.period + w.phase / (2.0 * M_PI);
      const double h = psi - floor(2.0 * psi) / 2.0;
      al = w.mean + w.amp * sin(2.0 * M_PI * h);
      ald = w.amp * om * cos(2.0 * M_PI * h);
    }
  }
  th = w.theta0 + w.sense * al;
  thd = w.sense * ald;
  hx = w.hinge0[0];
  hy = w.hinge0[1];
  vx = 0.0;
  vy = 0.0;
  if (w.tamp != 0.0) {
    const double om = 2.0 * M_PI / w.period;
    const double arg = om * t + w.phase;
    const double cb = cos(w.tang), sb = sin(w.tang);
    hx += w.tamp * cos(arg) * cb;
    hy += w.tamp * cos(arg) * sb;
    vx = -w.tamp * om * sin(arg) * cb;
    vy = -w.tamp * om * sin(arg) * sb;
  }
}

__device__ __forceinline__ int find_wing(const MarkerArgs& a, int m) {
  int w = 0;
  for (int k = 1; k < a.nw; ++k)
    if (m >= a.w[k].moff) w = k;
  return w;
}

// Position of marker (p, s) of foil w.
__device__ __forceinline__ void marker_pos(const MarkerArgs& a, const WingDev& w, int p, int s,
                                           double c, double sn, double hx, double hy,
                                           double& X, double& Y, double& Z, double& rx, double& ry) {
  const double px = a.ref[w.ref_off + 2 * p], py = a.ref[w.ref_off + 2 * p + 1];
  rx = c * px - sn * py;
  ry = sn * px + c * py;
  X = hx + rx;
  Y = hy + ry;
  Z = s + 0.5;
}

// 1D weights of a point: nodes b .. b+3 with b = floor(X) - 1.
__device__ __forceinline__ int weights4(double X, double w[4]) {
  const double fb = floor(X) - 1.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = delta_k(fb + k - X);
  return (int)fb;
}

__device__ __forceinline__ int wrapi(int i, int n, int per) {
  if (!per) return i;
  i %= n;
  return i < 0 ? i + n : i;
}

// a(p, q) = sum_j delta(j - p) delta(j - q): 1D factor of Eq. 18.
__device__ __forceinline__ double a1(const double wp[4], int bp, double q, int n, int per) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double r = (double)(bp + k) - q;
    if (per) r -= n * rint(r / n);
    s += wp[k] * delta_k(r);
  }
  return s;
}

// Perimeter block of M = I I^T (Eq. 18 with dA factored out):
// M_xy[p][q] = a(x_p, x_q) a(y_p, y_q), inverted in place by Gauss-Jordan
// (symmetric positive definite, no pivoting), in FP64 in LDS.
__global__ void __launch_bounds__(256) k_factor(MarkerArgs a) {
  extern __shared__ double lds[];
  const WingDev& w = a.w[blockIdx.x];
  const int n = w.np;
  double* M = lds;                       // n*n
  double* px = lds + n * n;              // n x-positions
  double* py = px + n;
  double th, thd, hx, hy, vx, vy;
  wing_pose(w, a.t, th, thd, hx, hy, vx, vy);
  const double c = cos(th), sn = sin(th);
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    double X, Y, Z, rx, ry;
    marker_pos(a, w, p, 0, c, sn, hx, hy, X, Y, Z, rx, ry);
    px[p] = X;
    py[p] = Y;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int p = e / n, q = e - p * n;
    double wx[4], wy[4];
    const int bx = weights4(px[p], wx), by = weights4(py[p], wy);
    M[e] = a1(wx, bx, px[q], a.g.nx, a.g.bclo == BC_PERIODIC) *
           a1(wy, by, py[q], a.g.ny, a.g.yper);
  }
  __syncthreads();
  __shared__ int singular;
  if (threadIdx.x == 0) singular = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = M[k * n + k];
    if (!(piv > 1e-300)) {
      if (threadIdx.x == 0) singular = 1;
      break;
    }
    const double ip = 1.0 / piv;
    __syncthreads();
    // column k of the other rows (saved before the row update overwrites it)
    double* colk = py;  // reuse: positions no longer needed
    for (int i = threadIdx.x; i < n; i += blockDim.x) colk[i] = M[i * n + k];
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) M[k * n + j] = (j == k ? 1.0 : M[k * n + j]) * ip;
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e - i * n;
      if (i == k) continue;
      const double base = (j == k) ? 0.0 : M[e];
      M[e] = base - colk[i] * M[k * n + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (singular && threadIdx.x == 0) atomicOr(a.flags, 2);
  double* out = a.Minv + w.minv_off;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) out[e] = M[e];
}

// One wave per marker, one lane per node of its 4x4x4 support.
template <class St>
__global__ void __launch_bounds__(256) k_interp(MarkerArgs a) {
  using T = typename St::T;
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= a.m_total) return;
  const int wi = find_wing(a, m);
  const WingDev& w = a.w[wi];
  const int local = m - w.moff;
  const int p = local / w.ns, s = local - p * w.ns;
  double th, thd, hx, hy, vx, vy;
  wing_pose(w, a.t, th, thd, hx, hy, vx, vy);
  const double c = cos(th), sn = sin(th);
  double X, Y, Z, rx, ry;
  marker_pos(a, w, p, s, c, sn, hx, hy, X, Y, Z, rx, ry);
  double wx[4], wy[4], wz[4];
  const int bx = weights4(X, wx), by = weights4(Y, wy), bz = weights4(Z, wz);
  const int ox = lane & 3, oy = (lane >> 2) & 3, oz = lane >> 4;
  const Geo& g = a.g;
  const int nx = wrapi(bx + ox, g.nx, g.bclo == BC_PERIODIC);
  const int ny = wrapi(by + oy, g.ny, g.yper);
  const int nz = wrapi(bz + oz, g.nz, g.zper);
  const double Dw = wx[ox] * wy[oy] * wz[oz];
  float f[kQ];
  pull19<St>(static_cast<const T*>(a.src), g, nx, ny, nz, f);
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    drho += f[i];
    jx += cxq(i) * f[i];
    jy += cyq(i) * f[i];
    jz += czq(i) * f[i];
  }
  const float rho = 1.0f + drho;
  const float ux = (jx + 0.5f * a.p.fb[0]) / rho;
  const float uy = (jy + 0.5f * a.p.fb[1]) / rho;
  const float uz = (jz + 0.5f * a.p.fb[2]) / rho;
  double s0 = Dw * (double)rho, s1 = Dw * (double)ux, s2 = Dw * (double)uy, s3 = Dw * (double)uz;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off);
    s1 += __shfl_xor(s1, off);
    s2 += __shfl_xor(s2, off);
    s3 += __shfl_xor(s3, off);
  }
  if (lane == 0) {
    const double Ux = vx - thd * ry, Uy = vy + thd * rx, Uz = 0.0;
    a.X[3 * m] = X; a.X[3 * m + 1] = Y; a.X[3 * m + 2] = Z;
    a.U[3 * m] = Ux; a.U[3 * m + 1] = Uy; a.U[3 * m + 2] = Uz;
    a.rhoB[m] = s0;
    a.B[3 * m] = Ux - s1;                 // Eq. 19: B = U_B - I u*
    a.B[3 * m + 1] = Uy - s2;
    a.B[3 * m + 2] = Uz - s3;
  }
}

// Block (foil w, span layer s): y = (M_xy^-1 (x) M_z^+) B restricted to the
// n_p markers of layer s, du_B = y / dA, and the force/moment of the layer.
__global__ void __launch_bounds__(256) k_solve(MarkerArgs a) {
  __shared__ double Cs[kMaxPerim * 3];
  __shared__ double red[4][256];
  __shared__ int last;
  int wi = 0, blk = blockIdx.x;
  while (wi + 1 < a.nw && blk >= a.w[wi].ns) { blk -= a.w[wi].ns; ++wi; }
  const WingDev& w = a.w[wi];
  const int s = blk, n = w.np, ns = w.ns;
  const double* G = a.G + w.g_off;
  // span convolution with the circulant pseudo-inverse row G
  for (int e = threadIdx.x; e < 3 * n; e += blockDim.x) {
    const int p = e / 3, comp = e - 3 * p;
    const double* Bp = a.B + 3 * (size_t)(w.moff + p * ns) + comp;
    double acc = 0.0;
    for (int s2 = 0; s2 < ns; ++s2) {
      int d = s - s2;
      if (d < 0) d += ns;
      acc += G[d] * Bp[3 * s2];
    }
    Cs[e] = acc;
  }
  __syncthreads();
  // perimeter inverse, then du_B and the per-marker body force -2 rho_B y
  const double* Mi = a.Minv + w.minv_off;
  double th, thd, hx, hy, vx, vy;
  wing_pose(w, a.t, th, thd, hx, hy, vx, vy);
  double fx = 0.0, fy = 0.0, fz = 0.0, mz = 0.0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    double y0 = 0.0, y1 = 0.0, y2 = 0.0;
    for (int q = 0; q < n; ++q) {
      const double mv = Mi[p * n + q];
      y0 += mv * Cs[3 * q];
      y1 += mv * Cs[3 * q + 1];
      y2 += mv * Cs[3 * q + 2];
    }
    const size_t m = (size_t)w.moff + (size_t)p * ns + s;
    a.duB[3 * m] = y0 / w.dA;
    a.duB[3 * m + 1] = y1 / w.dA;
    a.duB[3 * m + 2] = y2 / w.dA;
    const double r = a.rhoB[m];
    const double bx = -2.0 * r * y0, by = -2.0 * r * y1, bz = -2.0 * r * y2;   // Eq. 26, on the body
    fx += bx;
    fy += by;
    fz += bz;
    mz += (a.X[3 * m] - hx) * by - (a.X[3 * m + 1] - hy) * bx;
  }
  red[0][threadIdx.x] = fx;
  red[1][threadIdx.x] = fy;
  red[2][threadIdx.x] = fz;
  red[3][threadIdx.x] = mz;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  double* fp = a.fpart + 4 * ((size_t)w.layer_off + s);   // layer partials of this foil
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) fp[k] = red[k][0];
    __threadfence();
    const unsigned prev = atomicAdd(&a.counters[wi], 1u);
    last = (prev == (unsigned)(ns - 1));
  }
  __syncthreads();
  if (!last) return;
  // last layer of this foil: fixed-order sum over layers -> history row
  if (threadIdx.x == 0) {
    __threadfence();
    const double* base = a.fpart + 4 * (size_t)w.layer_off;
    double F[4] = {0.0, 0.0, 0.0, 0.0};
    for (int l = 0; l < ns; ++l)
      for (int k = 0; k < 4; ++k) F[k] += base[4 * l + k];
    const double qS = 0.5 * a.u_ref * a.u_ref * a.area_ref;
    double* h = a.hist + ((size_t)a.hist_row * a.nw + wi) * 8;
    h[0] = F[0];
    h[1] = F[1];
    h[2] = F[2];
    h[3] = F[3];
    h[4] = -w.sense * F[1] / qS;    // lift: lateral, outward for a mirrored pair
    h[5] = -F[0] / qS;              // thrust
    h[6] = F[0] / qS;               // drag = -thrust
    h[7] = F[3] / (qS * w.chord);
    a.counters[wi] = 0u;
  }
}

// One wave per marker: du(x) += D dA du_B at each node of its support.
__global__ void __launch_bounds__(256) k_spread(MarkerArgs a) {
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= a.m_total) return;
  const int wi = find_wing(a, m);
  const WingDev& w = a.w[wi];
  const double X = a.X[3 * m], Y = a.X[3 * m + 1], Z = a.X[3 * m + 2];
  double wx[4], wy[4], wz[4];
  const int bx = weights4(X, wx), by = weights4(Y, wy), bz = weights4(Z, wz);
  const int ox = lane & 3, oy = (lane >> 2) & 3, oz = lane >> 4;
  const Geo& g = a.g;
  const int nx = wrapi(bx + ox, g.nx, g.bclo == BC_PERIODIC);
  const int ny = wrapi(by + oy, g.ny, g.yper);
  const int nz = wrapi(bz + oz, g.nz, g.zper);
  const double wgt = wx[ox] * wy[oy] * wz[oz] * w.dA;
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const size_t cell = ((size_t)nz * g.ny + ny) * g.nx + nx;
  if (wgt != 0.0) {
    unsafeAtomicAdd(a.du + cell, (float)(wgt * a.duB[3 * m]));
    unsafeAtomicAdd(a.du + N + cell, (float)(wgt * a.duB[3 * m + 1]));
    unsafeAtomicAdd(a.du + 2 * N + cell, (float)(wgt * a.duB[3 * m + 2]));
  }
  const int tile = ((nz >> 3) * a.tny + (ny >> 3)) * a.tnx + (nx >> 3);
  a.stamps[tile] = a.stamp;
}

hipError_t launch_markers(int storage, const MarkerArgs& a, hipStream_t s) {
  int maxnp = 0, nlayers = 0;
  for (int k = 0; k < a.nw; ++k) {
    maxnp = a.w[k].np > maxnp ? a.w[k].np : maxnp;
    nlayers += a.w[k].ns;
  }
  const size_t lds = ((size_t)maxnp * maxnp + 2 * (size_t)maxnp) * sizeof(double);
  if (lds > 65536) {
    hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(k_factor),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  k_factor<<<a.nw, 256, lds, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned nbm = (unsigned)((a.m_total + 3) / 4);
  switch (storage) {
    case ST_F32: k_interp<StF32><<<nbm, 256, 0, s>>>(a); break;
    case ST_F16: k_interp<StF16><<<nbm, 256, 0, s>>>(a); break;
    default: k_interp<StBF16><<<nbm, 256, 0, s>>>(a); break;
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_solve<<<nlayers, 256, 0, s>>>(a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_spread<<<nbm, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace ibmk
