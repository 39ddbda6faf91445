// gfx950 lattice kernels of the D3Q19 BGK + implicit-IBM time step.
//
//  collide   fused pull-streaming, moments, IBM velocity correction, Guo
//            forcing and BGK relaxation over every cell (Eqs. 1-11, 16, 26);
//            rebuilds the entering populations of Zou-He face cells where a
//            solve has such faces; writes the x-face ghost layer of the next
//            state; on steps with foils, block 0 makes the fixed-order force
//            sum and the coefficients.
//  ghost     the same ghost rule for a freshly initialised state.
//  init_eq   equilibrium initial state from rho, u.
//  moments   rho and velocity of every cell (read-back).
//  mass      fixed-order sum of the per-block mass partials.
//
// Distributions are stored as deviations from the lattice weights,
// f~_i = f_i - w_i, so FP32 (and 16-bit) storage keeps the small velocity
// signal out of the rounding of the O(w_i) rest value.
#include "lattice_dev.h"

namespace ibmk {

// ---------------------------------------------------------------- collide --

// True if (x, y) lies in the node box of foil w.
__device__ __forceinline__ bool in_box(const FoilBox& b, int x, int y) {
  return y >= b.y0 && y < b.y0 + b.h && x >= b.x0 && x < b.x0 + b.w;
}

// du(x) of the IBM correction (Eq. 15): the sum over foils and the 4 span
// layers within reach of the layer images written by the spread kernel.
// Returns whether the cell is a support node of a foil's markers (elsewhere
// the correction is exactly zero and the images are not read).
__device__ __forceinline__ bool correction(const CollideArgs& a, int x, int y, int z, float& dux,
                                           float& duy, float& duz) {
  const Geo& g = a.g;
  dux = duy = duz = 0.f;
  bool hit = false;
  for (int w = 0; w < a.nw; ++w) {
    const FoilBox& b = a.box[w];
    if (y < b.y0 || y >= b.y0 + b.h) continue;         // wave-uniform: most rows miss
    if (!in_box(b, x, y)) continue;
    const int lx = x - b.x0, ly = y - b.y0;
    if (!((b.bits[ly * b.words + (lx >> 5)] >> (lx & 31)) & 1u)) continue;   // zero there
    hit = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int s = z - 2 + k;
      s = s < 0 ? s + g.nz : (s >= g.nz ? s - g.nz : s);
      s = s < 0 ? s + g.nz : s;                        // a span of one layer wraps twice
      const float4 v = b.corr[((long long)s * b.side + ly) * b.side + lx];
      dux += a.wz[k] * v.x;
      duy += a.wz[k] * v.y;
      duz += a.wz[k] * v.z;
    }
  }
  return hit;
}

// One cell update: pull-streaming, the Zou-He rebuild at the x faces (ZH:
// the solve has Zou-He faces), moments, optional IBM velocity
// correction and Guo forcing, BGK relaxation, streaming store of the
// post-collision values and, at x = 0 / nx-1, the ghost layer of the next
// state.  Returns the density deviation of the pre-collision state.
// Everything is computed in stored units
// (kS f~): the moments, the equilibrium (Eq. 4, with rho scaled) and the
// Guo term (Eq. 8, with F scaled) are linear in the distributions, and kS is
// a power of two, so the result is the same as in units of f~.
template <class St, bool IBM, bool FORCE, bool ZH = false>
__device__ __forceinline__ float collide_cell(const CollideArgs& a, const typename St::T* __restrict__ S,
                                              typename St::T* __restrict__ D, int x, int y, int z) {
  using T = typename St::T;
  constexpr float kS = St::kS, kInv = St::kInv;
  const Geo& g = a.g;
  float f[kQ];
  // wave-uniform row: the scalar-base pull where no y or z wall reflects
  // into the row
  if (pull_rows_inside(g, y, z))
    pull19_rows<St>(S, g, x, y, z, f);
  else
    pull19<St, true>(S, g, x, y, z, f);
  // IBM correction: with Zou-He faces it is fetched while the pull is in
  // flight (measured faster there), else after the moments
  float dux = 0.f, duy = 0.f, duz = 0.f;
  bool hit = false;
  if (IBM && ZH) hit = correction(a, x, y, z, dux, duy, duz);
  if constexpr (ZH) {
    // Zou-He x faces: rebuild the entering populations at the face lanes
    // (the rule of zou_he, each face's branch on its own so the rest of
    // the row keeps f in registers)
    if ((g.yper || (y > 0 && y < g.ny - 1)) && (g.zper || (z > 0 && z < g.nz - 1))) {
      if (x == 0 && g.bclo >= BC_ZH_VELOCITY) zou_he_face<St, true, 1>(a.p, g.bclo, f);
      if (x == g.nx - 1 && x != 0 && g.bchi >= BC_ZH_VELOCITY) zou_he_face<St, true, -1>(a.p, g.bchi, f);
    }
  }
  float dr, jx, jy, jz;                            // kS drho, kS j
  moments19(f, dr, jx, jy, jz);
  const float drho = dr * kInv;
  const float rho = 1.0f + drho;
  const float srho = kS * rho;
  const float inv = 1.0f / srho;
  float Fx = 0.f, Fy = 0.f, Fz = 0.f;                // kS F
  if (FORCE) {
    Fx = kS * a.p.fb[0]; Fy = kS * a.p.fb[1]; Fz = kS * a.p.fb[2];
    jx += 0.5f * Fx; jy += 0.5f * Fy; jz += 0.5f * Fz;
  }
  float ux = jx * inv, uy = jy * inv, uz = jz * inv;
  bool forced = FORCE;
  if (IBM) {
    if (!ZH) hit = correction(a, x, y, z, dux, duy, duz);
    if (hit) {
      ux += dux; uy += duy; uz += duz;                 // Eq. 16
      Fx += 2.0f * srho * dux;                         // Eq. 11 / Eq. 26
      Fy += 2.0f * srho * duy;
      Fz += 2.0f * srho * duz;
      forced = true;
    }
  }
  const float usq = ux * ux + uy * uy + uz * uz;
  const float om = a.p.omega;
  // Equilibrium (Eq. 4) by opposite pairs: with cu_opp = -cu, the even part
  // w (drho + rho (4.5 cu^2 - 1.5 u^2)) is shared and the odd part 3 w rho cu
  // changes sign, so each pair costs one evaluation
  const float c15 = 1.5f * usq;
  const float k1[2] = {wq(1) * srho, wq(7) * srho}, k3[2] = {3.0f * wq(1) * srho, 3.0f * wq(7) * srho},
              kd[2] = {wq(1) * dr, wq(7) * dr};
  float o[kQ];
  o[0] = f[0] - om * (f[0] - (wq(0) * dr - wq(0) * srho * c15));
#pragma unroll
  for (int i = 1; i < kQ; ++i) {
    if (oppq(i) < i) continue;
    const int c = i < 7 ? 0 : 1;                       // axis or diagonal weight
    const float cu = cdot(i, ux, uy, uz);
    const float A = k1[c] * (4.5f * cu * cu - c15) + kd[c];
    const float B = k3[c] * cu;
    const float fp = A + B, fm = A - B;                // feq of i and of opp(i)
    o[i] = f[i] - om * (f[i] - fp);
    o[oppq(i)] = f[oppq(i)] - om * (f[oppq(i)] - fm);
  }
  if (forced) {
    const float k = a.p.guo_k;
    const float uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const float cu = cdot(i, ux, uy, uz);
      const float cF = cdot(i, Fx, Fy, Fz);
      o[i] += k * wq(i) * (3.0f * (cF - uF) + 9.0f * cu * cF);   // Eq. 8
    }
  }
  T* own = D + rowbase(g, y, z);
  if constexpr (sizeof(T) == 2) {
    // 16-bit storage: one buffer descriptor over the cell row's 19
    // population rows, so each store takes its row as a scalar offset and
    // the lane's x as the vector offset, with no per-store address
    // arithmetic (FP32 measured faster with plain stores)
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(own, 0, (int)(kQ * g.ps * (long long)sizeof(T)), kRawBufferWord3);
    const int bo = x * (int)sizeof(T);
#pragma unroll
    for (int i = 0; i < kQ; ++i) St::stb(rs, bo, (int)(i * g.ps * (long long)sizeof(T)), o[i]);
  } else {
#pragma unroll
    for (int i = 0; i < kQ; ++i) St::stnr(own + (long long)i * g.ps + x, o[i]);
  }
  if (x == 0 || x == g.nx - 1) {
#pragma unroll
    for (int i = 0; i < kQ; ++i) o[i] *= kInv;
    write_ghosts<St>(D, g, a.p, x, y, z, o);
  }
  return drho;
}

// Block 0 of a collide launch after the marker kernels: per foil, the sum
// over span layers of the layer forces and moments in a fixed order, the
// coefficients (Sec. 3.6-3.7: lift is the lateral component, counted outward
// for a mirrored pair; thrust is -F_x; drag = -thrust) and the history row.
__device__ void reduce_forces(const CollideArgs& a) {
  __shared__ double red[4][kBlockX * kBlockRows];
  const int t = threadIdx.y * kBlockX + threadIdx.x, nt = kBlockX * kBlockRows;
  for (int w = 0; w < a.nw; ++w) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const double* fp = a.fpart + 4 * (size_t)w * a.g.nz;
    for (int l = t; l < a.g.nz; l += nt)
      for (int k = 0; k < 4; ++k) v[k] += fp[4 * l + k];
    for (int k = 0; k < 4; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int h = nt / 2; h > 0; h >>= 1) {
      if (t < h)
        for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + h];
      __syncthreads();
    }
    if (t == 0) {
      const double F0 = red[0][0], F1 = red[1][0], F2 = red[2][0], F3 = red[3][0];
      double* h = a.hist + ((size_t)a.hist_row * a.nw + w) * 8;
      h[0] = F0;
      h[1] = F1;
      h[2] = F2;
      h[3] = F3;
      h[4] = -a.sense[w] * F1 / a.qS;
      h[5] = -F0 / a.qS;
      h[6] = F0 / a.qS;
      h[7] = F3 / (a.qS * a.chord[w]);
    }
    __syncthreads();
  }
}

// Every cell, one row per wave, 64 cells along x per wave, 4 waves per block.
template <class St, bool IBM, bool FORCE, bool CHECK, bool ZH>
__device__ __forceinline__ void collide_block(const CollideArgs& __restrict__ a, int lb,
                                              const void* src, void* dst) {
  using T = typename St::T;
  const Geo& g = a.g;
  const T* __restrict__ S = static_cast<const T*>(src);
  T* __restrict__ D = static_cast<T*>(dst);
  if (IBM && lb == 0) reduce_forces(a);
  // Waves to (64-cell chunk, row).  FP32: a block is one chunk of 4
  // consecutive rows (tiles in XCD runs, below).  16-bit storage: waves run along x first, so the
  // chunks of a row sit in one block and the cache line each chunk shares
  // with its neighbour (the x -/+ 1 pulls) is fetched from memory once; at
  // 2 bytes a wave reads a single line per population row, so these shared
  // lines are a large part of its reads.
  int xc, row;
  if (sizeof(T) == 2) {
    const int gw = __builtin_amdgcn_readfirstlane(lb * kBlockRows + (int)threadIdx.y);
    row = a.nxc_mul ? (int)__umulhi((unsigned)gw, a.nxc_mul) : gw / a.nxc;
    xc = gw - row * a.nxc;
  } else {
    // Workgroups are dealt to the 8 XCDs in turn; a single solve's tiles are
    // reordered so that each XCD takes runs of 4 block rows (all chunks of
    // 16 lattice rows; 8 block rows where a row has 8 or more chunks,
    // measured faster there: 512x384x384 -1.1%, 256-cell rows +0.3%), and
    // the cache lines two chunks of a row share are fetched by one L2.
    // Bijective on the tiles; grouped launches keep the plain order.
    int lt = lb;
    const int G = (a.nxc >= 8 ? 8 : 4) * a.nxc;
    const int M = (int)(gridDim.x / (8 * G)) * 8 * G;
    if (lt < M && (int)gridDim.x == a.nblocks) {
      const int xcd = lt & 7, k = lt >> 3;
      lt = ((k / G) * 8 + xcd) * G + k % G;
    }
    xc = lt % a.nxc;
    row = (lt / a.nxc) * kBlockRows + (int)threadIdx.y;
  }
  const int x = xc * kBlockX + threadIdx.x;
  // one row per wave: make the row index wave-uniform for the compiler
  row = __builtin_amdgcn_readfirstlane(row);
  const bool active = x < g.nx && row < g.ny * g.nz;
  double dm = 0.0;
  bool bad = false;
  if (active) {
    const int z = __builtin_amdgcn_readfirstlane(
        sizeof(T) == 2 && a.ny_mul ? (int)__umulhi((unsigned)row, a.ny_mul) : row / g.ny);
    const int y = __builtin_amdgcn_readfirstlane(row - z * g.ny);
    const float drho = collide_cell<St, IBM, FORCE, ZH>(a, S, D, x, y, z);
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

// A grouped collide launch also carries each solve's state buffers as
// kernel arguments, so the compiler knows they are global memory.
struct CollideGroup {
  Group g;
  const void* src[kMaxGroup];
  void* dst[kMaxGroup];
};

template <class St, bool IBM, bool FORCE, bool CHECK, bool ZH>
__global__ void __launch_bounds__(kBlockX * kBlockRows)
k_collide(CollideGroup gr) {
  int lb;
  const int k = group_index(gr.g, lb);
  const CollideArgs* a = static_cast<const CollideArgs*>(gr.g.args[k]);
  collide_block<St, IBM, FORCE, CHECK, ZH>(*a, lb, gr.src[k], gr.dst[k]);
}

// One instantiation per (foils, body force, check step, Zou-He faces): the
// solves without Zou-He faces run a kernel without the rebuild.
template <class St, bool IBM, bool FORCE>
static hipError_t launch_collide_c(bool check, bool zh, const CollideGroup& g, int blocks, hipStream_t s) {
  const dim3 b(kBlockX, kBlockRows);
  switch ((check ? 2 : 0) | (zh ? 1 : 0)) {
    case 0: k_collide<St, IBM, FORCE, false, false><<<blocks, b, 0, s>>>(g); break;
    case 1: k_collide<St, IBM, FORCE, false, true><<<blocks, b, 0, s>>>(g); break;
    case 2: k_collide<St, IBM, FORCE, true, false><<<blocks, b, 0, s>>>(g); break;
    default: k_collide<St, IBM, FORCE, true, true><<<blocks, b, 0, s>>>(g); break;
  }
  return hipGetLastError();
}

template <class St>
static hipError_t launch_collide_s(bool ibm, bool force, bool check, bool zh, const CollideGroup& g,
                                   int blocks, hipStream_t s) {
  switch ((ibm ? 2 : 0) | (force ? 1 : 0)) {
    case 0: return launch_collide_c<St, false, false>(check, zh, g, blocks, s);
    case 1: return launch_collide_c<St, false, true>(check, zh, g, blocks, s);
    case 2: return launch_collide_c<St, true, false>(check, zh, g, blocks, s);
    default: return launch_collide_c<St, true, true>(check, zh, g, blocks, s);
  }
}

hipError_t launch_collide(int storage, bool ibm, bool force, bool check, bool zh,
                          const CollideArgs* const* host, const void* const* dev, int n,
                          hipStream_t s) {
  if (n < 1 || n > kMaxGroup) return hipErrorInvalidValue;
  CollideGroup g;
  int blocks[kMaxGroup];
  for (int k = 0; k < n; ++k) {
    blocks[k] = host[k]->nblocks;
    g.src[k] = host[k]->src;
    g.dst[k] = host[k]->dst;
  }
  const int total = group_fill(g.g, dev, blocks, n);
  if (total == 0) return hipSuccess;
  switch (storage) {
    case ST_F32: return launch_collide_s<StF32>(ibm, force, check, zh, g, total, s);
    case ST_F16: return launch_collide_s<StF16>(ibm, force, check, zh, g, total, s);
    default: return launch_collide_s<StBF16>(ibm, force, check, zh, g, total, s);
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
  zou_he<St, false>(g, p, x, y, z, f);
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

}  // namespace ibmk
