// gfx950 marker kernels of the implicit IBM (Sec. 2.2).
//
//  factor    marker kinematics (Eqs. 20-23), the perimeter block of the
//            no-slip matrix and its inverse (Eq. 18), for a window of steps.
//  band      rho, u* over the node box of each foil (Eqs. 2, 11).
//  interp_span  per marker, on every span layer: delta interpolation of rho
//            and u* (Eqs. 14, 17), B = U_B - I u* (Eq. 19), and the span part
//            of the minimum-norm solve (Eq. 19).
//  layer     the perimeter part of the solve, du_B, the force and moment of
//            each layer (Eq. 26) and sum_l du_B D dA over the layer (Eq. 15).
#include "lattice_dev.h"
#include "kinematics.h"

namespace ibmk {

// ---------------------------------------------------------------- markers --
//
// An extruded foil has the same perimeter section on every span layer
// z = s + 1/2, so D = delta_x delta_y delta_z splits into a perimeter part
// (per step) and a span part whose node weights are the constants
// delta(1.5), delta(0.5), delta(0.5), delta(1.5).  The no-slip matrix is then
// M_xy (x) M_z with M = I I^T, and its minimum-norm solution is
// (M_xy^-1 (x) M_z^+) B (Eqs. 18-19).
//
// Per-step perimeter record (stride kPw doubles): X, Y, rx, ry, wx[4], wy[4],
// bx, by; rx, ry = R(theta) ref, bx/by = floor(X) - 1 (first support node).
constexpr int kPw = 14;

// Eq. 14: (1 + cos(pi |r| / 2)) / 4 for |r| <= 2, else 0.
__device__ __forceinline__ double delta_k(double r) {
  r = fabs(r);
  return r <= 2.0 ? 0.25 * (1.0 + cos(0.5 * M_PI * r)) : 0.0;
}

// a(p, q) = sum_j delta(j - X_p) delta(j - X_q) from the two 4-node weight
// sets (1D factor of Eq. 18).
// Branch-free: every weight is loaded whatever the offset, so the loads of
// many entries can be in flight together; a term outside the overlap adds
// an exact zero.
__device__ __forceinline__ double a1(const double* wp, int bp, const double* wq, int bq) {
  const int d = bq - bp;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int kk = k - d;
    const bool in = kk >= 0 && kk < 4;
    const double t = wp[k] * wq[in ? kk : 0];
    s += in ? t : 0.0;
  }
  return s;
}

// Perimeter positions and weights of foil `wi` at time t, the block
// M_xy[p][q] = a(X_p, X_q) a(Y_p, Y_q) and its inverse by in-place
// Gauss-Jordan (symmetric positive definite: no pivoting), FP64 in
// registers.
// These depend on the prescribed kinematics only, so they are computed for a
// window of future steps at once, one block per (step, foil).
template <int NT>
__device__ __forceinline__ void factor_block(const MarkerArgs& __restrict__ a, int lb) {
  extern __shared__ double lds[];
  const int slot = lb / a.nw, wi = lb - slot * a.nw;
  const WingDev& w = a.w[wi];
  const int n = w.np;
  double* P = lds;              // n * kPw
  double* CR = P + n * kPw;     // 2 sets of (column k, row k) of the elimination, 4 n
  double th, thd, hx, hy, vx, vy;
  wing_pose(w, (double)(a.win_t0 + slot), th, thd, hx, hy, vx, vy);
  const double c = cos(th), sn = sin(th);
  double* Pg = a.pw + (size_t)slot * a.pw_step + w.pw_off;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const double px = a.ref[w.ref_off + 2 * p], py = a.ref[w.ref_off + 2 * p + 1];
    const double rx = c * px - sn * py, ry = sn * px + c * py;
    const double X = hx + rx, Y = hy + ry;
    double* r = P + p * kPw;
    r[0] = X;
    r[1] = Y;
    r[2] = rx;
    r[3] = ry;
    const double fx = floor(X) - 1.0, fy = floor(Y) - 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      r[4 + k] = delta_k(fx + k - X);
      r[8 + k] = delta_k(fy + k - Y);
    }
    r[12] = fx;
    r[13] = fy;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * kPw; e += blockDim.x) Pg[e] = P[e];
  {
    // support nodes of this step's node box: bit (lx, ly) for every node
    // floor(X) - 1 .. floor(X) + 2 of every marker (the nodes the
    // interpolation reads), relative to the box origin of that step; then
    // the set bits as a row-major list of ly << 16 | lx after their count
    const WingDev& ws = a.win_args[slot].w[wi];
    const int words = w.mask_words, rows = w.side;
    unsigned* bits = reinterpret_cast<unsigned*>(CR + 4 * n);   // side * words words
    int* rc = reinterpret_cast<int*>(bits + rows * words);    // side row counts
    for (int e = threadIdx.x; e < rows * words; e += blockDim.x) bits[e] = 0u;
    __syncthreads();
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
      const int bx = (int)P[p * kPw + 12] - ws.x0, by = (int)P[p * kPw + 13] - ws.y0;
      for (int oy = 0; oy < 4; ++oy)
        for (int ox = 0; ox < 4; ++ox) {
          const int lx = bx + ox, ly = by + oy;
          if (lx < 0 || ly < 0 || lx >= ws.bw || ly >= ws.bh) continue;
          atomicOr(&bits[ly * words + (lx >> 5)], 1u << (lx & 31));
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
      int c = 0;
      for (int q = 0; q < words; ++q) c += __popc(bits[r * words + q]);
      rc[r] = c;
    }
    __syncthreads();
    unsigned* out = a.sup + (size_t)slot * a.sup_step + w.sup_off;
    // the bitmap itself after the list, for the collide kernel
    for (int e = threadIdx.x; e < rows * words; e += blockDim.x) out[1 + 16 * n + e] = bits[e];
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
      int o = 0;
      for (int q = 0; q < r; ++q) o += rc[q];
      unsigned* e = out + 1 + o;
      for (int q = 0; q < words; ++q) {
        unsigned b = bits[r * words + q];
        while (b) {
          const int bit = __ffs(b) - 1;
          b &= b - 1;
          *e++ = ((unsigned)r << 16) | (unsigned)(q * 32 + bit);
        }
      }
      if (r == rows - 1) {
        out[0] = (unsigned)(o + rc[r]);
        // the band grid of that step covers sup_chunks * 64 entries
        if (o + rc[r] > 64 * ws.sup_chunks) atomicOr(a.flags, 4);
      }
    }
    __syncthreads();
  }
  // The block M[p][q] = a(X_p, X_q) a(Y_p, Y_q) and its inverse by
  // Gauss-Jordan without pivoting (symmetric positive definite), FP64.
  // Thread (ty, tx) of a 16 x 16 grid holds the elements (ty + 16 u,
  // tx + 16 v), u, v < NT (16 NT >= n), in registers; for pivot k the owners
  // of column k and of row k publish them in LDS (two sets, by the parity of
  // k, so one barrier per pivot).  Entries outside the n x n block are
  // carried along without branches and never read into the block.
  const int tx = (int)threadIdx.x & 15, ty = (int)threadIdx.x >> 4;
  double Mr[NT][NT];
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int v = 0; v < NT; ++v) {
      const int p = ty + 16 * u, q = tx + 16 * v;
      double val = 0.0;
      if (p < n && q < n) {
        const double* rp = P + p * kPw;
        const double* rq = P + q * kPw;
        val = a1(rp + 4, (int)rp[12], rq + 4, (int)rq[12]) * a1(rp + 8, (int)rp[13], rq + 8, (int)rq[13]);
      }
      Mr[u][v] = val;
    }
  __shared__ int singular;
  if (threadIdx.x == 0) singular = 0;
  for (int k = 0; k < n; ++k) {
    double* col = CR + (k & 1) * 2 * n;
    double* row = col + n;
    const int kb = k >> 4, kt = k & 15;
    if (tx == kt) {
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        double m = 0.0;
#pragma unroll
        for (int v = 0; v < NT; ++v) m = v == kb ? Mr[u][v] : m;
        if (ty + 16 * u < n) col[ty + 16 * u] = m;
      }
    }
    if (ty == kt) {
#pragma unroll
      for (int v = 0; v < NT; ++v) {
        double m = 0.0;
#pragma unroll
        for (int u = 0; u < NT; ++u) m = u == kb ? Mr[u][v] : m;
        if (tx + 16 * v < n) row[tx + 16 * v] = m;
      }
    }
    __syncthreads();
    const double piv = row[k];
    if (!(piv > 1e-300)) {
      if (threadIdx.x == 0) singular = 1;
      break;
    }
    const double ip = 1.0 / piv;
    double rk[NT];                                       // row k, scaled
#pragma unroll
    for (int v = 0; v < NT; ++v) {
      const int q = tx + 16 * v;
      rk[v] = (q == k ? 1.0 : row[q < n ? q : n - 1]) * ip;
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int p = ty + 16 * u;
      const double cp = col[p < n ? p : n - 1];
#pragma unroll
      for (int v = 0; v < NT; ++v) {
        const int q = tx + 16 * v;
        const double e = (q == k ? 0.0 : Mr[u][v]) - cp * rk[v];
        Mr[u][v] = p == k ? rk[v] : e;
      }
    }
  }
  __syncthreads();
  if (singular && threadIdx.x == 0) atomicOr(a.flags, 2);
  double* out = a.Minv + (size_t)slot * a.minv_step + w.minv_off;
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int v = 0; v < NT; ++v) {
      const int p = ty + 16 * u, q = tx + 16 * v;
      if (p < n && q < n) out[(size_t)p * n + q] = Mr[u][v];
    }
}

template <int NT>
__global__ void __launch_bounds__(256) k_factor(Group gr) {
  int lb;
  const MarkerArgs* a = static_cast<const MarkerArgs*>(group_find(gr, lb));
  factor_block<NT>(*a, lb);
}

// rho and u* = (sum c f + F_body/2)/rho (Eqs. 2, 9, 11) of the
// pre-collision state at the support nodes of every foil's markers, on every
// layer.  One wave per 64 entries of a foil's support list on one layer;
// waves past the list's length (the host sizes the grid from a bound) end at
// once.
template <class St>
__device__ __forceinline__ void band_block(const MarkerArgs& __restrict__ a, int lb) {
  using T = typename St::T;
  int R = __builtin_amdgcn_readfirstlane((int)(lb * 4 + (threadIdx.x >> 6)));
  const int lane = threadIdx.x & 63;
  int wi = 0;
  while (wi < a.nw) {
    const int units = a.w[wi].sup_chunks * a.g.nz;
    if (R < units) break;
    R -= units;
    ++wi;
  }
  if (wi >= a.nw) return;
  const WingDev& w = a.w[wi];
  const int z = R / w.sup_chunks, chunk = R - z * w.sup_chunks;
  const auto* list = gmem(a.sup + (size_t)a.slot * a.sup_step + w.sup_off);
  const int e = chunk * 64 + lane;
  // the count and the lane's entry are loaded together (the entry index
  // kept inside the list's 16 n_p entries), then the lane checks the count
  const int last = 16 * w.np;
  const unsigned cnt = list[0];
  const unsigned cell = list[1 + (e < last ? e : last - 1)];
  if (e >= (int)cnt) return;
  const int lx = (int)(cell & 0xffffu), ly = (int)(cell >> 16);
  float f[kQ];
  pull19<St>(static_cast<const T*>(a.src), a.g, w.x0 + lx, w.y0 + ly, z, f);
  zou_he<St, false>(a.g, a.p, w.x0 + lx, w.y0 + ly, z, f);
  float drho, jx, jy, jz;
  moments19(f, drho, jx, jy, jz);
  const float rho = 1.0f + drho;
  w.band[((long long)z * w.side + ly) * w.side + lx] =
      make_float4(rho, (jx + 0.5f * a.p.fb[0]) / rho, (jy + 0.5f * a.p.fb[1]) / rho, (jz + 0.5f * a.p.fb[2]) / rho);
}

template <class St>
__global__ void __launch_bounds__(256) k_band(Group gr) {
  int lb;
  const MarkerArgs* a = static_cast<const MarkerArgs*>(group_find(gr, lb));
  band_block<St>(*a, lb);
}

__device__ __forceinline__ int find_layer_block(const MarkerArgs& a, int blk, int& wi) {
  wi = 0;
  while (wi + 1 < a.nw && blk >= a.w[wi].ns) {
    blk -= a.w[wi].ns;
    ++wi;
  }
  return blk;
}

// Block (foil, perimeter marker p): the marker's delta interpolation on
// every span layer and the span part of the minimum-norm solve.
//  * D = D_xy wz factors, so per layer z the xy sum
//    R(z) = sum_nodes D_xy band(node, z) over the marker's 4 x 4 xy support
//    nodes is made once (FP64; a thread loads the 16 band records of its
//    layer together), and rho_B and
//    I u* at the marker on layer s are sum_k wz_k R(s - 1 + k), k = 0..3
//    (Eq. 17); B = U_B - I u* (Eq. 19).
//  * T(p, c, s) = sum_s2 G[(s - s2) mod ns] B(p, c, s2), G the pseudo-inverse
//    row of the circulant span factor: each item of the block makes the four
//    outputs t, t + Q, t + 2Q, t + 3Q (Q = ceil(ns / 4)) over one part of the
//    s2 range; the parts are added in a fixed order.  T is written
//    layer-major.
// One block holds every layer of its marker, so B never leaves the block.
__host__ __device__ inline int parts_at(int ns, int threads) {
  const int groups = (ns + 3) / 4;                   // threads per part
  const int parts = threads / groups;
  return parts < 1 ? 1 : (parts > 8 ? 8 : parts);
}

// LDS of a block: G (2 ns), B (3 ns), partial sums (parts x 3 ns) and the
// xy sums R (4 ns).
__host__ __device__ inline size_t interp_span_doubles(int ns, int parts) {
  const size_t d = (size_t)(9 + 3 * parts) * ns;
  return (d + 1) / 2 * 2;
}
__host__ __device__ inline size_t lds_at(int ns, int threads) {
  return interp_span_doubles(ns, parts_at(ns, threads)) * sizeof(double);
}

// Threads of an interp_span block for a span of ns layers: 512 (more parts
// of the span range in parallel) where its LDS fits, else 256.
__host__ __device__ inline int span_threads(int ns) { return lds_at(ns, 512) <= 150 * 1024 ? 512 : 256; }

// Parts of the span range and LDS of a block: fixed by ns alone, so a
// solve sums its span solve in the same order whatever block size a grouped
// launch runs it with (a smaller block takes the parts in turns).
__host__ __device__ inline int span_parts(int ns) { return parts_at(ns, span_threads(ns)); }
__host__ __device__ inline size_t interp_span_lds(int ns) { return lds_at(ns, span_threads(ns)); }

__device__ __forceinline__ void interp_span_block(const MarkerArgs& __restrict__ a, int lb) {
  extern __shared__ double lds[];
  // workgroups are dealt to the 8 XCDs in turn: blocks lb = 8 k + x take
  // the run of markers x * (M / 8) + k, so neighbouring markers, which
  // share most of their band records, read them through one L2 (a
  // permutation of the solve's blocks; the tail keeps the plain order)
  int tot = 0;
  for (int k = 0; k < a.nw; ++k) tot += a.w[k].np;
  const int per = tot >> 3;
  int wi = 0, p = lb < 8 * per ? (lb & 7) * per + (lb >> 3) : lb;
  while (wi + 1 < a.nw && p >= a.w[wi].np) {
    p -= a.w[wi].np;
    ++wi;
  }
  const WingDev& w = a.w[wi];
  const int ns = w.ns, n = w.np;
  const int groups = (ns + 3) / 4;
  const int parts = span_parts(ns);
  const int bd = (int)blockDim.x;
  double* G = lds;              // 2 * ns: G repeated so that G[d + ns] = G[d]
  double* Bc = G + 2 * ns;      // 3 * ns
  double* Pa = Bc + 3 * ns;     // parts * 3 * ns partial sums
  double* R = Pa + (size_t)parts * 3 * ns;                              // 4 * ns
  const auto* Gg = gmem(a.G + w.g_off);
  for (int i = threadIdx.x; i < ns; i += bd) {
    const double g = Gg[i];
    G[i] = g;
    G[i + ns] = g;
  }
  // the marker's record, read by every thread (one address per block), so
  // the band-record loads below wait on it and on nothing else
  double r[kPw];
  {
    const auto* rg = gmem(a.pw + (size_t)a.slot * a.pw_step + w.pw_off + (size_t)p * kPw);
#pragma unroll
    for (int k = 0; k < kPw; ++k) r[k] = rg[k];
  }
  const double thd = a.pose[wi][1], vx = a.pose[wi][4], vy = a.pose[wi][5];
  const double Ux = vx - thd * r[3], Uy = vy + thd * r[2];
  {
    // the 16 band records of layer z, loaded together straight from L2
    const int bx = (int)r[12] - w.x0, by = (int)r[13] - w.y0;
    typedef float v4f __attribute__((ext_vector_type(4)));   // one 16-byte load per record
    const auto* band = gmem(reinterpret_cast<const v4f*>(w.band));
    for (int z = threadIdx.x; z < ns; z += bd) {
      const auto* row0 = band + ((long long)z * w.side + by) * w.side + bx;
      v4f v[16];
#pragma unroll
      for (int node = 0; node < 16; ++node) v[node] = row0[(node >> 2) * w.side + (node & 3)];
      double R0 = 0.0, R1 = 0.0, R2 = 0.0, R3 = 0.0;
#pragma unroll
      for (int oy = 0; oy < 4; ++oy) {
#pragma unroll
        for (int ox = 0; ox < 4; ++ox) {
          const v4f q = v[oy * 4 + ox];
          const double D = r[4 + ox] * r[8 + oy];
          R0 += D * (double)q.x;
          R1 += D * (double)q.y;
          R2 += D * (double)q.z;
          R3 += D * (double)q.w;
        }
      }
      R[4 * z] = R0;
      R[4 * z + 1] = R1;
      R[4 * z + 2] = R2;
      R[4 * z + 3] = R3;
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < ns; s += bd) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int z = s - 1 + k;                             // the 4 layers of the span support
      z = z < 0 ? z + ns : (z >= ns ? z - ns : z);
      z = z >= ns ? z - ns : z;                      // a span of one layer wraps twice
      s0 += a.wz[k] * R[4 * z];
      s1 += a.wz[k] * R[4 * z + 1];
      s2 += a.wz[k] * R[4 * z + 2];
      s3 += a.wz[k] * R[4 * z + 3];
    }
    const size_t m = (size_t)w.moff + (size_t)p * ns + s;
    a.X[3 * m] = r[0];
    a.X[3 * m + 1] = r[1];
    a.X[3 * m + 2] = s + 0.5;
    a.U[3 * m] = Ux;
    a.U[3 * m + 1] = Uy;
    a.U[3 * m + 2] = 0.0;
    a.rhoB[m] = s0;
    const double b[3] = {Ux - s1, Uy - s2, 0.0 - s3};   // Eq. 19: B = U_B - I u*
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.B[3 * m + c] = b[c];
      Bc[c * ns + s] = b[c];
    }
  }
  __syncthreads();
  // items (part, four outputs t + j Q, j = 0..3, Q = ceil(ns / 4)) in turns
  // of the block: neighbouring threads read neighbouring G entries (no LDS
  // bank conflicts); each output sums its part of the s2 range in order
  const int Q = groups;
  for (int item = threadIdx.x; item < parts * Q; item += bd) {
    const int part = item / Q, t = item - part * Q;
    const int lo = part * ns / parts, hi = (part + 1) * ns / parts;
    double acc[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0;
    // output t + j Q takes G[(t + j Q - s2) mod ns] = G[t + j Q - s2 + ns]
    const double* G0 = G + t + ns;
#pragma unroll 4
    for (int s2 = lo; s2 < hi; ++s2) {
      const double b0 = Bc[s2], b1 = Bc[ns + s2], b2 = Bc[2 * ns + s2];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double g = G0[j * Q - s2];
        acc[j][0] += g * b0;
        acc[j][1] += g * b1;
        acc[j][2] += g * b2;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int so = t + j * Q;
      if (so < ns)
        for (int c = 0; c < 3; ++c) Pa[((size_t)part * ns + so) * 3 + c] = acc[j][c];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * ns; e += bd) {
    const int sj = e / 3, c = e - 3 * sj;
    double v = 0.0;
    for (int q = 0; q < parts; ++q) v += Pa[((size_t)q * ns + sj) * 3 + c];
    a.T[w.c_off + ((size_t)sj * n + p) * 3 + c] = v;
  }
}

__global__ void __launch_bounds__(512) k_interp_span(Group gr) {
  int lb;
  const MarkerArgs* a = static_cast<const MarkerArgs*>(group_find(gr, lb));
  interp_span_block(*a, lb);
}

// Block (foil, span layer s): the perimeter part of the solve,
// y(p) = sum_q M_xy^-1[p][q] T(q, s), du_B = y / dA (Eqs. 18-19); the body
// force and moment of the layer, -2 rho_B y (Eq. 26), reduced in a fixed
// order; and the xy image of sum_p du_B D_xy dA over the foil's box (Eq. 15
// without the span factor, which the collide kernel applies) at the
// support nodes of the step.  The image is built in `a.copies` partial
// images, each added by one wave over the markers p = copy (mod copies) in
// order, then summed copy by copy, so the sums are the same on every run.  The perimeter inverse is read from L2
// (measured faster than staging it in LDS, also where it fits).
__device__ __forceinline__ void layer_block(const MarkerArgs& __restrict__ a, int lb) {
  extern __shared__ double lds[];
  __shared__ double red[4][256];
  int wi;
  const int s = find_layer_block(a, lb, wi);
  const WingDev& w = a.w[wi];
  const int n = w.np, ns = w.ns, cells = w.bw * w.bh, copies = a.copies;
  const double* Minv_g = a.Minv + (size_t)a.slot * a.minv_step + w.minv_off;
  double* P = lds;                                   // n * kPw
  double* Tl = P + n * kPw;                          // n * 3
  double* Y = Tl + 3 * n;                            // n * 3
  float* img = reinterpret_cast<float*>(Y + 3 * n);  // copies * cells * 3
  // rho_B of this thread's first marker, fetched while the block loads
  const int p0 = (int)threadIdx.x;
  const double rho_p0 = p0 < n ? gmem(a.rhoB)[(size_t)w.moff + (size_t)p0 * ns + s] : 0.0;
  copy_to_lds(P, a.pw + (size_t)a.slot * a.pw_step + w.pw_off, n * kPw);
  copy_to_lds(Tl, a.T + w.c_off + (size_t)s * n * 3, 3 * n);
  for (int i = threadIdx.x; i < copies * 3 * cells; i += blockDim.x) img[i] = 0.f;
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * n; e += blockDim.x) {
    const int p = e / 3, c = e - 3 * p;
    double y0 = 0.0, y1 = 0.0;
    int q = 0;
    const auto* row = gmem(Minv_g + (size_t)p * n);
#pragma unroll 6
    for (; q + 1 < n; q += 2) {
      y0 += row[q] * Tl[3 * q + c];
      y1 += row[q + 1] * Tl[3 * (q + 1) + c];
    }
    if (q < n) y0 += row[q] * Tl[3 * q + c];
    Y[e] = y0 + y1;
  }
  __syncthreads();
  const double hx = a.pose[wi][2], hy = a.pose[wi][3];
  double fx = 0.0, fy = 0.0, fz = 0.0, mz = 0.0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const double y0 = Y[3 * p], y1 = Y[3 * p + 1], y2 = Y[3 * p + 2];
    const size_t m = (size_t)w.moff + (size_t)p * ns + s;
    a.duB[3 * m] = y0 / w.dA;
    a.duB[3 * m + 1] = y1 / w.dA;
    a.duB[3 * m + 2] = y2 / w.dA;
    const double r = p == p0 ? rho_p0 : a.rhoB[m];
    const double bx = -2.0 * r * y0, by = -2.0 * r * y1, bz = -2.0 * r * y2;   // on the body
    fx += bx;
    fy += by;
    fz += bz;
    mz += (P[p * kPw] - hx) * by - (P[p * kPw + 1] - hy) * bx;
  }
  red[0][threadIdx.x] = fx;
  red[1][threadIdx.x] = fy;
  red[2][threadIdx.x] = fz;
  red[3][threadIdx.x] = mz;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave < copies && lane < 48) {
    // du_B dA D_xy = y D_xy
    const int node = lane % 16, comp = lane / 16;
    const int ox = node & 3, oy = node >> 2;
    float* im = img + (size_t)wave * 3 * cells;
    for (int p = wave; p < n; p += copies) {
      const double* r = P + p * kPw;
      const double v = r[4 + ox] * r[8 + oy] * Y[3 * p + comp];
      const int lx = (int)r[12] + ox - w.x0, ly = (int)r[13] + oy - w.y0;
      im[3 * (ly * w.bw + lx) + comp] += (float)v;
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) a.fpart[4 * ((size_t)w.layer_off + s) + threadIdx.x] = red[threadIdx.x][0];
  // only the support nodes of this step are written: the collide kernel
  // reads the image nowhere else (its support bitmap)
  float4* out = w.corr + (size_t)s * w.side * w.side;
  const auto* list = gmem(a.sup + (size_t)a.slot * a.sup_step + w.sup_off);
  const int cnt = (int)list[0];
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const unsigned cell = list[1 + e];
    const int lx = (int)(cell & 0xffffu), ly = (int)(cell >> 16);
    const int i = ly * w.bw + lx;
    float v[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < copies; ++k)
      for (int c = 0; c < 3; ++c) v[c] += img[(size_t)k * 3 * cells + 3 * i + c];
    out[ly * w.side + lx] = make_float4(v[0], v[1], v[2], 0.f);
  }
}

__global__ void __launch_bounds__(256) k_layer(Group gr) {
  int lb;
  const MarkerArgs* a = static_cast<const MarkerArgs*>(group_find(gr, lb));
  layer_block(*a, lb);
}

size_t marker_span_lds(int ns) { return interp_span_lds(ns); }

static hipError_t raise_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_factor(const MarkerArgs* const* host, const void* const* dev, int n, int count,
                         hipStream_t s) {
  if (n < 1 || n > kMaxGroup) return hipErrorInvalidValue;
  int maxnp = 0, maxmask = 0, blocks[kMaxGroup];
  for (int j = 0; j < n; ++j) {
    const MarkerArgs& a = *host[j];
    for (int k = 0; k < a.nw; ++k) {
      maxnp = a.w[k].np > maxnp ? a.w[k].np : maxnp;
      const int mw = a.w[k].side * (a.w[k].mask_words + 1);   // bitmap and row counts
      maxmask = mw > maxmask ? mw : maxmask;
    }
    blocks[j] = count * a.nw;
  }
  const size_t lds = (size_t)(kPw + 4) * maxnp * sizeof(double) + (size_t)maxmask * sizeof(unsigned);
  // register tile of the elimination: the smallest NT with 16 NT >= n_p
  const int nt = maxnp <= 32 ? 2 : (maxnp <= 64 ? 4 : (maxnp <= 96 ? 6 : 8));
  const void* fn = nt == 2   ? reinterpret_cast<const void*>(k_factor<2>)
                   : nt == 4 ? reinterpret_cast<const void*>(k_factor<4>)
                   : nt == 6 ? reinterpret_cast<const void*>(k_factor<6>)
                             : reinterpret_cast<const void*>(k_factor<8>);
  hipError_t e = raise_lds(fn, lds);
  if (e != hipSuccess) return e;
  Group g;
  const int total = group_fill(g, dev, blocks, n);
  if (total == 0) return hipSuccess;
  switch (nt) {
    case 2: k_factor<2><<<(unsigned)total, 256, lds, s>>>(g); break;
    case 4: k_factor<4><<<(unsigned)total, 256, lds, s>>>(g); break;
    case 6: k_factor<6><<<(unsigned)total, 256, lds, s>>>(g); break;
    default: k_factor<8><<<(unsigned)total, 256, lds, s>>>(g); break;
  }
  return hipGetLastError();
}

hipError_t launch_markers(int storage, const MarkerArgs* const* host, const void* const* dev, int n,
                          hipStream_t s) {
  if (n < 1 || n > kMaxGroup) return hipErrorInvalidValue;
  int nb[kMaxGroup], nl[kMaxGroup], np[kMaxGroup];
  size_t lds_l = 0, lds_s = 0;
  for (int j = 0; j < n; ++j) {
    const MarkerArgs& a = *host[j];
    int maxnp = 0, layers = 0, perims = 0, maxcells = 0;
    for (int k = 0; k < a.nw; ++k) {
      maxnp = a.w[k].np > maxnp ? a.w[k].np : maxnp;
      layers += a.w[k].ns;
      perims += a.w[k].np;
      const int c = a.w[k].bw * a.w[k].bh;
      maxcells = c > maxcells ? c : maxcells;
    }
    const size_t ll = (size_t)(kPw + 6) * maxnp * sizeof(double) + (size_t)a.copies * maxcells * 3 * sizeof(float);
    lds_l = ll > lds_l ? ll : lds_l;
    nb[j] = a.band_blocks;   // 4 waves per block, 64 support-list entries per wave
    nl[j] = layers;
    np[j] = perims;
  }
  // one block size for the group: 512 threads unless a solve's span needs 256
  int thr = 512;
  for (int j = 0; j < n; ++j) thr = span_threads(host[j]->g.nz) < thr ? span_threads(host[j]->g.nz) : thr;
  for (int j = 0; j < n; ++j) {
    const size_t ls = interp_span_lds(host[j]->g.nz);
    lds_s = ls > lds_s ? ls : lds_s;
  }
  hipError_t e = raise_lds(reinterpret_cast<const void*>(k_layer), lds_l);
  if (e == hipSuccess) e = raise_lds(reinterpret_cast<const void*>(k_interp_span), lds_s);
  if (e != hipSuccess) return e;
  Group g;
  int total = group_fill(g, dev, nb, n);
  if (total > 0) {
    switch (storage) {
      case ST_F32: k_band<StF32><<<total, 256, 0, s>>>(g); break;
      case ST_F16: k_band<StF16><<<total, 256, 0, s>>>(g); break;
      default: k_band<StBF16><<<total, 256, 0, s>>>(g); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int tp = group_fill(g, dev, np, n);
  if (tp == 0) return hipSuccess;
  k_interp_span<<<tp, thr, lds_s, s>>>(g);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  total = group_fill(g, dev, nl, n);
  k_layer<<<total, 256, lds_l, s>>>(g);
  return hipGetLastError();
}

}  // namespace ibmk
