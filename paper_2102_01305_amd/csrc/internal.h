// Internal declarations shared by the host API (api.cpp) and the gfx950
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ibmk {

constexpr int kQ = 19;
constexpr int kMaxWings = 8;
constexpr int kMaxPerim = 128;     // perimeter markers per foil (LDS of the inversion)
constexpr int kTile = 8;           // tile edge of the marker-band flags
constexpr int kBlockX = 64;        // collide block: 64 cells along x ...
constexpr int kBlockRows = 4;      // ... times 4 rows

enum Bc { BC_PERIODIC = 0, BC_WALL = 1, BC_VELOCITY = 2, BC_PRESSURE = 3 };
enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

// Padded distribution layout: population q, row r = z*ny + y, cell x lives at
// element q*ps + (r+1)*px + x.  Element (r+1)*px - 1 is the x = -1 ghost of
// row r and (r+1)*px + nx the x = nx ghost; px >= nx + 2 and px*elem is a
// multiple of 128 bytes so every row starts on a cache line.
struct Geo {
  int nx, ny, nz, px;
  long long ps;
  int yper, zper;      // periodic y / z
  int bclo, bchi;      // kinds of the -x / +x faces
};

struct Phys {
  float omega;         // 1/tau
  float guo_k;         // 1 - 1/(2 tau)
  float fb[3];         // body force density
  float u_in[3];       // velocity of VELOCITY faces
  float rho_out;       // density of PRESSURE faces
};

struct CollideArgs {
  Geo g;
  Phys p;
  const void* src;
  void* dst;
  float* du;                 // 3 planes of N floats (marker-band velocity correction)
  const int* stamps;         // per-tile stamp of the last spread
  int stamp;                 // stamp value meaning "spread this step"
  int tnx, tny;              // tiles along x and y
  int nxc;                   // 64-wide chunks along x
  int nblocks;
  double* mass_part;         // per-block partial sums (check steps)
  int* flags;                // bit 0: non-finite density seen
};

struct WingDev {
  int np, ns, moff;          // perimeter markers, span layers, first marker index
  int ref_off;               // offset of this foil's (np x 2) reference coordinates
  int g_off;                 // offset of this foil's span pseudo-inverse row (ns)
  int minv_off;              // offset of this foil's perimeter inverse (np x np)
  int layer_off;             // offset of this foil's span layers in the force partials
  int shape;
  double hinge0[2], theta0, sense, mean, amp, period, phase, tamp, tang;
  double dA, chord;
};

struct MarkerArgs {
  Geo g;
  Phys p;
  int nw;
  int m_total;
  WingDev w[kMaxWings];
  double t;
  const void* src;           // current state (post-collision of the previous step)
  const double* ref;
  const double* G;
  double* Minv;
  double* X;                 // 3 per marker
  double* U;                 // 3 per marker
  double* B;                 // 3 per marker
  double* rhoB;              // 1 per marker
  double* duB;               // 3 per marker
  double* fpart;             // per (wing, span layer): Fx, Fy, Fz, Mz
  unsigned int* counters;    // per wing: finished span blocks this step
  double* hist;              // [H][nw][8]
  long long hist_row;        // row of this step in the ring
  double u_ref, area_ref;
  float* du;                 // lattice velocity-correction planes
  int* stamps;
  int stamp;
  int tnx, tny;
  int* flags;                // bit 1: singular perimeter system
};

// launch wrappers (kernels.hip); all enqueue on `s` and return hipError_t
hipError_t launch_collide(int storage, bool ibm, bool force, bool check,
                          const CollideArgs& a, hipStream_t s);
hipError_t launch_ghost(int storage, const Geo& g, const Phys& p, void* buf, hipStream_t s);
hipError_t launch_init_eq(int storage, const Geo& g, const double* rho, const double* u,
                          void* dst, hipStream_t s);
hipError_t launch_moments(int storage, const Geo& g, const Phys& p, const void* src,
                          float* out, hipStream_t s);
hipError_t launch_mass_reduce(const double* part, int n, double ncells, double* out,
                              long long step, hipStream_t s);
hipError_t launch_markers(int storage, const MarkerArgs& a, hipStream_t s);

}  // namespace ibmk
