// Internal declarations shared by the host API (api.cpp) and the gfx950
// kernels (collide.hip, markers.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ibmk {

constexpr int kQ = 19;
constexpr int kMaxWings = 8;
constexpr int kMaxPerim = 128;     // perimeter markers per foil (LDS of the inversion)
constexpr int kBlockX = 64;        // collide block: 64 cells along x ...
constexpr int kBlockRows = 4;      // ... times 4 rows, one row per wave
constexpr int kFactorWindow = 64;  // steps whose perimeter factors (and launch arguments) are made at once
constexpr int kMaxGroup = 64;      // solves in one grouped launch

enum Bc { BC_PERIODIC = 0, BC_WALL = 1, BC_VELOCITY = 2, BC_PRESSURE = 3, BC_ZH_VELOCITY = 4,
          BC_ZH_PRESSURE = 5 };
enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

// FP16 storage keeps 2^12 (f_i - w_i): a power of two, so the scaling is
// exact, and it lifts the deviations of a slow background flow (~1e-5) out
// of the FP16 subnormal range while |f_i - w_i| up to 16 stays finite.
constexpr float kF16Scale = 4096.0f;
constexpr float kF16Unscale = 1.0f / 4096.0f;

// Padded distribution layout, row-major slabs: population q of row
// r = z*ny + y, cell x, lives at element ((r+1)*19 + q)*px + x; px >= nx + 2
// and px*elem is a multiple of 128 bytes so every population row starts on a
// cache line.  The first slab is padding.  After the slabs, at byte offset
// goff, each state keeps its x-face ghost records: 32 bytes per row and side.
struct Geo {
  int nx, ny, nz, px;
  long long ps;        // population stride within a slab (= px)
  long long goff;      // byte offset of a state's ghost records from its base
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

// Per foil and step: the xy box of lattice nodes that its markers' kernel
// supports can reach (identical for every span layer of an extruded foil).
// Band moments and the spread correction are stored over this box, with a
// fixed pitch `side` (the largest box the motion can produce).
struct FoilBox {
  int x0, y0, w, h;    // box origin and size for this step
  int side;            // pitch of the per-layer images
  int words;           // 32-bit words per row of `bits`
  // per-layer images over the box, written and read at this step's support
  // nodes only (below)
  const float4* band;  // [nz][side][side] rho, u*x, u*y, u*z
  const float4* corr;  // [nz][side][side] du_x, du_y, du_z, 0 (spread result)
  // this step's support nodes of the foil's markers, bit (lx, ly) relative
  // to the box origin: the only cells the spread can reach, so the cells
  // of the box outside it have a zero correction
  const unsigned* bits;
};

struct CollideArgs {
  Geo g;
  Phys p;
  const void* src;
  void* dst;
  int nw;                    // foils whose correction the kernel applies
  FoilBox box[kMaxWings];
  float wz[4];               // span weights delta(1.5), delta(0.5), delta(0.5), delta(1.5)
  int nxc;                   // 64-wide chunks along x
  int nblocks;               // row groups of 4 rows x 64 cells
  // n / nxc and n / ny as umulhi(n, m) for the wave indices the kernel
  // divides (m = floor(2^32 / d) + 1, exact when n d < 2^32; 0: divide)
  unsigned nxc_mul, ny_mul;
  double* mass_part;         // per-block partial sums (check steps); face blocks after nblocks
  int* flags;                // bit 0: non-finite density seen
  // force reduction by block 0 on steps with foils
  const double* fpart;       // [nw][nz][4] layer forces and moments
  double* hist;              // [H][nw][8]
  long long hist_row;
  double qS;                 // 0.5 u_ref^2 area_ref
  double sense[kMaxWings], chord[kMaxWings];
};

// A grouped launch: the blocks of solve k are start[k] .. start[k+1]-1 and
// read that solve's arguments from device memory at args[k].  One solve is a
// group of one, so a solve runs the same code alone and in a group.
struct Group {
  int n;
  int start[kMaxGroup + 1];
  const void* args[kMaxGroup];
};

// launch wrappers of collide.hip (the marker kernels' are in marker_args.h);
// all enqueue on `s` and return hipError_t.  `host[k]` is the host copy of the arguments that `dev[k]`
// holds on the device (used for grid and LDS sizing only).
hipError_t launch_collide(int storage, bool ibm, bool force, bool check, bool zh,
                          const CollideArgs* const* host, const void* const* dev, int n,
                          hipStream_t s);
hipError_t launch_ghost(int storage, const Geo& g, const Phys& p, void* buf, hipStream_t s);
hipError_t launch_init_eq(int storage, const Geo& g, const double* rho, const double* u,
                          void* dst, hipStream_t s);
hipError_t launch_moments(int storage, const Geo& g, const Phys& p, const void* src,
                          float* out, hipStream_t s);
hipError_t launch_mass_reduce(const double* part, int n, double ncells, double* out,
                              long long step, hipStream_t s);
constexpr size_t kMaxLds = 160 * 1024;  // LDS per block on gfx950

// Static scratch of ibmlbm_create_noalloc (scratch.hip): its size, and the
// device address of a device's copy (looked up once per device).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
hipError_t scratch_address(int device, void** out);

}  // namespace ibmk
