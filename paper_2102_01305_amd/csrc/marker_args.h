// Arguments of the marker kernels (markers.hip) and their launch wrappers,
// shared with the host API (api.cpp).  Kept apart from internal.h, which
// holds what the collide kernel is compiled from.
#pragma once

#include "internal.h"

namespace ibmk {

struct WingDev {
  int np, ns, moff;          // perimeter markers, span layers, first marker index
  int ref_off;               // offset of this foil's (np x 2) reference coordinates
  int g_off;                 // offset of this foil's span pseudo-inverse row (ns)
  int minv_off;              // offset of this foil's perimeter inverse (np x np)
  int pw_off;                // offset of this foil's per-step perimeter records (np x 14)
  int sup_off;               // offset of this foil's support list in a window slot (1 + np*16 words, then side * mask_words of bitmap)
  int mask_words;            // 32-bit words per node-box row of the support bitmap
  int sup_chunks;            // this step's band waves per layer: 64-cell chunks of a bound on its support count
  int c_off;                 // offset of this foil's span-solved T (ns x np x 3)
  int layer_off;             // offset of this foil's layers in the force partials
  int shape;
  double hinge0[2], theta0, sense, mean, amp, period, phase, tamp, tang;
  double dA, chord;
  int x0, y0, bw, bh, side;  // this step's node box (see FoilBox)
  float4* band;              // band moments over the box
  float4* corr;              // spread correction over the box
};

struct MarkerArgs {
  Geo g;
  Phys p;
  int nw;
  int m_total;
  int band_blocks;           // blocks of 4 band waves (64 support cells of one foil's layer each)
  WingDev w[kMaxWings];
  double wz[4];              // span weights of a node at offsets -1.5, -0.5, 0.5, 1.5
  double t;
  double pose[kMaxWings][6]; // per foil at t: theta, dtheta/dt, pivot x, y, pivot velocity x, y
  const void* src;           // current state (post-collision of the previous step)
  const double* ref;
  const double* G;
  double* Minv;              // [window slot][sum np^2] perimeter inverses
  double* pw;                // [window slot][sum np x 14] perimeter records
  // per window slot and foil: the support nodes of its perimeter markers
  // (the only node-box cells whose band moments the interpolation reads),
  // as a count and then ly << 16 | lx per cell, row-major
  unsigned* sup;
  int sup_step;              // words per slot
  const MarkerArgs* win_args;  // the window's per-step arguments (device), for the node-box origins
  long long win_t0;          // first step of the precomputed window
  int slot;                  // this step's slot in the window
  int pw_step, minv_step;    // doubles per slot
  double* T;                 // span-solved B, layer-major: [layer][marker p][component]
  double* fpart;             // [layer]: Fx, Fy, Fz, Mz of each span layer
  double* X;                 // 3 per marker
  double* U;                 // 3 per marker
  double* B;                 // 3 per marker
  double* rhoB;              // 1 per marker
  double* duB;               // 3 per marker
  int copies;                // partial spread images per layer block (1..4)
  int* flags;                // bit 1: singular perimeter system; bit 2: a support list longer than its bound
};

// launch wrappers (markers.hip); enqueue on `s` and return hipError_t.
// `host[k]` is the host copy of the arguments that `dev[k]` holds on the
// device (used for grid and LDS sizing only).
hipError_t launch_factor(const MarkerArgs* const* host, const void* const* dev, int n, int count,
                         hipStream_t s);
hipError_t launch_markers(int storage, const MarkerArgs* const* host, const void* const* dev, int n,
                          hipStream_t s);
// LDS bytes of the per-marker interpolation and span-solve block for a span
// of ns layers, against the device's kMaxLds per block.
size_t marker_span_lds(int ns);

}  // namespace ibmk
