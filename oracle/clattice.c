/*
 * D3Q19 lattice Boltzmann BGK with Guo forcing, FP64, plain C with OpenMP
 * over z-planes (oracle; test infrastructure only).
 *
 * The same three operations as lattice.py (streaming with the boundary
 * rules, moments, collision), written a second time in C so that long
 * oracle runs on large boxes finish in minutes instead of hours.  It is a
 * separate implementation with its own tables, checked against lattice.py
 * and against the closed forms in tests/test_oracle_clattice.py.  Nothing
 * here is shared with the GPU library.
 *
 * Arrays are C-contiguous float64 in the oracle's layout: distributions
 * (19, nz, ny, nx), vectors (3, nz, ny, nx), scalars (nz, ny, nx), x fastest.
 * Lattice units dx = dt = 1, c_s^2 = 1/3.
 */
#include <stddef.h>

#include <omp.h>

enum { Q = 19 };
enum { PERIODIC = 0, WALL = 1, VELOCITY = 2, PRESSURE = 3, ZH_VELOCITY = 4, ZH_PRESSURE = 5 };

/* D3Q19 velocities: rest, 6 faces, 12 edges (canonical order). */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
static const double CS2 = 1.0 / 3.0;

static double weight(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

/* Eq. 4 (standard second-order form): w_i rho [1 + c.u/cs^2 + (c.u)^2/(2 cs^4) - u.u/(2 cs^2)]. */
static double feq(int i, double rho, double ux, double uy, double uz) {
  const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
  const double usq = ux * ux + uy * uy + uz * uz;
  return weight(i) * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
}

/* Eq. 2 at one cell of a distribution array: rho and sum_i c_i f_i. */
static void cell_moments(const double* f, size_t N, size_t cell, double* rho, double m[3]) {
  double r = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
  for (int i = 0; i < Q; ++i) {
    const double v = f[(size_t)i * N + cell];
    r += v;
    mx += CX[i] * v;
    my += CY[i] * v;
    mz += CZ[i] * v;
  }
  *rho = r;
  m[0] = mx;
  m[1] = my;
  m[2] = mz;
}

/* Zou-He rebuild of one boundary cell of an x face (Sec. 3.1, ref. [21]),
 * in place; n = +1 on the -x face, -1 on the +x face, the unknowns are the
 * populations with c_x = n.  K = sum_{c_x=0} f + 2 sum_{c_x=-n} f gives
 * rho (1 - n u_x) = K; each unknown is its opposite plus the equilibrium
 * difference 2 w rho c.u / cs^2, less the transverse corrections c_t N_t
 * with N_t = (1/2) sum_{c_x=0} c_t f - rho u_t / 3. */
static void zou_he_cell(double* f, size_t N, size_t cell, int n, int kind, const double u_in[3],
                        double rho_out) {
  double K = 0.0, sy = 0.0, sz = 0.0;
  for (int i = 0; i < Q; ++i) {
    const double v = f[(size_t)i * N + cell];
    if (CX[i] == 0) {
      K += v;
      sy += CY[i] * v;
      sz += CZ[i] * v;
    } else if (CX[i] == -n) {
      K += 2.0 * v;
    }
  }
  double rho, ux, uy, uz;
  if (kind == ZH_VELOCITY) {
    ux = u_in[0];
    uy = u_in[1];
    uz = u_in[2];
    rho = K / (1.0 - n * ux);
  } else {
    rho = rho_out;
    ux = n * (1.0 - K / rho);
    uy = 0.0;
    uz = 0.0;
  }
  const double Ny = 0.5 * sy - rho * uy / 3.0;
  const double Nz = 0.5 * sz - rho * uz / 3.0;
  for (int i = 0; i < Q; ++i) {
    if (CX[i] != n) continue;
    const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
    f[(size_t)i * N + cell] = f[(size_t)OPP[i] * N + cell] + 2.0 * weight(i) * rho * cu / CS2 -
                              CY[i] * Ny - CZ[i] * Nz;
  }
}

/* Streaming with the boundary rules of Sec. 2.1 (the left-hand side of
 * Eqs. 1 and 7): f_i(x) = S_i(x - c_i) where the source lies in the box.
 * Across a face: periodic axes wrap; a WALL face gives half-way bounce-back
 * f_i(x) = S_opp(i)(x), and a link leaving through a wall and an x
 * inlet/outlet face at once takes that rule; a VELOCITY face gives the
 * equilibrium of (rho of S at the adjacent boundary cell, u_in), a PRESSURE
 * face that of (rho_out, velocity of S at the adjacent boundary cell), each
 * taken at the ghost row the link comes from; ZH_ faces use the same ghosts
 * and then rebuild their boundary cells by Zou-He, except cells whose
 * entering links touch a y or z wall. */
void ora_stream(const double* S, double* f, int nx, int ny, int nz, const int bc[6],
                const double u_in[3], double rho_out) {
  const size_t N = (size_t)nx * ny * nz;
  const int dims[3] = {nx, ny, nz};
  const int per[3] = {bc[0] == PERIODIC, bc[2] == PERIODIC, bc[4] == PERIODIC};
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t cell = ((size_t)z * ny + y) * nx + x;
        const int c[3] = {x, y, z};
        for (int i = 0; i < Q; ++i) {
          const int ci[3] = {CX[i], CY[i], CZ[i]};
          int s[3], lo[3], hi[3];
          for (int d = 0; d < 3; ++d) {
            s[d] = c[d] - ci[d];
            if (per[d]) s[d] = (s[d] % dims[d] + dims[d]) % dims[d];
            lo[d] = s[d] < 0;
            hi[d] = s[d] >= dims[d];
            if (s[d] < 0) s[d] = 0;
            if (s[d] >= dims[d]) s[d] = dims[d] - 1;
          }
          int wall = 0;
          for (int d = 0; d < 3; ++d) {
            if (bc[2 * d] == WALL && lo[d]) wall = 1;
            if (bc[2 * d + 1] == WALL && hi[d]) wall = 1;
          }
          if (wall) {
            f[(size_t)i * N + cell] = S[(size_t)OPP[i] * N + cell];
            continue;
          }
          const size_t src = ((size_t)s[2] * ny + s[1]) * nx + s[0];
          double v = S[(size_t)i * N + src];
          for (int face = 0; face < 2; ++face) {
            const int crossed = face == 0 ? lo[0] : hi[0];
            const int kind = bc[face];
            if (!crossed || kind == PERIODIC || kind == WALL) continue;
            /* the ghost of row (s_y, s_z), fed by boundary cell xb of that row */
            const int xb = face == 0 ? 0 : nx - 1;
            const size_t bcell = ((size_t)s[2] * ny + s[1]) * nx + xb;
            double rb, mb[3];
            cell_moments(S, N, bcell, &rb, mb);
            if (kind == VELOCITY || kind == ZH_VELOCITY)
              v = feq(i, rb, u_in[0], u_in[1], u_in[2]);
            else
              v = feq(i, rho_out, mb[0] / rb, mb[1] / rb, mb[2] / rb);
          }
          f[(size_t)i * N + cell] = v;
        }
      }
  /* Zou-He faces, after the pull */
  for (int face = 0; face < 2; ++face) {
    const int kind = bc[face];
    if (kind != ZH_VELOCITY && kind != ZH_PRESSURE) continue;
    const int xb = face == 0 ? 0 : nx - 1;
    const int n = face == 0 ? 1 : -1;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
      if (!per[2] && (z == 0 || z == nz - 1)) continue;
      for (int y = 0; y < ny; ++y) {
        if (!per[1] && (y == 0 || y == ny - 1)) continue;
        zou_he_cell(f, N, ((size_t)z * ny + y) * nx + xb, n, kind, u_in, rho_out);
      }
    }
  }
  (void)dims;
}

/* Eq. 2: rho = sum_i f_i and the momentum sum_i c_i f_i of every cell. */
void ora_moments(const double* f, double* rho, double* mom, int nx, int ny, int nz) {
  const size_t N = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; ++z)
    for (size_t cell = (size_t)z * ny * nx; cell < (size_t)(z + 1) * ny * nx; ++cell) {
      double m[3];
      cell_moments(f, N, cell, &rho[cell], m);
      mom[cell] = m[0];
      mom[N + cell] = m[1];
      mom[2 * N + cell] = m[2];
    }
}

/* Eq. 7 with Eq. 4 and Eq. 8: f* = f - (f - f^eq(rho, u))/tau + F_i,
 * F_i = (1 - 1/(2 tau)) w_i [(c_i - u)/cs^2 + (c_i.u) c_i/cs^4] . F
 * (Guo's form, the c_i factor of the second term restored), with the
 * force-corrected velocity u. */
void ora_collide(const double* f, const double* rho, const double* u, const double* F, double tau,
                 double* out, int nx, int ny, int nz) {
  const size_t N = (size_t)nx * ny * nz;
  const double k = 1.0 - 0.5 / tau;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; ++z)
    for (size_t cell = (size_t)z * ny * nx; cell < (size_t)(z + 1) * ny * nx; ++cell) {
      const double r = rho[cell];
      const double ux = u[cell], uy = u[N + cell], uz = u[2 * N + cell];
      const double Fx = F[cell], Fy = F[N + cell], Fz = F[2 * N + cell];
      const double uF = ux * Fx + uy * Fy + uz * Fz;
      for (int i = 0; i < Q; ++i) {
        const double fi = f[(size_t)i * N + cell];
        const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        const double cF = CX[i] * Fx + CY[i] * Fy + CZ[i] * Fz;
        const double src = k * weight(i) * ((cF - uF) / CS2 + cu * cF / (CS2 * CS2));
        out[(size_t)i * N + cell] = fi - (fi - feq(i, r, ux, uy, uz)) / tau + src;
      }
    }
}

/* Eq. 4 over whole arrays (initial state). */
void ora_equilibrium(const double* rho, const double* u, double* out, int nx, int ny, int nz) {
  const size_t N = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; ++z)
    for (size_t cell = (size_t)z * ny * nx; cell < (size_t)(z + 1) * ny * nx; ++cell)
      for (int i = 0; i < Q; ++i)
        out[(size_t)i * N + cell] = feq(i, rho[cell], u[cell], u[N + cell], u[2 * N + cell]);
}

/* Threads of the parallel loops above (the OpenMP default is the host's). */
void ora_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}
