/* clb3d.h -- C ABI of the three-dimensional CLB path of libclb (gfx950): D3Q27 central-moment
 * flow, D3Q7 central-moment temperature, Boussinesq coupling with gravity along -z, on one GPU.
 *
 * The paper (Fei, Luo, Lin, Li; arXiv 1710.10569) derives the method in two dimensions
 * (Secs. 2.1-2.2) and states that it extends directly to three (Sec. 4).  This path takes every
 * definition dimension by dimension:
 *   - velocity set {0, +1, -1}^3; central moments k~_abc, a, b, c in {0, 1, 2} (Eq. 5);
 *   - equilibrium central moments rho m(a) m(b) m(c), m = (1, 0, 1/3) (Eq. 9's pattern);
 *   - forcing central moments sum_d F_d [a_d = 1] prod_{d' != d} m(a_d') (Eq. 11's pattern);
 *   - collision Gamma~* = (I - S) Gamma~ + S Gamma~^eq + (I - S/2) C (Eq. 8): trace of the
 *     second-order diagonal moments with s_b, their deviatoric part and k~110, k~101, k~011 with
 *     s_nu = 1/tau_nu, orders 3, 4, 5, 6 with s3, s4, s5, s6;
 *   - D3Q7 temperature collision (Eq. 19) to [T, 0, 0, 0, T/4, T/4, T/4], lambda1 = 1/tau_alpha;
 *   - rho, u = (sum f e + F/2)/rho (Eq. 13), T = sum g (Eq. 23), F = F_v + g beta (T - T0) e_z
 *     (Eq. 3);
 *   - nu = (tau_nu - 1/2)/3, alpha = (tau_alpha - 1/2)/4.
 * Domain: nx x ny x nz nodes, periodic in x and y; z periodic, or bounded by walls on the nodes
 * z = 0 (bottom) and z = nz - 1 (top), H = nz - 1.  Walls: tangential velocity (ux, uy), a
 * Dirichlet temperature or adiabatic (T_b = (4 T(x_f) - T(x_ff))/3).  The paper gives no 3D wall
 * scheme; wall nodes take non-equilibrium extrapolation from the inner neighbour x_f for every
 * population of both lattices (the paper's temperature wall scheme), at the wall velocity and
 * temperature, with the node's mass-balance density (the populations known after streaming plus
 * those the node sent out of the domain the step before), so closed boxes conserve mass.
 *
 * Ownership: the handle owns its device memory and (unless a stream is given) its stream; host
 * arrays are borrowed for the duration of a call, FP64, index (z ny + y) nx + x.  Errors: the
 * CLB_* codes of clb.h (negative), never an abort; clb_last_error() holds the message.  A handle
 * is single-threaded.  Calls are ordered on the handle's stream; clb3d_step does not block,
 * clb3d_moments and clb3d_diagnostics synchronise.
 */
#ifndef CLB3D_H
#define CLB3D_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct clb3d_lattice clb3d_lattice;

enum { CLB3D_PERIODIC = 0, CLB3D_DIRICHLET = 1, CLB3D_ADIABATIC = 2 };

/* One z wall: kind (CLB3D_DIRICHLET or CLB3D_ADIABATIC; CLB3D_PERIODIC for a periodic z),
 * tangential velocity (ux, uy) and temperature T (Dirichlet). */
typedef struct { int kind; double ux, uy, T; } clb3d_wall;

/* Lattice description: nodes (nx, ny >= 1; nz >= 1, >= 3 with walls), precision (clb.h:
 * CLB_FP64 and CLB_FP64_DEV both store and collide FP64 deviations from the rest state, CLB_FP32_DEV
 * FP32 deviations collided in FP32, CLB_FP32_SR FP32 deviations collided in FP64 and rounded
 * stochastically on store), bottom and top walls (both CLB3D_PERIODIC or both walls), T0 of Eq. 3. */
typedef struct {
    int nx, ny, nz, precision;
    clb3d_wall bottom, top;
    double T0;
} clb3d_desc;

/* Diagnostics of the current state, in FP64 (every sum in a fixed order, so repeatable):
 *   mass = sum rho, momentum = sum rho u, heat = sum T over all nodes;
 *   uzT = sum w_z u_z (T - T0) with w_z = 1/2 on the two wall planes and 1 elsewhere (the
 *         numerator of Eq. 29's volume average; divide by nx ny H, H = nz - 1, with walls);
 *   plane_T = sum over x, y of T on the planes z = 0, 1, 2, nz - 3, nz - 2, nz - 1 (wall fluxes);
 *   max_speed = max |u|; step = steps taken. */
typedef struct {
    double mass, momentum[3], heat, uzT, plane_T[6], max_speed;
    long long step;
} clb3d_diag;

/* Create a lattice in the rest state (rho = 1, u = 0, T = T0) with tau_nu = tau_alpha = 1, no
 * buoyancy, all other rates 1.  hip_stream: a hipStream_t to run on, or NULL for an own stream.
 * Errors: CLB_EINVAL (bad description), CLB_ENOMEM, CLB_EDEVICE. */
int clb3d_create(const clb3d_desc* desc, void* hip_stream, clb3d_lattice** out);

/* tau_nu = 1/s_nu, tau_alpha = 1/lambda1 (both > 1/2), g beta of Eq. 3.  CLB_EINVAL otherwise. */
int clb3d_set_params(clb3d_lattice* h, double tau_nu, double tau_alpha, double g_beta);

/* s_b, s3, s4, s5, s6 in (0, 2) and lambda2 in (0, 2); defaults 1.  CLB_EINVAL otherwise. */
int clb3d_set_relaxation(clb3d_lattice* h, double s_b, double s3, double s4, double s5, double s6, double lambda2);

/* Body force F_v of Eq. 3 (force density, lattice units). */
int clb3d_set_body_force(clb3d_lattice* h, double Fx, double Fy, double Fz);

/* Initial state from fields (NULL: rho = 1, u = 0, T = T0): f = f^eq(rho, u - F/(2 rho)) with F
 * from T, g = g^eq(T, u), so clb3d_moments returns the given fields at t = 0 (at wall nodes the
 * wall velocity and temperature).  u holds three planes of n values (u_x, u_y, u_z).  Resets the
 * step count. */
int clb3d_init(clb3d_lattice* h, const double* rho, const double* u, const double* T);

/* Advance n >= 0 steps (per step one launch, or two with walls: the wall planes and the rest); does
 * not block. */
int clb3d_step(clb3d_lattice* h, long long n);

/* rho, u (three planes), T of the current time into host arrays of n = nx ny nz values (any may be
 * NULL).  Synchronises. */
int clb3d_moments(clb3d_lattice* h, double* rho, double* u, double* T);

/* Diagnostics (above).  Synchronises. */
int clb3d_diagnostics(clb3d_lattice* h, clb3d_diag* out);

/* Time n steps with HIP events on the handle's stream; writes the milliseconds.  Synchronises. */
int clb3d_time_steps(clb3d_lattice* h, long long n, double* ms);

/* Wait for the handle's stream and report a pending launch error (CLB_EDEVICE). */
int clb3d_synchronize(clb3d_lattice* h);

/* Bytes of device memory a lattice of this description holds (two population buffers and the
 * FP64 field and reduction buffers); 0 for an invalid description. */
size_t clb3d_footprint(const clb3d_desc* desc);

/* Checkpoint / resume, as clb_checkpoint_* of clb.h: the size of the blob; a copy of the header
 * (description, parameters, step count) and the current population buffer into the caller's host
 * buffer (synchronises); and its restore into a lattice of the same description, after which
 * stepping on gives bitwise the uninterrupted run.  Errors: CLB_EINVAL (NULL, too small, another
 * version or description), CLB_EDEVICE. */
int clb3d_checkpoint_size(clb3d_lattice* h, size_t* bytes);
int clb3d_checkpoint_save(clb3d_lattice* h, void* host, size_t bytes);
int clb3d_checkpoint_load(clb3d_lattice* h, const void* host, size_t bytes);

/* Destroy the lattice and free its memory (NULL-safe). */
void clb3d_destroy(clb3d_lattice* h);

#ifdef __cplusplus
}
#endif

#endif
