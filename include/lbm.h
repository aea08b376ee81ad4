/*
 * lbm.h - C ABI of the MI355X (gfx950) thermal pseudopotential D3Q19 lattice
 * Boltzmann step.
 *
 * The method is the two-population scheme of Biferale, Perlekar, Sbragaglia &
 * Toschi, "Convection in multiphase flows using Lattice Boltzmann methods"
 * (arXiv:1111.0905), section "Algorithm": eqs. (LBEQ)/(LBEQ2) for the mass
 * populations f and the rho*T populations g, eq. (HYDRO) for the moments,
 * eq. (FORCE) for the pseudopotential force with psi = exp(-1/rho), the
 * velocity shift u' = u + tau_nu F / rho, the f/g coupling giving the ideal
 * pressure rho T, and a counter-term in the g dynamics giving the
 * compressive work P0 div u of eq. (eq).  Walls at the bottom and top are
 * no-slip with imposed temperatures T_d / T_u (Fig. 1 caption, text before
 * eq. (heat2)); x and y are periodic.
 *
 * Lattice and layout
 * ------------------
 * Nodes (i, j, k), 0 <= i < nx, 0 <= j < ny, 0 <= k < nz; the walls sit
 * half a spacing below k = 0 and above k = nz-1 (cell height H = nz).
 * D3Q19 velocities, in this order (an interface: state buffers use it):
 *    0:( 0, 0, 0)
 *    1:(+1, 0, 0)  2:(-1, 0, 0)  3:( 0,+1, 0)  4:( 0,-1, 0)  5:( 0, 0,+1)  6:( 0, 0,-1)
 *    7:(+1,+1, 0)  8:(-1,-1, 0)  9:(+1,-1, 0) 10:(-1,+1, 0)
 *   11:(+1, 0,+1) 12:(-1, 0,-1) 13:(+1, 0,-1) 14:(-1, 0,+1)
 *   15:( 0,+1,+1) 16:( 0,-1,-1) 17:( 0,+1,-1) 18:( 0,-1,+1)
 * A canonical state is 38 * N doubles, N = nx*ny*nz: population q
 * (q < 19: f_q, q >= 19: g_{q-19}) of node (i,j,k) at
 *   state[((q * nz + k) * ny + j) * nx + i],
 * holding the post-streaming populations at the current time level.
 * Fields are (nz, ny, nx) row-major, i fastest.
 *
 * Memory ownership
 * ----------------
 * The caller owns every buffer.  The library never allocates device memory:
 * lbm_init carves its two population buffers and its scratch out of one
 * caller-provided device workspace of lbm_workspace_bytes() bytes, which must
 * stay alive (and untouched) until lbm_destroy.  Pointers documented "device"
 * must be device memory of the current HIP device; "host" pointers are host
 * memory.  All work is enqueued on the HIP stream given to lbm_init (NULL =
 * the default stream).
 *
 * Errors
 * ------
 * Functions return 0 on success or a negative LBM_E* code; lbm_last_error()
 * returns a thread-local message describing the last failure.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* storage of the populations; arithmetic is FP64 for LBM_FP64, FP32 else.
 * Bytes per node and buffer: FP64 304, FP32 152, the 16-bit forms 80: the 18
 * moving (f_l, g_l) pairs as 16-bit deviations from the reference pops
 * (round to nearest even), the rest pair in FP32.  FP32 and the 16-bit forms
 * update the rest pair in remainder form: old value + what the moving pairs
 * gave up in the collision (+ the rounding residuals of their 16-bit stores)
 * (+ the energy source for g), so the stored mass is conserved to the
 * rounding of small per-node sums instead of drifting with correlated FP32
 * roundings of the node sums and of f_0 (which carries most of the mass). */
enum {
  LBM_FP64 = 0,      /* double storage, double arithmetic */
  LBM_FP32 = 1,      /* float storage, float arithmetic */
  LBM_FP16DEV = 2,   /* IEEE half of (pop - reference pop), float arithmetic */
  LBM_BF16DEV = 3    /* bfloat16 of (pop - reference pop), float arithmetic */
};

/* which implementation of the step */
enum {
  LBM_KERNEL_FUSED = 0,        /* one z-marching kernel per step (default).  With tile_x = tile_y = 0
                                  the library picks: FP32 and the 16-bit forms the pipelined kernel
                                  (LBM_KERNEL_PIPELINED) on 512-thread tiles 128 x 4 (nx >= 128),
                                  64 x 8 (nx >= 64) or 32 x 16; FP64 the register-resident kernel on
                                  64 x 2 tiles.  With an explicit tile (of at most 512 threads) it is
                                  the register-resident kernel on that tile */
  LBM_KERNEL_REFERENCE = 1,    /* two plain kernels per step (moments, then collide+stream) */
  LBM_KERNEL_FUSED_RELOAD = 2, /* one z-marching kernel per step, populations re-read from cache */
  LBM_KERNEL_PIPELINED = 3     /* one z-marching kernel per step with the loads of plane k+2 in
                                  flight while plane k collides (FP32 and 16-bit storage only;
                                  tiles 128 x 4, 256 x 2, 64 x 8, 32 x 16, 32 x 8, 16 x 16; 0 x 0 picks
                                  the widest 512-thread tile the plane fills) */
};

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* invalid argument or parameter */
  LBM_EWORKSPACE = -2,  /* workspace too small or misaligned */
  LBM_EHIP = -3,        /* a HIP runtime call failed */
  LBM_ENUMERIC = -4     /* a diagnostic found a non-finite value or rho <= 0 */
};

/*
 * Problem statement (eqs. (ns), (LBEQ)-(FORCE), Table 1).
 *   tau_nu, tau_kappa > 1/2: relaxation times of f and g;
 *     nu = (tau_nu - 1/2)/3, kappa = c_v (tau_kappa - 1/2) rho_kappa / 3.
 *   G: strength of eq. (FORCE), G < 0 (attraction); critical point
 *     rho_c = 1, T_c = -G / e^2, bulk pressure rho T + (G/2) exp(-2/rho)
 *     (with psi_form = 1: rho_c = ln 2, T_c = -G / 4, rho T + (G/2) psi^2).
 *   T_d, T_u > 0: bottom and top wall temperatures.
 *   gravity >= 0: body force rho * (0, 0, -gravity).
 *   c_v > 0: specific heat at constant volume.
 *   rho_kappa > 0: density that sets the conductivity of g^eq.
 *   T_lat: lattice temperature of f^eq (its second moment is rho T_lat delta
 *     + rho u u); the rest of the ideal pressure, rho (T - T_lat), acts as a
 *     force.  <= 0 picks the mean wall temperature.
 *   rho_ref, T_ref: reference state of the FP16/BF16 deviation storage
 *     (pop_ref = equilibrium at rest of (rho_ref, T_ref)); ignored otherwise.
 *   periodic_z: 0 = walls (nz >= 2), 1 = periodic in z as well.
 *   rho_wall_d, rho_wall_u, psi_form: see the fields below.
 *   kernel: LBM_KERNEL_*.
 *   tile_x x tile_y: x-y tile of one z-marching work-group; supported
 *     64 x {1, 2, 4, 8, 16} and 32 x {8, 16, 32} (fused kernels), 128 x 4,
 *     64 x 8, 32 x 16, 32 x 8 and 16 x 16 (pipelined); 0 picks the default.
 */
typedef struct lbm_params {
  int32_t nx, ny, nz;
  int32_t storage;
  int32_t periodic_z;
  int32_t kernel;
  int32_t tile_x;      /* fused-kernel tile width: 0 (default 64), 32 or 64 */
  int32_t tile_y;      /* fused-kernel tile height: 0 (default), 1..32, see lbm_init */
  int32_t z_chunk;     /* planes per fused-kernel work-group column; 0 = chosen at
                          init: the chunking (chunks of at least 4 planes) that
                          makes the launch shortest, counted as rounds of the
                          work-groups the GPU holds at once (the runtime's
                          occupancy) times the planes each marches plus its two
                          halo planes; the whole height when the tiles fill
                          whole rounds */
  int32_t adjoint;     /* 1 = reserve workspace for the lbm_adjoint_* entry points */
  double tau_nu, tau_kappa;
  double G;
  double T_d, T_u;
  double gravity;
  double c_v;
  double rho_kappa;
  double rho_ref, T_ref;
  double T_lat;        /* lattice temperature of f^eq; <= 0 picks (T_d + T_u) / 2 */
  double rho_wall_d;   /* wetting of the bottom wall: > 0 gives the psi ghost plane below
                          k = 0 the constant value psi(rho_wall_d) (a prescribed wall
                          density); <= 0 mirrors psi of the wall plane (neutral wetting,
                          90 degree contact angle).  The paper is silent on wettability;
                          this is the wall-density method of Benzi et al., Phys. Rev. E 74,
                          021509 (2006).  Ignored with periodic_z. */
  double rho_wall_u;   /* the same for the top wall (ghost plane above k = nz - 1) */
  int32_t psi_form;    /* pseudopotential of eq. (FORCE): 0 = exp(-1/rho), the paper's choice
                          (coexistence on the Maxwell construction); 1 = 1 - exp(-rho), the
                          original Shan-Chen form, one of the alternatives the paper cites as
                          prior art (coexistence on its own mechanical-stability rule).
                          Other values: LBM_EINVAL */
} lbm_params;

typedef struct lbm_handle lbm_handle;

/* Library version string (static storage). */
const char* lbm_version(void);

/* Thread-local message of the last failure ("" if none). */
const char* lbm_last_error(void);

/* Bytes of device workspace lbm_init needs for these parameters, or 0 if the
 * parameters are invalid (then lbm_last_error says why). */
size_t lbm_workspace_bytes(const lbm_params* p);

/*
 * Set up a lattice at rest in local equilibrium (Algorithm section):
 *   f = f^eq(rho0, u = 0),  g = g^eq(rho0 T0, v = 0).
 * rho0: device, N doubles (> 0), the initial density field.
 * T0:   device, N doubles, or NULL for the conduction profile
 *       T0(k) = T_d + (T_u - T_d)(k + 1/2)/nz.
 * workspace: device, >= lbm_workspace_bytes(p) bytes, 256-byte aligned;
 *   owned by the caller, used by the handle until lbm_destroy.
 * stream: hipStream_t (as void*) on which all work of this handle runs.
 * On success *out is a new handle (host memory owned by the library).
 * Synchronous with respect to the stream on return.
 */
int lbm_init(const lbm_params* p, void* workspace, size_t workspace_bytes,
             const double* rho0, const double* T0, void* stream, lbm_handle** out);

/*
 * The seeded initial density of the workloads (row a10 of the step's set-up):
 *   rho0[n] = rho_mean (1 + noise_amp (2 u_n - 1)),  n = i + nx (j + ny k),
 * u_n = (SplitMix64 output for state seed + (n + 1) 0x9E3779B97F4A7C15) >> 11,
 * divided by 2^53 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014), in IEEE double without contraction, so the field
 * is bit-identical to any implementation of the same definition.
 *   rho0: device, nx*ny*nz doubles, written (caller-owned); stream as lbm_init.
 * Asynchronous.  LBM_EINVAL for empty sizes, rho_mean <= 0 or noise_amp
 * outside [0, 1).
 */
int lbm_seeded_density(int32_t nx, int32_t ny, int32_t nz, uint64_t seed, double rho_mean,
                       double noise_amp, double* rho0, void* stream);

/*
 * Advance n >= 0 time steps of eqs. (LBEQ)/(LBEQ2): per step one collision
 * (BGK with the velocity-shifted f equilibrium, the pseudopotential force
 * of eq. (FORCE) with the thermal and gravity forces, the g equilibrium with
 * the counter-term) and one streaming with the walls, on the handle's
 * stream (asynchronous unless the numeric guard below is on).
 */
int lbm_step(lbm_handle* h, int64_t n);

/*
 * Numeric guard of lbm_step (failure detection; the paper has none).  With
 * every > 0, after each step whose count since lbm_init / lbm_set_state is a
 * multiple of `every`, lbm_step reads the state once more (FP64 sums of the
 * stored populations per node), synchronises the stream and returns
 * LBM_ENUMERIC (message: the step and what failed) if a node's populations
 * sum to a non-finite value or to rho <= 0, or if the stored mass differs
 * from its value at the first check (after lbm_set_check or lbm_set_state)
 * by more than mass_tol relative.  every = 0 turns the guard off (default).
 * LBM_EINVAL for every < 0 or mass_tol <= 0.
 */
int lbm_set_check(lbm_handle* h, int64_t every, double mass_tol);

/* Number of steps taken since lbm_init / lbm_set_state. */
int64_t lbm_time(const lbm_handle* h);

/*
 * Global FP64 diagnostics of the current state (eqs. (HYDRO), (internal)):
 * totals (host, 6 doubles) = [sum rho, sum rho v_x, sum rho v_y, sum rho v_z,
 *   sum rho T, sum rho U] with v = (j + F/2)/rho the physical velocity and
 *   U = c_v T + (G/4) exp(-2/rho) the internal energy.
 * fields (device, 5*N doubles, or NULL): rho, v_x, v_y, v_z, T.
 * Synchronises the stream.  Returns LBM_ENUMERIC if a value is non-finite or
 * rho <= 0 somewhere.
 */
int lbm_moments(lbm_handle* h, double* totals, double* fields);

/*
 * Nusselt numbers (eq. (flux), Fig. 2 bottom) in units of kappa (T_d-T_u)/nz:
 *   nu_bot = 2 nz (T_d - Tbar(0)) / (T_d - T_u)  (half-cell wall flux),
 *   nu_top = 2 nz (Tbar(nz-1) - T_u) / (T_d - T_u),
 *   nu_z[k] = [<rho U v_z>(k) - kappa (Tbar(k+1) - Tbar(k-1))/2] nz / (kappa (T_d-T_u))
 *     with ghost planes Tbar(-1) = 2 T_d - Tbar(0), Tbar(nz) = 2 T_u - Tbar(nz-1),
 *   T_z[k] = Tbar(k), the horizontal mean of T.
 * nu_bot, nu_top: host, may be NULL; nu_z, T_z: host, nz doubles, may be NULL.
 * Synchronises the stream.  Needs walls and T_d != T_u (else LBM_EINVAL).
 */
int lbm_nusselt(lbm_handle* h, double* nu_bot, double* nu_top, double* nu_z, double* T_z);

/*
 * Plane profile of the pressure work, the right-hand side of the layer heat
 * balance eq. (heat2) and the integrand of the constraint eq. (flux),
 * Nu(z) - Nu(0) = -integral_0^z <P d_j u_j>:
 *   pw_z[k] = horizontal mean over plane k of P d_j v_j,
 * with P = rho T + (G/2) psi(rho)^2 the bulk equation of state (text after
 * eq. (ns); psi of the handle's psi_form), v = (j + F/2)/rho the physical
 * velocity and d_j v_j its divergence on the W stencil of eq. (FORCE)
 * (central differences; at the no-slip walls the ghost planes hold the
 * negative mirror image of v, periodic otherwise), all in FP64 from the
 * moment fields of lbm_moments.
 *   work: device, >= 5 * nx * ny * nz doubles, caller-owned; receives the
 *     moment fields (rho, v_x, v_y, v_z, T) as lbm_moments writes them.
 *   pw_z: host, nz doubles.
 * Synchronises the stream.  LBM_EWORKSPACE if work is too small;
 * LBM_ENUMERIC as lbm_moments.
 */
int lbm_pressure_work(lbm_handle* h, double* work, size_t work_bytes, double* pw_z);

/* node quantities for lbm_histogram */
enum {
  LBM_Q_RHO = 0,       /* density */
  LBM_Q_T = 1,         /* temperature E / rho */
  LBM_Q_VZ = 2,        /* vertical physical velocity */
  LBM_Q_HEATFLUX = 3   /* convective heat flux rho U v_z, U = c_v T + (G/4) exp(-2/rho) */
};

/*
 * Histogram of node quantities over the planes k0 <= k < k1: the joint
 * (rho, T) distribution of Fig. 2 (top panel, T-rho scatter against the
 * equilibrium curves, per region of the cell) and the pdf of the bulk heat
 * flux rho U u_z of Fig. 2 (inset of the bottom panel), eq. (flux).
 *   qx, qy: LBM_Q_*; qy = -1 for a 1-D histogram (then ny_bins = 1).
 *   Uniform bins: a node falls in bin (bx, by) = (floor((x - x_lo) nx_bins /
 *   (x_hi - x_lo)), likewise y) when 0 <= bx < nx_bins and 0 <= by < ny_bins,
 *   the scale computed once in FP64 as nx_bins / (x_hi - x_lo); x, y in FP64
 *   (rho and E summed in FP64 from the stored populations).
 *   counts: device, nx_bins * ny_bins uint64 (row-major, by fastest),
 *     overwritten.  out_of_range (host, may be NULL): nodes in no bin.
 *   sums (host, 5 doubles, may be NULL): [nodes, sum x, sum x^2, sum y, sum y^2]
 *     over all nodes of the planes, in or out of range (FP64).
 * Synchronises the stream.  LBM_EINVAL for an empty plane or bin range, an
 * unknown quantity or more than 2^26 bins.
 */
int lbm_histogram(lbm_handle* h, int32_t k0, int32_t k1, int32_t qx, double x_lo, double x_hi,
                  int32_t nx_bins, int32_t qy, double y_lo, double y_hi, int32_t ny_bins,
                  uint64_t* counts, uint64_t* out_of_range, double* sums);

/*
 * Structure functions with horizontal increments (Fig. 3): for r = 1..r_max
 *   S_2(r) = < (a(x + r e) - a(x))^2 >,  S_4(r) = < (a(x + r e) - a(x))^4 >,
 * averaged over the nodes of planes k0 <= k < k1 and over e = x and e = y
 * (periodic), a one of LBM_Q_* (u_z: LBM_Q_VZ; T: LBM_Q_T) in FP64; the
 * flatness is S_4 / S_2^2.
 *   work: device, >= lbm_structure_work_bytes(h, k0, k1, r_max) bytes
 *     (the field over the planes, per-block partial sums), caller-owned.
 *   out: host, 2 * r_max doubles: [S_2(1..r_max), S_4(1..r_max)].
 * 1 <= r_max <= 256 and r_max < nx, ny; nx, ny <= 8192.  Deterministic
 * (fixed-order sums).  Synchronises the stream.
 */
size_t lbm_structure_work_bytes(const lbm_handle* h, int32_t k0, int32_t k1, int32_t r_max);
int lbm_structure_functions(lbm_handle* h, int32_t k0, int32_t k1, int32_t q, int32_t r_max,
                            double* work, size_t work_bytes, double* out);

/*
 * lbm_structure_functions without a work buffer, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the field over the planes and the
 * per-block partial sums go to a static device array of the library, 32 MiB
 * per GPU (held until the process ends), instead of the caller's work
 * buffer.  Same arguments, results and errors as lbm_structure_functions
 * (the same kernels), plus LBM_EWORKSPACE when lbm_structure_work_bytes()
 * for these planes exceeds 33554432 bytes (e.g. more than about 3.6 million
 * nodes over the planes).  Allocates nothing, host or device.  Every call on
 * one GPU uses that GPU's one array, so calls that overlap on one GPU (from
 * several host threads or streams) race; calls in sequence are safe.
 */
int lbm_structure_functions_noalloc(lbm_handle* h, int32_t k0, int32_t k1, int32_t q,
                                    int32_t r_max, double* out);

/* Checkpoint and restore (resume a run, or the adjoint's recomputation of a
 * segment from its checkpoint): copy the current state to / from a canonical
 * FP64 state (device, 38*N doubles, layout above, caller-owned).  set_state
 * encodes to the handle's storage (16-bit forms: the rounding residuals of
 * the moving pairs go to the rest pair, so the stored sums equal the given
 * ones) and resets lbm_time to 0.  Both are asynchronous on the stream;
 * LBM_EINVAL for NULL arguments. */
int lbm_get_state(lbm_handle* h, double* state);
int lbm_set_state(lbm_handle* h, const double* state);

/*
 * Discrete adjoint (reverse mode) of one step, for gradients of objectives of
 * the trajectory (the step is eqs. (LBEQ)/(LBEQ2) with everything of the
 * Algorithm section, so its transposed Jacobian is exact up to rounding).
 * Needs a handle made with adjoint = 1 (which adds 88 bytes per node of
 * workspace).  The arithmetic is FP64 for every storage form: the adjoint
 * linearises the FP64 step about the given state, which for a reduced-precision
 * handle is a state of its own (rounded) trajectory.
 *   state:   device, canonical FP64 state s_t (the input of the step t -> t+1);
 *   adj_in:  device, 38*N doubles, lambda_{t+1} = dJ/ds_{t+1};
 *   adj_out: device, 38*N doubles, receives lambda_t = (ds_{t+1}/ds_t)^T lambda_{t+1}
 *            (must not alias adj_in);
 *   grads:   host, 2 doubles, accumulated: [dJ/dG, dJ/dT_d] through this step
 *            (T_d enters through the bottom-wall rule), may be NULL.
 * Synchronises the stream.
 */
int lbm_adjoint_step(lbm_handle* h, const double* state, const double* adj_in, double* adj_out,
                     double* grads);

/*
 * Wall heat flux q_bot = 2 kappa (T_d - Tbar(0)) of a canonical state (text
 * before eq. (heat2); half-cell wall difference) and its adjoint:
 *   q (host, may be NULL) receives q_bot;
 *   adj (device, 38*N doubles, may be NULL) += weight * dq_bot/dstate;
 *   grads (host, may be NULL): grads[1] += weight * dq_bot/dT_d = weight * 2 kappa.
 * Needs walls.  Synchronises the stream.
 */
int lbm_adjoint_qbot(lbm_handle* h, const double* state, double weight, double* adj, double* q,
                     double* grads);

/*
 * Gradient with respect to the initial density field of lbm_init, from
 * lambda_0 (device, 38*N doubles) and the initial temperature T0 (device, N
 * doubles, or NULL for the conduction profile): dJ_drho0 (device, N doubles).
 */
int lbm_adjoint_init_rho(lbm_handle* h, const double* adj0, const double* T0, double* dJ_drho0);

/* Release the handle (the workspace stays the caller's). */
void lbm_destroy(lbm_handle* h);

/*
 * Bandwidth references for the roofline of the step (not part of the
 * method): plain streaming kernels that show what HBM delivers on this
 * device, timed beside the step by the caller.
 *
 * lbm_stream_copy: dst[0, bytes) = src[0, bytes), one 16-byte vector per
 *   thread; nontemporal != 0 marks the loads and stores non-temporal.
 *   src, dst: device, 16-byte aligned, not overlapping; bytes a positive
 *   multiple of 16.  Asynchronous on stream.
 * lbm_stream_rows: the step's streaming pattern without its arithmetic:
 *   every thread reads 8 bytes at the same offset of each of `rows` rows
 *   (row_stride bytes apart) and writes them to the same places of dst,
 *   all loads before the stores (the step reads 19 population rows and
 *   writes 19).  rows: 1, 2, 4 or 19; row_bytes: bytes moved per row
 *   (multiple of 8); row_stride >= row_bytes (multiple of 8); src, dst:
 *   device, 8-byte aligned, rows * row_stride bytes each, not overlapping.
 *   Asynchronous on stream.
 * Both return LBM_EINVAL for arguments outside these ranges.
 */
int lbm_stream_copy(const void* src, void* dst, size_t bytes, int32_t nontemporal, void* stream);
int lbm_stream_rows(const void* src, void* dst, int32_t rows, size_t row_stride, size_t row_bytes,
                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
