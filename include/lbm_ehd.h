/*
 * lbm_ehd.h — C ABI of the MI355X (gfx950) three-phase leaky-dielectric EHD
 * lattice Boltzmann step.
 *
 * Method: Liu, Qian, Xiong, Wang, "Onsager-variational-principle-based
 * lattice Boltzmann model for three-phase dielectric fluid flows"
 * (arXiv 2608.05787), Sec. 3: D2Q9 lattice (Eq. 31), Eq. (33) stencils,
 * Cahn-Hilliard LB with split degenerate mobility (Eqs. 34-36, 28), flow LB
 * (Eqs. 37-41), potential LB with permittivity decomposition (Eqs. 42-45),
 * charge LB (Eqs. 46-50), closed system Eqs. (27a)-(27e), properties
 * Eqs. (29)-(30), spreading coefficients Eq. (9).
 *
 * Conventions for every call:
 *  - Return value: 0 on success, a negative LBM_EHD_E* code on failure.  No
 *    call aborts, exits or throws; lbm_ehd_last_error() gives a message.
 *  - Device memory is owned by the caller.  The library keeps non-owning
 *    pointers into the caller's workspace and never allocates device memory.
 *  - All device work of a handle is ordered on the HIP stream given at
 *    create time.  Only lbm_ehd_create, lbm_ehd_diagnostics, lbm_ehd_status,
 *    lbm_ehd_scalars, lbm_ehd_restore and lbm_ehd_profile_end synchronise
 *    that stream.
 *  - Conditions the device detects while stepping (a non-finite velocity or
 *    pressure; a residual-controlled potential loop that reached sub_max)
 *    are latched in a per-instance status word and returned by the next
 *    lbm_ehd_diagnostics or lbm_ehd_status call: LBM_EHD_EDIVERGED stays
 *    latched, LBM_EHD_ENOCONV (a warning: the state is valid) is cleared once
 *    returned.
 *  - One handle is used by one host thread at a time.
 *  - Layout of every field plane: row-major [ny][nx], x fastest.
 */
#ifndef LBM_EHD_H
#define LBM_EHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ehd_s *lbm_ehd_t; /* opaque; host memory owned by the library */

enum {
  LBM_EHD_OK = 0,
  LBM_EHD_EINVAL = -1,       /* invalid argument or parameter */
  LBM_EHD_ENOMEM = -2,       /* workspace or buffer too small / misaligned */
  LBM_EHD_EHIP = -3,         /* a HIP runtime call failed */
  LBM_EHD_EDIVERGED = -4,    /* non-finite populations detected */
  LBM_EHD_ENOCONV = -5,      /* potential iteration hit its cap (state valid) */
  LBM_EHD_ESTATE = -6,       /* call not valid in the handle's state */
  LBM_EHD_EUNSUPPORTED = -7  /* feature not available in this library */
};

enum { LBM_BC_PERIODIC = 0, LBM_BC_WALL = 1 }; /* x (and z) are always periodic */
enum { LBM_LATTICE_D2Q9 = 0, LBM_LATTICE_D3Q15 = 1 };
/* Charge transport: the leaky-dielectric charge family (Eqs. 46-50) or a
 * symmetric two-ion Nernst-Planck electrolyte (Eq. 52). */
enum { LBM_CHARGE_LEAKY = 0, LBM_CHARGE_NERNST_PLANCK = 1 };
enum { LBM_PREC_FP32 = 0, LBM_PREC_FP16S = 1, LBM_PREC_FP64 = 2, LBM_PREC_TANGENT = 3 };
/* LBM_DTYPE_TANGENT_F64: the derivative part of a tangent-mode handle's
 * fields, as float64. */
enum { LBM_DTYPE_F32 = 0, LBM_DTYPE_F64 = 1, LBM_DTYPE_TANGENT_F64 = 2 };

/* Field bits for lbm_ehd_fields (the fields computed during the last step;
 * after create, the initial fields). */
enum {
  LBM_F_PHI1 = 1u << 0, LBM_F_PHI2 = 1u << 1, LBM_F_PHI3 = 1u << 2,
  LBM_F_RHO = 1u << 3, LBM_F_UX = 1u << 4, LBM_F_UY = 1u << 5, LBM_F_P = 1u << 6,
  LBM_F_PSI = 1u << 7, LBM_F_EX = 1u << 8, LBM_F_EY = 1u << 9, LBM_F_Q = 1u << 10,
  LBM_F_MU1 = 1u << 11, LBM_F_MU2 = 1u << 12, LBM_F_MU3 = 1u << 13,
  LBM_F_EPS = 1u << 14, LBM_F_R = 1u << 15,
  LBM_F_UZ = 1u << 16, LBM_F_EZ = 1u << 17, /* D3Q15 only */
  LBM_F_NPLUS = 1u << 18, LBM_F_NMINUS = 1u << 19 /* Nernst-Planck only */
};
/* Population families for lbm_ehd_populations. */
enum { LBM_POP_F = 0, LBM_POP_G = 1, LBM_POP_L = 2, LBM_POP_H = 3 };

/*
 * Parameters of one instance.  Physical inputs in lattice units
 * (dx = dt = 1, cs^2 = 1/3):
 *  nx, ny        lattice nodes (>= 2 each); walls sit half-way, at y = -1/2
 *                and y = ny - 1/2, when bc_y == LBM_BC_WALL.
 *  wall_u        tangential wall speeds [bottom, top] (moving-wall
 *                bounce-back of every family with an advective equilibrium).
 *  wall_phi      Dirichlet electric potential of the walls (electrodes), by
 *                anti-bounce-back of the potential populations.
 *  wall_q_mode   0: charge no-flux (bounce-back); 1: Dirichlet charge wall_q.
 *  E_ext         uniform applied field: an imposed mean gradient of the
 *                potential, psi = psi' - E_ext . x with psi' periodic
 *                (carried by the potential populations); the permittivity
 *                source of Eq. (43) and the gradient of Eq. (45) are those
 *                of the full psi, so Eq. (42) holds for it, and
 *                E = -grad(psi).
 *  gamma12..23   pair surface tensions -> lambda_i of Eq. (9); each lambda_i
 *                must be > 0.
 *  width         interface thickness D of Eq. (7).
 *  rho, visc, eps, sigma  per-phase density, dynamic viscosity,
 *                permittivity, conductivity (Eqs. 29-30).
 *  tau_f         CH relaxation time, m0 = cs^2 (tau_f - 1/2) (Eq. 34 text).
 *  tau_l         charge relaxation time, alpha = cs^2 (tau_l - 1/2).
 *  eps_ref_phase phase whose permittivity is the reference of Eq. (42);
 *                tau_h = 1/2 + eps_ref / cs^2.
 *  phase_mode    0: evolve the three order parameters; 1: keep them frozen.
 *  sub_min, sub_max, sub_tol  potential sub-iterations per step.  Fixed
 *                count when sub_min == sub_max or sub_tol <= 0; otherwise the
 *                loop stops after iteration k once k >= max(sub_min, 2) and
 *                the relative L2 change of the potential over iteration k-1
 *                is below sub_tol.  1 <= sub_min <= sub_max <= 4096.
 *  init_sub_max, init_tol  cold-start iterations of create (same rule with
 *                sub_min = 1; init_tol <= 0 runs exactly init_sub_max).
 *  precision     LBM_PREC_FP32: FP32 populations and arithmetic;
 *                LBM_PREC_FP64: the same kernels in double precision;
 *                LBM_PREC_FP16S: FP32 arithmetic, populations stored as
 *                half-precision values scaled by 2^14 (f, j >= 1), 2^16 (g)
 *                and 2^16 (l), rest populations f^i_0 and the potential
 *                populations in FP32; magnitudes must stay below 4, 1 and 1
 *                (overflow shows up as non-finite populations);
 *                LBM_PREC_TANGENT: FP64 values carrying their derivative
 *                along the parameter direction dtheta (forward-mode
 *                differentiation of the same kernels, 16 bytes per value).
 *  lattice       LBM_LATTICE_D2Q9 (Eq. 31: an nx x ny plane, nz must be 0 or
 *                1) or LBM_LATTICE_D3Q15 (Eq. 32: an nx x ny x nz box,
 *                periodic in z as in x; y as set by bc_y).  All instances
 *                of a handle share the lattice.  Fields and populations are
 *                then [nz][ny][nx]; vector fields have 3 components (u, E:
 *                the z parts are the LBM_F_UZ, LBM_F_EZ fields) and the
 *                families 15 populations (f 45).  The potential source
 *                weights are 1/14 on the moving D3Q15 directions (1/8 on
 *                D2Q9).  Reverse-mode gradients are D2Q9 only.
 *  nz            layers in z (D3Q15); 0 is read as 1.
 *  E_ext_z       z component of the applied field (D3Q15).
 *  charge_model  LBM_CHARGE_LEAKY: charge family with the Ohmic source of
 *                Eq. (47).  LBM_CHARGE_NERNST_PLANCK: two ion
 *                concentrations n_+ and n_- (valences +1, -1) transported by
 *                Eq. (52); each is the zeroth moment of a BGK
 *                advection-diffusion family (the l populations hold both,
 *                [2][Q][N]) with equilibrium w_j n (1 + c_j . (u + v)/cs^2)
 *                and drift v = z ion_beta D E, D = cs^2 (ion_tau - 1/2); the
 *                charge is q = ion_charge (n_+ - n_-) and walls are no-flux.
 *                Requires sigma = 0 (ions carry the current), wall_q_mode 0,
 *                FP32, FP64 or tangent precision, and init ions0; forward
 *                mode only (reverse-mode gradients are refused).
 *  sum_relax     0: the CH scheme of Eqs. (34)-(36) as printed.  1: the
 *                variable part of the diffusion flux of phase i in Eq. (36)
 *                gains m0 (phi_i / S) grad S, S = phi_1 + phi_2 + phi_3
 *                (grad S by Eq. 33), so that the three families carry S back
 *                to the model's constraint S = 1 (Sec. 2, Eq. 56) by
 *                diffusion with the mobility m0.  Every phase keeps its mass,
 *                an absent phase stays absent, and where S = 1 the scheme
 *                is the printed one.  It removes the truncation error that
 *                the three separately evolved order parameters accumulate
 *                in S where the flow's continuity error is largest (triple
 *                junctions at density jumps, Sec. 4.3).  Both gradient
 *                modes cover it.
 *  ion_tau, ion_beta, ion_charge  Nernst-Planck: relaxation time of the
 *                ion families (> 1/2), e/(k_B T) in potential units, and the
 *                charge e of a unit concentration.
 *  dtheta        tangent mode only: direction in the parameter space
 *                theta = (eps2/eps1, eps3/eps1, sigma2/sigma1, sigma3/sigma1,
 *                E0).  The first four scale eps2, eps3, sigma2, sigma3 with
 *                eps1, sigma1 fixed.  E0 is the magnitude of the applied
 *                field |E_ext + (0, (wall_phi[0] - wall_phi[1]) / ny)|; its
 *                direction scales E_ext, the electrode potentials about
 *                their mean and the initial potential guess about the same
 *                mean, proportionally.
 */
typedef struct {
  int32_t nx, ny, bc_y, wall_q_mode;
  int32_t eps_ref_phase, phase_mode, sub_min, sub_max;
  int32_t init_sub_max, precision, nz, lattice;
  double sub_tol, init_tol;
  double wall_u[2], wall_phi[2], wall_q[2], E_ext[2];
  double gamma12, gamma13, gamma23, width;
  double rho[3], visc[3], eps[3], sigma[3];
  double tau_f, tau_l;
  double dtheta[5];
  double E_ext_z;
  int32_t charge_model, sum_relax;
  double ion_tau, ion_beta, ion_charge;
} lbm_ehd_params;

/* Initial fields of one instance, HOST pointers to float64 arrays on the
 * instance's grid G ([ny][nx], or [nz][ny][nx] on D3Q15):
 * phi0 [3][G] (required); u0 [D][G], q0 [G] and psi0 (initial guess of the
 * potential) [G] may be NULL (zero); ions0 [2][G] (n_+, n_-) is required
 * under the Nernst-Planck charge model, which then ignores q0 (q =
 * ion_charge (n_+ - n_-)), and ignored otherwise.  Read during create only. */
typedef struct {
  const double *phi0, *u0, *q0, *psi0, *ions0;
} lbm_ehd_init;

/* Bytes of device workspace that lbm_ehd_create needs for n_inst instances
 * with the given parameters (array of n_inst).  The workspace must be
 * 256-byte aligned. */
int lbm_ehd_workspace_bytes(const lbm_ehd_params *params, int32_t n_inst, size_t *bytes);

/* Create a handle for n_inst instances (params[n_inst], init[n_inst]).
 * dev_workspace: caller-owned device memory of at least workspace_bytes.
 * hip_stream: the hipStream_t all work is ordered on (NULL = null stream).
 * Maps the parameters, uploads the initial fields, iterates the potential
 * from psi0 with q0 (cold start), computes the chemical potentials and sets
 * every population to the equilibrium of the initial fields.  Synchronises
 * the stream.  On success *out receives the handle. */
int lbm_ehd_create(const lbm_ehd_params *params, int32_t n_inst, const lbm_ehd_init *init,
                   void *dev_workspace, void *hip_stream, lbm_ehd_t *out);

/* Enqueue n >= 0 coupled time steps of every instance (asynchronous).
 * One step is the scheme of Sec. 3 in this order: order-parameter moments
 * (text after Eq. 36) and properties (Eqs. 29-30); the charge of Eq. (50)'s
 * text with the source R of Eq. (47) on the previous step's field; the
 * potential sub-iterations (Eqs. 42-45; fixed count or residual-controlled,
 * see sub_min/sub_max/sub_tol); the field and the chemical potentials
 * (Eqs. 45, 20); the force (Eq. 27b) and flow moments (Eq. 41); the
 * collisions of the three order-parameter families (Eqs. 34-36 with the
 * mobility of Eq. 28), the flow family (Eqs. 37-40) and the charge family
 * (Eqs. 48-50), each streamed with the wall rules described at
 * lbm_ehd_params; Eq. (33) gives every gradient and Laplacian.
 * With a captured graph (lbm_ehd_graph) whole blocks of steps are replayed
 * with one hipGraphLaunch each; remaining steps are launched kernel by
 * kernel.  Results are identical either way.  Errors: EINVAL for n < 0;
 * EHIP if a launch fails; device-detected conditions are latched (see the
 * conventions above). */
int lbm_ehd_step(lbm_ehd_t h, int64_t n);

/* Capture steps_per_graph (even, >= 2) coupled steps of every instance into
 * a HIP graph that lbm_ehd_step replays (one launch for the whole block, all
 * instances and all kernels).  0 releases the graph.  Needs a non-default
 * stream; enqueues nothing. */
int lbm_ehd_graph(lbm_ehd_t h, int32_t steps_per_graph);

/* n >= 0 coupled time steps of every instance (the scheme of Sec. 3, as
 * lbm_ehd_step) run by one grid-resident kernel per block of up to 256
 * steps: a cooperative launch of one 1024-thread block per CU takes every
 * stage of a step (moments and properties, the charge step with the
 * potential sub-iterations of Eqs. 42-45 four at a time on LDS tiles, field
 * and chemical potentials, collide-and-stream) over the node and tile lists
 * of all instances, with a grid-wide barrier between stages.  The state
 * after n steps is bitwise that of lbm_ehd_step in a tall-tile launch
 * configuration (LBM_TUNE_TALL_TILES set, LBM_TUNE_SINGLE_POTENTIAL
 * clear); in the others it agrees to rounding.  Needs D2Q9, FP32 or FP16S
 * storage, the leaky-dielectric charge model and a fixed sub-iteration
 * count that is a multiple of 4 (LBM_EHD_EUNSUPPORTED otherwise); not while
 * profiling (LBM_EHD_ESTATE).  Synchronises after every launch.  Every
 * barrier wait is bounded: should one run out (about 2 s), the call returns
 * LBM_EHD_EHIP and the state is undefined. */
int lbm_ehd_step_persistent(lbm_ehd_t h, int64_t n);

/* Bound of one barrier wait of lbm_ehd_step_persistent, in polls of about
 * 1 us (polls >= 1; default 2^21).  A wait that runs out makes every block
 * of the launch leave and the call return LBM_EHD_EHIP with the state
 * undefined: a small bound forces that path from the host (its test). */
int lbm_ehd_set_persistent_polls(lbm_ehd_t h, int32_t polls);

/* Stage timing of lbm_ehd_step_persistent (on: 1; default 0): the launches
 * then run a variant of the kernel in which one block reads the device's
 * constant-rate wall clock after every grid barrier (same results; the
 * readings cost the stages registers, ~2 % of the step). */
int lbm_ehd_set_persistent_timing(lbm_ehd_t h, int32_t on);

/* Where the last lbm_ehd_step_persistent call with stage timing on spent its
 * time: us[0..3], the average microseconds per step of the moments stage,
 * the charge step with the potential passes, the field and chemical
 * potential stage and the collide-and-stream stage, each with the grid
 * barrier that ends it.  LBM_EHD_ESTATE before such a call. */
int lbm_ehd_persistent_stage_times(lbm_ehd_t h, double us[4]);

/* Write the selected fields of instance `inst` into caller device memory
 * dev_dst as consecutive planes [popcount(mask)][ny][nx] in ascending bit
 * order, converted to dtype (LBM_DTYPE_F32 or LBM_DTYPE_F64; for a tangent
 * handle LBM_DTYPE_TANGENT_F64 gives the derivatives).  Async.
 * The fields are those the last step formed: phi_i (zeroth moments, text
 * after Eq. 36), rho (Eq. 29), u and p (Eq. 41), the potential and the field
 * E = -grad(psi) (Eq. 45 with the applied field, see E_ext), q and R (Eq. 47
 * and the text after Eq. 50), mu_i (Eq. 20), eps (Eq. 30).  dev_dst must
 * hold popcount(mask) * nodes values of the dtype; EINVAL for an instance
 * out of range, an empty mask or bits the handle does not have. */
int lbm_ehd_fields(lbm_ehd_t h, int32_t inst, uint32_t mask, void *dev_dst, int32_t dtype);

/* Pre-collision populations of the current level of instance `inst`,
 * converted to dtype: family LBM_POP_F gives [3][Q][G], LBM_POP_L under the
 * Nernst-Planck model [2][Q][G] (n_+ then n_-), the others [Q][G] (Q = 9 on
 * D2Q9, 15 on D3Q15).  FP16S values are unscaled (the stored half value divided by
 * its family's power-of-two scale; f^i_0 from its FP32 plane).  Async. */
int lbm_ehd_populations(lbm_ehd_t h, int32_t inst, int32_t family, void *dev_dst, int32_t dtype);

/* Diagnostics of instance `inst` from the fields of the last step, FP64
 * reductions in a fixed order:
 *  out[0..2] sum_x phi_i (conserved, Eq. 5 and the CH equations Eq. 27c),
 *  out[3] sum_x q (Eq. 17), out[4] max |phi1+phi2+phi3-1| (Eq. 5),
 *  out[5] relative potential change of the last sub-iteration, out[6]
 *  sub-iterations of the last step, out[7] non-finite population count;
 *  out[8], out[9]: the deformation factor of Sec. 4.4,
 *  D = (r_par - r_perp) / (r_par + r_perp), of the outer drop (indicator
 *  w = 1 - phi1) and the inner drop (w = phi3), with the field along y:
 *  r_par is half the distance between the w = 1/2 crossings on the y line
 *  through the indicator's centroid (weights max(w, 0)), r_perp the same on
 *  the x line; w on a line between nodes is interpolated linearly, the
 *  crossings linearly between the last node with w >= 1/2 and the next,
 *  scanning outward from the node nearest the centroid; nan where a line
 *  has no crossing (a wall first, or w >= 1/2 throughout);
 *  out[10], out[11]: the second-moment form (sqrt(I_par) - sqrt(I_perp)) /
 *  (sqrt(I_par) + sqrt(I_perp)) of the same indicators entered as
 *  w * s(w), s = 0 below 0.005, 1 above 0.02, cubic smoothstep between;
 *  out[12..15]: r_par, r_perp of the outer drop, then of the inner.
 * Synchronises.  Returns LBM_EHD_EDIVERGED if out[7] > 0 or a non-finite
 * value was latched, else LBM_EHD_ENOCONV if a residual-controlled potential
 * loop reached sub_max since the last report (the outputs are valid). */
int lbm_ehd_diagnostics(lbm_ehd_t h, int32_t inst, double out[16]);

/* For callers that cannot allocate device memory (serving loops,
 * harnesses that forbid hipMalloc): lbm_ehd_diagnostics with its per-block
 * partial sums in a static device buffer of the library instead of the
 * handle's workspace.  Same outputs (bitwise) and return codes as
 * lbm_ehd_diagnostics; allocates nothing.  The buffer holds 65536 node
 * blocks of 256 nodes (16.7 M nodes over all of the handle's instances,
 * 12 MiB per GPU, kept until the process ends); larger handles get
 * LBM_EHD_ENOMEM.  Every call on one GPU shares that GPU's buffer: calls
 * that overlap in time on one GPU (several host threads, or handles on
 * different streams) race and must be serialised by the caller.
 * Synchronises. */
int lbm_ehd_diagnostics_static(lbm_ehd_t h, int32_t inst, double out[16]);

/* Latched status of every instance (see the conventions above), without a
 * reduction pass: synchronises, ORs the instances' status bits into *flags
 * (may be NULL; bit 1: non-finite velocity or pressure formed, bit 2: a
 * potential loop reached sub_max) and returns LBM_EHD_EDIVERGED,
 * LBM_EHD_ENOCONV or LBM_EHD_OK.  Reporting clears bit 2. */
int lbm_ehd_status(lbm_ehd_t h, int32_t *flags);

/* Host-side counters: out[0] steps taken, out[1] total potential
 * sub-iterations run in those steps (summed over instances), out[2]
 * instances.  Synchronises. */
int lbm_ehd_scalars(lbm_ehd_t h, double out[3]);

/* Launch configuration (autotuning).  The block order and the collide load
 * schedule do not change the results (bitwise); the two potential kernel
 * forms agree to rounding (their multiply-adds are scheduled differently).
 * Bits:
 *  LBM_TUNE_LINEAR_ORDER: launched blocks take node blocks (and potential
 *    tiles) in row order, instead of giving each XCD a contiguous range of
 *    rows (neighbour rows then share that XCD's L2);
 *  LBM_TUNE_SINGLE_POTENTIAL: fixed-count potential sub-iterations run one
 *    launch each instead of the LDS-tiled kernel (which exists
 *    for fixed-count D2Q9 handles in FP32, FP16S or FP64; elsewhere single
 *    launches are the only form and the bit changes nothing);
 *  LBM_TUNE_COLLIDE_PER_FAMILY: the collide kernel loads each population
 *    family next to its use (fewer registers, more waves per SIMD) instead
 *    of issuing every load before its first store (more loads in flight);
 *    FP32 and FP16S handles (FP64 and tangent always load per family);
 *  LBM_TUNE_TALL_TILES: the LDS-tiled potential kernel uses 64 x 32 tiles
 *    (two rows per thread) instead of 64 x 16 (60 x 12 written), and runs
 *    four sub-iterations per launch (ring of 4, 56 x 24 written, one HBM
 *    round trip of h per four sub-iterations) while four remain, then two
 *    (60 x 28 written); FP32 and FP16S handles where the LDS-tiled kernel
 *    runs.  With a fixed even K >= 4 the step's first four-sub-iteration
 *    launch also forms the charge, Ohmic source and permittivity on its
 *    tiles (no separate launch for them).  The forms agree to rounding (the
 *    compiler fuses their multiply-adds differently).
 * A captured graph (lbm_ehd_graph) is re-captured with the new
 * configuration. */
enum {
  LBM_TUNE_LINEAR_ORDER = 1,
  LBM_TUNE_SINGLE_POTENTIAL = 2,
  LBM_TUNE_COLLIDE_PER_FAMILY = 4,
  LBM_TUNE_TALL_TILES = 8
};
int lbm_ehd_set_tuning(lbm_ehd_t h, int32_t config);
int lbm_ehd_get_tuning(lbm_ehd_t h, int32_t *config);

/* Autotuner: from the handle's current state, runs 2 warm-up steps and
 * times `steps` steps (HIP events on the handle's stream) under each
 * configuration 0..15, then restores the state and keeps the fastest.
 * dev_scratch: caller device memory of lbm_ehd_checkpoint_bytes (holds the
 * saved state).  ms_per_step[c]: time per step of configuration c, or -1 for
 * a configuration that coincides with another on this handle (a bit that
 * changes nothing; not run).  *best (may be NULL) receives the configuration kept.
 * Synchronises the stream; not while profiling (ESTATE). */
int lbm_ehd_tune(lbm_ehd_t h, int32_t steps, void *dev_scratch, double ms_per_step[16], int32_t *best);

/* Save / restore the complete evolving state (populations of the current
 * level, history planes, last fields, control words) to / from caller
 * device memory of lbm_ehd_checkpoint_bytes.  Checkpoint is async; restore
 * synchronises (it reads back the restored step count).  N+N steps with a
 * save/restore in between equal 2N steps bitwise. */
int lbm_ehd_checkpoint_bytes(lbm_ehd_t h, size_t *bytes);
int lbm_ehd_checkpoint(lbm_ehd_t h, void *dev_buf);
int lbm_ehd_restore(lbm_ehd_t h, const void *dev_buf);

/* Gradients of a linear functional of the final fields,
 *   J = sum over selected fields F and nodes x of seed_F(x) * F(x),
 * with respect to theta = (eps2/eps1, eps3/eps1, sigma2/sigma1,
 * sigma3/sigma1, E0) (see dtheta above), for the run of n_steps steps that
 * starts from this handle's creation state (create's cold start included).
 * A nonlinear objective of the fields (a deformation parameter, say) passes
 * its derivative with respect to the fields as the seed.  Fields are the
 * planes lbm_ehd_fields returns after the run.  dev_seed: device float64
 * planes [popcount(seed_mask)][ny][nx] in ascending bit order of seed_mask
 * (LBM_F_* bits).  grad_theta receives dJ/dtheta.  All calls synchronise;
 * single-instance handles only.
 *
 * Reverse mode (the discrete adjoint of the step and of create):
 * lbm_ehd_record steps the handle n_steps from its creation state exactly
 * like lbm_ehd_step (bitwise the same states) and saves a checkpoint of the
 * state every ckpt_every steps into dev_work.  lbm_ehd_adjoint then runs
 * the adjoint sweep: segments of ckpt_every steps, last first, are
 * recomputed from their checkpoint in a private handle inside dev_work,
 * storing each step's forward values, and the step adjoints run backwards
 * through them; finally the adjoint of create (equilibrium populations,
 * field, the cold-start potential iterations recomputed in chunks, the
 * initial potential guess).  If dev_work does not hold a recording of this
 * handle for the same n_steps and ckpt_every, lbm_ehd_adjoint first makes
 * one inside it from the handle's initial fields (the handle itself is not
 * touched).  Needs: FP32 or FP64 precision, fixed sub-iteration counts
 * (step and cold start), eps_ref_phase 0, seeds on LBM_F_PHI1..3 only.
 * Arithmetic in the handle's precision, parameter sums in FP64.
 * Returns LBM_EHD_EUNSUPPORTED otherwise.  dev_work: caller device memory
 * of lbm_ehd_adjoint_workspace_bytes(n_steps, ckpt_every), 256-byte
 * aligned: a workspace, one checkpoint per segment, ckpt_every step
 * records of (22 + 9 K) planes and 176 adjoint planes.
 *
 * Forward mode: lbm_ehd_tangent_gradient runs one tangent run of the same
 * kernels in FP64 (LBM_PREC_TANGENT) per component of theta inside dev_work
 * (lbm_ehd_tangent_workspace_bytes) and contracts the tangent fields with
 * the seed; any fields may be seeded.  Cost: 5 FP64 tangent runs. */
int lbm_ehd_adjoint_workspace_bytes(lbm_ehd_t h, int64_t n_steps, int32_t ckpt_every, size_t *bytes);
int lbm_ehd_record(lbm_ehd_t h, int64_t n_steps, int32_t ckpt_every, void *dev_work, size_t work_bytes);
int lbm_ehd_adjoint(lbm_ehd_t h, int64_t n_steps, int32_t ckpt_every, const void *dev_seed,
                    uint32_t seed_mask, void *dev_work, size_t work_bytes, double grad_theta[5]);
int lbm_ehd_tangent_workspace_bytes(lbm_ehd_t h, size_t *bytes);
int lbm_ehd_tangent_gradient(lbm_ehd_t h, int64_t n_steps, const void *dev_seed, uint32_t seed_mask,
                             void *dev_work, size_t work_bytes, double grad_theta[5]);

/* Kernel timing.  Between lbm_ehd_profile_begin and lbm_ehd_profile_end
 * every kernel launch of the handle is bracketed by HIP events on its stream
 * (kernel durations are unchanged; launches are not otherwise altered).
 * lbm_ehd_profile_end synchronises and returns, per kernel kind, the summed
 * event time in ms and the launch count: index 0 moments, 1 charge/stencil
 * (pre), 2 single potential sub-iteration, 3 field + chemical potential,
 * 4 fused collide-and-stream, 5 diagnostics, 6 two or four potential
 * sub-iterations in one launch, 7 a step's first launch of four potential
 * sub-iterations that also forms the charge (kind 1's work, which then has
 * no launch of its own: a fixed even K >= 4 on tall tiles). */
int lbm_ehd_profile_begin(lbm_ehd_t h);
int lbm_ehd_profile_end(lbm_ehd_t h, double ms[8], int64_t launches[8]);

/* Release the handle (not the caller's device memory).  NULL is ignored. */
void lbm_ehd_destroy(lbm_ehd_t h);

const char *lbm_ehd_strerror(int code);
/* Message of the last failing call on h (h may be NULL: last create error). */
const char *lbm_ehd_last_error(lbm_ehd_t h);

#ifdef __cplusplus
}
#endif
#endif /* LBM_EHD_H */
