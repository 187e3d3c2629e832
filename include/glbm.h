/*
 * glbm.h — C ABI of the MI355X generalized lattice Boltzmann (GLBM) library.
 *
 * The library solves the generalized lattice Boltzmann equation of
 * Wang, Chen, Kang & Rahman, "Permeability prediction of organic shale with
 * generalized lattice Boltzmann model considering surface diffusion effect"
 * (arXiv:1601.00704), Sec. 2.3, Eq. (27)-(37): a Brinkman-type stream-and-
 * collide sweep over a voxelised shale map in which every node carries its own
 * porosity eps and apparent permeability K_app (Sec. 2.1, Eq. 18-19).  The
 * sweep is iterated to steady state and the sample's apparent permeability is
 * read off Darcy's law from the volume-averaged velocity (Eq. 26, Sec. 3.2).
 *
 * Conventions for every entry point
 *   - Return value: GLBM_OK (0) or a negative GLBM_E* code; glbm_last_error()
 *     then returns a thread-local message describing the failure.
 *   - Units: everything crossing this ABI is in lattice units (dx = dt = 1,
 *     c_s^2 = 1/3) except glbm_class_table, which converts SI inputs.
 *   - Layout: node index n = (z * ny + y) * nx + x (x fastest).  Velocity
 *     fields are three planes ux[N], uy[N], uz[N].
 *   - Ownership: host arrays passed in are copied before the call returns;
 *     host arrays passed out are written by the call and owned by the caller.
 *     A device population buffer passed to glbm_init_geometry stays owned by
 *     the caller and must outlive the context; all other device memory is
 *     allocated and freed by the library.
 *   - Streams: all device work of a context is issued on the HIP stream given
 *     to glbm_init_geometry (NULL = the null stream).  Calls that return
 *     values to the host synchronise that stream.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef GLBM_H
#define GLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Velocity sets (Eq. 29-31 leave the stencil open; the standard ones are used). */
enum { GLBM_D2Q9 = 9, GLBM_D3Q19 = 19 };

/* Population storage.  Arithmetic is FP64 for F64 and FP32 otherwise; the
 * residual and flux reductions are always accumulated in FP64.
 *   F64     f_i - w_i stored as double                       (145 B per D2Q9 update)
 *   F32     f_i - w_i stored as float                        (73 B).  The node
 *           collides in the local form (its own density part w_i (rho - 1)
 *           split off and put back with fused multiply-adds), so each stored
 *           value carries one rounding at the scale of the density deviation
 *           and solves reach r <= 1e-8 on shale maps (k within 1e-5 of FP64).
 *   F16DEV  (f_i - w_i) 2^s stored as IEEE half, rounded to nearest even (37 B).
 *           The velocity part of f is then resolved only relative to the
 *           density deviation: on the 128^2 shale map k is off by several
 *           percent, far outside 1e-3.  Accepted only with
 *           GLBM_FLAG_F16DEV_OPT_IN (a study form); use F16LOC.
 *   F16LOC  (f_i - w_i rho(x)) 2^s as IEEE half, with rho(x) - 1 of the node
 *           x that wrote the value kept in an extra float plane (45 B).
 *           Removing the node's own density leaves the velocity and
 *           non-equilibrium parts at full half precision (k within ~1e-4).
 *   F32LOC  (f_i - w_i rho(x)) as float with the same float density plane
 *           (81 B): FP32 storage whose rounding no longer scales with the
 *           density deviation, so the residual can fall further before
 *           rounding noise stops it. */
enum { GLBM_STORE_F64 = 0, GLBM_STORE_F32 = 1, GLBM_STORE_F16DEV = 2, GLBM_STORE_F16LOC = 3,
       GLBM_STORE_F32LOC = 4 };

enum {
    GLBM_OK = 0,
    GLBM_EINVAL = -1,        /* invalid argument (shape, tau <= 1/2, eps outside (0,1], K <= 0, ...) */
    GLBM_ENOMEM = -2,        /* device or host allocation failed, or caller buffer too small */
    GLBM_EDEVICE = -3,       /* a HIP runtime call failed */
    GLBM_ESTATE = -4,        /* call out of order (e.g. stepping before glbm_set_local_perm) */
    GLBM_ENONFINITE = -5,    /* a NaN or Inf population was seen by a check */
    GLBM_ENOTCONVERGED = -6, /* glbm_step_n reached its step budget with tol > 0 unmet */
    GLBM_EUNSTABLE = -7      /* a check saw a node velocity |u| > 0.1 (lattice units): outside the
                                low-Mach range where the equilibrium of Eq. (30) holds */
};

#define GLBM_WALL_CLASS 255           /* class code of a solid wall node (no fluid) */
#define GLBM_SCALE_AUTO (-2147483647 - 1) /* let the library pick the FP16 scale */

typedef struct glbm_ctx_s* glbm_ctx;

/* One problem instance.  lattice, store and check_every must be equal for
 * every instance of a context. */
typedef struct {
    int32_t lattice;         /* GLBM_D2Q9 or GLBM_D3Q19 */
    int32_t store;           /* GLBM_STORE_* */
    int32_t nx, ny, nz;      /* grid; nz = 1 for GLBM_D2Q9 */
    uint32_t wall_faces;     /* bit 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+: halfway bounce-back
                                at that domain face; faces without a bit are periodic.
                                Both faces of an axis must be set or clear together. */
    double tau;              /* BGK relaxation time of Eq. (29), > 1/2; nu = (tau - 1/2)/3 */
    double g[3];             /* external body force G of Eq. (27), lattice units */
    int32_t dev_scale_log2;  /* s of the F16DEV scale 2^s in [0, 30], or GLBM_SCALE_AUTO */
    int32_t check_every;     /* n_c > 0, even: residual and flux are evaluated every n_c steps */
    uint32_t flags;          /* GLBM_FLAG_* bits; 0 for the defaults */
    int32_t pressure_axis;   /* 0: no pressure faces; 1, 2, 3: pressure faces normal to x, y, z
                                (the inlet / outlet pressures of the paper's Tab. 4 and Tab. 7).
                                The face at coordinate 0 is held at density rho_in, the face at
                                n - 1 at rho_out, by the Zou-He rule (the populations entering
                                through a face are rebuilt from the known ones so that the node
                                has the face density and no tangential momentum).  The other
                                faces must be periodic; wall nodes are allowed.  Every instance
                                of a context has pressure faces or none does. */
    double rho_in, rho_out;  /* face densities (lattice units, > 0, different) */
} glbm_instance_desc;

/* Descriptor flags.  GLBM_FLAG_F16DEV_OPT_IN: accept GLBM_STORE_F16DEV, whose
 * k is outside the FP16 accuracy target on shale maps (see the store list). */
enum { GLBM_FLAG_F16DEV_OPT_IN = 1 };

/*
 * Bytes of device memory that the populations of these instances need (both
 * ping-pong buffers, with the library's padding).  The arrangement inside is
 * the library's own (node blocks of 4096 nodes for the FP64 and FP32 stores,
 * planes for the FP16 stores) and may change; read populations with
 * glbm_get_populations.  Returns 0 if the descriptors are invalid, including
 * when (q + 3) times the node count, rounded up to whole blocks, reaches 2^31
 * (32-bit element indices).
 */
size_t glbm_required_bytes(int32_t n_inst, const glbm_instance_desc* desc);

/*
 * Create a context for n_inst instances and upload their class maps.
 *   out         receives the context
 *   desc        n_inst descriptors
 *   cls_host    n_inst host pointers to uint8 class maps of nx*ny*nz nodes
 *               (x fastest); class 255 is a wall node, every other class
 *               must be given a table entry by glbm_set_local_perm
 *   pop_dev     device buffer of at least glbm_required_bytes() bytes owned
 *               by the caller (256-byte aligned), or NULL to let the library
 *               allocate it
 *   pop_bytes   size of pop_dev (ignored when pop_dev is NULL)
 *   hip_stream  hipStream_t for all work of the context (NULL: null stream)
 * The populations start at rest, f_i = w_i (rho = 1, u = 0) — the paper
 * leaves the initial state open.
 * Errors: GLBM_EINVAL (n_inst < 1, empty grid, tau <= 1/2, mixed lattice /
 * store / check_every, nz != 1 for D2Q9, odd check_every, pop_dev not
 * 256-byte aligned, scale outside
 * [0, 30], a wall face without its opposite face, unknown flag bits,
 * GLBM_STORE_F16DEV without GLBM_FLAG_F16DEV_OPT_IN); GLBM_ENOMEM; GLBM_EDEVICE.
 */
int glbm_init_geometry(glbm_ctx* out, int32_t n_inst, const glbm_instance_desc* desc,
                       const uint8_t* const* cls_host, void* pop_dev, size_t pop_bytes,
                       void* hip_stream);

/*
 * Set the per-class porosity eps, local permeability K (Eq. 27-28, K -> K_app)
 * and Forchheimer coefficient F_eps (Eq. 27) of instance inst (-1: every
 * instance).  Arrays hold n_classes entries for classes 0 .. n_classes-1
 * (n_classes <= 255).  k_lattice is K_app / dx^2; +INF marks an open pore (no
 * drag).  f_eps may be NULL (F_eps = 0: the paper drops the Forchheimer
 * term, Sec. 2.3).  The per-node constants of Eq. (36)-(37) are derived here.
 * Every class present in the map must be covered.
 * On an instance with pressure faces K is constant (the pressure-independent
 * case of glbm_set_pressure_perm) and F_eps must be 0.
 * Errors: GLBM_EINVAL (eps outside (0, 1], K <= 0 or NaN, F_eps < 0, a class
 * of the map without an entry, F_eps > 0 with pressure faces).
 */
int glbm_set_local_perm(glbm_ctx ctx, int32_t inst, int32_t n_classes, const double* eps,
                        const double* k_lattice, const double* f_eps);

/*
 * Pressure-dependent local permeability of an instance with pressure faces:
 * the apparent permeability of Eq. (18)-(19) evaluated at every node and step
 * at the local pressure,
 *     K(P) = k_const + k_knudsen / P + k_surface / (P (1 + langmuir_b P)),
 * which is Eq. (18) (K_0 + eta D_K / P) plus the surface-diffusion term of
 * Eq. (19) with the ideal-gas density (glbm_class_table_pressure computes the
 * coefficients).  Arrays of n_classes entries (classes 0 .. n_classes-1), K in
 * lattice units (K / dx^2), P in the unit of p_in / p_out (langmuir_b in its
 * inverse); k_const = +INF marks an open pore (no drag; the other coefficients
 * are ignored).  The local pressure is the affine image of the local lattice
 * density, which carries the pressure of Eq. (26):
 *     P(x) = p_out + (rho(x) - rho_out) (p_in - p_out) / (rho_in - rho_out).
 * Errors: GLBM_EINVAL (no pressure faces, eps outside (0, 1], k_const <= 0,
 * k_knudsen, k_surface or langmuir_b < 0 or not finite, p_in or p_out <= 0,
 * a class of the map without an entry, a class whose K(P) is not positive and
 * finite for every P between p_out and p_in).
 */
int glbm_set_pressure_perm(glbm_ctx ctx, int32_t inst, int32_t n_classes, const double* eps, const double* k_const,
                           const double* k_knudsen, const double* k_surface, const double* langmuir_b, double p_in,
                           double p_out);

/*
 * Advance every active instance by up to n time steps of Eq. (29).  At every
 * step count that is a multiple of check_every the library evaluates, per
 * instance, the residual r = ||u(t) - u(t - n_c)||_2 / (n_c ||u(t)||_2) over
 * fluid nodes (FP64 sums) and the Darcy flux.  tol <= 0: exactly n steps.
 * tol > 0: an instance stops at the first check with r <= tol; the call
 * returns when all instances have stopped (GLBM_OK) or after n steps
 * (GLBM_ENOTCONVERGED).  GLBM_ENONFINITE if a check saw NaN/Inf;
 * GLBM_EUNSTABLE if a check saw |u| > 0.1 at a fluid node (the state is kept
 * as of that check, stepping stops there).  GLBM_ESTATE before
 * glbm_set_local_perm.
 */
int glbm_step_n(glbm_ctx ctx, int64_t n, double tol);

/*
 * Per instance: r at the most recent check (+INF before the first) and the
 * number of steps taken.  Either pointer may be NULL.  Synchronises.
 */
int glbm_residual(glbm_ctx ctx, double* r, int64_t* steps);

/*
 * Apparent permeability of each instance by Darcy's law on the current state:
 * k[3*i + d] = nu <u_d> / G_d, <.> the mean over fluid nodes of the
 * volume-averaged velocity of Eq. (34); NaN where G_d = 0.  Along the axis of
 * pressure faces: nu <u_a> (n_a - 1) / (c_s^2 (rho_in - rho_out)), Darcy's law
 * with the lattice pressure c_s^2 rho over the node distance between the faces
 * (in a uniform medium of porosity eps this is K / eps, because c_s^2 rho
 * carries eps P).  Lattice units (multiply by dx^2 for m^2).  Synchronises.
 */
int glbm_permeability(glbm_ctx ctx, double* k_lattice);

/*
 * Replace the state of instance inst by the equilibrium of Eq. (30) at the
 * given density (N doubles) and velocity (3N doubles): a warm start.  The
 * residual snapshot is reset; step counts are kept.
 */
int glbm_set_fields(glbm_ctx ctx, int32_t inst, const double* rho, const double* u);

/* Same as glbm_set_fields from device arrays of floats: drho_dev[N] holds
 * rho - 1 (a float of rho itself would round a small density deviation
 * against 1), u_dev[3N] the velocity planes. */
int glbm_set_fields_device(glbm_ctx ctx, int32_t inst, const float* drho_dev, const float* u_dev);

/*
 * Density (N doubles) and velocity (3N doubles, Eq. 34) of the current state
 * of instance inst; wall nodes get zeros.  Either pointer may be NULL.
 */
int glbm_get_fields(glbm_ctx ctx, int32_t inst, double* rho, double* u);

/*
 * Post-streaming populations f_i(x, t) of instance inst as q planes of N
 * doubles (f_i, not deviations); wall-node slots are zero.  For tests and
 * inspection.
 */
int glbm_get_populations(glbm_ctx ctx, int32_t inst, double* f_host);

/*
 * Bitwise checkpoint of a whole context: glbm_state_bytes() bytes of host
 * memory hold the populations, residual snapshots and step counters.
 * glbm_load_state restores a checkpoint taken from a context created with
 * identical descriptors and tables.
 */
size_t glbm_state_bytes(glbm_ctx ctx);
int glbm_save_state(glbm_ctx ctx, void* host, size_t bytes);
int glbm_load_state(glbm_ctx ctx, const void* host, size_t bytes);

/*
 * Options (value in parentheses: default).
 *   GLBM_OPT_GRAPH (1)       replay full n_c-step chunks from a captured HIP graph
 *   GLBM_OPT_TIMING (0)      bracket every sweep launch with HIP events on the
 *                            context's stream; glbm_sweep_time reports the summed
 *                            time and the number of sweeps since the option was
 *                            set (a two-step launch, policy bit 6, counts as two)
 *   GLBM_OPT_TILE_WIDTH      nodes along x per workgroup tile: 64 .. 1024, a power
 *                            of two (default: 256, or the largest <= max nx)
 *   GLBM_OPT_TILE_ROWS       rows per tile, 1 .. 256; width x rows must be a
 *                            multiple of 256 (default: 256 / width)
 *   GLBM_OPT_CACHE (13)      memory policy bits: 0 nontemporal population stores;
 *                            1 nontemporal loads of the planes without an x shift;
 *                            2 workgroups in launch order (clear: grouped per XCD);
 *                            3 per-class constants read through L1 (clear: staged
 *                            in LDS); 4 LDS staging of the population and density
 *                            rows in the D2Q9 FP16 sweep (periodic instances with
 *                            nx a multiple of 8, tiles at most 256 nodes wide with
 *                            1, 2 or 4 rows; ignored elsewhere); 5 two x-adjacent
 *                            nodes per lane in the D2Q9 FP16 sweep (periodic
 *                            instances with nx even, tiles at least 128 nodes
 *                            wide and an even number of nodes per thread;
 *                            ignored elsewhere and when bit 4 applies); 6 two
 *                            time steps per launch, the intermediate state kept
 *                            in LDS (D2Q9; periodic instances with the F32,
 *                            F32LOC and F16LOC stores and tiles 64 x 4/8/16,
 *                            128 x 4/8 or 256 x 4, or the F64 store and tiles
 *                            64 x 4/8 or 128 x 4; pressure faces, with or
 *                            without wall nodes, with the F64 and F32 stores and
 *                            tiles 64 x 4/8 or 128 x 4; runs of 4k steps that
 *                            start at an even step go as 2k such launches, the
 *                            rest of a run as single steps; ignored elsewhere, see
 *                            glbm_sweeps_per_launch).  Same results bit for bit
 *                            under every policy.
 * Errors: GLBM_EINVAL for unknown options or values.
 */
enum { GLBM_OPT_GRAPH = 1, GLBM_OPT_TIMING = 2, GLBM_OPT_TILE_ROWS = 3, GLBM_OPT_TILE_WIDTH = 4,
       GLBM_OPT_CACHE = 5 };
int glbm_set_option(glbm_ctx ctx, int32_t option, int64_t value);
int glbm_sweep_time(glbm_ctx ctx, double* ms_total, int64_t* launches);

/*
 * Time steps that one sweep launch performs under the context's current
 * tile shape and cache policy: 2 where policy bit 6 (two time steps per
 * launch) applies to the context, else 1.  Host only, no device work.
 * Errors: GLBM_EINVAL for a null context or output pointer.
 */
int glbm_sweeps_per_launch(glbm_ctx ctx, int32_t* sweeps);

/*
 * Autotuner: time every (tile width, tile rows, cache policy) candidate for
 * `steps` sweeps and keep the fastest.  Widths 64 .. 1024 (up to twice the
 * widest instance), rows 1 .. 16, cache policies 1, 3, 4, 5, 9, 12, 13, 15
 * (and 29, 31 where the LDS-staged FP16 sweep applies, 37, 45, 47 where the
 * paired-node FP16 sweep does, 69, 71, 77, 79 where two steps per launch do and
 * `steps` is a multiple of 4).
 * The state advances by those sweeps (an even number per candidate); the
 * residual snapshot is reset.  If chosen is not NULL it receives {width,
 * rows, cache}.  Errors: GLBM_EINVAL for a null context or odd or < 2 steps;
 * a failing launch is returned as is, with the caller's stream joined.
 */
int glbm_autotune(glbm_ctx ctx, int32_t steps, int32_t* chosen);

/*
 * Velocity set of a lattice in the library's direction order: e receives q*3
 * ints (e_x, e_y, e_z per direction), w the q weights; either may be NULL.
 * This is the plane order of glbm_get_populations.
 * D2Q9:  rest, +x, +y, -x, -y, (+x,+y), (-x,+y), (-x,-y), (+x,-y).
 * D3Q19: rest, +x, -x, +y, -y, +z, -z, then the 12 edges as opposite pairs.
 */
int glbm_velocity_set(int32_t lattice, int32_t* e, double* w);

/*
 * Copy `bytes` of device memory with nontemporal 16-byte loads and stores (the
 * memory pattern of a sweep without its gathers and arithmetic): a measured
 * streaming ceiling of the GPU, for reporting a kernel's bandwidth against.
 * Queued on hip_stream; does not synchronise.  Errors: GLBM_EINVAL (null
 * pointers, or pointers or size not multiples of 16 bytes); GLBM_EDEVICE.
 */
int glbm_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Release every resource of the context (the caller's population buffer is not freed). */
int glbm_destroy(glbm_ctx ctx);

/* Message of the last failure on this thread ("" if none). */
const char* glbm_last_error(void);

/*
 * Physical inputs of the class table (SI units).
 */
typedef struct {
    double pressure;       /* P, Pa */
    double temperature;    /* T, K */
    double viscosity;      /* eta, Pa s */
    double molar_mass;     /* M, kg/mol */
    double tortuosity;     /* tau_t of Eq. (4) */
    double dx;             /* lattice spacing, m */
    double eps_iom;        /* porosity of inorganic matter */
    double eps_om;         /* porosity of organic matter */
    double langmuir_b;     /* b of Eq. (13), 1/Pa */
    double q_sat;          /* mol/m^3; <= 0: from langmuir_vl and toc by Eq. (38) */
    double langmuir_vl;    /* Langmuir volume, m^3 of methane at 273.15 K, 101.325 kPa per kg of rock */
    double toc;            /* organic volume fraction used by Eq. (38) */
    double d_s;            /* Maxwell-Stefan surface diffusivity, m^2/s */
} glbm_gas_params;

/*
 * Class table of a three-phase shale map: class 0 open pore (eps 1, K +INF);
 * classes 1 .. n_iom inorganic matter of radii r_iom (Eq. 18); classes
 * 128 .. 127 + n_om organic matter of radii r_om (Eq. 19).  Radii in m; the
 * pore diameter of Eq. (3)-(4) is twice the radius.  The gas density is the
 * ideal-gas P M / (R T).  eps_out and k_lattice_out receive 256 entries each
 * (unused classes: eps 1, K +INF); K is returned as K_app / dx^2.
 * Errors: GLBM_EINVAL (n_iom or n_om outside [0, 127], non-positive inputs).
 */
int glbm_class_table(const glbm_gas_params* p, int32_t n_iom, const double* r_iom, int32_t n_om,
                     const double* r_om, double* eps_out, double* k_lattice_out);

/*
 * The same classes as coefficients of K_app(P) = k_const + k_knudsen / P +
 * k_surface / (P (1 + b P)) (Eq. 18-19 with rho_g = P M / (R T); P in Pa), in
 * lattice units (divided by dx^2), for glbm_set_pressure_perm:
 *   k_const = K_0, k_knudsen = eta D_K, k_surface = eta R T (1 - eps) q_sat b D_s
 * (organic classes only), b_out = b of Eq. (13).  p->pressure is used only when
 * q_sat comes from Eq. (38) (it does not depend on it).  Open pores and unused
 * classes: eps 1, k_const +INF, the rest 0.  Each output holds 256 entries.
 * Errors: as glbm_class_table.
 */
int glbm_class_table_pressure(const glbm_gas_params* p, int32_t n_iom, const double* r_iom, int32_t n_om,
                              const double* r_om, double* eps_out, double* k_const_out, double* k_knudsen_out,
                              double* k_surface_out, double* b_out);

/* ---------------------------------------------- pore-size distributions -- */

#define GLBM_GMM_MAX_COMPONENTS 8

/*
 * Batched EM fit of one-dimensional Gaussian mixtures to pore-size samples
 * (Sec. 2.2, Eq. 20-24): the E-step responsibilities of Eq. (20) with the
 * Gaussian of Eq. (21) (input length 1, exponent negative), and the M-step
 * updates of Eq. (22)-(24), the variance taken about the updated mean.
 *   n_sets      independent sample sets
 *   offsets     host, n_sets + 1 entries: set s holds x_dev[offsets[s] ..
 *               offsets[s + 1]) (increasing, non-empty)
 *   x_dev       device array of the samples (double; e.g. pore radii or their
 *               logarithms)
 *   k           components, 1 .. GLBM_GMM_MAX_COMPONENTS
 *   phi, mu, var  host arrays of n_sets * k (set-major): in, the starting
 *               point (fractions > 0 summing to 1, variances > 0); out, the fit
 *   iters       maximum iterations
 *   tol         0: run exactly `iters` iterations; > 0: a set stops after the
 *               first iteration (from the second on) whose log-likelihood gain
 *               is <= tol times the log-likelihood
 *   loglik      host, n_sets (may be NULL): log-likelihood of the returned
 *               parameters, sum_i log sum_j Phi_j g_j(x_i)
 *   iters_done  host, n_sets (may be NULL): iterations each set ran
 * FP64 throughout; the sums are reduced in a fixed order, so results are
 * deterministic and do not depend on the other sets of the batch.  A
 * component whose responsibilities all vanish gets Phi = 0 (Eq. 22) and keeps
 * its mean and variance (Eq. 23-24 are then 0/0).  Work is
 * queued on hip_stream (NULL: null stream) and the call synchronises it.
 * Each call allocates its own device buffers and frees them before it returns,
 * so calls from several threads on different streams are independent.
 * Errors: GLBM_EINVAL (bad sizes or starting point), GLBM_ENOMEM, GLBM_EDEVICE.
 */
int glbm_gmm_fit(int32_t n_sets, const int64_t* offsets, const double* x_dev, int32_t k, double* phi, double* mu,
                 double* var, int32_t iters, double tol, double* loglik, int32_t* iters_done, void* hip_stream);

/*
 * Radius classes of one pore-size mode fitted in the logarithm of the radius
 * (a Gaussian of mean mu_ln and standard deviation sigma_ln in ln r): n
 * equal-probability bins, r_k = exp(mu_ln + sigma_ln z_k) with z_k the standard
 * normal quantile of (k + 1/2) / n, for the r_iom / r_om arguments of
 * glbm_class_table.  Errors: GLBM_EINVAL (n outside [1, 127], sigma_ln <= 0 or
 * a non-finite input).
 */
int glbm_radius_bins(double mu_ln, double sigma_ln, int32_t n, double* r_out);

/*
 * Whether the open pores (class 0) of a class map connect the two faces
 * normal to the drive axis: a chain of open-pore nodes, each linked to the
 * next by a velocity of the lattice (D2Q9: the 8 neighbours; D3Q19: the 18
 * face and edge neighbours), from coordinate 0 to coordinate n - 1 of that
 * axis, with the other axes periodic.  Near the site-percolation threshold of
 * that neighbourhood the k of random maps is bimodal across seeds (an
 * open-pore path or none); this flag tells the two branches apart.
 *   lattice, nx, ny, nz   as in glbm_instance_desc (nz = 1 for D2Q9)
 *   cls                   host class map, x fastest (not retained)
 *   axis                  1 = x, 2 = y, 3 = z (as pressure_axis)
 *   percolates            receives 1 or 0
 * Host only; no device work.  Errors: GLBM_EINVAL (null pointers, empty grid,
 * an unknown lattice, nz != 1 for D2Q9, axis out of range).
 */
int glbm_pore_percolates(int32_t lattice, int32_t nx, int32_t ny, int32_t nz, const uint8_t* cls, int32_t axis,
                         int32_t* percolates);

#ifdef __cplusplus
}
#endif

#endif /* GLBM_H */
