/*
 * lbmd.h -- C ABI of the MI355X (gfx950) coupled lattice-Boltzmann / bead-dynamics library.
 *
 * The library advances the hybrid scheme of Fyta, Melchionna, Kaxiras and Succi,
 * "Coupling Lattice Boltzmann with Atomistic Dynamics for the multiscale
 * simulation of nano-biological flows" (arXiv:0710.1272), Sec. II:
 *   - a D3Q19 BGK lattice-Boltzmann solvent (Eq. lbe, f_eq eq.), with periodic or
 *     specular free-slip outer faces and half-way bounce-back on solid nodes
 *     (the separating wall with a square pore of Sec. III);
 *   - bead chains moved by Langevin dynamics (Eq. force: harmonic bonds, WCA
 *     bead-bead and bead-wall repulsion, a pulling force inside the pore,
 *     frictional drag against the local fluid velocity, random force);
 *   - the two-way coupling of Sec. II: nearest-grid-point velocity interpolation
 *     at each bead, M MD substeps per LB step with that velocity frozen, and the
 *     equal and opposite force spread back as the source S_p (S_p eq.).
 * Any number of independent replicas (boxes of different sizes, each with its own
 * chains and random seed) advance together.
 *
 * Conventions used throughout:
 *   - Node index of (x,y,z) in a replica of nx*ny*nz nodes: x + nx*(y + ny*z).
 *   - Populations p = 0..18 in the order: rest; +x,-x,+y,-y,+z,-z;
 *     (+1,+1,0),(-1,-1,0),(+1,-1,0),(-1,+1,0),(+1,0,+1),(-1,0,-1),(+1,0,-1),
 *     (-1,0,+1),(0,+1,+1),(0,-1,-1),(0,+1,-1),(0,-1,+1).
 *   - Lattice units: Delta x = Delta t = 1; c_s^2 = 1/3; omega = 1/tau.
 *   - Host arrays that cover several replicas hold the replicas back to back in
 *     replica order, each block in the layout stated for one replica.
 *   - Every call returns LB_OK (0) or a negative LB_E* code; on error,
 *     lb_last_error_message() describes it.  No C++ exception crosses this ABI.
 *   - All calls on one context must come from one host thread at a time.
 */
#ifndef LBMD_H
#define LBMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------------ */
#define LB_OK 0
#define LB_EINVAL (-1)    /* invalid argument or configuration */
#define LB_ENOMEM (-2)    /* device or host allocation failed */
#define LB_EDEVICE (-3)   /* HIP runtime error, or no usable gfx950 device */
#define LB_EUNSTABLE (-4) /* the device error word is set (see LB_ERR_* bits) */
#define LB_ESTATE (-5)    /* call not valid in the context's current state */
#define LB_ESIZE (-6)     /* caller buffer too small */

/* bits of the device error word (reported through LB_MOM_STATUS) */
#define LB_ERR_BEAD_IN_SOLID 1u   /* a bead centre lies inside a solid node cube */
#define LB_ERR_BEAD_OUTSIDE 2u    /* a bead crossed a free-slip outer face */
#define LB_ERR_NONFINITE 4u       /* a bead coordinate is not finite */
#define LB_ERR_BOND_STRETCH 8u    /* a bond is longer than 2 r0 */
#define LB_ERR_DENSITY 16u        /* a fluid node met rho <= 0 or a non-finite rho */
#define LB_ERR_CONSTRAINT 32u     /* rigid bonds: SHAKE did not converge in shake_iter iterations */

/* ---- configuration ---------------------------------------------------------- */
#define LB_BC_PERIODIC 0
#define LB_BC_FREESLIP 1

#define LB_STORE_F64 0     /* populations stored and collided in FP64 */
#define LB_STORE_F32 1     /* populations stored and collided in FP32 */
#define LB_STORE_F16DEV 2  /* FP16 store of s_p (f_p - w_p rho0), FP32 collision */
#define LB_STORE_BF16DEV 3 /* BF16 store of s_p (f_p - w_p rho0), FP32 collision */

#define LB_MAX_WALLS 2

/* A separating wall (Sec. III): solid node planes x0..x1 over the whole
 * cross-section, except the open pore y0..y1 x z0..z1 (no pore if y0 > y1). */
typedef struct lbmd_wall {
    int x0, x1;
    int y0, y1;
    int z0, z1;
} lbmd_wall;

typedef struct lbmd_replica {
    int nx, ny, nz;        /* box size in nodes, each >= 2 */
    int bc[3];             /* LB_BC_PERIODIC or LB_BC_FREESLIP per axis */
    int n_walls;           /* 0..LB_MAX_WALLS */
    lbmd_wall wall[LB_MAX_WALLS];
    double tau;            /* BGK relaxation time, > 1/2 (nu = (tau - 1/2)/3, Sec. II) */
    double rho0;           /* reference density; also the 16-bit deviation origin */
    double fluid_kT;       /* temperature of the thermal source F_p of Eq. lbe (the
                              fluctuating LB the paper cites; formula: lb_step); 0 = no F_p */
    int n_chains;          /* number of linear chains */
    const int* chain_len;  /* host, n_chains lengths >= 1; read during lb_init only */
    uint64_t seed;         /* Philox key (low word, high word) of this replica */
} lbmd_replica;

/* Bead-model parameters shared by all replicas (Sec. II Eq. force; Sec. III). */
typedef struct lbmd_md_params {
    int M;             /* MD substeps per LB step, Delta t_MD = 1/M */
    double mass;       /* bead mass m */
    double gamma;      /* friction coefficient: F_drag = -m gamma (v - u) */
    double kT;         /* temperature of the random force */
    double k_bond;     /* harmonic bond k (r - r0)^2 / 2 between chain neighbours */
    double r0;
    double eps, sigma; /* WCA between non-bonded beads, cut at 2^(1/6) sigma */
    double eps_w, sigma_w; /* WCA on the distance to the nearest solid surface / free-slip face */
    double f_drive;    /* pulling force on beads whose nearest node is a pore node */
    int drive_sign;    /* +1: along +x; -1: along -x */
    int rigid;         /* 0: harmonic bonds (k_bond, r0); 1: rigid bonds of length r0, the
                          N-1 holonomic constraints of Sec. II, enforced on positions by
                          SHAKE (Newton iterations) and on velocities by RATTLE; at most
                          512 beads per replica */
    double kappa_phi;  /* angular term kappa_phi phi^2 / 2 between consecutive bonds (>= 0) */
    double shake_tol;  /* rigid bonds: |s^2 - r0^2| <= shake_tol r0^2 for every bond */
    int shake_iter;    /* rigid bonds: most Newton iterations per substep; not converging
                          sets LB_ERR_CONSTRAINT */
    int stencil;       /* coupling stencil of steps 1 and 3 (Sec. II): LB_STENCIL_* */
} lbmd_md_params;

/* stencil: the node(s) a bead takes the fluid velocity from and gives its reaction to */
#define LB_STENCIL_NGP 0       /* the nearest node floor(r + 1/2) (Sec. II, Fig. 1) */
#define LB_STENCIL_TRILINEAR 1 /* the 8 surrounding nodes floor(r_a) + {0, 1}, weights
                                  prod_a (1 - |r_a - x_a|); periodic axes wrap, a node beyond a
                                  free-slip face is the face node; solid nodes give u = 0 and
                                  drop their share of the reaction; the reaction uses the
                                  stencil of the start-of-step position.  LB_MOM_COUPLING then
                                  reports node -1 for every bead */

/* Optional initial state (host arrays, read during lb_init only). */
typedef struct lbmd_initial_state {
    const double* rho;    /* [V] per replica, or NULL for rho0 everywhere */
    const double* u;      /* [3][V] per replica (u_x block, u_y, u_z), or NULL for rest */
    const double* pops;   /* [19][V] per replica pre-collision populations; overrides rho/u */
    const double* bead_r; /* [n_beads][3] per replica positions; required if there are beads */
    const double* bead_v; /* [n_beads][3] per replica velocities, or NULL for rest */
    int64_t step0;        /* initial value of the LB step counter (Philox counter word) */
} lbmd_initial_state;

#define LB_CFG_NO_GRAPH 1u   /* enqueue plain launches instead of captured HIP graphs */
#define LB_CFG_AUTOTUNE 2u   /* time candidate launch shapes (lattice kernel, lanes per bead of
                                the bead kernel) at lb_init and keep the fastest; the bead
                                state is restored after the trial steps */
#define LB_CFG_DETERMINISTIC 4u /* bitwise identical results from run to run for one configuration.
                                   The nearest-node path always is: one leader bead per node adds
                                   the summed reaction of the node's beads in bead order.  With it,
                                   the trilinear spread (step 3 of Sec. II) rounds each contribution
                                   -w_c (w_p / c_s^2) Fbar . c_p once to a multiple of 2^-48, sums a
                                   node's contributions as 64-bit integers (exact, so in any order)
                                   and adds each node's sums to its populations once, instead of
                                   floating-point atomic adds whose order varies; and LB_CFG_AUTOTUNE
                                   leaves the lanes per bead at their choice by bead count, since
                                   they set the order of the bead-force sums.  The lattice kernel's
                                   launch shape never changes results.  A contribution above 512
                                   in magnitude is dropped and sets LB_ERR_NONFINITE (so that no
                                   node's 64-bit sum can overflow below 64 contributions).  FP16 and
                                   BF16 storage take this fixed-point spread with or without the
                                   flag (it is faster there than a floating-point add into a 16-bit
                                   element) */

typedef struct lbmd_config {
    int n_replicas;
    const lbmd_replica* replicas;      /* host array of n_replicas */
    int storage;                       /* LB_STORE_* for every replica */
    lbmd_md_params md;
    const lbmd_initial_state* init;    /* may be NULL: rest fluid at rho0, no beads allowed */
    int block_size;                    /* threads per block of the lattice kernel, 0 = default */
    int lattice_mapping;               /* LB_MAP_*: how lattice-kernel threads map to nodes */
    int xcd_order;                     /* LB_XCD_* or a chunk size > 0: tile order over the 8 XCDs */
    int md_lanes;                      /* lanes per bead in the bead kernel: 0 = by bead count,
                                          1, 2 (up to 512 beads in the largest replica), or
                                          4/8/16 with lanes x (beads of the largest replica)
                                          <= 512; LB_CFG_AUTOTUNE times the choices */
    unsigned flags;                    /* LB_CFG_* */
    int obs_every;                     /* record the translocation observables (LB_MOM_OBSERVABLES)
                                          after every step whose new step count is a multiple of
                                          obs_every; 0 = none */
    int obs_capacity;                  /* rows kept per replica (later rows are counted, not kept) */
} lbmd_config;

/* lattice_mapping */
#define LB_MAP_AUTO 0  /* flat (LB_CFG_AUTOTUNE also tries rows, shifted and flat2) */
#define LB_MAP_FLAT 1  /* each wave takes 64 consecutive nodes of a replica */
#define LB_MAP_ROWS 2  /* each wave takes one segment of at most 64 nodes of one x-row */
#define LB_MAP_SHIFTED 3 /* flat, with each x-row rotated by whole 128-byte lines so that
                            the planes within one node of a wall share as few waves as
                            possible (the other waves skip the bounce-back tests); the same
                            as flat unless nx is a multiple of 64 and the replica has walls */
#define LB_MAP_FLAT2 4   /* two nodes per lane, 64 apart (a wave takes 128 consecutive nodes):
                            twice the bytes in flight per wave; blocks of 128-512 threads */
/* xcd_order (a value C > 0 deals chunks of C consecutive tiles round-robin to the XCDs) */
#define LB_XCD_AUTO 0        /* contiguous for one replica, hardware order for several */
#define LB_XCD_HARDWARE (-1) /* blocks in launch order (the hardware deals them round-robin) */
#define LB_XCD_CONTIGUOUS (-2) /* each XCD takes one contiguous eighth of the tiles */

/* Device buffers.  Either all NULL-free (caller-owned, sizes from
 * lb_required_bytes) or the whole struct pointer NULL (library-owned).
 * Population buffer layout: the replicas' blocks one after another, each [19][S] elements of
 * the storage type, population p of node n (linear index x + nx (y + ny z)) at p S + n, with
 * the plane stride S = lb_plane_stride(replica, storage) >= V (elements n >= V of a plane are
 * padding that no call reads or writes).  The slots hold post-collision values of the pull
 * scheme (Sec. II Eq. lbe), FP16/BF16 as deviations from w_p rho0 scaled per weight class. */
typedef struct lbmd_buffers {
    void* pops[2]; /* device, lb_required_bytes(cfg, LB_BUF_POPS) bytes each, 256-byte aligned */
    void* beads;   /* device, lb_required_bytes(cfg, LB_BUF_BEADS) bytes, 256-byte aligned */
    void* work;    /* device, lb_required_bytes(cfg, LB_BUF_WORK) bytes, 256-byte aligned */
} lbmd_buffers;

#define LB_BUF_POPS 0
#define LB_BUF_BEADS 1
#define LB_BUF_WORK 2

typedef struct lbmd_ctx lbmd_ctx;

/* Bytes the caller must provide for buffer `which` (LB_BUF_*), 0 on an invalid
 * configuration.  Pure host computation. */
size_t lb_required_bytes(const lbmd_config* cfg, int which);

/* Checks a configuration on the host, without touching the device.  Rejects
 * tau <= 1/2, boxes below 2 nodes, boxes above 2^30 nodes or whose one population exceeds
 * 4 GiB (FP64 storage: 2^29 nodes), walls or pores outside the box, walls closer
 * than 2 nodes to a periodic x face, M < 1, an unstable bond/substep ratio
 * (2 sqrt(k/m)/M >= 2, the kick-drift stability limit), chain lengths that do
 * not add up, and unknown storage. Returns LB_OK or LB_EINVAL. */
int lb_validate_config(const lbmd_config* cfg);

/* Sec. II, the lattice-Boltzmann and bead state of every replica.
 * Validates cfg, binds (or allocates) the device buffers, writes the initial
 * populations (f_eq of the given rho/u, or the given pre-collision populations),
 * uploads beads, optionally autotunes, and prepares the step sequence.
 * hip_stream: a hipStream_t (NULL = default stream) on which every later call
 * enqueues its work.  *out receives a library-owned context freed by lb_destroy.
 * Synchronises the stream before returning. */
int lb_init(const lbmd_config* cfg, const lbmd_buffers* bufs, void* hip_stream, lbmd_ctx** out);

#define LB_STEP_COUPLED 1u  /* steps 1-4 of Sec. II; without it: lattice update only */
#define LB_STEP_NO_HYDRO 2u /* beads only, in a fluid at rest (the no-solvent comparison of
                               Sec. III): u_i = 0, no spreading, populations untouched */

/* Enqueues n_steps LB time steps (Eq. lbe with Delta t = 1).  The thermal source
 * F_p (replicas with fluid_kT > 0; Sec. II gives no formula and cites the fluctuating LB
 * of Adhikari et al.) is noise on the non-conserved moments of the collision with the
 * covariance that keeps the equilibrium population fluctuations mu rho w_p at every
 * node, mu = fluid_kT / c_s^2: F = phi Pi eta, phi = sqrt(mu rho (1 - (1 - omega)^2)),
 * eta_p = sqrt(w_p) xi_p, (Pi x)_p = x_p - w_p (sum x + 3 c_p . sum c x), rho the
 * pre-collision density; xi_p = sqrt(12) ((k_p + 1/2) / 2^24 - 1/2) with k_p the top 24
 * bits of Philox4x32-10 word p of the counters (node, step, j, 2), j = 0..4, keyed by the
 * replica seed (node = x + nx (y + ny z), step = the low word of the step counter).  With
 * LB_STEP_COUPLED each step is: nearest-node velocity interpolation at the beads,
 * M MD substeps with that velocity frozen, then the lattice update with the
 * spread reaction force S_p = -(w_p / c_s^2) Fbar_i . c_p added after collision
 * at each bead's node (Fbar_i = mean over the substeps of drag + random force).
 * Without it, only the lattice stream-and-collide runs.  With LB_STEP_NO_HYDRO
 * (exclusive with LB_STEP_COUPLED) only the beads advance: M substeps with drag
 * against u_i = 0 and the random force, no lattice update, no spreading; the step
 * counter advances as for any step.  Asynchronous: returns launch errors, or
 * LB_EINVAL for both flags together. */
int lb_step(lbmd_ctx* ctx, int n_steps, unsigned flags);

/* Captures and instantiates, for either population-buffer parity, the HIP graphs that
 * lb_step(ctx, n_steps, flags) launches (graphs of 16 steps and one of n_steps mod 16), so
 * that later lb_step calls of that length capture and instantiate nothing.  Enqueues no work
 * and leaves the state unchanged; does nothing with LB_CFG_NO_GRAPH.  Returns LB_EINVAL for
 * n_steps < 0 or both step flags, LB_EDEVICE if a capture fails. */
int lb_graph_prepare(lbmd_ctx* ctx, int n_steps, unsigned flags);

#define LB_COUPLE_INTERP 1u /* step 1 of Sec. II alone: u(x) -> u_i, nearest node of each bead */
#define LB_COUPLE_SPREAD 2u /* step 3 alone: add the spread reaction of the last MD call's Fbar */

/* One half of the coupling, for checking each half separately.  INTERP reads
 * the current pre-collision state; SPREAD adds S_p to the current (post-collision,
 * not yet streamed) state at the nodes found by the last INTERP.  The sequence
 * INTERP, md_step, lb_step(1, 0), SPREAD equals one coupled step.  Asynchronous. */
int lb_couple(lbmd_ctx* ctx, unsigned dir);

/* Step 2 of Sec. II alone: M substeps of every replica's beads with the fluid
 * velocity of the last INTERP frozen; accumulates Fbar.  Asynchronous. */
int md_step(lbmd_ctx* ctx);

#define LB_MOM_CONSERVED 1u   /* 4 doubles: total mass, momentum x, y, z over fluid nodes (FP64) */
#define LB_MOM_FIELDS 2u      /* [4][V] doubles: rho, u_x, u_y, u_z per node (0 on solid nodes) */
#define LB_MOM_POPULATIONS 3u /* [19][V] doubles: pre-collision populations (0 on solid nodes) */
#define LB_MOM_BEADS 4u       /* [n][3] positions then [n][3] velocities, doubles */
#define LB_MOM_TRANSLOC 5u    /* 6 doubles: N_T, completion step (-1 if none), COM x, y, z, step */
#define LB_MOM_COUPLING 6u    /* [n][3] u_i, [n][3] Fbar_i, [n] node index (-1 on solid), doubles */
#define LB_MOM_STATUS 7u      /* 2 doubles: device error word, LB step counter */
#define LB_MOM_OBSERVABLES 8u /* [1 + obs_capacity][8] doubles: row 0 = (rows recorded, obs_every,
                                 obs_capacity, 0...); then one row per recorded bead step:
                                 step count after it, N_T, S_H, S_E, K, R_U^2, R_T^2, x of the centre of
                                 mass (the Sec. III analysis: S_H = m gamma sum v_i . u_i (eq. Shydro)
                                 with u_i the fluid velocity interpolated for that step, S_E = sum
                                 F_drive,i . v_i (eq. Selec) over beads whose nearest node is a pore
                                 node, K = m/2 sum |v_i|^2, R_U^2 / R_T^2 the squared radii of
                                 gyration of the beads at x <= / > the mid-plane of wall 0, 0 for an
                                 empty part); recorded in coupled, no-solvent and md_step bead steps */

/* Observables of one replica (Sec. II Eqs. dens and vel; Sec. III translocation
 * coordinate).  Synchronises the stream and copies into host_out (bytes long).
 * Returns LB_ESIZE if bytes is too small, LB_EUNSTABLE if the device error word
 * is non-zero (the output is still written), LB_OK otherwise. */
int lb_moments(lbmd_ctx* ctx, int replica, unsigned what, void* host_out, size_t bytes);

/* Bytes lb_moments needs for (replica, what); 0 if invalid. */
size_t lb_moments_bytes(const lbmd_ctx* ctx, int replica, unsigned what);

/* LB_MOM_FIELDS or LB_MOM_POPULATIONS for the `count` consecutive nodes node0 ..
 * node0 + count - 1 of one replica (linear index x + nx (y + ny z)), written to host_out
 * as [4][count] or [19][count] doubles (caller-owned, at least 8 * ncomp * count bytes),
 * for sampling boxes too large to copy whole.  Synchronises like lb_moments.  Returns
 * LB_EINVAL for another `what` or a range outside the replica, LB_ESIZE for a short
 * buffer, LB_EUNSTABLE (output still written) when the device error word is set. */
int lb_moments_range(lbmd_ctx* ctx, int replica, unsigned what, long long node0, int count, void* host_out,
                     size_t bytes);

/* For callers that cannot allocate (code under HIP graph capture, tight loops, harnesses that
 * forbid hipMalloc): the FP64 totals of lb_moments(LB_MOM_CONSERVED) for one replica's block of
 * populations, with no context and no allocation of any kind.  The reduction's partial sums go
 * to a static device array of the library: 1 MiB on each GPU it runs on, held until the process
 * ends and shared by every call on that GPU, so calls that overlap in time on one GPU (other
 * streams or host threads) race and return wrong sums.
 *   pops:       device: the replica's [19][S] block of a population buffer in `storage` (S =
 *               lb_plane_stride(rep, storage)), as lb_init lays it out (the current state is
 *               buffer pops[0] after an even number of lattice updates since lb_init); read
 *               only; aligned to its element size
 *   storage:    LB_STORE_*
 *   rep:        host: the replica's box, faces, walls and rho0, read during the call (its chains
 *               are ignored)
 *   out4:       device, 4 doubles written: total mass and momentum x, y, z over the fluid nodes
 *               of the pre-collision state (Sec. II Eqs. dens and vel), summed in a fixed order
 *   hip_stream: a hipStream_t to enqueue on (NULL = the default stream)
 * Asynchronous, no synchronisation (it can be captured into a graph).  Returns LB_EINVAL for a
 * NULL or misaligned pointer, unknown storage or an invalid replica, LB_ESIZE for a replica of
 * more than 2^27 nodes (the array holds 32768 blocks of partial sums, one per 4096 nodes), and
 * LB_EDEVICE for a launch error. */
int lb_conserved_noalloc(const void* pops, int storage, const lbmd_replica* rep, double* out4, void* hip_stream);

/* Plane stride S (elements) of a replica's population block in `storage`: the smallest odd
 * multiple of 256 bytes at least 12032 bytes beyond the V nodes of a plane, so that the 19
 * planes of a sweep (Sec. II Eq. lbe) do not start a multiple of a large power of two apart,
 * which puts their streams on the same HBM channels.
 * Returns -1 (with lb_last_error_message set) for a NULL replica, unknown storage or a
 * non-positive box size. */
long long lb_plane_stride(const lbmd_replica* rep, int storage);

/* Lattice-kernel launch shape in use (threads per block). */
int lb_block_size(const lbmd_ctx* ctx);

/* Lattice-kernel launch shape in use: threads per block, LB_MAP_FLAT/ROWS/SHIFTED/FLAT2, the XCD
 * tile order (LB_XCD_HARDWARE, LB_XCD_CONTIGUOUS or a chunk size) and whether the
 * populations are written with non-temporal stores (1: both buffers together exceed
 * 160 MB, so they are streamed past the last-level cache; 0: they stay cached between
 * steps).  Any pointer may be NULL.  Returns LB_OK or LB_EINVAL for a NULL context. */
int lb_launch_shape(const lbmd_ctx* ctx, int* block, int* mapping, int* xcd_order, int* nt_stores);

/* Measurement reference for the lattice kernel (the streaming of Eq. lbe without the collision):
 * one launch that reads the 19 populations of every node of the current state at the lattice
 * kernel's pull addresses (the node index minus c_p's offset, wrapped into the replica; no face
 * or wall handling) and writes them unchanged to the node's slots in the other population
 * buffer, with the launch shape in use (block size, XCD tile order, store policy; one node per
 * lane).  Its duration bounds what the lattice kernel's access pattern reaches on this GPU.
 * alternate = 0: the copy overwrites the other buffer, which the next lattice update rewrites
 * wherever a later step reads it; the current state is unchanged.  alternate != 0: the copy
 * becomes the current state, so that back-to-back copies alternate between the two buffers as
 * lattice updates do (repeated copies out of one buffer find it in the last-level cache when
 * both buffers together fit there, which lattice updates do not); the populations are then a
 * shifted copy with no physical meaning, and the context should only be measured or destroyed
 * afterwards.  Asynchronous. */
int lb_pattern_copy(lbmd_ctx* ctx, int alternate);

/* Lanes per bead of the bead kernel in use (1, 2, 4, 8 or 16; each bead's neighbour
 * loop is split over its lanes), 0 if no replica has beads, LB_EINVAL for a NULL
 * context. */
int lb_md_lanes(const lbmd_ctx* ctx);

/* Synchronises the stream, frees library-owned buffers and the context. */
int lb_destroy(lbmd_ctx* ctx);

/* Static description of an error code. */
const char* lb_strerror(int code);

/* Message of the last failing call on this thread ("" if none). */
const char* lb_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMD_H */
