// lbmd_internal.hpp -- host-side internals shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "lbmd.h"
#include "lbmd_device.hpp"

namespace lbmd {

// Scalar bead-model parameters as the MD kernel uses them.
struct MDDev {
    int M;
    double h, inv_M;
    double mass, inv_mass, gamma, A;  // A = sqrt(24 m gamma kT / h)
    double k_bond, r0;
    double eps, sigma2, rc2;          // WCA bead-bead: rc^2 = 2^(1/3) sigma^2
    double eps_w, sigma_w2, rcw2, rcw; // WCA bead-surface
    double rl2, half_skin2;           // Verlet list radius^2 (rc + skin)^2 and (skin/2)^2
    int node_scan_all;                // 1: find the beads sharing a node by scanning every bead
                                      // (the WCA cutoff is shorter than a node cell's diagonal
                                      // sqrt(3), so such beads need not be list neighbours)
    double f_drive;                   // signed along x
    int rigid;                        // rigid bonds (SHAKE/RATTLE) instead of harmonic ones
    int shake_iter;
    double kappa_phi;                 // angular term between consecutive bonds
    int stencil;                      // LB_STENCIL_*
    double b2, shake_tol_b2;          // rigid bond length^2 and the SHAKE tolerance on |s^2 - b^2|
};

enum MDMode : int { MD_INTERP = 1, MD_SUBSTEPS = 2, MD_COUPLED = 3, MD_NO_HYDRO = 4 };
enum StepMode : int { STEP_LB = 0, STEP_COUPLED = 1, STEP_NO_HYDRO = 2 };

// Lattice-kernel launch description for one block size.
struct LatticeLaunch {
    int block = 0;
    int mapping = 0;          // 0: 64 consecutive nodes per wave; 1: one row segment per wave;
                              // 2: as 0 with x-rows rotated; 3: two nodes per lane, 64 apart
    int total_tiles = 0;
    int* d_prefix = nullptr;  // [n_reps + 1] first block of each replica (one row segment per wave)
};

struct Context {
    lbmd_config cfg{};                 // copy; pointer members not kept
    int storage = LB_STORE_F32;
    std::vector<Replica> reps;         // host copies
    std::vector<int> chain_len_all;
    lbmd_md_params md_params{};
    MDDev md{};
    long long total_nodes = 0;         // sum of V over replicas
    long long pop_elems = 0;           // 19 S summed over replicas (one population buffer)
    int ntot_beads = 0;
    int max_beads = 0;
    int max_V = 0;

    hipStream_t stream = nullptr;      // caller's stream
    hipStream_t side = nullptr;        // MD branch of the coupled step
    hipStream_t cap = nullptr;         // private stream used only to capture graphs
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    void* pops[2] = {nullptr, nullptr};
    void* beads = nullptr;
    void* work = nullptr;
    bool owns_buffers = false;
    double* h_small = nullptr;         // pinned host staging for small read-outs (32 doubles)
    int cur = 0;                       // which pops buffer holds the current state
    long long host_step = 0;           // mirror of the device step counter

    // carved from `work`
    Replica* d_reps = nullptr;
    RunState* d_state = nullptr;
    double* d_partials = nullptr;      // reduction partials
    double* d_stage = nullptr;         // lb_moments staging
    size_t stage_doubles = 0;
    int partial_blocks = 0;
    void* bead_ptrs = nullptr;         // BeadPtrs<float> or BeadPtrs<double> (by storage)

    LatticeLaunch lat;                 // current lattice launch shape
    int lat_chunk = -1;                // lattice tile order over XCDs (-1 contiguous, 0 none, C chunks)
    bool lat_nt = true;                // non-temporal population stores
    bool thermal = false;              // some replica has a thermal source (fluid_kT > 0)
    int obs_every = 0, obs_capacity = 0;  // observable record (0: none)
    std::vector<LatticeLaunch> lat_all;
    int md_lanes = 0;                  // lanes per bead of the bead kernel (0: by bead count)

    bool use_graph = true;
    bool deterministic = false;        // LB_CFG_DETERMINISTIC
    // instantiated graphs of 1..kGraphSteps steps, by (coupled, parity of cur, length)
    static constexpr int kGraphSteps = 16;
    hipGraphExec_t graphs[3][2][kGraphSteps + 1] = {};  // [StepMode][parity][length]
};

// work-buffer layout (byte offsets), computed on the host
struct WorkLayout {
    size_t reps, state, partials, stage, prefix, total;
    size_t stage_doubles;
    int partial_blocks;
    int n_prefix_tables;
};
WorkLayout work_layout(int n_reps, int max_V, long long max_stage_nodes);

// bead-buffer layout
struct BeadLayout {
    size_t r, v, u, fbar, node, bond_next, agg_at, agg_f, rep_of, diag, nlist, ncount, rref, rs, obs;
    size_t hkey, hrep, hsum, total;
    unsigned hcap;
};
// obs_rows: rows of the observable record per replica (capacity + 1 header row; 0 = none);
// trilinear: room for the node table of the deterministic trilinear spread
BeadLayout bead_layout(int ntot, int n_reps, size_t real_size, int obs_rows, bool trilinear);

// kernel launchers (lb_kernels.hip / md_kernels.hip); all enqueue on `s`
hipError_t launch_stream_collide(const Context& c, const void* src, void* dst, bool bump_step,
                                 hipStream_t s);
// the same-pattern reference of the lattice kernel (current launch shape): src -> dst
hipError_t launch_pattern(const Context& c, const void* src, void* dst, hipStream_t s);
hipError_t launch_init(const Context& c, int r, void* dst, const double* d_rho, const double* d_u,
                       const double* d_pops, hipStream_t s);
hipError_t launch_gather(const Context& c, int r, const void* src, int mode, long long node0,
                         int count, double* out, hipStream_t s);
hipError_t launch_conserved(const Context& c, int r, const void* src, double* d_out4, hipStream_t s);
// the same reduction for a replica description passed by value (its pop_base applies to src),
// with nblk partial-sum blocks written to partials ([nblk][4] doubles)
hipError_t launch_conserved_desc(const Replica& R, int storage, const void* src, double* partials, int nblk,
                                 double* out4, hipStream_t s);
// the kernel-side description of one replica (pop_base, bead0 and x_shift are left 0)
Replica make_replica(const lbmd_replica& in, size_t elem);
// host-side checks of one replica's box, faces, walls, tau, rho0 and fluid_kT; "" if valid
std::string replica_problem(const lbmd_replica& R);
hipError_t launch_md(const Context& c, const void* cur, int mode, hipStream_t s);
hipError_t launch_spread(const Context& c, void* dst, bool bump_step, hipStream_t s);
hipError_t launch_bump(const Context& c, hipStream_t s);
// step 1 with the trilinear stencil (a kernel of its own; the bead kernel then runs its
// substeps on the interpolated velocities)
hipError_t launch_interp_trilinear(const Context& c, const void* cur, hipStream_t s);
// appends a row to every replica's observable record after a bead step, when the new step
// count is a multiple of obs_every (no_hydro: the beads saw a fluid at rest, u = 0)
hipError_t launch_observe(const Context& c, bool no_hydro, hipStream_t s);
int md_default_lanes(int max_beads);
bool md_lanes_valid(int lanes, int max_beads);
// most beads one replica may hold: the bead kernel's per-replica LDS arrays must fit one
// compute unit (positions, node and bond arrays; with rigid bonds also the constraint work area)
int md_max_beads(bool rigid);

}  // namespace lbmd
