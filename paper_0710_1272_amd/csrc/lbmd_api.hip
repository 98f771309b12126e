// lbmd_api.hip -- the C ABI of lbmd.h: validation, buffers, step sequencing, observables.
//
// One coupled LB step (arXiv:0710.1272 Sec. II, steps 1-4) is enqueued as
//   fork:  side stream  -> k_md (interpolate u_i, M substeps, Fbar, N_T/COM, node sums)
//          main stream  -> k_stream_collide (current -> other buffer)
//   join:  main stream  -> k_spread (S_p into the other buffer), step counter += 1
// The lattice update does not need the beads (S_p is added after collision), so
// the latency-bound MD of one workgroup per replica runs under the bandwidth-bound
// lattice sweep.  The steps are captured once per buffer parity into HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbmd_internal.hpp"

using namespace lbmd;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE,                  \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t store_size(int storage) {
    switch (storage) {
        case LB_STORE_F64: return 8;
        case LB_STORE_F32: return 4;
        case LB_STORE_F16DEV:
        case LB_STORE_BF16DEV: return 2;
        default: return 0;
    }
}

// Population plane stride (elements) of a replica of V nodes.  Plane starts a multiple of
// a large power of two apart (a 512^3 box: 2^29 bytes in FP32) put the same offset of all
// 19 planes on the same HBM channels, so that the 19 read and 19 write streams of a sweep
// queue on a few channels at a time.  The stride is an odd multiple of 256 bytes (every
// plane starts on a 256-byte boundary, so whole-wave stores stay whole lines) at least
// 47 x 256 bytes beyond the plane: on MI355X a 19-read + 19-write pull copy then ran
// 7-14 % faster than with unpadded planes (512^3 and 256x128x128 boxes, 4- and 2-byte
// elements).
long long plane_stride(long long V, size_t elem) {
    const long long units = ((V * (long long)elem + 255) / 256 + 47) | 1;  // 256-byte units
    return units * 256 / (long long)elem;
}

size_t real_size(int storage) { return storage == LB_STORE_F64 ? 8 : 4; }

const int kBlockSizes[] = {64, 128, 256, 512, 1024};
const int kNumBlockSizes = 5;
const long long kStageNodes = 1 << 20;

struct Totals {
    long long nodes = 0;
    long long pop_elems = 0;  // 19 S summed over replicas (one population buffer)
    int beads = 0, max_beads = 0, max_V = 0;
};

Totals totals(const lbmd_config* cfg) {
    Totals t;
    for (int r = 0; r < cfg->n_replicas; ++r) {
        const lbmd_replica& R = cfg->replicas[r];
        const long long V = (long long)R.nx * R.ny * R.nz;
        t.nodes += V;
        t.pop_elems += 19 * plane_stride(V, store_size(cfg->storage));
        t.max_V = std::max<long long>(t.max_V, V);
        int nb = 0;
        for (int c = 0; c < R.n_chains; ++c) nb += R.chain_len[c];
        t.beads += nb;
        t.max_beads = std::max(t.max_beads, nb);
    }
    return t;
}

}  // namespace

namespace lbmd {

std::string replica_problem(const lbmd_replica& R) {
    if (R.nx < 2 || R.ny < 2 || R.nz < 2) return "box sides must be >= 2";
    if ((long long)R.nx * R.ny * R.nz > (1LL << 30)) return "box above 2^30 nodes";
    for (int a = 0; a < 3; ++a)
        if (R.bc[a] != LB_BC_PERIODIC && R.bc[a] != LB_BC_FREESLIP) return "unknown boundary type";
    if (!(R.tau > 0.5) || !std::isfinite(R.tau)) return "tau must be > 1/2";
    if (!(R.rho0 > 0.0) || !std::isfinite(R.rho0)) return "rho0 must be > 0";
    if (!(R.fluid_kT >= 0.0) || !std::isfinite(R.fluid_kT)) return "fluid_kT must be >= 0";
    if (R.n_walls < 0 || R.n_walls > LB_MAX_WALLS) return "n_walls out of range";
    for (int k = 0; k < R.n_walls; ++k) {
        const lbmd_wall& w = R.wall[k];
        if (w.x0 > w.x1 || w.x0 < 2 || w.x1 > R.nx - 3) return "wall planes must satisfy 2 <= x0 <= x1 <= nx-3";
        if (w.y0 <= w.y1 || w.z0 <= w.z1) {
            if (w.y0 > w.y1 || w.z0 > w.z1 || w.y0 < 0 || w.y1 >= R.ny || w.z0 < 0 || w.z1 >= R.nz)
                return "pore outside the cross-section";
        }
        if (k > 0 && w.x0 <= R.wall[k - 1].x1 + 2) return "walls must be ordered along x and at least 2 planes apart";
    }
    return "";
}

Replica make_replica(const lbmd_replica& in, size_t elem) {
    Replica R{};
    R.nx = in.nx;
    R.ny = in.ny;
    R.nz = in.nz;
    R.V = in.nx * in.ny * in.nz;
    R.S = (int)plane_stride(R.V, elem);
    for (int a = 0; a < 3; ++a) R.fs[a] = in.bc[a] == LB_BC_FREESLIP ? 1 : 0;
    R.n_walls = in.n_walls;
    R.wzone_lo = 1 << 30;
    R.wzone_hi = -1;
    for (int k = 0; k < in.n_walls; ++k) {
        const lbmd_wall& w = in.wall[k];
        const int v6[6] = {w.x0, w.x1, w.y0, w.y1, w.z0, w.z1};
        for (int m = 0; m < 6; ++m) R.wall[k][m] = v6[m];
        R.wzone_lo = std::min(R.wzone_lo, w.x0 - 1);
        R.wzone_hi = std::max(R.wzone_hi, w.x1 + 1);
    }
    R.seed_lo = (uint32_t)(in.seed & 0xFFFFFFFFu);
    R.seed_hi = (uint32_t)(in.seed >> 32);
    R.omega = 1.0 / in.tau;
    R.rho0 = in.rho0;
    // thermal source amplitude: phi^2 / rho = (kT / c_s^2) (1 - gamma^2), gamma = 1 - omega
    const double g = 1.0 - R.omega;
    R.noise_c = 3.0 * in.fluid_kT * (1.0 - g * g);
    R.xmid = in.n_walls > 0 ? 0.5 * (in.wall[0].x0 + in.wall[0].x1) : 0.5 * (in.nx - 1);
    R.div_nx = make_fastdiv((uint32_t)in.nx);
    R.div_ny = make_fastdiv((uint32_t)in.ny);
    return R;
}

WorkLayout work_layout(int n_reps, int max_V, long long max_stage_nodes) {
    WorkLayout L{};
    size_t off = 0;
    L.reps = off;
    off += align256(sizeof(Replica) * (size_t)n_reps);
    L.state = off;
    off += align256(sizeof(RunState));
    L.partial_blocks = 32768;  // capacity: one block of partial sums per 4096 nodes up to 2^27 nodes
    L.partials = off;
    off += align256(sizeof(double) * (4 * (size_t)L.partial_blocks + 4));
    const long long stage_nodes = std::min<long long>(max_V, max_stage_nodes);
    L.stage_doubles = (size_t)(19 * stage_nodes);
    L.stage = off;
    off += align256(sizeof(double) * L.stage_doubles);
    L.n_prefix_tables = 3 * kNumBlockSizes;
    L.prefix = off;
    off += align256(sizeof(int) * (size_t)(n_reps + 1) * kNumBlockSizes * 3);
    L.total = off;
    return L;
}

BeadLayout bead_layout(int ntot, int n_reps, size_t rs, int obs_rows, bool trilinear) {
    BeadLayout L{};
    size_t off = 0;
    const size_t N = (size_t)std::max(ntot, 1);
    L.r = off;        off += align256(3 * N * sizeof(double));
    L.v = off;        off += align256(3 * N * rs);
    L.u = off;        off += align256(3 * N * rs);
    L.fbar = off;     off += align256(3 * N * rs);
    L.node = off;     off += align256(N * sizeof(int));
    L.bond_next = off; off += align256(N);
    L.agg_at = off;   off += align256(2 * N * sizeof(long long));
    L.agg_f = off;    off += align256(3 * N * rs);
    L.rep_of = off;   off += align256(N * sizeof(int));
    L.diag = off;     off += align256(8 * (size_t)std::max(n_reps, 1) * sizeof(double));
    L.nlist = off;    off += align256((size_t)kNeighbourMax * N * sizeof(unsigned short));
    L.ncount = off;   off += align256(N * sizeof(int));
    L.rref = off;     off += align256(3 * N * sizeof(double));
    L.rs = off;       off += align256(3 * N * sizeof(double));
    L.obs = off;      off += align256((size_t)std::max(n_reps, 1) * (size_t)obs_rows * 8 * sizeof(double));
    // a bead's stencil touches at most 8 nodes: a table of at least 16 slots a bead stays at
    // most half full
    L.hcap = 0;
    if (trilinear) {
        L.hcap = 64;
        while (L.hcap < 16 * N) L.hcap <<= 1;
    }
    L.hkey = off;     off += align256((size_t)L.hcap * sizeof(unsigned long long));
    L.hrep = off;     off += align256((size_t)L.hcap * sizeof(int));
    L.hsum = off;     off += align256((size_t)18 * L.hcap * sizeof(long long));
    L.total = off;
    return L;
}

}  // namespace lbmd

struct lbmd_ctx {
    Context c;
};

extern "C" {

const char* lb_strerror(int code) {
    switch (code) {
        case LB_OK: return "success";
        case LB_EINVAL: return "invalid argument or configuration";
        case LB_ENOMEM: return "out of memory";
        case LB_EDEVICE: return "HIP device or runtime error";
        case LB_EUNSTABLE: return "device error word set (unstable or invalid state)";
        case LB_ESTATE: return "call not valid in the current state";
        case LB_ESIZE: return "output buffer too small";
        default: return "unknown error code";
    }
}

const char* lb_last_error_message(void) { return g_last_error.c_str(); }

int lb_validate_config(const lbmd_config* cfg) {
    if (!cfg) return fail(LB_EINVAL, "cfg is NULL");
    if (cfg->n_replicas < 1 || !cfg->replicas) return fail(LB_EINVAL, "need n_replicas >= 1 and replicas");
    if (!store_size(cfg->storage)) return fail(LB_EINVAL, "unknown storage");
    if (cfg->block_size != 0) {
        bool ok = false;
        for (int b : kBlockSizes) ok = ok || b == cfg->block_size;
        if (!ok) return fail(LB_EINVAL, "block_size must be 0, 64, 128, 256, 512 or 1024");
    }
    if (cfg->lattice_mapping < LB_MAP_AUTO || cfg->lattice_mapping > LB_MAP_FLAT2)
        return fail(LB_EINVAL, "unknown lattice_mapping");
    if (cfg->lattice_mapping == LB_MAP_FLAT2 && (cfg->block_size == 64 || cfg->block_size == 1024))
        return fail(LB_EINVAL, "LB_MAP_FLAT2 runs blocks of 128, 256 or 512 threads");
    if (cfg->xcd_order < LB_XCD_CONTIGUOUS) return fail(LB_EINVAL, "unknown xcd_order");
    int total_beads = 0, max_beads = 0;
    for (int r = 0; r < cfg->n_replicas; ++r) {
        const lbmd_replica& R = cfg->replicas[r];
        const std::string at = "replica " + std::to_string(r) + ": ";
        const std::string why = replica_problem(R);
        if (!why.empty()) return fail(LB_EINVAL, at + why);
        // the lattice kernel addresses one population of a replica with 32-bit byte offsets
        const long long nodes = (long long)R.nx * R.ny * R.nz;
        if (nodes * (long long)store_size(cfg->storage) > (1LL << 32) ||
            plane_stride(nodes, store_size(cfg->storage)) > 0x7FFFFFFFLL)
            return fail(LB_EINVAL, at + "one population of the box exceeds 4 GiB (FP64 storage: at most 2^29 nodes)");
        if (R.n_chains < 0 || (R.n_chains > 0 && !R.chain_len))
            return fail(LB_EINVAL, at + "chain_len missing");
        int nb = 0;
        for (int c = 0; c < R.n_chains; ++c) {
            if (R.chain_len[c] < 1) return fail(LB_EINVAL, at + "chain lengths must be >= 1");
            nb += R.chain_len[c];
            if (nb > 4096) return fail(LB_EINVAL, at + "more than 4096 beads in one replica");
        }
        total_beads += nb;
        max_beads = std::max(max_beads, nb);
    }
    // the bead kernel keeps a replica's positions (two buffers), node and bond arrays, and
    // for rigid chains the constraint work area, in one compute unit's LDS
    if (max_beads > md_max_beads(cfg->md.rigid != 0))
        return fail(LB_EINVAL, "more than " + std::to_string(md_max_beads(cfg->md.rigid != 0)) +
                                   " beads in one replica (the bead kernel's LDS limit)");
    if (cfg->obs_every < 0 || (cfg->obs_every > 0 && (cfg->obs_capacity < 1 || cfg->obs_capacity > (1 << 24))))
        return fail(LB_EINVAL, "obs_every must be >= 0, and obs_capacity in 1..2^24 when recording");
    if (cfg->md_lanes != 0 && !md_lanes_valid(cfg->md_lanes, max_beads))
        return fail(LB_EINVAL, "md_lanes must be 0, 1, or 2/4/8/16 with md_lanes x beads per replica <= 512");
    const lbmd_md_params& m = cfg->md;
    if (total_beads > 0) {
        if (m.M < 1) return fail(LB_EINVAL, "md.M must be >= 1");
        if (!(m.mass > 0) || !(m.gamma >= 0) || !(m.kT >= 0) || !(m.k_bond >= 0) || !(m.r0 > 0) ||
            !(m.eps >= 0) || !(m.sigma > 0) || !(m.eps_w >= 0) || !(m.sigma_w > 0) ||
            !std::isfinite(m.f_drive))
            return fail(LB_EINVAL, "md parameters out of range");
        if (m.drive_sign != 1 && m.drive_sign != -1) return fail(LB_EINVAL, "md.drive_sign must be +-1");
        if (m.stencil != LB_STENCIL_NGP && m.stencil != LB_STENCIL_TRILINEAR)
            return fail(LB_EINVAL, "md.stencil must be LB_STENCIL_NGP or LB_STENCIL_TRILINEAR");
        if (m.rigid != 0 && m.rigid != 1) return fail(LB_EINVAL, "md.rigid must be 0 or 1");
        if (!(m.kappa_phi >= 0) || !std::isfinite(m.kappa_phi)) return fail(LB_EINVAL, "md.kappa_phi must be >= 0");
        if (m.rigid) {
            if (!(m.shake_tol > 0) || m.shake_iter < 1)
                return fail(LB_EINVAL, "rigid bonds need shake_tol > 0 and shake_iter >= 1");
            if (max_beads > 512) return fail(LB_EINVAL, "rigid bonds: at most 512 beads per replica");
        } else if (2.0 * std::sqrt(m.k_bond / m.mass) / m.M >= 2.0) {
            // kick-drift is stable for omega h < 2; the stiffest chain mode has omega = 2 sqrt(k/m)
            return fail(LB_EINVAL, "bond stiffness unstable at this M: need 2 sqrt(k/m)/M < 2");
        }
        if (!cfg->init || !cfg->init->bead_r) return fail(LB_EINVAL, "beads need init->bead_r");
    }
    return LB_OK;
}

static int obs_rows(const lbmd_config* cfg) { return cfg->obs_every > 0 ? cfg->obs_capacity + 1 : 0; }

size_t lb_required_bytes(const lbmd_config* cfg, int which) {
    if (lb_validate_config(cfg) != LB_OK) return 0;
    const Totals t = totals(cfg);
    switch (which) {
        case LB_BUF_POPS: return align256((size_t)t.pop_elems * store_size(cfg->storage));
        case LB_BUF_BEADS:
            return bead_layout(t.beads, cfg->n_replicas, real_size(cfg->storage), obs_rows(cfg),
                               t.beads > 0 && cfg->md.stencil == LB_STENCIL_TRILINEAR)
                .total;
        case LB_BUF_WORK: return work_layout(cfg->n_replicas, t.max_V, kStageNodes).total;
        default: g_last_error = "unknown buffer id"; return 0;
    }
}

}  // extern "C"

namespace {

// Row rotation of the shifted flat mapping: among shifts that keep every wave's accesses
// aligned to 128-byte lines, the one that leaves the fewest 64-node waves of a row within
// one node of a wall, the most aligned one (0 first) on ties.  Rows must be whole waves
// (nx a multiple of 64).  A shift of 64-byte granularity measured 28 % slower for 16-bit
// storage in a streamed box (the non-temporal stores then split lines).
int wall_x_shift(const Replica& R, size_t elem_bytes) {
    const int g = (int)(128 / elem_bytes);
    if (R.n_walls == 0 || R.nx % 64 != 0) return 0;
    auto zone_waves = [&](int s) {
        int cnt = 0;
        for (int w0 = 0; w0 < R.nx; w0 += 64) {
            bool hit = false;
            for (int j = 0; j < 64 && !hit; ++j) {
                const int x = (w0 + j + s) % R.nx;
                for (int k = 0; k < R.n_walls; ++k)
                    hit = hit || (x >= R.wall[k][0] - 1 && x <= R.wall[k][1] + 1);
            }
            cnt += hit;
        }
        return cnt;
    };
    auto align = [](int s) { return s == 0 ? 1 << 30 : (s & -s); };
    int best = 0, best_cnt = zone_waves(0);
    for (int s = g; s < R.nx; s += g) {
        const int cnt = zone_waves(s);
        if (cnt < best_cnt || (cnt == best_cnt && align(s) > align(best))) {
            best = s;
            best_cnt = cnt;
        }
    }
    return best;
}

int set_lattice_shape(Context& c, int block, int mapping = -1) {
    if (mapping < 0) mapping = c.lat.mapping;
    for (auto& L : c.lat_all)
        if (L.block == block && L.mapping == mapping) {
            c.lat = L;
            return LB_OK;
        }
    return fail(LB_EINVAL, "no launch table for block size");
}

template <class Real>
int setup_beads(Context& c, const lbmd_config* cfg) {
    const BeadLayout L = bead_layout(c.ntot_beads, (int)c.reps.size(), sizeof(Real),
                                     c.obs_every > 0 ? c.obs_capacity + 1 : 0,
                                     c.ntot_beads > 0 && c.md.stencil == LB_STENCIL_TRILINEAR);
    char* base = (char*)c.beads;
    BeadPtrs<Real>* p = new (std::nothrow) BeadPtrs<Real>;
    if (!p) return fail(LB_ENOMEM, "host allocation");
    p->r = (double*)(base + L.r);
    p->v = (Real*)(base + L.v);
    p->u = (Real*)(base + L.u);
    p->fbar = (Real*)(base + L.fbar);
    p->node = (int*)(base + L.node);
    p->bond_next = (unsigned char*)(base + L.bond_next);
    p->agg_at = (long long*)(base + L.agg_at);
    p->agg_f = (Real*)(base + L.agg_f);
    p->rep_of = (int*)(base + L.rep_of);
    p->diag = (double*)(base + L.diag);
    p->nlist = (unsigned short*)(base + L.nlist);
    p->ncount = (int*)(base + L.ncount);
    p->rref = (double*)(base + L.rref);
    p->rs = (double*)(base + L.rs);
    p->obs = (double*)(base + L.obs);
    p->hkey = (unsigned long long*)(base + L.hkey);
    p->hrep = (int*)(base + L.hrep);
    p->hsum = (long long*)(base + L.hsum);
    p->hcap = L.hcap;
    p->obs_every = c.obs_every;
    p->obs_cap = c.obs_capacity;
    p->ntot = c.ntot_beads;
    c.bead_ptrs = p;

    const int N = c.ntot_beads;
    const size_t nz = (size_t)std::max(N, 1);
    std::vector<double> r(3 * nz, 0.0);
    std::vector<Real> v(3 * nz, Real(0));
    std::vector<unsigned char> bn(nz, 0);
    std::vector<int> rep_of(nz, 0), minus1(nz, -1);
    std::vector<double> diag(8 * std::max<size_t>(c.reps.size(), 1), 0.0);
    const lbmd_initial_state* in = cfg->init;
    int g = 0;
    for (size_t ri = 0; ri < c.reps.size(); ++ri) {
        const lbmd_replica& R = cfg->replicas[ri];
        for (int ch = 0; ch < R.n_chains; ++ch) {
            for (int k = 0; k < R.chain_len[ch]; ++k, ++g) {
                for (int a = 0; a < 3; ++a) {
                    r[a * nz + g] = in->bead_r[3 * g + a];
                    v[a * nz + g] = in->bead_v ? (Real)in->bead_v[3 * g + a] : Real(0);
                }
                bn[g] = k + 1 < R.chain_len[ch] ? 1 : 0;
                rep_of[g] = (int)ri;
            }
        }
        diag[8 * ri + 1] = -1.0;  // no completion yet
    }
    // SoA blocks are sized by ntot; when N == 0 nothing is copied
    if (N > 0) {
        for (int a = 0; a < 3; ++a) {
            HIP_TRY(hipMemcpy(p->r + (size_t)a * N, r.data() + a * nz, N * sizeof(double), hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(p->v + (size_t)a * N, v.data() + a * nz, N * sizeof(Real), hipMemcpyHostToDevice));
        }
        HIP_TRY(hipMemset(p->u, 0, 3 * (size_t)N * sizeof(Real)));
        HIP_TRY(hipMemset(p->fbar, 0, 3 * (size_t)N * sizeof(Real)));
        HIP_TRY(hipMemset(p->agg_f, 0, 3 * (size_t)N * sizeof(Real)));
        HIP_TRY(hipMemcpy(p->node, minus1.data(), N * sizeof(int), hipMemcpyHostToDevice));
        std::vector<long long> none(2 * (size_t)N, -1);
        HIP_TRY(hipMemcpy(p->agg_at, none.data(), 2 * (size_t)N * sizeof(long long), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->bond_next, bn.data(), N, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->rep_of, rep_of.data(), N * sizeof(int), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(p->diag, diag.data(), 8 * c.reps.size() * sizeof(double), hipMemcpyHostToDevice));
    if (L.hcap > 0) {
        // the table starts empty; the spread leaves it empty after every step
        HIP_TRY(hipMemset(p->hkey, 0, (size_t)L.hcap * sizeof(unsigned long long)));
        HIP_TRY(hipMemset(p->hsum, 0, (size_t)18 * L.hcap * sizeof(long long)));
    }
    if (c.obs_every > 0) {
        // header rows (rows recorded, every, capacity); the rows themselves start unset (step -1)
        const size_t rows = (size_t)c.obs_capacity + 1;
        std::vector<double> rec(c.reps.size() * rows * 8, 0.0);
        for (size_t r = 0; r < c.reps.size(); ++r) {
            double* h = rec.data() + r * rows * 8;
            h[1] = c.obs_every;
            h[2] = c.obs_capacity;
            for (size_t k = 1; k < rows; ++k) h[k * 8] = -1.0;
        }
        HIP_TRY(hipMemcpy(p->obs, rec.data(), rec.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    return LB_OK;
}

int init_populations(Context& c, const lbmd_config* cfg) {
    const lbmd_initial_state* in = cfg->init;
    long long node_off = 0;
    double* d_tmp = nullptr;
    size_t tmp_bytes = 0;
    for (size_t r = 0; r < c.reps.size(); ++r) {
        const long long V = c.reps[r].V;
        const double *d_rho = nullptr, *d_u = nullptr, *d_pops = nullptr;
        size_t need = 0;
        if (in && in->pops) need = 19 * V;
        else if (in && (in->rho || in->u)) need = 4 * V;
        if (need * sizeof(double) > tmp_bytes) {
            if (d_tmp) (void)hipFree(d_tmp);
            d_tmp = nullptr;
            tmp_bytes = need * sizeof(double);
            hipError_t e = hipMalloc(&d_tmp, tmp_bytes);
            if (e != hipSuccess) return fail(LB_ENOMEM, "staging for initial state");
        }
        if (in && in->pops) {
            HIP_TRY(hipMemcpy(d_tmp, in->pops + 19 * node_off, 19 * V * sizeof(double), hipMemcpyHostToDevice));
            d_pops = d_tmp;
        } else if (in && (in->rho || in->u)) {
            if (in->rho) {
                HIP_TRY(hipMemcpy(d_tmp, in->rho + node_off, V * sizeof(double), hipMemcpyHostToDevice));
                d_rho = d_tmp;
            }
            if (in->u) {
                HIP_TRY(hipMemcpy(d_tmp + V, in->u + 3 * node_off, 3 * V * sizeof(double), hipMemcpyHostToDevice));
                d_u = d_tmp + V;
            }
        }
        HIP_TRY(launch_init(c, (int)r, c.pops[c.cur], d_rho, d_u, d_pops, c.stream));
        HIP_TRY(hipStreamSynchronize(c.stream));
        node_off += V;
    }
    if (d_tmp) HIP_TRY(hipFree(d_tmp));
    return LB_OK;
}

int autotune(Context& c) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct EventGuard {
        hipEvent_t* a;
        hipEvent_t* b;
        ~EventGuard() {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } guard{&e0, &e1};
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    struct Shape {
        int map, block, chunk;
        float ms;
    };
    std::vector<Shape> shapes;
    bool shifted = false;
    for (const Replica& R : c.reps) shifted = shifted || R.x_shift != 0;
    for (int map : {0, 1, 2, 3})
        for (int b : {128, 256, 512}) {
            if (map == 2 && !shifted) continue;  // the same launches as the flat mapping
            for (int chunk : {-1, 0, 16, 64}) shapes.push_back({map, b, chunk, 1e30f});
        }
    // `reps` back-to-back launches of one shape, best of `rounds`, in ms per launch
    auto time_shape = [&](Shape& sh, int reps, int rounds) -> int {
        int rc = set_lattice_shape(c, sh.block, sh.map);
        if (rc != LB_OK) return rc;
        c.lat_chunk = sh.chunk;
        HIP_TRY(launch_stream_collide(c, c.pops[c.cur], c.pops[1 - c.cur], false, c.stream));
        float ms = 1e30f;
        for (int round = 0; round < rounds; ++round) {
            HIP_TRY(hipEventRecord(e0, c.stream));
            for (int k = 0; k < reps; ++k)
                HIP_TRY(launch_stream_collide(c, c.pops[c.cur], c.pops[1 - c.cur], false, c.stream));
            HIP_TRY(hipEventRecord(e1, c.stream));
            HIP_TRY(hipEventSynchronize(e1));
            float t = 0;
            HIP_TRY(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t / reps);
        }
        sh.ms = ms;
        return LB_OK;
    };
    // a short pass over every shape (about 1 ms of launches each, at least 2), then the four
    // fastest timed again as best of three rounds of 10 launches (short kernels are noisy):
    // a large box spends a few launches per shape instead of 31
    int rc = time_shape(shapes[0], 2, 1);
    if (rc != LB_OK) return rc;
    const int reps1 = std::max(2, std::min(10, (int)(1.0f / std::max(shapes[0].ms, 1e-3f))));
    for (Shape& sh : shapes)
        if ((rc = time_shape(sh, reps1, 1)) != LB_OK) return rc;
    std::stable_sort(shapes.begin(), shapes.end(), [](const Shape& a, const Shape& b) { return a.ms < b.ms; });
    const size_t finalists = std::min<size_t>(4, shapes.size());
    for (size_t k = 0; k < finalists; ++k)
        if ((rc = time_shape(shapes[k], 10, 3)) != LB_OK) return rc;
    size_t best = 0;
    for (size_t k = 1; k < finalists; ++k)
        if (shapes[k].ms < shapes[best].ms) best = k;
    c.lat_chunk = shapes[best].chunk;
    return set_lattice_shape(c, shapes[best].block, shapes[best].map);
}

// Lanes per bead of the bead kernel: times coupled-mode launches (interpolation and M
// substeps) for every valid choice, each from the same saved bead state and each beside a
// lattice sweep into the spare population buffer, as in a coupled step (the sweep shares the
// bead kernel's compute unit, which changes the best choice); then puts the bead buffer and
// the run state back as they were.
int autotune_md(Context& c) {
    if (c.ntot_beads == 0 || c.md_lanes != 0) return LB_OK;
    std::vector<int> cand;
    for (int G : {1, 2, 4, 8, 16})
        if (md_lanes_valid(G, c.max_beads)) cand.push_back(G);
    if (cand.size() < 2) return LB_OK;
    const size_t real = c.storage == LB_STORE_F64 ? sizeof(double) : sizeof(float);
    const size_t bytes = bead_layout(c.ntot_beads, (int)c.reps.size(), real, c.obs_every > 0 ? c.obs_capacity + 1 : 0,
                                     c.md.stencil == LB_STENCIL_TRILINEAR)
                             .total;
    void* save = nullptr;
    HIP_TRY(hipMalloc(&save, bytes + sizeof(RunState)));
    RunState* save_st = (RunState*)((char*)save + bytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = LB_OK;
    float best = 1e30f;
    int best_G = md_default_lanes(c.max_beads);
    auto body = [&]() -> hipError_t {
        hipError_t e;
        if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
        if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(save, c.beads, bytes, hipMemcpyDeviceToDevice, c.stream)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(save_st, c.d_state, sizeof(RunState), hipMemcpyDeviceToDevice, c.stream)) !=
            hipSuccess)
            return e;
        for (int G : cand) {
            c.md_lanes = G;
            if ((e = hipMemcpyAsync(c.beads, save, bytes, hipMemcpyDeviceToDevice, c.stream)) != hipSuccess) return e;
            if ((e = launch_md(c, c.pops[c.cur], MD_COUPLED, c.stream)) != hipSuccess) return e;
            float ms = 1e30f;
            for (int round = 0; round < 3; ++round) {
                if ((e = hipEventRecord(e0, c.stream)) != hipSuccess) return e;
                for (int k = 0; k < 5; ++k) {
                    if ((e = hipEventRecord(c.ev_fork, c.stream)) != hipSuccess) return e;
                    if ((e = hipStreamWaitEvent(c.side, c.ev_fork, 0)) != hipSuccess) return e;
                    if ((e = launch_md(c, c.pops[c.cur], MD_COUPLED, c.side)) != hipSuccess) return e;
                    if ((e = hipEventRecord(c.ev_join, c.side)) != hipSuccess) return e;
                    if ((e = launch_stream_collide(c, c.pops[c.cur], c.pops[1 - c.cur], false, c.stream)) !=
                        hipSuccess)
                        return e;
                    if ((e = hipStreamWaitEvent(c.stream, c.ev_join, 0)) != hipSuccess) return e;
                }
                if ((e = hipEventRecord(e1, c.stream)) != hipSuccess) return e;
                if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
                float t = 0;
                if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return e;
                ms = std::min(ms, t);
            }
            if (ms < best) {
                best = ms;
                best_G = G;
            }
        }
        if ((e = hipMemcpyAsync(c.beads, save, bytes, hipMemcpyDeviceToDevice, c.stream)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(c.d_state, save_st, sizeof(RunState), hipMemcpyDeviceToDevice, c.stream)) !=
            hipSuccess)
            return e;
        return hipStreamSynchronize(c.stream);
    };
    const hipError_t e = body();
    if (e != hipSuccess)
        rc = fail(e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE,
                  std::string("bead-kernel autotune: ") + hipGetErrorString(e));
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(save);
    c.md_lanes = best_G;
    return rc;
}

void destroy_graphs(Context& c) {
    for (int k = 0; k < 3; ++k) {
        for (int par = 0; par < 2; ++par)
            for (int len = 0; len <= Context::kGraphSteps; ++len) {
                if (c.graphs[k][par][len]) (void)hipGraphExecDestroy(c.graphs[k][par][len]);
                c.graphs[k][par][len] = nullptr;
            }
    }
}

void release(Context& c) {
    destroy_graphs(c);
    if (c.side) (void)hipStreamDestroy(c.side);
    if (c.cap) (void)hipStreamDestroy(c.cap);
    if (c.ev_fork) (void)hipEventDestroy(c.ev_fork);
    if (c.ev_join) (void)hipEventDestroy(c.ev_join);
    if (c.h_small) (void)hipHostFree(c.h_small);
    c.h_small = nullptr;
    if (c.owns_buffers) {
        for (int k = 0; k < 2; ++k)
            if (c.pops[k]) (void)hipFree(c.pops[k]);
        if (c.beads) (void)hipFree(c.beads);
        if (c.work) (void)hipFree(c.work);
    }
    if (c.bead_ptrs) {
        if (c.storage == LB_STORE_F64) delete (BeadPtrs<double>*)c.bead_ptrs;
        else delete (BeadPtrs<float>*)c.bead_ptrs;
    }
    c.bead_ptrs = nullptr;
}

// enqueue one LB step on the context's streams (no graph)
hipError_t enqueue_step(Context& c, int mode, int cur, hipStream_t main) {
    void* src = c.pops[cur];
    void* dst = c.pops[1 - cur];
    if (mode == STEP_NO_HYDRO) {
        // beads alone; the counter moves in its own launch, after every replica has read it
        hipError_t e;
        if (c.ntot_beads > 0 && (e = launch_md(c, src, MD_SUBSTEPS | MD_NO_HYDRO, main)) != hipSuccess) return e;
        if (c.ntot_beads > 0 && c.obs_every > 0 && (e = launch_observe(c, true, main)) != hipSuccess) return e;
        return launch_bump(c, main);
    }
    const bool coupled = mode == STEP_COUPLED;
    if (coupled && c.ntot_beads > 0) {
        // the bead work goes first: its workgroup needs nearly all of one compute unit's LDS,
        // and a sweep enqueued ahead of it fills every unit, so that the bead kernel would
        // wait for the sweep's blocks to drain instead of running beside them
        hipError_t e;
        // the trilinear interpolation (8 x 19 population reads a bead, a launch of its own) goes
        // on the main stream ahead of the fork, where no sweep competes with its reads: on
        // 128x64x64 (FP32) it took 19 us beside the sweep and 11 us ahead of it, and the step
        // fell from 68 to 60 us
        const bool tri = c.md.stencil == LB_STENCIL_TRILINEAR;
        if (tri && (e = launch_interp_trilinear(c, src, main)) != hipSuccess) return e;
        if ((e = hipEventRecord(c.ev_fork, main)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(c.side, c.ev_fork, 0)) != hipSuccess) return e;
        if ((e = launch_md(c, src, tri ? MD_SUBSTEPS : MD_COUPLED, c.side)) != hipSuccess) return e;
        if (c.obs_every > 0 && (e = launch_observe(c, false, c.side)) != hipSuccess) return e;
        if ((e = hipEventRecord(c.ev_join, c.side)) != hipSuccess) return e;
        if ((e = launch_stream_collide(c, src, dst, false, main)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(main, c.ev_join, 0)) != hipSuccess) return e;
        return launch_spread(c, dst, true, main);
    }
    // the thermal source reads the step counter in every block: it moves in a launch of
    // its own after the sweep
    if (c.thermal) {
        hipError_t e = launch_stream_collide(c, src, dst, false, main);
        return e != hipSuccess ? e : launch_bump(c, main);
    }
    return launch_stream_collide(c, src, dst, true, main);
}

int build_graph(Context& c, int mode, int parity, int len, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    // the caller's stream may be the null stream, which cannot be captured: capture on
    // a private stream; the instantiated graph is then launched on the caller's stream
    HIP_TRY(hipStreamBeginCapture(c.cap, hipStreamCaptureModeThreadLocal));
    int cur = parity;
    hipError_t e = hipSuccess;
    for (int k = 0; k < len && e == hipSuccess; ++k) {
        e = enqueue_step(c, mode, cur, c.cap);
        if (mode != STEP_NO_HYDRO) cur = 1 - cur;
    }
    hipError_t e2 = hipStreamEndCapture(c.cap, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(LB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(LB_EDEVICE, std::string("end capture: ") + hipGetErrorString(e2));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    return LB_OK;
}

}  // namespace

extern "C" {

int lb_init(const lbmd_config* cfg, const lbmd_buffers* bufs, void* hip_stream, lbmd_ctx** out) {
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = lb_validate_config(cfg);
    if (rc != LB_OK) return rc;
    if (bufs && (!bufs->pops[0] || !bufs->pops[1] || !bufs->beads || !bufs->work))
        return fail(LB_EINVAL, "caller buffers: all four pointers are required");

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(LB_EDEVICE, std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");

    lbmd_ctx* ctx = new (std::nothrow) lbmd_ctx;
    if (!ctx) return fail(LB_ENOMEM, "host allocation");
    Context& c = ctx->c;
    c.cfg = *cfg;
    c.storage = cfg->storage;
    c.md_params = cfg->md;
    c.stream = (hipStream_t)hip_stream;
    c.use_graph = !(cfg->flags & LB_CFG_NO_GRAPH);
    c.deterministic = (cfg->flags & LB_CFG_DETERMINISTIC) != 0;

    const Totals t = totals(cfg);
    c.total_nodes = t.nodes;
    c.pop_elems = t.pop_elems;
    c.ntot_beads = t.beads;
    c.max_beads = t.max_beads;
    c.max_V = t.max_V;
    c.md_lanes = cfg->md_lanes;
    c.obs_every = cfg->obs_every;
    c.obs_capacity = cfg->obs_every > 0 ? cfg->obs_capacity : 0;

    // replica descriptors
    long long pop_base = 0;
    int bead0 = 0;
    for (int r = 0; r < cfg->n_replicas; ++r) {
        const lbmd_replica& in = cfg->replicas[r];
        Replica R = make_replica(in, store_size(cfg->storage));
        R.x_shift = wall_x_shift(R, store_size(cfg->storage));
        R.pop_base = pop_base;
        pop_base += 19LL * R.S;
        int nb = 0;
        for (int ch = 0; ch < in.n_chains; ++ch) nb += in.chain_len[ch];
        R.bead0 = bead0;
        R.n_beads = nb;
        bead0 += nb;
        if (in.fluid_kT > 0.0) c.thermal = true;
        c.reps.push_back(R);
    }

    // bead-model constants
    const lbmd_md_params& m = cfg->md;
    MDDev& md = c.md;
    md.M = std::max(m.M, 1);
    md.h = 1.0 / md.M;
    md.inv_M = 1.0 / md.M;
    md.mass = m.mass;
    md.inv_mass = m.mass > 0 ? 1.0 / m.mass : 0.0;
    md.gamma = m.gamma;
    md.A = std::sqrt(24.0 * m.mass * m.gamma * m.kT / md.h);
    md.k_bond = m.k_bond;
    md.r0 = m.r0;
    md.eps = m.eps;
    md.sigma2 = m.sigma * m.sigma;
    md.rc2 = std::pow(2.0, 1.0 / 3.0) * md.sigma2;
    md.eps_w = m.eps_w;
    md.sigma_w2 = m.sigma_w * m.sigma_w;
    md.rcw2 = std::pow(2.0, 1.0 / 3.0) * md.sigma_w2;
    md.rcw = std::sqrt(md.rcw2);
    // Verlet skin: the list holds pairs closer than rc + skin (plus 1e-3 for the rounding
    // of the FP32 displacement test) and is rebuilt as soon as any bead has moved skin/2
    // since the last build, so no interacting pair is missed.  Lists are kept across LB
    // steps; a wide skin makes rebuilds rare (pore beads drift ~0.2 per LB step) while
    // the register slots still hold the typical 3-4 neighbours.
    const double skin = 1.0;
    md.rl2 = (std::sqrt(md.rc2) + skin + 1e-3) * (std::sqrt(md.rc2) + skin + 1e-3);
    md.half_skin2 = 0.25 * skin * skin;
    // two beads on one node are at most sqrt(3) apart (the node's unit cell); a kept list
    // holds every non-bonded pair closer than rc, so it names them only when rc covers that
    md.node_scan_all = std::sqrt(md.rc2) < std::sqrt(3.0) + 1e-3 ? 1 : 0;
    md.f_drive = m.drive_sign * m.f_drive;
    md.rigid = m.rigid;
    md.shake_iter = m.shake_iter;
    md.kappa_phi = m.kappa_phi;
    md.stencil = m.stencil;
    md.b2 = m.r0 * m.r0;
    md.shake_tol_b2 = m.shake_tol * md.b2;

    // buffers
    const size_t pop_bytes = lb_required_bytes(cfg, LB_BUF_POPS);
    const size_t bead_bytes = lb_required_bytes(cfg, LB_BUF_BEADS);
    const size_t work_bytes = lb_required_bytes(cfg, LB_BUF_WORK);
    auto bail = [&](int code) {
        release(c);
        delete ctx;
        return code;
    };
    if (bufs) {
        c.pops[0] = bufs->pops[0];
        c.pops[1] = bufs->pops[1];
        c.beads = bufs->beads;
        c.work = bufs->work;
        c.owns_buffers = false;
    } else {
        c.owns_buffers = true;
        if (hipMalloc(&c.pops[0], pop_bytes) != hipSuccess || hipMalloc(&c.pops[1], pop_bytes) != hipSuccess ||
            hipMalloc(&c.beads, bead_bytes) != hipSuccess || hipMalloc(&c.work, work_bytes) != hipSuccess)
            return bail(fail(LB_ENOMEM, "device allocation of " + std::to_string(2 * pop_bytes + bead_bytes + work_bytes) + " bytes"));
    }
    for (void* p : {c.pops[0], c.pops[1], c.beads, c.work})
        if (((uintptr_t)p & 255) != 0) return bail(fail(LB_EINVAL, "buffers must be 256-byte aligned"));

    const WorkLayout W = work_layout((int)c.reps.size(), c.max_V, kStageNodes);
    char* wb = (char*)c.work;
    c.d_reps = (Replica*)(wb + W.reps);
    c.d_state = (RunState*)(wb + W.state);
    c.d_partials = (double*)(wb + W.partials);
    c.partial_blocks = W.partial_blocks;
    c.d_stage = (double*)(wb + W.stage);
    c.stage_doubles = W.stage_doubles;

    auto check = [&](hipError_t e, const char* what) -> int {
        if (e == hipSuccess) return LB_OK;
        return fail(e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    if ((rc = check(hipMemcpy(c.d_reps, c.reps.data(), sizeof(Replica) * c.reps.size(), hipMemcpyHostToDevice), "upload replicas")))
        return bail(rc);
    RunState st{};
    st.step = cfg->init ? cfg->init->step0 : 0;
    c.host_step = st.step;
    if ((rc = check(hipMemcpy(c.d_state, &st, sizeof st, hipMemcpyHostToDevice), "upload state"))) return bail(rc);

    // tile prefix tables for every lattice block size and both thread mappings
    int* prefix_base = (int*)(wb + W.prefix);
    for (int mi = 0; mi < 3; ++mi) {
        for (int bi = 0; bi < kNumBlockSizes; ++bi) {
            const int b = kBlockSizes[bi];
            std::vector<int> pre(c.reps.size() + 1, 0);
            for (size_t r = 0; r < c.reps.size(); ++r) {
                const Replica& R = c.reps[r];
                long long tiles;
                if (mi == 0) {
                    tiles = (R.V + b - 1) / b;
                } else if (mi == 1) {
                    // one wave per row segment of at most 64 nodes
                    const long long units = (long long)R.ny * R.nz * ((R.nx + 63) / 64);
                    tiles = (units + b / 64 - 1) / (b / 64);
                } else {
                    // two nodes per lane
                    tiles = (R.V + 2 * b - 1) / (2 * b);
                }
                pre[r + 1] = pre[r] + (int)tiles;
            }
            LatticeLaunch L;
            L.block = b;
            L.mapping = mi == 2 ? 3 : mi;
            L.total_tiles = pre.back();
            L.d_prefix = prefix_base + (mi * kNumBlockSizes + bi) * (int)(c.reps.size() + 1);
            if ((rc = check(hipMemcpy(L.d_prefix, pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice),
                            "upload tiles")))
                return bail(rc);
            c.lat_all.push_back(L);
            if (mi == 0) {
                // the shifted flat mapping has the flat mapping's tiles
                L.mapping = 2;
                c.lat_all.push_back(L);
            }
        }
    }
    // launch shape: flattened mapping; contiguous XCD ranges for one box, hardware order
    // for several (uneven) boxes; LB_CFG_AUTOTUNE times the alternatives
    bool rows_fit = true;
    for (const Replica& R : c.reps) rows_fit = rows_fit && (R.nx % 64 == 0);
    // measured: row segments win only marginally (FP32, one box), so flat is the default
    (void)rows_fit;
    c.lat.mapping = cfg->lattice_mapping == LB_MAP_ROWS      ? 1
                    : cfg->lattice_mapping == LB_MAP_SHIFTED ? 2
                    : cfg->lattice_mapping == LB_MAP_FLAT2   ? 3
                                                             : 0;
    if (cfg->xcd_order == LB_XCD_AUTO) c.lat_chunk = c.reps.size() == 1 ? -1 : 0;
    else if (cfg->xcd_order == LB_XCD_HARDWARE) c.lat_chunk = 0;
    else if (cfg->xcd_order == LB_XCD_CONTIGUOUS) c.lat_chunk = -1;
    else c.lat_chunk = cfg->xcd_order;
    if ((rc = set_lattice_shape(c, cfg->block_size ? cfg->block_size : 256))) return bail(rc);
    // both population buffers within 160 MB stay in the 256 MB last-level cache between
    // sweeps when stored normally; larger ones are streamed past it
    c.lat_nt = 2.0 * (double)c.pop_elems * (double)store_size(c.storage) > 160e6;

    if ((rc = check(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking), "side stream"))) return bail(rc);
    if ((rc = check(hipStreamCreateWithFlags(&c.cap, hipStreamNonBlocking), "capture stream"))) return bail(rc);
    if ((rc = check(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming), "event"))) return bail(rc);
    if ((rc = check(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming), "event"))) return bail(rc);
    if ((rc = check(hipHostMalloc((void**)&c.h_small, 32 * sizeof(double), hipHostMallocDefault),
                    "pinned staging")))
        return bail(rc);

    rc = c.storage == LB_STORE_F64 ? setup_beads<double>(c, cfg) : setup_beads<float>(c, cfg);
    if (rc) return bail(rc);
    c.cur = 0;
    if ((rc = init_populations(c, cfg))) return bail(rc);
    if (c.ntot_beads > 0) {
        // a mode-0 launch of the bead kernel changes nothing; it sets the kernel's
        // LDS attribute here rather than inside a later graph capture
        if ((rc = check(launch_md(c, c.pops[c.cur], 0, c.stream), "bead kernel warm-up"))) return bail(rc);
    }
    if (cfg->flags & LB_CFG_AUTOTUNE) {
        if ((rc = autotune(c))) return bail(rc);
        // the lanes per bead set the order of the bead-force sums: a deterministic context
        // keeps the choice by bead count (or the configured one) rather than a timed one
        if (!c.deterministic && (rc = autotune_md(c))) return bail(rc);
    }
    if ((rc = check(hipStreamSynchronize(c.stream), "sync"))) return bail(rc);
    *out = ctx;
    return LB_OK;
}

int lb_step(lbmd_ctx* ctx, int n_steps, unsigned flags) {
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    if (n_steps < 0) return fail(LB_EINVAL, "n_steps < 0");
    Context& c = ctx->c;
    if ((flags & LB_STEP_COUPLED) && (flags & LB_STEP_NO_HYDRO))
        return fail(LB_EINVAL, "LB_STEP_COUPLED and LB_STEP_NO_HYDRO exclude each other");
    const int mode = (flags & LB_STEP_COUPLED) ? STEP_COUPLED : (flags & LB_STEP_NO_HYDRO) ? STEP_NO_HYDRO : STEP_LB;
    const bool flips = mode != STEP_NO_HYDRO;  // the populations change buffers
    int done = 0;
    if (c.use_graph) {
        // graphs of kGraphSteps steps, then one graph for the remainder (each length and
        // buffer parity is captured once and kept)
        while (done < n_steps) {
            const int len = std::min(n_steps - done, (int)Context::kGraphSteps);
            hipGraphExec_t& g = c.graphs[mode][c.cur][len];
            if (!g) {
                int rc = build_graph(c, mode, c.cur, len, &g);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(g, c.stream));
            if (flips && (len & 1)) c.cur = 1 - c.cur;
            done += len;
        }
    }
    for (; done < n_steps; ++done) {
        HIP_TRY(enqueue_step(c, mode, c.cur, c.stream));
        if (flips) c.cur = 1 - c.cur;
    }
    c.host_step += n_steps;
    return LB_OK;
}

int lb_graph_prepare(lbmd_ctx* ctx, int n_steps, unsigned flags) {
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    if (n_steps < 0) return fail(LB_EINVAL, "n_steps < 0");
    if ((flags & LB_STEP_COUPLED) && (flags & LB_STEP_NO_HYDRO))
        return fail(LB_EINVAL, "LB_STEP_COUPLED and LB_STEP_NO_HYDRO exclude each other");
    Context& c = ctx->c;
    if (!c.use_graph || n_steps == 0) return LB_OK;
    const int mode = (flags & LB_STEP_COUPLED) ? STEP_COUPLED : (flags & LB_STEP_NO_HYDRO) ? STEP_NO_HYDRO : STEP_LB;
    // lb_step launches graphs of kGraphSteps steps and one of the remainder, starting from
    // either buffer parity
    const int lens[2] = {n_steps >= Context::kGraphSteps ? (int)Context::kGraphSteps : 0,
                         n_steps % Context::kGraphSteps};
    for (int parity = 0; parity < 2; ++parity)
        for (int len : lens) {
            if (len == 0) continue;
            hipGraphExec_t& g = c.graphs[mode][parity][len];
            if (!g) {
                const int rc = build_graph(c, mode, parity, len, &g);
                if (rc) return rc;
            }
        }
    return LB_OK;
}

int lb_couple(lbmd_ctx* ctx, unsigned dir) {
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    Context& c = ctx->c;
    if (dir != LB_COUPLE_INTERP && dir != LB_COUPLE_SPREAD) return fail(LB_EINVAL, "unknown direction");
    if (c.ntot_beads == 0) return LB_OK;
    if (dir == LB_COUPLE_INTERP && c.md.stencil == LB_STENCIL_TRILINEAR)
        HIP_TRY(launch_interp_trilinear(c, c.pops[c.cur], c.stream));
    else if (dir == LB_COUPLE_INTERP) HIP_TRY(launch_md(c, c.pops[c.cur], MD_INTERP, c.stream));
    else HIP_TRY(launch_spread(c, c.pops[c.cur], false, c.stream));
    return LB_OK;
}

int md_step(lbmd_ctx* ctx) {
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    Context& c = ctx->c;
    if (c.ntot_beads == 0) return LB_OK;
    HIP_TRY(launch_md(c, c.pops[c.cur], MD_SUBSTEPS, c.stream));
    if (c.obs_every > 0) HIP_TRY(launch_observe(c, false, c.stream));
    return LB_OK;
}

size_t lb_moments_bytes(const lbmd_ctx* ctx, int replica, unsigned what) {
    if (!ctx || replica < 0 || replica >= (int)ctx->c.reps.size()) return 0;
    const Replica& R = ctx->c.reps[replica];
    const size_t V = (size_t)R.V, n = (size_t)R.n_beads;
    switch (what) {
        case LB_MOM_CONSERVED: return 4 * sizeof(double);
        case LB_MOM_FIELDS: return 4 * V * sizeof(double);
        case LB_MOM_POPULATIONS: return 19 * V * sizeof(double);
        case LB_MOM_BEADS: return 6 * n * sizeof(double);
        case LB_MOM_TRANSLOC: return 6 * sizeof(double);
        case LB_MOM_COUPLING: return 7 * n * sizeof(double);
        case LB_MOM_STATUS: return 2 * sizeof(double);
        case LB_MOM_OBSERVABLES:
            return ctx->c.obs_every > 0 ? ((size_t)ctx->c.obs_capacity + 1) * 8 * sizeof(double) : 0;
        default: return 0;
    }
}

long long lb_plane_stride(const lbmd_replica* rep, int storage) {
    const size_t elem = store_size(storage);
    if (!rep || !elem || rep->nx < 1 || rep->ny < 1 || rep->nz < 1) {
        fail(LB_EINVAL, !rep ? "rep is NULL" : !elem ? "unknown storage" : "box sizes must be >= 1");
        return -1;
    }
    return plane_stride((long long)rep->nx * rep->ny * rep->nz, elem);
}

int lb_block_size(const lbmd_ctx* ctx) { return ctx ? ctx->c.lat.block : 0; }

int lb_launch_shape(const lbmd_ctx* ctx, int* block, int* mapping, int* xcd_order, int* nt_stores) {
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    const Context& c = ctx->c;
    if (nt_stores) *nt_stores = c.lat_nt ? 1 : 0;
    if (block) *block = c.lat.block;
    if (mapping)
        *mapping = c.lat.mapping == 1   ? LB_MAP_ROWS
                   : c.lat.mapping == 2 ? LB_MAP_SHIFTED
                   : c.lat.mapping == 3 ? LB_MAP_FLAT2
                                        : LB_MAP_FLAT;
    if (xcd_order) *xcd_order = c.lat_chunk < 0 ? LB_XCD_CONTIGUOUS : (c.lat_chunk == 0 ? LB_XCD_HARDWARE : c.lat_chunk);
    return LB_OK;
}

int lb_pattern_copy(lbmd_ctx* ctx, int alternate) {
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    Context& c = ctx->c;
    HIP_TRY(launch_pattern(c, c.pops[c.cur], c.pops[1 - c.cur], c.stream));
    if (alternate) c.cur = 1 - c.cur;
    return LB_OK;
}

int lb_md_lanes(const lbmd_ctx* ctx) {
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    const Context& c = ctx->c;
    if (c.ntot_beads == 0) return 0;
    return c.md_lanes > 0 ? c.md_lanes : md_default_lanes(c.max_beads);
}

}  // extern "C"

namespace {

template <class Real>
int copy_bead_field(Context& c, const Replica& R, const Real* dev, int ncomp, double* out) {
    const int n = R.n_beads, N = c.ntot_beads;
    std::vector<Real> tmp((size_t)n);
    for (int a = 0; a < ncomp; ++a) {
        HIP_TRY(hipMemcpyAsync(tmp.data(), dev + (size_t)a * N + R.bead0, n * sizeof(Real), hipMemcpyDeviceToHost, c.stream));
        HIP_TRY(hipStreamSynchronize(c.stream));
        for (int i = 0; i < n; ++i) out[(size_t)ncomp * i + a] = (double)tmp[i];
    }
    return LB_OK;
}

template <class Real>
int moments_beads(Context& c, int replica, unsigned what, double* out) {
    const BeadPtrs<Real>& b = *(const BeadPtrs<Real>*)c.bead_ptrs;
    const Replica& R = c.reps[replica];
    const int n = R.n_beads;
    if (n == 0) return LB_OK;
    int rc;
    if (what == LB_MOM_BEADS) {
        if ((rc = copy_bead_field<double>(c, R, b.r, 3, out))) return rc;
        return copy_bead_field<Real>(c, R, b.v, 3, out + 3 * (size_t)n);
    }
    if ((rc = copy_bead_field<Real>(c, R, b.u, 3, out))) return rc;
    if ((rc = copy_bead_field<Real>(c, R, b.fbar, 3, out + 3 * (size_t)n))) return rc;
    std::vector<int> nd((size_t)n);
    HIP_TRY(hipMemcpyAsync(nd.data(), b.node + R.bead0, n * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
    for (int i = 0; i < n; ++i) out[6 * (size_t)n + i] = nd[i];
    return LB_OK;
}

}  // namespace

extern "C" {

int lb_moments(lbmd_ctx* ctx, int replica, unsigned what, void* host_out, size_t bytes) {
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    Context& c = ctx->c;
    if (replica < 0 || replica >= (int)c.reps.size()) return fail(LB_EINVAL, "replica out of range");
    const size_t need = lb_moments_bytes(ctx, replica, what);
    if (!need) return fail(LB_EINVAL, "unknown observable");
    if (!host_out || bytes < need) return fail(LB_ESIZE, "need " + std::to_string(need) + " bytes");
    double* out = (double*)host_out;
    const Replica& R = c.reps[replica];
    const void* cur = c.pops[c.cur];
    // every read below is ordered on the context's stream after the queued steps; small
    // results travel through pinned staging with the run state, one synchronisation
    double* hs = c.h_small;
    RunState* hst = (RunState*)(hs + 16);
    switch (what) {
        case LB_MOM_CONSERVED: {
            double* d_out4 = c.d_partials + 4 * (size_t)c.partial_blocks;
            HIP_TRY(launch_conserved(c, replica, cur, d_out4, c.stream));
            HIP_TRY(hipMemcpyAsync(hs, d_out4, 4 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
            break;
        }
        case LB_MOM_FIELDS:
        case LB_MOM_POPULATIONS: {
            const int ncomp = what == LB_MOM_FIELDS ? 4 : 19;
            const long long chunk = (long long)(c.stage_doubles / 19);
            for (long long n0 = 0; n0 < R.V; n0 += chunk) {
                const int cnt = (int)std::min<long long>(chunk, R.V - n0);
                HIP_TRY(launch_gather(c, replica, cur, ncomp == 4 ? 1 : 0, n0, cnt, c.d_stage, c.stream));
                for (int k = 0; k < ncomp; ++k)
                    HIP_TRY(hipMemcpyAsync(out + (size_t)k * R.V + n0, c.d_stage + (size_t)k * cnt,
                                           cnt * sizeof(double), hipMemcpyDeviceToHost, c.stream));
            }
            break;
        }
        case LB_MOM_BEADS:
        case LB_MOM_COUPLING: {
            int rc = c.storage == LB_STORE_F64 ? moments_beads<double>(c, replica, what, out)
                                               : moments_beads<float>(c, replica, what, out);
            if (rc) return rc;
            break;
        }
        case LB_MOM_TRANSLOC: {
            const double* diag = c.storage == LB_STORE_F64 ? ((BeadPtrs<double>*)c.bead_ptrs)->diag
                                                           : ((BeadPtrs<float>*)c.bead_ptrs)->diag;
            HIP_TRY(hipMemcpyAsync(hs, diag + 8 * replica, 8 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
            break;
        }
        case LB_MOM_STATUS:
            break;
        case LB_MOM_OBSERVABLES: {
            const double* obs = c.storage == LB_STORE_F64 ? ((BeadPtrs<double>*)c.bead_ptrs)->obs
                                                          : ((BeadPtrs<float>*)c.bead_ptrs)->obs;
            const size_t rows = (size_t)c.obs_capacity + 1;
            HIP_TRY(hipMemcpyAsync(out, obs + (size_t)replica * rows * 8, rows * 8 * sizeof(double),
                                   hipMemcpyDeviceToHost, c.stream));
            break;
        }
    }
    HIP_TRY(hipMemcpyAsync(hst, c.d_state, sizeof(RunState), hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
    const RunState st = *hst;
    if (what == LB_MOM_CONSERVED) {
        for (int k = 0; k < 4; ++k) out[k] = hs[k];
    } else if (what == LB_MOM_TRANSLOC) {
        for (int k = 0; k < 5; ++k) out[k] = hs[k];
        out[5] = (double)c.host_step;
    } else if (what == LB_MOM_STATUS) {
        out[0] = (double)st.err;
        out[1] = (double)st.step;
    }
    if (st.err) return fail(LB_EUNSTABLE, "device error word " + std::to_string(st.err));
    return LB_OK;
}

int lb_moments_range(lbmd_ctx* ctx, int replica, unsigned what, long long node0, int count, void* host_out,
                     size_t bytes) {
    if (!ctx) return fail(LB_EINVAL, "ctx is NULL");
    Context& c = ctx->c;
    if (replica < 0 || replica >= (int)c.reps.size()) return fail(LB_EINVAL, "replica out of range");
    if (what != LB_MOM_FIELDS && what != LB_MOM_POPULATIONS) return fail(LB_EINVAL, "only fields or populations");
    const Replica& R = c.reps[replica];
    if (node0 < 0 || count < 0 || node0 + count > R.V) return fail(LB_EINVAL, "node range outside the replica");
    const int ncomp = what == LB_MOM_FIELDS ? 4 : 19;
    if (!host_out || bytes < (size_t)ncomp * count * sizeof(double))
        return fail(LB_ESIZE, "need " + std::to_string((size_t)ncomp * count * sizeof(double)) + " bytes");
    double* out = (double*)host_out;
    HIP_TRY(hipStreamSynchronize(c.stream));
    const long long chunk = (long long)(c.stage_doubles / 19);
    for (long long k0 = 0; k0 < count; k0 += chunk) {
        const int cnt = (int)std::min<long long>(chunk, count - k0);
        HIP_TRY(launch_gather(c, replica, c.pops[c.cur], ncomp == 4 ? 1 : 0, node0 + k0, cnt, c.d_stage, c.stream));
        for (int k = 0; k < ncomp; ++k)
            HIP_TRY(hipMemcpyAsync(out + (size_t)k * count + k0, c.d_stage + (size_t)k * cnt, cnt * sizeof(double),
                                   hipMemcpyDeviceToHost, c.stream));
    }
    RunState st;
    HIP_TRY(hipMemcpyAsync(&st, c.d_state, sizeof st, hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
    if (st.err) return fail(LB_EUNSTABLE, "device error word " + std::to_string(st.err));
    return LB_OK;
}

int lb_destroy(lbmd_ctx* ctx) {
    if (!ctx) return LB_OK;
    Context& c = ctx->c;
    (void)hipStreamSynchronize(c.stream);
    release(c);
    delete ctx;
    return LB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Conserved sums without allocation (lb_conserved_noalloc): the partial sums of the FP64
// reduction go to a static device array instead of a context's work buffer.
// ---------------------------------------------------------------------------------
namespace {
// one block of partial sums per kNodesPerBlock nodes, at most kScratchBlocks blocks: replicas
// of up to 2^27 nodes (512^3)
constexpr int kScratchBlocks = 32768;
constexpr long long kNodesPerBlock = 4096;
constexpr int kMaxDevices = 64;
}  // namespace

// [kScratchBlocks][4] doubles, 1 MiB on every GPU the library runs on, held until the process
// ends; every call on a GPU shares that GPU's copy
static __device__ __align__(256) double scratch[4 * kScratchBlocks];

namespace {
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of the current device's `scratch` (in host code the array's name is a
// host-side stand-in, not a device address), looked up on the first call on each device.
int scratch_on_current_device(double** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LB_EDEVICE, "device ordinal beyond the library's table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LB_EDEVICE, "no device address for the scratch array");
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return LB_OK;
}
}  // namespace

extern "C" int lb_conserved_noalloc(const void* pops, int storage, const lbmd_replica* rep, double* out4,
                                    void* hip_stream) {
    if (!pops || !rep || !out4) return fail(LB_EINVAL, "pops, rep and out4 are required");
    const size_t elem = store_size(storage);
    if (!elem) return fail(LB_EINVAL, "unknown storage");
    if (((uintptr_t)pops % elem) != 0 || ((uintptr_t)out4 % sizeof(double)) != 0)
        return fail(LB_EINVAL, "pops and out4 must be aligned to their element sizes");
    const std::string why = replica_problem(*rep);
    if (!why.empty()) return fail(LB_EINVAL, "replica: " + why);
    const long long V = (long long)rep->nx * rep->ny * rep->nz;
    const long long nblk = (V + kNodesPerBlock - 1) / kNodesPerBlock;
    if (nblk > kScratchBlocks)
        return fail(LB_ESIZE, "a replica of " + std::to_string(V) + " nodes needs " + std::to_string(nblk) +
                                  " blocks of partial sums; the static scratch array holds " +
                                  std::to_string(kScratchBlocks) + " (replicas of at most 2^27 nodes)");
    double* partials = nullptr;
    const int rc = scratch_on_current_device(&partials);
    if (rc != LB_OK) return rc;
    // pops is the replica's own [19][S] block: its description keeps pop_base = 0
    const Replica R = make_replica(*rep, elem);
    HIP_TRY(launch_conserved_desc(R, storage, pops, partials, (int)nblk, out4, (hipStream_t)hip_stream));
    return LB_OK;
}
