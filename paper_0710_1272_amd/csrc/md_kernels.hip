// md_kernels.hip -- bead kernels (gfx950).
//
// k_md: one workgroup per replica.  Depending on the mode it performs
//   step 1 of Sec. II (arXiv:0710.1272): nearest-grid-point interpolation of the fluid
//          velocity at every bead, u_i = j/rho of the pre-collision populations of the
//          node floor(r + 1/2) (pull-gathered from the current post-collision buffer);
//   step 2: M substeps h = 1/M with u_i frozen: harmonic bonds, WCA between non-bonded
//          beads, WCA on the distance to the nearest solid surface and to free-slip
//          faces, the pulling force in the pore (Sec. III), drag -m gamma (v - u_i) and
//          the random force A c (Philox4x32-10, A = sqrt(24 m gamma kT / h)),
//          integrated kick-drift; Fbar_i = mean of drag + random force;
//   epilogue: translocation count N_T, centre of mass (FP64), completion latch, and a
//          deterministic per-node sum of Fbar (one leader bead per node).
// Bead positions are accumulated in FP64 (they integrate ~10^5-10^6 small increments);
// velocities and forces use the lattice's arithmetic type.  Positions live in LDS.
//
// k_spread: step 3, S_p = -(w_p / c_s^2) Fbar . c_p added to the post-collision
// populations of each leader's node (S_p eq.); nodes are unique within a replica,
// so there are no write conflicts and no floating-point atomics.
#include <algorithm>
#include <utility>

#include "lbmd_internal.hpp"

namespace lbmd {

template <class F, int... Ps>
__device__ __forceinline__ void md_for_pops_impl(F&& f, std::integer_sequence<int, Ps...>) {
    (f(std::integral_constant<int, Ps>{}), ...);
}
template <class F>
__device__ __forceinline__ void md_for_pops(F&& f) {
    md_for_pops_impl(f, std::make_integer_sequence<int, Q>{});
}

template <int S>
struct MDReal {
    using type = float;
};
template <>
struct MDReal<LB_STORE_F64> {
    using type = double;
};

template <class Real>
struct MDKArgs {
    const Replica* reps;
    MDDev md;
    BeadPtrs<Real> b;
    const void* cur;
    RunState* st;
    int mode;
    int nmax;
    int list_in_lds;
};

// nearest node: floor(r + 1/2); periodic axes wrap, free-slip axes clamp (NaN -> 0)
__device__ __forceinline__ void ngp3(const Replica& R, const double* r, int* g) {
    const int n[3] = {R.nx, R.ny, R.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double t = floor(r[a] + 0.5);
        if (!(t >= -1e15 && t <= 1e15)) t = 0.0;  // non-finite
        if (R.fs[a]) {
            t = t < 0.0 ? 0.0 : (t > n[a] - 1 ? (double)(n[a] - 1) : t);
        } else {
            t = t - n[a] * floor(t / n[a]);
        }
        g[a] = (int)t;
    }
}

__device__ __forceinline__ double min_image(double d, int n, int periodic) {
    return periodic ? d - n * floor(d / n + 0.5) : d;
}

// distance to the nearest solid surface (unit cubes around solid nodes; a wall is
// its slab minus the pore prism, as four boxes), and the vector from it to r
__device__ inline double wall_distance(const Replica& R, const double* rin, double* dv) {
    const int n[3] = {R.nx, R.ny, R.nz};
    double r[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) r[a] = R.fs[a] ? rin[a] : rin[a] - n[a] * floor((rin[a] + 0.5) / n[a]);
    double best2 = HUGE_VAL;
    dv[0] = dv[1] = dv[2] = 0.0;
#pragma unroll
    for (int k = 0; k < LB_MAX_WALLS; ++k) {
        if (k >= R.n_walls) break;
        const int* w = R.wall[k];
        const double X0 = w[0] - 0.5, X1 = w[1] + 0.5;
        const bool open = pore_open(w);
        const double Y0 = w[2] - 0.5, Y1 = w[3] + 0.5, Z0 = w[4] - 0.5, Z1 = w[5] + 0.5;
        const int nb = open ? 4 : 1;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (m >= nb) break;
            double lo[3] = {X0, -HUGE_VAL, -HUGE_VAL}, hi[3] = {X1, HUGE_VAL, HUGE_VAL};
            if (open) {
                if (m == 0) { hi[1] = Y0; }
                else if (m == 1) { lo[1] = Y1; }
                else if (m == 2) { lo[1] = Y0; hi[1] = Y1; hi[2] = Z0; }
                else { lo[1] = Y0; hi[1] = Y1; lo[2] = Z1; }
            }
            double d[3], d2 = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double c = fmin(fmax(r[a], lo[a]), hi[a]);
                d[a] = r[a] - c;
                d2 += d[a] * d[a];
            }
            if (d2 < best2) {
                best2 = d2;
                dv[0] = d[0];
                dv[1] = d[1];
                dv[2] = d[2];
            }
        }
    }
    return sqrt(best2);
}

// The part of a replica's description the substep loop reads, copied into registers
// at kernel entry (before any store, so the copy is made with scalar loads).
struct Geom {
    int n[3];
    int fs[3];
    int n_walls;
    int wall[LB_MAX_WALLS][6];
};

__device__ __forceinline__ Geom load_geom(const Replica& R) {
    // every field is the same for the whole workgroup: keep it in scalar registers
    auto u = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
    Geom g;
#pragma unroll
    for (int a = 0; a < 3; ++a) g.fs[a] = u(R.fs[a]);
    g.n[0] = u(R.nx);
    g.n[1] = u(R.ny);
    g.n[2] = u(R.nz);
    g.n_walls = u(R.n_walls);
#pragma unroll
    for (int k = 0; k < LB_MAX_WALLS; ++k)
#pragma unroll
        for (int m = 0; m < 6; ++m) g.wall[k][m] = u(R.wall[k][m]);
    return g;
}

__device__ __forceinline__ bool geom_is_pore(const Geom& G, const int* c) {
    bool s = false;
#pragma unroll
    for (int k = 0; k < LB_MAX_WALLS; ++k) {
        if (k >= G.n_walls) break;
        const int* w = G.wall[k];
        s = s || (c[0] >= w[0] && c[0] <= w[1] && pore_open(w) && c[1] >= w[2] && c[1] <= w[3] &&
                  c[2] >= w[4] && c[2] <= w[5]);
    }
    return s;
}

// nearest node floor(r + 1/2): free-slip axes clamp (NaN -> 0), periodic axes wrap
template <bool PERIODIC>
__device__ __forceinline__ void geom_ngp(const Geom& G, const double* r, int* c) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double t = floor(r[a] + 0.5);
        if (!(t >= -1e9 && t <= 1e9)) t = 0.0;  // non-finite or absurd
        int k = (int)t;
        if (PERIODIC && !G.fs[a]) {
            k %= G.n[a];
            if (k < 0) k += G.n[a];
        } else {
            k = k < 0 ? 0 : (k > G.n[a] - 1 ? G.n[a] - 1 : k);
        }
        c[a] = k;
    }
}

// distance to the nearest solid surface and the vector from it to r (see wall_distance)
template <bool PERIODIC>
__device__ inline double geom_wall_distance(const Geom& G, const double* rin, double* dv) {
    double r[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        r[a] = (PERIODIC && !G.fs[a]) ? rin[a] - G.n[a] * floor((rin[a] + 0.5) / G.n[a]) : rin[a];
    double best2 = HUGE_VAL;
    dv[0] = dv[1] = dv[2] = 0.0;
#pragma unroll
    for (int k = 0; k < LB_MAX_WALLS; ++k) {
        if (k >= G.n_walls) break;
        const int* w = G.wall[k];
        const double X0 = w[0] - 0.5, X1 = w[1] + 0.5;
        const bool open = pore_open(w);
        const double Y0 = w[2] - 0.5, Y1 = w[3] + 0.5, Z0 = w[4] - 0.5, Z1 = w[5] + 0.5;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (m >= (open ? 4 : 1)) break;
            double lo[3] = {X0, -HUGE_VAL, -HUGE_VAL}, hi[3] = {X1, HUGE_VAL, HUGE_VAL};
            if (open) {
                if (m == 0) { hi[1] = Y0; }
                else if (m == 1) { lo[1] = Y1; }
                else if (m == 2) { lo[1] = Y0; hi[1] = Y1; hi[2] = Z0; }
                else { lo[1] = Y0; hi[1] = Y1; lo[2] = Z1; }
            }
            double d[3], d2 = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double c = fmin(fmax(r[a], lo[a]), hi[a]);
                d[a] = r[a] - c;
                d2 += d[a] * d[a];
            }
            if (d2 < best2) {
                best2 = d2;
                dv[0] = d[0];
                dv[1] = d[1];
                dv[2] = d[2];
            }
        }
    }
    return sqrt(best2);
}

// 1/x: the hardware reciprocal in FP32 (about 1 ulp), an exact division in FP64
template <class Real>
__device__ __forceinline__ Real fast_rcp(Real x) {
    if constexpr (sizeof(Real) == 4) return __builtin_amdgcn_rcpf(x);
    else return Real(1) / x;
}

// -(1/r) dV/dr of WCA at squared distance r2 (0 beyond the cutoff)
template <class Real>
__device__ __forceinline__ Real wca_coef(Real r2, Real eps, Real sig2, Real rc2) {
    if (!(r2 < rc2)) return Real(0);
    const Real ir2 = fast_rcp<Real>(r2);
    const Real s2 = sig2 * ir2;
    const Real s6 = s2 * s2 * s2;
    return Real(24) * eps * (Real(2) * s6 * s6 - s6) * ir2;
}

template <class Real>
__device__ __forceinline__ void block_sums(double* vals, int nv, double* scratch) {
    // sums nv doubles over the block; result valid in every thread; scratch >= 16*nv
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nv; ++k) {
        double v = vals[k];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) scratch[k * 16 + wave] = v;
    }
    __syncthreads();
    for (int k = 0; k < nv; ++k) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += scratch[k * 16 + w];
        vals[k] = t;
    }
    __syncthreads();
}


// pre-collision populations of one node, decoded (storage chosen at run time)
template <int S, class Real>
__device__ __forceinline__ void node_moments(const Replica& R, const void* cur, const int* g, Real* rho,
                                             Real* j) {
    using C = Codec<S>;
    const typename C::T* src = (const typename C::T*)cur;
    Real m = 0, jx = 0, jy = 0, jz = 0;
    md_for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        int q;
        const int s = pull_source<p>(R, g[0], g[1], g[2], &q);
        Real fp = (Real)C::template load<p>(src[R.pop_base + (long long)q * R.V + s]);
        if constexpr (C::deviation) fp += w_of<Real>(p) * (Real)R.rho0;
        m += fp;
        if constexpr (cx_of(p) != 0) jx += Real(cx_of(p)) * fp;
        if constexpr (cy_of(p) != 0) jy += Real(cy_of(p)) * fp;
        if constexpr (cz_of(p) != 0) jz += Real(cz_of(p)) * fp;
    });
    *rho = m;
    j[0] = jx;
    j[1] = jy;
    j[2] = jz;
}

template <class Real>
__device__ __forceinline__ void node_velocity(int storage, const Replica& R, const void* cur, const int* g,
                                              Real* u) {
    Real rho = 1, j[3] = {0, 0, 0};
    switch (storage) {
        case LB_STORE_F64: node_moments<LB_STORE_F64, Real>(R, cur, g, &rho, j); break;
        case LB_STORE_F32: node_moments<LB_STORE_F32, Real>(R, cur, g, &rho, j); break;
        case LB_STORE_F16DEV: node_moments<LB_STORE_F16DEV, Real>(R, cur, g, &rho, j); break;
        default: node_moments<LB_STORE_BF16DEV, Real>(R, cur, g, &rho, j); break;
    }
    u[0] = j[0] / rho;
    u[1] = j[1] / rho;
    u[2] = j[2] / rho;
}

// sum over the G consecutive lanes of a group (G a power of two <= 64)
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Pairwise separation r_i - r_j as FP32/FP64 components (minimum image on periodic
// axes) and its square.
template <class Real, bool PERIODIC>
__device__ __forceinline__ Real separation(const double* ri, const double* PX, const double* PY,
                                           const double* PZ, int j, const int* per, const double* nd,
                                           Real* d) {
    double dd[3] = {ri[0] - PX[j], ri[1] - PY[j], ri[2] - PZ[j]};
    if constexpr (PERIODIC) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (per[c]) dd[c] -= nd[c] * floor(dd[c] / nd[c] + 0.5);
    }
    d[0] = (Real)dd[0];
    d[1] = (Real)dd[1];
    d[2] = (Real)dd[2];
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

// Verlet list of bead i (group of G lanes): every non-bonded bead closer than the list
// radius, in lane-then-index order.  Returns the count (may exceed the capacity).
template <class Real, int G, bool PERIODIC>
__device__ __forceinline__ int build_list(int i, int n, bool bn, bool bp, const double* ri, const double* PX,
                                          const double* PY, const double* PZ, const int* per,
                                          const double* nd, Real rl2, int gl, unsigned short* list,
                                          int stride) {
    if constexpr (G == 1) {
        // one lane per bead: append directly, keep counting past the capacity
        int total = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i || (j == i + 1 && bn) || (j == i - 1 && bp)) continue;
            Real d[3];
            if (separation<Real, PERIODIC>(ri, PX, PY, PZ, j, per, nd, d) < rl2) {
                if (total < kNeighbourMax) list[(size_t)total * stride] = (unsigned short)j;
                ++total;
            }
        }
        return total;
    } else {
        int mine = 0;
        for (int j = gl; j < n; j += G) {
            if (j == i || (j == i + 1 && bn) || (j == i - 1 && bp)) continue;
            Real d[3];
            if (separation<Real, PERIODIC>(ri, PX, PY, PZ, j, per, nd, d) < rl2) ++mine;
        }
        // exclusive prefix over the group's lanes
        int incl = mine;
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            const int t = __shfl_up(incl, off, G);
            if (gl >= off) incl += t;
        }
        int pos = incl - mine;
        const int total = __shfl(incl, G - 1, G);
        if (total <= kNeighbourMax) {
            for (int j = gl; j < n; j += G) {
                if (j == i || (j == i + 1 && bn) || (j == i - 1 && bp)) continue;
                Real d[3];
                if (separation<Real, PERIODIC>(ri, PX, PY, PZ, j, per, nd, d) < rl2)
                    list[(size_t)(pos++) * stride] = (unsigned short)j;
            }
        }
        return total;
    }
}

// Each bead is owned by a group of G lanes that split its neighbour loop; every lane
// of the group keeps the bead's state, so the per-bead terms are computed redundantly
// without divergence.  BPT beads per group when there are more beads than groups
// (then G = 1).  WCA pairs come from a Verlet list (radius rc + skin) rebuilt at the
// start of every LB step and whenever a bead has moved skin/2 since the last build,
// so the set of interacting pairs is exactly that of the all-pairs definition.
// Positions are double-buffered in LDS: one barrier per substep.
template <class Real, int G, int BPT, bool PERIODIC, int MAXT>
__global__ __launch_bounds__(MAXT) void k_md(MDKArgs<Real> a, int storage) {
    extern __shared__ double lds[];
    __shared__ double red[16 * 4];
    const int NG = blockDim.x / G;  // groups per block
    const Replica& R = a.reps[blockIdx.x];
    const Geom GM = load_geom(R);
    const uint32_t seed_lo = R.seed_lo, seed_hi = R.seed_hi;
    const double xmid = R.xmid;
    const int n = R.n_beads;
    if (n == 0) return;
    const int b0 = R.bead0, NT = a.b.ntot, tid = threadIdx.x, nmax = a.nmax;
    const int grp = tid / G, gl = tid % G;
    double* P = lds;                                    // [2][3][nmax] positions
    int* NODE = (int*)(P + 6 * nmax);                   // [nmax]
    unsigned char* BN = (unsigned char*)(NODE + nmax);  // [nmax]
    // Verlet lists: [kNeighbourMax][nmax] in LDS when they fit, else global memory
    unsigned short* lists = a.list_in_lds ? (unsigned short*)(BN + nmax) : a.b.nlist + b0;
    const int lstride = a.list_in_lds ? nmax : NT;
    const MDDev md = a.md;
    const int M = md.M;
    const long long step = a.st->step;
    const int* nn = GM.n;
    const double nd[3] = {(double)GM.n[0], (double)GM.n[1], (double)GM.n[2]};
    const int per[3] = {GM.fs[0] ? 0 : 1, GM.fs[1] ? 0 : 1, GM.fs[2] ? 0 : 1};
    unsigned flags = 0;
    int cur = 0;

    double r[BPT][3];
    Real v[BPT][3], u[BPT][3], fb[BPT][3];
    int node[BPT];
    bool own[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        own[k] = i < n;
        node[k] = -1;
#pragma unroll
        for (int c = 0; c < 3; ++c) { r[k][c] = 0; v[k][c] = 0; u[k][c] = 0; fb[k][c] = 0; }
        if (own[k]) {
            const int g = b0 + i;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                r[k][c] = a.b.r[c * NT + g];
                v[k][c] = a.b.v[c * NT + g];
            }
            if (gl == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) P[c * nmax + i] = r[k][c];
                BN[i] = a.b.bond_next[g];
            }
        }
    }
    __syncthreads();

    if (a.mode & MD_INTERP) {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            if (!own[k]) continue;
            int g[3];
            ngp3(R, r[k], g);
            if (is_solid(R, g[0], g[1], g[2])) {
                node[k] = -1;
                u[k][0] = u[k][1] = u[k][2] = 0;
            } else {
                node[k] = g[0] + R.nx * (g[1] + R.ny * g[2]);
                node_velocity<Real>(storage, R, a.cur, g, u[k]);
            }
            if (gl == 0) {
                const int gi = b0 + i;
                a.b.node[gi] = node[k];
#pragma unroll
                for (int c = 0; c < 3; ++c) a.b.u[c * NT + gi] = u[k][c];
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            if (!own[k]) continue;
            node[k] = a.b.node[b0 + i];
#pragma unroll
            for (int c = 0; c < 3; ++c) u[k][c] = a.b.u[c * NT + b0 + i];
        }
    }
    if (!(a.mode & MD_SUBSTEPS)) return;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        if (own[k] && gl == 0) NODE[i] = node[k];
    }

    const Real h = (Real)md.h, hm = (Real)(md.h * md.inv_mass), invM = (Real)md.inv_M;
    const Real mg = (Real)(md.mass * md.gamma), A = (Real)md.A;
    const Real kb = (Real)md.k_bond, r0 = (Real)md.r0;
    const Real eps24 = (Real)(24.0 * md.eps), sig2 = (Real)md.sigma2, rc2 = (Real)md.rc2;
    const Real epsw = (Real)md.eps_w, sigw2 = (Real)md.sigma_w2, rcw2 = (Real)md.rcw2;
    const double rcw = md.rcw;
    const Real rl2 = (Real)md.rl2, hs2 = (Real)md.half_skin2;
    const Real fdrive = (Real)md.f_drive;

    // neighbour lists (reference positions kept in registers)
    double rref[BPT][3];
    int cnt[BPT];
    int builds = 1;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        cnt[k] = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) rref[k][c] = r[k][c];
        if (!own[k]) continue;
        cnt[k] = build_list<Real, G, PERIODIC>(i, n, BN[i] != 0, i > 0 && BN[i - 1] != 0, r[k], P, P + nmax,
                                               P + 2 * nmax, per, nd, rl2, gl, lists + i, lstride);
    }
    __syncthreads();
    // Beads on one node at the start of the step are closer than sqrt(3) < rc, so they
    // are bonded neighbours or in this list: flag whether a bead shares its node and
    // whether a lower-index bead does (then it is not the node's leader).
    bool shared[BPT], before[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        int sh = 0, bf = 0;
        if (own[k] && node[k] >= 0) {
            const bool ovf = cnt[k] > kNeighbourMax;
            const int lim = ovf ? n : cnt[k] + 2;
            for (int q = gl; q < lim; q += G) {
                int j;
                if (ovf) j = q;
                else if (q < cnt[k]) j = lists[i + q * lstride];
                else j = (q == cnt[k]) ? i - 1 : i + 1;
                if (j < 0 || j >= n || j == i || NODE[j] != node[k]) continue;
                sh = 1;
                if (j < i) bf = 1;
            }
        }
        shared[k] = group_sum<G>(sh) != 0;
        before[k] = group_sum<G>(bf) != 0;
    }

    for (int sub = 0; sub < M; ++sub) {
        const double* PX = P + cur * 3 * nmax;
        const double* PY = PX + nmax;
        const double* PZ = PY + nmax;
        double* QX = P + (cur ^ 1) * 3 * nmax;
        Real F[BPT][3];
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            F[k][0] = F[k][1] = F[k][2] = 0;
            if (!own[k]) continue;
            const bool bn = BN[i] != 0;
            const bool bp = i > 0 && BN[i - 1] != 0;
            // WCA against the Verlet neighbours (all pairs if the list overflowed)
            Real fx = 0, fy = 0, fz = 0;
            const bool overflow = cnt[k] > kNeighbourMax;
            const int lim = overflow ? n : cnt[k];
            const unsigned short* li = lists + i;
            for (int q = gl; q < lim; q += G) {
                int j;
                if (overflow) {
                    j = q;
                    if (j == i || (j == i + 1 && bn) || (j == i - 1 && bp)) continue;
                } else {
                    j = li[q * lstride];
                }
                Real d[3];
                const Real r2 = separation<Real, PERIODIC>(r[k], PX, PY, PZ, j, per, nd, d);
                if (r2 < rc2) {
                    const Real ir2 = fast_rcp<Real>(r2);
                    const Real s2 = sig2 * ir2;
                    const Real s6 = s2 * s2 * s2;
                    const Real c = eps24 * (Real(2) * s6 * s6 - s6) * ir2;
                    fx += c * d[0];
                    fy += c * d[1];
                    fz += c * d[2];
                }
            }
            F[k][0] = group_sum<G>(fx);
            F[k][1] = group_sum<G>(fy);
            F[k][2] = group_sum<G>(fz);
            // harmonic bonds to the chain neighbours
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool on = side == 0 ? bp : bn;
                if (!on) continue;
                const int j = side == 0 ? i - 1 : i + 1;
                Real d[3];
                const Real len = sqrt(separation<Real, PERIODIC>(r[k], PX, PY, PZ, j, per, nd, d));
                if (len > Real(2) * r0) flags |= LB_ERR_BOND_STRETCH;
                // d points from j to i: the bond pulls i towards j when stretched
                const Real coef = -kb * (len - r0) * fast_rcp<Real>(len);
#pragma unroll
                for (int c = 0; c < 3; ++c) F[k][c] += coef * d[c];
            }
            // nearest solid surface (only near a wall)
            if (!(isfinite(r[k][0]) && isfinite(r[k][1]) && isfinite(r[k][2]))) flags |= LB_ERR_NONFINITE;
            bool near_wall = false;
#pragma unroll
            for (int w = 0; w < LB_MAX_WALLS; ++w) {
                if (w >= GM.n_walls) break;
                near_wall = near_wall || (r[k][0] > GM.wall[w][0] - 0.5 - rcw && r[k][0] < GM.wall[w][1] + 0.5 + rcw);
            }
            if (near_wall) {
                double dv[3];
                const double dist = geom_wall_distance<PERIODIC>(GM, r[k], dv);
                if (dist == 0.0) {
                    flags |= LB_ERR_BEAD_IN_SOLID;
                } else {
                    const Real c = wca_coef<Real>((Real)(dist * dist), epsw, sigw2, rcw2);
#pragma unroll
                    for (int q = 0; q < 3; ++q) F[k][q] += c * (Real)dv[q];
                }
            }
            // free-slip faces at -1/2 and n - 1/2
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!GM.fs[c]) continue;
                const Real dlo = (Real)(r[k][c] + 0.5), dhi = (Real)((nn[c] - 0.5) - r[k][c]);
                if (!(dlo > Real(0)) || !(dhi > Real(0))) {
                    flags |= LB_ERR_BEAD_OUTSIDE;
                    continue;
                }
                F[k][c] += wca_coef<Real>(dlo * dlo, epsw, sigw2, rcw2) * dlo;
                F[k][c] -= wca_coef<Real>(dhi * dhi, epsw, sigw2, rcw2) * dhi;
            }
            // pulling force on beads whose nearest node is a pore node
            int g[3];
            geom_ngp<PERIODIC>(GM, r[k], g);
            if (geom_is_pore(GM, g)) F[k][0] += fdrive;
            // drag against the frozen fluid velocity and the random force
            const U4 rnd = philox4x32_10(U4{(uint32_t)i, (uint32_t)step, (uint32_t)sub, 1u}, seed_lo, seed_hi);
            const uint32_t rr[3] = {rnd.x, rnd.y, rnd.z};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const Real drag = -mg * (v[k][c] - u[k][c]);
                const Real noise = A * centred_uniform<Real>(rr[c]);
                F[k][c] += drag + noise;
                fb[k][c] += (drag + noise) * invM;
            }
        }
        // kick-drift into the other position buffer; the single barrier below both
        // publishes the new positions and votes on a list rebuild
        int moved = 0;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            if (!own[k]) continue;
            Real disp2 = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[k][c] += hm * F[k][c];
                r[k][c] += (double)(h * v[k][c]);
                const Real dd = (Real)(r[k][c] - rref[k][c]);
                disp2 += dd * dd;
            }
            moved |= !(disp2 <= hs2);  // also catches a non-finite position
            if (gl == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) QX[c * nmax + i] = r[k][c];
            }
        }
        cur ^= 1;
        if (__syncthreads_or(moved) && sub + 1 < M) {
            ++builds;
            const double* NX = P + cur * 3 * nmax;
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const int i = grp + k * NG;
#pragma unroll
                for (int c = 0; c < 3; ++c) rref[k][c] = r[k][c];
                if (!own[k]) continue;
                cnt[k] = build_list<Real, G, PERIODIC>(i, n, BN[i] != 0, i > 0 && BN[i - 1] != 0, r[k], NX,
                                                       NX + nmax, NX + 2 * nmax, per, nd, rl2, gl, lists + i,
                                                       lstride);
            }
            __syncthreads();
        }
    }

    // write back, translocation count, centre of mass
    double acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        if (!own[k] || gl != 0) continue;
        const int gi = b0 + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a.b.r[c * NT + gi] = r[k][c];
            a.b.v[c * NT + gi] = v[k][c];
            a.b.fbar[c * NT + gi] = fb[k][c];
        }
        acc[0] += r[k][0] > xmid ? 1.0 : 0.0;
        acc[1] += r[k][0];
        acc[2] += r[k][1];
        acc[3] += r[k][2];
    }
    block_sums<Real>(acc, 4, red);

    // one leader per occupied node (its lowest-index bead) sums the Fbar of the beads on
    // it in index order; a bead alone on its node is its own sum
    double* FX = P;  // positions are no longer needed
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        if (!own[k] || gl != 0) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) FX[c * nmax + i] = (double)fb[k][c];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        if (!own[k]) continue;
        const int me = node[k];
        const bool lead = me >= 0 && !before[k];
        Real s[3] = {fb[k][0], fb[k][1], fb[k][2]};
        if (lead && shared[k]) {
            Real t[3] = {0, 0, 0};
            for (int j = i + 1 + gl; j < n; j += G)
                if (NODE[j] == me) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) t[c] += (Real)FX[c * nmax + j];
                }
#pragma unroll
            for (int c = 0; c < 3; ++c) s[c] += group_sum<G>(t[c]);
        }
        if (gl == 0) {
            const int gi = b0 + i;
            a.b.agg_node[gi] = lead ? me : -1;
#pragma unroll
            for (int c = 0; c < 3; ++c) a.b.agg_f[c * NT + gi] = lead ? s[c] : Real(0);
        }
    }
    if (tid == 0) {
        double* dg = a.b.diag + 8 * blockIdx.x;
        dg[0] = acc[0];
        if (dg[1] < 0.0 && (int)acc[0] == n) dg[1] = (double)(step + 1);
        dg[2] = acc[1] / n;
        dg[3] = acc[2] / n;
        dg[4] = acc[3] / n;
        dg[5] = (double)(step + 1);
        dg[6] += (double)builds;
    }
    if (flags) atomicOr(&a.st->err, flags);
}

template <int S>
__global__ __launch_bounds__(256) void k_spread(const Replica* __restrict__ reps,
                                                BeadPtrs<typename MDReal<S>::type> b,
                                                typename Codec<S>::T* __restrict__ dst, RunState* st,
                                                int bump_step) {
    using C = Codec<S>;
    using Rl = typename C::R;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (bump_step && i == 0) st->step += 1;
    if (i >= b.ntot) return;
    const int node = b.agg_node[i];
    if (node < 0) return;
    const Replica& R = reps[b.rep_of[i]];
    const Rl F[3] = {(Rl)b.agg_f[i], (Rl)b.agg_f[b.ntot + i], (Rl)b.agg_f[2 * b.ntot + i]};
    typename C::T* __restrict__ base = dst + R.pop_base + node;
    const long long V = R.V;
    // all 18 moving populations are read before any is written
    Rl f[Q];
    md_for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (p != 0) f[p] = C::template load<p>(base[(long long)p * V]);
    });
    md_for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (p != 0) {
            Rl fc = 0;
            if constexpr (cx_of(p) != 0) fc += Rl(cx_of(p)) * F[0];
            if constexpr (cy_of(p) != 0) fc += Rl(cy_of(p)) * F[1];
            if constexpr (cz_of(p) != 0) fc += Rl(cz_of(p)) * F[2];
            // S_p = -(w_p / c_s^2) Fbar . c_p with c_s^2 = 1/3
            base[(long long)p * V] = C::template store<p>(f[p] - Rl(3) * w_of<Rl>(p) * fc);
        }
    });
}

__global__ void k_bump(RunState* st) { st->step += 1; }

// ---------------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------------
static int md_nmax(const Context& c) { return (c.max_beads + 63) / 64 * 64; }

// Verlet lists go to LDS when positions (two buffers), node/bond arrays and lists fit
static bool md_lists_in_lds(const Context& c) {
    const size_t nmax = (size_t)md_nmax(c);
    return nmax * (6 * sizeof(double) + sizeof(int) + 1 + kNeighbourMax * sizeof(unsigned short)) <= 150 * 1024;
}

size_t md_lds_bytes(const Context& c) {
    const size_t nmax = (size_t)md_nmax(c);
    size_t b = nmax * (6 * sizeof(double) + sizeof(int) + 1);
    if (md_lists_in_lds(c)) b += nmax * kNeighbourMax * sizeof(unsigned short);
    return b;
}

template <class Real, int G, int BPT, bool PER, int MAXT>
static hipError_t launch_md_t(const Context& c, const void* cur, int mode, int block, hipStream_t s) {
    MDKArgs<Real> a;
    a.reps = c.d_reps;
    a.md = c.md;
    a.b = *(const BeadPtrs<Real>*)c.bead_ptrs;
    a.cur = cur;
    a.st = c.d_state;
    a.mode = mode;
    a.nmax = md_nmax(c);
    a.list_in_lds = md_lists_in_lds(c) ? 1 : 0;
    const size_t lds = md_lds_bytes(c);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_md<Real, G, BPT, PER, MAXT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_md<Real, G, BPT, PER, MAXT>), dim3((unsigned)c.reps.size()), dim3(block), lds, s, a,
                       c.storage);
    return hipGetLastError();
}

template <class Real, bool PER>
static hipError_t launch_md_g(const Context& c, const void* cur, int mode, hipStream_t s) {
    // lanes per bead: up to ~512 threads, so that each SIMD has two waves to interleave
    // (measured faster than one wave per SIMD for 100 beads, although the per-bead work
    // is repeated by every lane of a group); beyond 256 beads one lane per bead, beyond
    // 512 the 1024-thread bound, beyond 1024 up to 4 beads per lane
    const int m = std::max(c.max_beads, 1);
    auto blk = [](int t) { return std::min(1024, (t + 63) / 64 * 64); };
    if (m <= 32) return launch_md_t<Real, 16, 1, PER, 512>(c, cur, mode, blk(16 * m), s);
    if (m <= 64) return launch_md_t<Real, 8, 1, PER, 512>(c, cur, mode, blk(8 * m), s);
    if (m <= 128) return launch_md_t<Real, 4, 1, PER, 512>(c, cur, mode, blk(4 * m), s);
    if (m <= 256) return launch_md_t<Real, 2, 1, PER, 512>(c, cur, mode, blk(2 * m), s);
    if (m <= 512) return launch_md_t<Real, 1, 1, PER, 512>(c, cur, mode, blk(m), s);
    if (m <= 1024) return launch_md_t<Real, 1, 1, PER, 1024>(c, cur, mode, blk(m), s);
    if (m <= 2048) return launch_md_t<Real, 1, 2, PER, 1024>(c, cur, mode, 1024, s);
    if (m <= 3072) return launch_md_t<Real, 1, 3, PER, 1024>(c, cur, mode, 1024, s);
    if (m <= 4096) return launch_md_t<Real, 1, 4, PER, 1024>(c, cur, mode, 1024, s);
    return hipErrorInvalidValue;
}

template <class Real>
static hipError_t launch_md_r(const Context& c, const void* cur, int mode, hipStream_t s) {
    bool any_periodic = false;
    for (const Replica& R : c.reps)
        if (R.n_beads > 0 && (!R.fs[0] || !R.fs[1] || !R.fs[2])) any_periodic = true;
    return any_periodic ? launch_md_g<Real, true>(c, cur, mode, s) : launch_md_g<Real, false>(c, cur, mode, s);
}

hipError_t launch_md(const Context& c, const void* cur, int mode, hipStream_t s) {
    if (c.storage == LB_STORE_F64) return launch_md_r<double>(c, cur, mode, s);
    return launch_md_r<float>(c, cur, mode, s);
}

template <int S>
static hipError_t launch_spread_t(const Context& c, void* dst, bool bump, hipStream_t s) {
    using Real = typename MDReal<S>::type;
    const BeadPtrs<Real> b = *(const BeadPtrs<Real>*)c.bead_ptrs;
    const int grid = (c.ntot_beads + 255) / 256;
    hipLaunchKernelGGL((k_spread<S>), dim3(grid > 0 ? grid : 1), dim3(256), 0, s, c.d_reps, b,
                       (typename Codec<S>::T*)dst, c.d_state, bump ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_spread(const Context& c, void* dst, bool bump, hipStream_t s) {
    switch (c.storage) {
        case LB_STORE_F64: return launch_spread_t<LB_STORE_F64>(c, dst, bump, s);
        case LB_STORE_F32: return launch_spread_t<LB_STORE_F32>(c, dst, bump, s);
        case LB_STORE_F16DEV: return launch_spread_t<LB_STORE_F16DEV>(c, dst, bump, s);
        case LB_STORE_BF16DEV: return launch_spread_t<LB_STORE_BF16DEV>(c, dst, bump, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bump(const Context& c, hipStream_t s) {
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(1), 0, s, c.d_state);
    return hipGetLastError();
}

}  // namespace lbmd
