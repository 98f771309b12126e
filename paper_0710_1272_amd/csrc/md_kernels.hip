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
    double best = HUGE_VAL;
    dv[0] = dv[1] = dv[2] = 0.0;
    for (int k = 0; k < R.n_walls; ++k) {
        const int* w = R.wall[k];
        const double X0 = w[0] - 0.5, X1 = w[1] + 0.5;
        const bool open = pore_open(w);
        const double Y0 = w[2] - 0.5, Y1 = w[3] + 0.5, Z0 = w[4] - 0.5, Z1 = w[5] + 0.5;
        const int nb = open ? 4 : 1;
        for (int m = 0; m < nb; ++m) {
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
            const double dist = sqrt(d2);
            if (dist < best) {
                best = dist;
                dv[0] = d[0];
                dv[1] = d[1];
                dv[2] = d[2];
            }
        }
    }
    return best;
}

// -(1/r) dV/dr of WCA at squared distance r2 (0 beyond the cutoff)
template <class Real>
__device__ __forceinline__ Real wca_coef(Real r2, Real eps, Real sig2, Real rc2) {
    if (!(r2 < rc2)) return Real(0);
    const Real s2 = sig2 / r2;
    const Real s6 = s2 * s2 * s2;
    return Real(24) * eps * (Real(2) * s6 * s6 - s6) / r2;
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

// Each bead is owned by a group of G lanes that split its partner loop; every lane
// of the group keeps the bead's state, so the per-bead terms are computed
// redundantly without divergence.  BPT beads per group when there are more beads
// than groups (then G = 1).
template <class Real, int BLOCK, int G, int BPT, bool PERIODIC>
__global__ __launch_bounds__(BLOCK) void k_md(MDKArgs<Real> a, int storage) {
    extern __shared__ double lds[];
    __shared__ double red[16 * 4];
    constexpr int NG = BLOCK / G;  // groups per block
    const Replica& R = a.reps[blockIdx.x];
    const int n = R.n_beads;
    if (n == 0) return;
    const int b0 = R.bead0, NT = a.b.ntot, tid = threadIdx.x;
    const int grp = tid / G, gl = tid % G;
    double* PX = lds;
    double* PY = PX + a.nmax;
    double* PZ = PY + a.nmax;
    int* NODE = (int*)(PZ + a.nmax);
    unsigned char* BN = (unsigned char*)(NODE + a.nmax);
    const MDDev& md = a.md;
    const long long step = a.st->step;
    const int nn[3] = {R.nx, R.ny, R.nz};
    const double nd[3] = {(double)R.nx, (double)R.ny, (double)R.nz};
    const int per[3] = {R.fs[0] ? 0 : 1, R.fs[1] ? 0 : 1, R.fs[2] ? 0 : 1};
    unsigned flags = 0;

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
                PX[i] = r[k][0];
                PY[i] = r[k][1];
                PZ[i] = r[k][2];
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

    const Real h = (Real)md.h, hm = (Real)(md.h * md.inv_mass), invM = (Real)md.inv_M;
    const Real mg = (Real)(md.mass * md.gamma), A = (Real)md.A;
    const Real kb = (Real)md.k_bond, r0 = (Real)md.r0;
    const Real eps24 = (Real)(24.0 * md.eps), sig2 = (Real)md.sigma2, rc2 = (Real)md.rc2;
    const Real epsw = (Real)md.eps_w, sigw2 = (Real)md.sigma_w2, rcw2 = (Real)md.rcw2;
    const Real fdrive = (Real)md.f_drive;

    for (int sub = 0; sub < md.M; ++sub) {
        Real F[BPT][3];
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            F[k][0] = F[k][1] = F[k][2] = 0;
            if (!own[k]) continue;
            const bool bn = BN[i] != 0;
            const bool bp = i > 0 && BN[i - 1] != 0;
            // WCA against every non-bonded bead: this lane takes j = gl, gl + G, ...
            Real fx = 0, fy = 0, fz = 0;
            for (int j = gl; j < n; j += G) {
                if (j == i || (j == i + 1 && bn) || (j == i - 1 && bp)) continue;
                double ddx = r[k][0] - PX[j], ddy = r[k][1] - PY[j], ddz = r[k][2] - PZ[j];
                if constexpr (PERIODIC) {
                    if (per[0]) ddx -= nd[0] * floor(ddx / nd[0] + 0.5);
                    if (per[1]) ddy -= nd[1] * floor(ddy / nd[1] + 0.5);
                    if (per[2]) ddz -= nd[2] * floor(ddz / nd[2] + 0.5);
                }
                const Real dx = (Real)ddx, dy = (Real)ddy, dz = (Real)ddz;
                const Real r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < rc2) {
                    const Real ir2 = Real(1) / r2;
                    const Real s2 = sig2 * ir2;
                    const Real s6 = s2 * s2 * s2;
                    const Real c = eps24 * (Real(2) * s6 * s6 - s6) * ir2;
                    fx += c * dx;
                    fy += c * dy;
                    fz += c * dz;
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
                double dd[3] = {PX[j] - r[k][0], PY[j] - r[k][1], PZ[j] - r[k][2]};
                if constexpr (PERIODIC) {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        if (per[c]) dd[c] -= nd[c] * floor(dd[c] / nd[c] + 0.5);
                }
                const Real d[3] = {(Real)dd[0], (Real)dd[1], (Real)dd[2]};
                const Real len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (len > Real(2) * r0) flags |= LB_ERR_BOND_STRETCH;
                const Real coef = kb * (len - r0) / len;
#pragma unroll
                for (int c = 0; c < 3; ++c) F[k][c] += coef * d[c];
            }
            // nearest solid surface
            if (!(isfinite(r[k][0]) && isfinite(r[k][1]) && isfinite(r[k][2]))) flags |= LB_ERR_NONFINITE;
            if (R.n_walls > 0) {
                double dv[3];
                const double dist = wall_distance(R, r[k], dv);
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
                if (!R.fs[c]) continue;
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
            ngp3(R, r[k], g);
            if (is_pore(R, g[0], g[1], g[2])) F[k][0] += fdrive;
            // drag against the frozen fluid velocity and the random force
            const U4 rnd = philox4x32_10(U4{(uint32_t)i, (uint32_t)step, (uint32_t)sub, 1u}, R.seed_lo,
                                         R.seed_hi);
            const uint32_t rr[3] = {rnd.x, rnd.y, rnd.z};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const Real drag = -mg * (v[k][c] - u[k][c]);
                const Real noise = A * centred_uniform<Real>(rr[c]);
                F[k][c] += drag + noise;
                fb[k][c] += (drag + noise) * invM;
            }
        }
        __syncthreads();  // every read of the old positions is done
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            if (!own[k]) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[k][c] += hm * F[k][c];
                r[k][c] += (double)(h * v[k][c]);
            }
            if (gl == 0) {
                PX[i] = r[k][0];
                PY[i] = r[k][1];
                PZ[i] = r[k][2];
            }
        }
        __syncthreads();
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
        acc[0] += r[k][0] > R.xmid ? 1.0 : 0.0;
        acc[1] += r[k][0];
        acc[2] += r[k][1];
        acc[3] += r[k][2];
    }
    block_sums<Real>(acc, 4, red);

    // one leader per occupied node (its lowest-index bead) sums the Fbar of the beads on it
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        if (!own[k] || gl != 0) continue;
        NODE[i] = node[k];
        PX[i] = (double)fb[k][0];
        PY[i] = (double)fb[k][1];
        PZ[i] = (double)fb[k][2];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        if (!own[k]) continue;
        const int me = node[k];
        int before = 0;
        Real s[3] = {0, 0, 0};
        if (me >= 0) {
            for (int j = gl; j < n; j += G) {
                if (NODE[j] != me) continue;
                if (j < i) {
                    before = 1;
                } else {
                    s[0] += (Real)PX[j];
                    s[1] += (Real)PY[j];
                    s[2] += (Real)PZ[j];
                }
            }
        }
        before = group_sum<G>(before);
        s[0] = group_sum<G>(s[0]);
        s[1] = group_sum<G>(s[1]);
        s[2] = group_sum<G>(s[2]);
        if (gl == 0) {
            const int gi = b0 + i;
            a.b.agg_node[gi] = (me >= 0 && before == 0) ? me : -1;
#pragma unroll
            for (int c = 0; c < 3; ++c) a.b.agg_f[c * NT + gi] = s[c];
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
size_t md_lds_bytes(const Context& c) {
    const size_t nmax = (size_t)((c.max_beads + 63) / 64 * 64);
    return nmax * (3 * sizeof(double) + sizeof(int) + 1);
}

template <class Real, int G, int BPT, bool PER>
static hipError_t launch_md_t(const Context& c, const void* cur, int mode, hipStream_t s) {
    MDKArgs<Real> a;
    a.reps = c.d_reps;
    a.md = c.md;
    a.b = *(const BeadPtrs<Real>*)c.bead_ptrs;
    a.cur = cur;
    a.st = c.d_state;
    a.mode = mode;
    a.nmax = (c.max_beads + 63) / 64 * 64;
    const size_t lds = md_lds_bytes(c);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_md<Real, 1024, G, BPT, PER>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_md<Real, 1024, G, BPT, PER>), dim3((unsigned)c.reps.size()), dim3(1024), lds, s, a,
                       c.storage);
    return hipGetLastError();
}

template <class Real, bool PER>
static hipError_t launch_md_g(const Context& c, const void* cur, int mode, hipStream_t s) {
    // lanes per bead: as many as fit 1024 threads (at most 32); beyond 1024 beads,
    // one lane per bead and up to 4 beads per lane
    const int m = std::max(c.max_beads, 1);
    if (m <= 32) return launch_md_t<Real, 32, 1, PER>(c, cur, mode, s);
    if (m <= 64) return launch_md_t<Real, 16, 1, PER>(c, cur, mode, s);
    if (m <= 128) return launch_md_t<Real, 8, 1, PER>(c, cur, mode, s);
    if (m <= 256) return launch_md_t<Real, 4, 1, PER>(c, cur, mode, s);
    if (m <= 512) return launch_md_t<Real, 2, 1, PER>(c, cur, mode, s);
    if (m <= 1024) return launch_md_t<Real, 1, 1, PER>(c, cur, mode, s);
    if (m <= 2048) return launch_md_t<Real, 1, 2, PER>(c, cur, mode, s);
    if (m <= 4096) return launch_md_t<Real, 1, 4, PER>(c, cur, mode, s);
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
