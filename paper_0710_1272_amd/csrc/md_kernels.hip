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
    int noise_in_lds;  // random forces of all substeps tabulated in LDS at step start
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

// Whether the nearest node floor(r + 1/2) of r is a node of wall w's pore.  On a
// free-slip axis floor(t) in [lo, hi] is decided as lo <= t < hi + 1 on the same rounded
// t = r + 1/2, with the index clamping into the box kept (a bound on the box face always
// holds); a periodic axis wraps the index as the node lookup does.
template <bool PERIODIC>
__device__ __forceinline__ bool wall_pore_node(const Geom& G, const int* w, const double* r) {
    if (!pore_open(w)) return false;
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int lo = w[2 * a], hi = w[2 * a + 1];
        const double t = r[a] + 0.5;
        if (PERIODIC && !G.fs[a]) {
            double f = floor(t);
            if (!(f >= -1e9 && f <= 1e9)) f = 0.0;  // non-finite or absurd
            int k = (int)f % G.n[a];
            if (k < 0) k += G.n[a];
            in = in && k >= lo && k <= hi;
        } else {
            in = in && (lo <= 0 || t >= (double)lo) && (hi >= G.n[a] - 1 || t < (double)(hi + 1));
        }
    }
    return in;
}

// Squared distance from r to the nearest solid surface of wall w, and the vector from
// that surface point to r (xw: x wrapped into the box on a periodic axis).  Solid node
// cubes span [i - 1/2, i + 1/2], so a wall is its slab X0..X1 minus the pore prism
// Y0..Y1 x Z0..Z1.  Outside the prism (in y, z) the nearest solid point lies straight
// along x, on the slab; inside it, on the nearest of the four prism sides, at x clamped
// into the slab.  Ties go to the sides in the order y-low, y-high, z-low, z-high.
template <bool PERIODIC>
__device__ __forceinline__ double wall_dist2(const Geom& G, const int* w, const double* rin, double xw,
                                             double* dv) {
    double ry = rin[1], rz = rin[2];
    if (PERIODIC && !G.fs[1]) ry -= G.n[1] * floor((ry + 0.5) / G.n[1]);
    if (PERIODIC && !G.fs[2]) rz -= G.n[2] * floor((rz + 0.5) / G.n[2]);
    const double X0 = w[0] - 0.5, X1 = w[1] + 0.5;
    const double Y0 = w[2] - 0.5, Y1 = w[3] + 0.5, Z0 = w[4] - 0.5, Z1 = w[5] + 0.5;
    const double dx = xw - fmin(fmax(xw, X0), X1);
    double dy = 0.0, dz = 0.0;
    if (pore_open(w) && ry >= Y0 && ry <= Y1 && rz >= Z0 && rz <= Z1) {
        double side = ry - Y0;
        dy = side;
        double t = Y1 - ry;
        if (t < side) { side = t; dy = -t; }
        t = rz - Z0;
        if (t < side) { side = t; dy = 0.0; dz = t; }
        t = Z1 - rz;
        if (t < side) { side = t; dy = 0.0; dz = -t; }
    }
    dv[0] = dx;
    dv[1] = dy;
    dv[2] = dz;
    return dx * dx + dy * dy + dz * dz;
}

// 1/x: the hardware reciprocal in FP32 (about 1 ulp), an exact division in FP64
template <class Real>
__device__ __forceinline__ Real fast_rcp(Real x) {
    if constexpr (sizeof(Real) == 4) return __builtin_amdgcn_rcpf(x);
    else return Real(1) / x;
}

// 1/sqrt(x): the hardware reciprocal square root in FP32 (about 1 ulp), sqrt and an
// exact division in FP64
template <class Real>
__device__ __forceinline__ Real fast_rsqrt(Real x) {
    if constexpr (sizeof(Real) == 4) return __builtin_amdgcn_rsqf(x);
    else return Real(1) / sqrt(x);
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
        Real fp = (Real)C::template load<p>(src[R.pop_base + (long long)q * R.S + s]);
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

// One DPP lane exchange (no LDS round trip): quad_perm [1,0,3,2] swaps neighbouring lanes,
// [2,3,0,1] swaps lane pairs, row_half_mirror reverses each group of 8 lanes, row_mirror
// each row of 16.
constexpr int kDppSwap1 = 0xB1, kDppSwap2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_x(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_x(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)(b & 0xFFFFFFFFll));
    const int hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ int dpp_x(int v) {
    return dpp_i<CTRL>(v);
}

// Sum over the G consecutive lanes of a group (G a power of two <= 64).  Each step adds
// the partial sum of the partner half, so every lane of the group ends with the same
// bits (a + b and b + a round alike): the redundant per-bead state of the group's
// lanes stays identical.
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
    if constexpr (G >= 2) v += dpp_x<kDppSwap1>(v);
    if constexpr (G >= 4) v += dpp_x<kDppSwap2>(v);
    if constexpr (G >= 8) v += dpp_x<kDppHalfMirror>(v);
    if constexpr (G >= 16) v += dpp_x<kDppMirror>(v);
    if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
    if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

// Pairwise separation r_i - r_j as FP32/FP64 components (minimum image on periodic
// axes) and its square.
template <class Real, bool PERIODIC>
__device__ __forceinline__ Real separation_v(const double* ri, const double* pj, const int* per,
                                             const double* nd, Real* d) {
    double dd[3] = {ri[0] - pj[0], ri[1] - pj[1], ri[2] - pj[2]};
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

template <class Real, bool PERIODIC>
__device__ __forceinline__ Real separation(const double* ri, const double* PX, const double* PY,
                                           const double* PZ, int j, const int* per, const double* nd,
                                           Real* d) {
    const double pj[3] = {PX[j], PY[j], PZ[j]};
    return separation_v<Real, PERIODIC>(ri, pj, per, nd, d);
}

// Angular term of Sec. II at the middle bead of (a, b, c): V = kappa phi^2 / 2 with phi
// the angle between the consecutive bonds d1 = r_b - r_a and d2 = r_c - r_b (0 for a
// straight chain).  With cos(phi) = d1.d2 / (|d1||d2|), the forces are
// f_a = -kappa (phi / sin phi) dcos/dd1, f_c = kappa (phi / sin phi) dcos/dd2, and the
// middle bead takes -(f_a + f_c); phi / sin phi -> 1 as phi -> 0.
template <class Real, bool PERIODIC>
__device__ __forceinline__ void angle_forces(const double* ra, const double* rb, const double* rc, const int* per,
                                             const double* nd, Real kappa, Real* fa, Real* fc) {
    Real d1[3], d2[3];
    const Real q1 = separation_v<Real, PERIODIC>(rb, ra, per, nd, d1);
    const Real q2 = separation_v<Real, PERIODIC>(rc, rb, per, nd, d2);
    const Real l1 = sqrt(q1), l2 = sqrt(q2);
    const Real dot = d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2];
    const Real cx = d1[1] * d2[2] - d1[2] * d2[1], cy = d1[2] * d2[0] - d1[0] * d2[2],
               cz = d1[0] * d2[1] - d1[1] * d2[0];
    const Real cross = sqrt(cx * cx + cy * cy + cz * cz);
    const Real phi = atan2(cross, dot);
    const Real il12 = Real(1) / (l1 * l2);
    const Real sn = cross * il12;
    const Real small = sizeof(Real) == 4 ? Real(1e-4) : Real(1e-8);
    const Real phi_over_sin = sn > small ? phi / sn : Real(1) + phi * phi / Real(6);
    const Real c = dot * il12;
    const Real kk = kappa * phi_over_sin;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        fa[a] = -kk * (d2[a] * il12 - c * d1[a] / q1);
        fc[a] = kk * (d1[a] * il12 - c * d2[a] / q2);
    }
}

// One tridiagonal system a_t x_{t-1} + b_t x_t + c_t x_{t+1} = d_t per workgroup, row t
// held by thread t (t < m), solved by parallel cyclic reduction: at stride s each row
// eliminates its couplings to rows t - s and t + s (rows outside 0..m-1 are identities),
// so after ceil(log2 m) levels x_t = d_t / b_t.  Each row publishes 1/b with a, c, d, so a
// level takes one division (the row's own new 1/b) instead of two.  Double-buffered in LDS
// (W: [2][4][nmax] doubles: a, 1/b, c, d); one barrier per level.  Every thread of the
// block must call it.
// With `vote`, the barrier after the first writes also returns whether any thread passed
// need = true in *any; without any, or with solve = false, no level runs and 0 is returned
// (a Newton step folds its convergence test into the solve that follows it this way).
__device__ __forceinline__ double pcr_solve(double* W, int nmax, int m, int t, double a, double b, double c,
                                            double d, bool vote = false, bool need = true, bool solve = true,
                                            bool* any = nullptr) {
    const bool row = t < m;
    int buf = 0;
    double ib = 1.0 / b;
    if (row) {
        W[(0 * 4 + 0) * nmax + t] = a;
        W[(0 * 4 + 1) * nmax + t] = ib;
        W[(0 * 4 + 2) * nmax + t] = c;
        W[(0 * 4 + 3) * nmax + t] = d;
    }
    if (vote) {
        const bool any_need = __syncthreads_or(need) != 0;
        *any = any_need;
        if (!any_need || !solve) return 0.0;
    } else {
        __syncthreads();
    }
    for (int s = 1; s < m; s <<= 1) {
        const double* Ws = W + buf * 4 * nmax;
        double* Wd = W + (buf ^ 1) * 4 * nmax;
        if (row) {
            const int lo = t - s, hi = t + s;
            const double al = lo >= 0 ? Ws[lo] : 0.0, ibl = lo >= 0 ? Ws[nmax + lo] : 1.0;
            const double cl = lo >= 0 ? Ws[2 * nmax + lo] : 0.0, dl = lo >= 0 ? Ws[3 * nmax + lo] : 0.0;
            const double ah = hi < m ? Ws[hi] : 0.0, ibh = hi < m ? Ws[nmax + hi] : 1.0;
            const double ch = hi < m ? Ws[2 * nmax + hi] : 0.0, dh = hi < m ? Ws[3 * nmax + hi] : 0.0;
            const double k1 = a * ibl, k2 = c * ibh;
            const double na = -al * k1, nc = -ch * k2;
            b = b - cl * k1 - ah * k2;
            d = d - dl * k1 - dh * k2;
            a = na;
            c = nc;
            ib = 1.0 / b;
            Wd[t] = a;
            Wd[nmax + t] = ib;
            Wd[2 * nmax + t] = c;
            Wd[3 * nmax + t] = d;
        }
        buf ^= 1;
        __syncthreads();
    }
    return row ? d * ib : 0.0;
}

// Verlet-list entries each lane keeps in registers (slot s of lane gl is entry gl + s G);
// entries beyond them are read from the list
// (fewer under the 1024-thread bound, where registers are scarcer)
template <int G, int BPT, int MAXT>
struct SlotsPerLane {
    static constexpr int K = MAXT > 512 ? (BPT > 1 ? 1 : 2) : (BPT > 1 ? 4 : (G >= 8 ? 1 : 8 / G));
};

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
        // one pass: each lane marks its hits j = gl + m G in a mask of 64 W bits, then the
        // group places them by an exclusive prefix of counts.  m < n / G: at most
        // 512 / G^2 <= 128 for G >= 4 (lanes x beads <= 512) and 256 for G = 2 (up to 512
        // beads)
        constexpr int W = G == 2 ? 4 : 2;
        unsigned long long hit[W];
#pragma unroll
        for (int w = 0; w < W; ++w) hit[w] = 0ull;
        int mine = 0, m = 0;
        for (int j = gl; j < n; j += G, ++m) {
            if (j == i || (j == i + 1 && bn) || (j == i - 1 && bp)) continue;
            Real d[3];
            if (separation<Real, PERIODIC>(ri, PX, PY, PZ, j, per, nd, d) < rl2) {
                const unsigned long long bit = 1ull << (m & 63);
#pragma unroll
                for (int w = 0; w < W; ++w) hit[w] |= (m >> 6) == w ? bit : 0ull;
                ++mine;
            }
        }
        int incl = mine;
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            const int t = __shfl_up(incl, off, G);
            if (gl >= off) incl += t;
        }
        int pos = incl - mine;
        const int total = __shfl(incl, G - 1, G);
        if (total <= kNeighbourMax) {
#pragma unroll
            for (int w = 0; w < W; ++w) {
                unsigned long long h = hit[w];
                while (h) {
                    const int b = __builtin_ctzll(h);
                    h &= h - 1;
                    list[(size_t)(pos++) * stride] = (unsigned short)(gl + (64 * w + b) * G);
                }
            }
        }
        return total;
    }
}

// Each bead is owned by a group of G lanes that split its neighbour loop; every lane
// of the group keeps the bead's state, so the per-bead terms are computed redundantly
// without divergence.  BPT beads per group when there are more beads than groups
// (then G = 1).  WCA pairs come from a Verlet list (radius rc + skin), kept across LB
// steps and rebuilt whenever a bead has moved skin/2 since the last build, so the set
// of interacting pairs is exactly that of the all-pairs definition.
// Positions are double-buffered in LDS: one barrier per substep.  POLY compiles in the
// angular term and rigid bonds (the kernel without them is the harmonic-chain model).
template <class Real, int G, int BPT, bool PERIODIC, int MAXT, bool POLY>
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
    // random forces [M][3][nmax], after the lists (or after BN when the lists are global)
    Real* NZ = (Real*)(a.list_in_lds ? (unsigned char*)(BN + nmax) + (size_t)kNeighbourMax * nmax * 2
                                     : (unsigned char*)(BN + nmax));
    const bool noise_lds = G > 1 && a.noise_in_lds;
    const MDDev md = a.md;
    // rigid bonds: SHAKE/RATTLE work area after the random-force table, doubles:
    // reference bond vectors [3][nmax], multipliers [nmax], velocities [3][nmax], and
    // the cyclic-reduction buffers [2][4][nmax]
    double* RW = (double*)((unsigned char*)NZ +
                           (noise_lds ? (size_t)md.M * 3 * nmax * sizeof(Real) : (size_t)0));
    double* SDV = RW;
    double* LAM = RW + 3 * nmax;
    double* VXV = RW + 4 * nmax;
    double* PCRW = RW + 7 * nmax;
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
    // the kept Verlet list's state (the positions it was built at, its length, whether it is
    // valid) does not depend on this step's positions: with one bead per lane it is fetched in
    // the same round trip as the bead state instead of after the interpolation
    double* dg = a.b.diag + 8 * blockIdx.x;
    const double kept = dg[7];
    double pre_rref[BPT][3];
    int pre_cnt[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        own[k] = i < n;
        node[k] = -1;
        pre_cnt[k] = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) { r[k][c] = 0; v[k][c] = 0; u[k][c] = 0; fb[k][c] = 0; pre_rref[k][c] = 0; }
        if (own[k]) {
            const int g = b0 + i;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                r[k][c] = a.b.r[c * NT + g];
                v[k][c] = a.b.v[c * NT + g];
            }
            if constexpr (BPT == 1) {
                if (kept != 0.0) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) pre_rref[k][c] = a.b.rref[c * NT + g];
                    pre_cnt[k] = a.b.ncount[g];
                }
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
    } else if (!(a.mode & MD_NO_HYDRO)) {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            if (!own[k]) continue;
            node[k] = a.b.node[b0 + i];
#pragma unroll
            for (int c = 0; c < 3; ++c) u[k][c] = a.b.u[c * NT + b0 + i];
        }
    }  // without hydrodynamics: u = 0 and no node (nothing is spread)
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
    // beyond this distance from a face the face WCA term is zero (a margin over the cutoff
    // keeps the skipped terms zero under any rounding of the distance)
    const Real rcw_gate = (Real)(md.rcw + 1e-3);
    const Real rl2 = (Real)md.rl2, hs2 = (Real)md.half_skin2;
    const Real fdrive = (Real)md.f_drive;

    // Verlet lists: kept from the previous launch (stored with the positions they were
    // built at) unless a bead has moved skin/2 since, else rebuilt here
    double rref[BPT][3];
    int cnt[BPT];
    int builds = 0;
    bool reuse = kept != 0.0;
    if (reuse) {
        int moved = 0;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int gi = b0 + grp + k * NG;
            cnt[k] = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) rref[k][c] = r[k][c];
            if (!own[k]) continue;
            Real disp2 = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                rref[k][c] = BPT == 1 ? pre_rref[k][c] : a.b.rref[c * NT + gi];
                const Real dd = (Real)(r[k][c] - rref[k][c]);
                disp2 += dd * dd;
            }
            moved |= !(disp2 <= hs2);
            cnt[k] = BPT == 1 ? pre_cnt[k] : a.b.ncount[gi];
        }
        reuse = !__syncthreads_or(moved);
    }
    if (reuse) {
        if (a.list_in_lds) {
            // the kept list into LDS, 8 entries a lane per round trip (a load and its LDS
            // store per entry would make every entry a dependent round trip)
            constexpr int U = 8;
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const int i = grp + k * NG;
                if (!own[k]) continue;
                const int m = cnt[k] < kNeighbourMax ? cnt[k] : kNeighbourMax;
                for (int q0 = gl; q0 < m; q0 += U * G) {
                    unsigned short e[U];
#pragma unroll
                    for (int t = 0; t < U; ++t) {
                        const int q = q0 + t * G;
                        e[t] = q < m ? a.b.nlist[(size_t)q * NT + b0 + i] : (unsigned short)0;
                    }
#pragma unroll
                    for (int t = 0; t < U; ++t) {
                        const int q = q0 + t * G;
                        if (q < m) lists[i + q * lstride] = e[t];
                    }
                }
            }
        }
    } else {
        builds = 1;
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
    }
    if (noise_lds) {
        // the G lanes of a bead share its M Philox draws instead of each lane drawing all
        // of them; the table is read from the next barrier on
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            if (!own[k]) continue;
            for (int s = gl; s < M; s += G) {
                const U4 rnd = philox4x32_10(U4{(uint32_t)i, (uint32_t)step, (uint32_t)s, 1u}, seed_lo, seed_hi);
                NZ[(3 * s + 0) * nmax + i] = A * centred_uniform<Real>(rnd.x);
                NZ[(3 * s + 1) * nmax + i] = A * centred_uniform<Real>(rnd.y);
                NZ[(3 * s + 2) * nmax + i] = A * centred_uniform<Real>(rnd.z);
            }
        }
    }
    __syncthreads();
    // Flag whether a bead shares its node and whether a lower-index bead does (then it is
    // not the node's leader).  Beads on one node lie in its unit cell, at most sqrt(3) apart:
    // when the WCA cutoff rc covers that, they are bonded neighbours or in this list (which
    // holds every non-bonded pair closer than rc); otherwise every bead's node is scanned.
    bool shared[BPT], before[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        int sh = 0, bf = 0;
        if (own[k] && node[k] >= 0) {
            const bool ovf = cnt[k] > kNeighbourMax;
            const bool all = ovf || md.node_scan_all;
            const int lim = all ? n : cnt[k] + 2;
            for (int q = gl; q < lim; q += G) {
                int j;
                if (all) j = q;
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

    // chain neighbours (constant over the step) and the register slots of the lists
    bool bnk[BPT], bpk[BPT], bnn[BPT], bpp[BPT];  // bonded to i+1, i-1, and i+1 to i+2, i-1 to i-2
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int i = grp + k * NG;
        bnk[k] = own[k] && BN[i] != 0;
        bpk[k] = own[k] && i > 0 && BN[i - 1] != 0;
        bnn[k] = bnk[k] && BN[i + 1] != 0;
        bpp[k] = bpk[k] && i > 1 && BN[i - 2] != 0;
    }
    // rigid chains (at most 512 beads, one bond row per thread) only run with one bead per group
    const bool rigid = POLY && BPT == 1 && md.rigid != 0;
    const Real kappa = POLY ? (Real)md.kappa_phi : Real(0);
    constexpr int K = SlotsPerLane<G, BPT, MAXT>::K;
    int slot[BPT][K], nslot[BPT];
    // Beads within reach of a wall slab or a free-slip face.  Decided at each list build
    // with the margin skin/2: until the next build no bead moves farther than that, so a
    // bead outside these zones needs none of the wall, pore or face terms (all zero) and
    // cannot have left the box.
    const bool x_periodic = PERIODIC && !GM.fs[0];
    const double zone = md.rcw + sqrt(md.half_skin2) + 1e-3;
    bool nearw[BPT], nearf[BPT];
    auto load_slots = [&]() {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            const double xw = x_periodic ? r[k][0] - nd[0] * floor((r[k][0] + 0.5) / nd[0]) : r[k][0];
            bool w_near = false, f_near = false;
#pragma unroll
            for (int w = 0; w < LB_MAX_WALLS; ++w) {
                if (w >= GM.n_walls) break;
                w_near = w_near || (xw > GM.wall[w][0] - 0.5 - zone && xw < GM.wall[w][1] + 0.5 + zone);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (GM.fs[c]) f_near = f_near || !(r[k][c] + 0.5 >= zone && (nn[c] - 0.5) - r[k][c] >= zone);
            nearw[k] = w_near;
            nearf[k] = f_near;
            nslot[k] = 0;
#pragma unroll
            for (int s = 0; s < K; ++s) {
                const int q = gl + s * G;
                slot[k][s] = own[k] ? i : 0;  // an unused slot reads the bead itself
                if (own[k] && cnt[k] <= kNeighbourMax && q < cnt[k]) {
                    slot[k][s] = lists[i + q * lstride];
                    ++nslot[k];
                }
            }
        }
    };
    load_slots();
    // rebuild vote: one flag per wave, double-buffered so that one barrier per substep
    // separates the writes of a substep from its reads and from the next substep's writes
    __shared__ __align__(16) unsigned char vote[2][16];
    const int wave = tid >> 6, n_waves = (blockDim.x + 63) >> 6;
    // flags of absent waves stay 0 (they are read whole, as 16 bytes, after each barrier;
    // no wave writes them, so clearing them here races with nothing)
    if (tid < 32 && (tid & 15) >= n_waves) vote[tid >> 4][tid & 15] = 0;

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
            // every position this substep reads, issued together: the register slots of
            // the Verlet list and the two chain neighbours (the bead itself when absent)
            double pj[K][3];
#pragma unroll
            for (int s = 0; s < K; ++s) {
                const int j = slot[k][s];
                pj[s][0] = PX[j];
                pj[s][1] = PY[j];
                pj[s][2] = PZ[j];
            }
            const int jm = bpk[k] ? i - 1 : i, jp = bnk[k] ? i + 1 : i;
            const double pm[3] = {PX[jm], PY[jm], PZ[jm]};
            const double pp[3] = {PX[jp], PY[jp], PZ[jp]};
            Real noise[3];
            if (noise_lds) {
#pragma unroll
                for (int c = 0; c < 3; ++c) noise[c] = NZ[(3 * sub + c) * nmax + i];
            } else {
                const U4 rnd = philox4x32_10(U4{(uint32_t)i, (uint32_t)step, (uint32_t)sub, 1u}, seed_lo, seed_hi);
                noise[0] = A * centred_uniform<Real>(rnd.x);
                noise[1] = A * centred_uniform<Real>(rnd.y);
                noise[2] = A * centred_uniform<Real>(rnd.z);
            }
            // WCA against the Verlet neighbours: register slots, then any further list
            // entries, or all pairs if the list overflowed
            Real fx = 0, fy = 0, fz = 0;
            auto wca = [&](const Real* d, Real r2) {
                if (r2 < rc2) {
                    const Real ir2 = fast_rcp<Real>(r2);
                    const Real s2 = sig2 * ir2;
                    const Real s6 = s2 * s2 * s2;
                    const Real c = eps24 * (Real(2) * s6 * s6 - s6) * ir2;
                    fx += c * d[0];
                    fy += c * d[1];
                    fz += c * d[2];
                }
            };
#pragma unroll
            for (int s = 0; s < K; ++s) {
                // without branches: an unused slot or a pair beyond the cutoff adds 0
                Real d[3];
                const Real r2 = separation_v<Real, PERIODIC>(r[k], pj[s], per, nd, d);
                const bool hit = s < nslot[k] && r2 < rc2;
                const Real ir2 = fast_rcp<Real>(hit ? r2 : Real(1));
                const Real s2 = sig2 * ir2;
                const Real s6 = s2 * s2 * s2;
                const Real c = hit ? eps24 * (Real(2) * s6 * s6 - s6) * ir2 : Real(0);
                fx += c * d[0];
                fy += c * d[1];
                fz += c * d[2];
            }
            const bool overflow = cnt[k] > kNeighbourMax;
            const int lim = overflow ? n : cnt[k];
            const unsigned short* li = lists + i;
            for (int q = overflow ? gl : gl + K * G; q < lim; q += G) {
                int j;
                if (overflow) {
                    j = q;
                    if (j == i || (j == i + 1 && bnk[k]) || (j == i - 1 && bpk[k])) continue;
                } else {
                    j = li[q * lstride];
                }
                Real d[3];
                const Real r2 = separation<Real, PERIODIC>(r[k], PX, PY, PZ, j, per, nd, d);
                wca(d, r2);
            }
            F[k][0] = group_sum<G>(fx);
            F[k][1] = group_sum<G>(fy);
            F[k][2] = group_sum<G>(fz);
            // harmonic bonds to the chain neighbours, -k (len - r0)/len d = -k (1 - r0/len) d
            // (d points from j to i: the bond pulls i towards j when stretched); an
            // absent neighbour is the bead itself and adds 0
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool on = (side == 0 ? bpk[k] : bnk[k]) && !rigid;
                Real d[3];
                const Real b2 = separation_v<Real, PERIODIC>(r[k], side == 0 ? pm : pp, per, nd, d);
                if (on && b2 > Real(4) * r0 * r0) flags |= LB_ERR_BOND_STRETCH;
                const Real coef = on ? -kb * (Real(1) - r0 * fast_rsqrt<Real>(b2)) : Real(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) F[k][c] += coef * d[c];
            }
            // angular terms centred on i - 1, i and i + 1 (each needs both of its bonds)
            if (POLY && kappa != Real(0) && (bpk[k] || bnk[k])) {
                const int jmm = bpp[k] ? i - 2 : i, jpp = bnn[k] ? i + 2 : i;
                const double pmm[3] = {PX[jmm], PY[jmm], PZ[jmm]};
                const double ppp[3] = {PX[jpp], PY[jpp], PZ[jpp]};
                Real fa[3], fc[3];
                if (bpk[k] && bnk[k]) {
                    angle_forces<Real, PERIODIC>(pm, r[k], pp, per, nd, kappa, fa, fc);
#pragma unroll
                    for (int c = 0; c < 3; ++c) F[k][c] -= fa[c] + fc[c];
                }
                if (bpp[k]) {
                    angle_forces<Real, PERIODIC>(pmm, pm, r[k], per, nd, kappa, fa, fc);
#pragma unroll
                    for (int c = 0; c < 3; ++c) F[k][c] += fc[c];
                }
                if (bnn[k]) {
                    angle_forces<Real, PERIODIC>(r[k], pp, ppp, per, nd, kappa, fa, fc);
#pragma unroll
                    for (int c = 0; c < 3; ++c) F[k][c] += fa[c];
                }
            }
            if (!(isfinite(r[k][0]) && isfinite(r[k][1]) && isfinite(r[k][2]))) flags |= LB_ERR_NONFINITE;
            // nearest solid surface over the walls (min, earlier wall on ties) and the pore
            // drive, each wall only within reach of its slab (x wrapped on a periodic
            // axis): a bead whose nearest node is a pore node lies within half a node of
            // its wall's slab
            if (nearw[k]) {
            const double xw = x_periodic ? r[k][0] - nd[0] * floor((r[k][0] + 0.5) / nd[0]) : r[k][0];
            double best2 = HUGE_VAL, dvw[3] = {0.0, 0.0, 0.0};
            bool pore = false;
#pragma unroll
            for (int w = 0; w < LB_MAX_WALLS; ++w) {
                if (w >= GM.n_walls) break;
                const int* W = GM.wall[w];
                if (xw > W[0] - 0.5 - rcw && xw < W[1] + 0.5 + rcw) {
                    double dv[3];
                    const double q = wall_dist2<PERIODIC>(GM, W, r[k], xw, dv);
                    if (q < best2) {
                        best2 = q;
                        dvw[0] = dv[0];
                        dvw[1] = dv[1];
                        dvw[2] = dv[2];
                    }
                    pore = pore || wall_pore_node<PERIODIC>(GM, W, r[k]);
                }
            }
            if (best2 == 0.0) flags |= LB_ERR_BEAD_IN_SOLID;
            if (best2 < (double)rcw2 && best2 > 0.0) {
                const Real c = wca_coef<Real>((Real)best2, epsw, sigw2, rcw2);
#pragma unroll
                for (int q = 0; q < 3; ++q) F[k][q] += c * (Real)dvw[q];
            }
            if (pore) F[k][0] += fdrive;
            }
            // free-slip faces at -1/2 and n - 1/2 (the WCA terms only within the cutoff)
            if (nearf[k]) {
            Real dlo[3], dhi[3];
            bool near_face = false;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dlo[c] = (Real)(r[k][c] + 0.5);
                dhi[c] = (Real)((nn[c] - 0.5) - r[k][c]);
                if (!GM.fs[c]) continue;
                if (!(dlo[c] > Real(0)) || !(dhi[c] > Real(0))) flags |= LB_ERR_BEAD_OUTSIDE;
                near_face = near_face || !(dlo[c] >= rcw_gate && dhi[c] >= rcw_gate);
            }
            if (near_face) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (!GM.fs[c] || !(dlo[c] > Real(0)) || !(dhi[c] > Real(0))) continue;
                    F[k][c] += wca_coef<Real>(dlo[c] * dlo[c], epsw, sigw2, rcw2) * dlo[c];
                    F[k][c] -= wca_coef<Real>(dhi[c] * dhi[c], epsw, sigw2, rcw2) * dhi[c];
                }
            }
            }
            // drag against the frozen fluid velocity and the random force
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const Real drag = -mg * (v[k][c] - u[k][c]);
                F[k][c] += drag + noise[c];
                fb[k][c] += (drag + noise[c]) * invM;
            }
        }
        // kick-drift into the other position buffer; the single barrier below both
        // publishes the new positions and collects the rebuild vote
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
#pragma unroll
                for (int c = 0; c < 3; ++c) QX[c * nmax + i] = r[k][c];
            }
        }
        if (POLY && rigid) {
            // SHAKE and RATTLE on the unconstrained positions now in QX (PX still holds
            // the positions of the start of the substep); row t of the bond systems is
            // thread t, bond t joining beads t and t + 1
            __syncthreads();
            const int m = n - 1, t = tid;
            const bool on = t < m && BN[t] != 0;
            const double ih = 1.0 / md.h, im = md.inv_mass;
            double dref[3] = {0.0, 0.0, 0.0}, ut[3] = {0.0, 0.0, 0.0}, ut1[3] = {0.0, 0.0, 0.0};
            if (on) {
                const double pa[3] = {PX[t], PY[t], PZ[t]}, pb[3] = {PX[t + 1], PY[t + 1], PZ[t + 1]};
                (void)separation_v<double, PERIODIC>(pa, pb, per, nd, dref);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    ut[c] = QX[c * nmax + t];
                    ut1[c] = QX[c * nmax + t + 1];
                }
            }
            if (t < nmax) {
#pragma unroll
                for (int c = 0; c < 3; ++c) SDV[c * nmax + t] = dref[c];
                LAM[t] = 0.0;
            }
            __syncthreads();
            // Newton iterations on the multipliers: positions r'_i = u_i + (lam_i d_i -
            // lam_{i-1} d_{i-1})/m, residuals g_t = |r'_t - r'_{t+1}|^2 - b^2
            double dm1[3] = {0.0, 0.0, 0.0}, dp1[3] = {0.0, 0.0, 0.0};
            if (on) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    dm1[c] = t > 0 ? SDV[c * nmax + t - 1] : 0.0;
                    dp1[c] = t + 1 < m ? SDV[c * nmax + t + 1] : 0.0;
                }
            }
            for (int it = 0;; ++it) {
                double sv[3] = {0.0, 0.0, 0.0}, g = 0.0;
                if (on) {
                    const double lm = t > 0 ? LAM[t - 1] : 0.0, l0 = LAM[t], lp = t + 1 < m ? LAM[t + 1] : 0.0;
                    double ra[3], rb[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        ra[c] = ut[c] + im * (l0 * dref[c] - lm * dm1[c]);
                        rb[c] = ut1[c] + im * (lp * dp1[c] - l0 * dref[c]);
                    }
                    g = (double)separation_v<double, PERIODIC>(ra, rb, per, nd, sv) - md.b2;
                }
                const bool bad = on && !(fabs(g) <= md.shake_tol_b2);
                // the Jacobian is assembled before the vote, which the solve's first barrier takes
                const double B = on ? 4.0 * im * (sv[0] * dref[0] + sv[1] * dref[1] + sv[2] * dref[2]) : 1.0;
                const double Aa = on ? -2.0 * im * (sv[0] * dm1[0] + sv[1] * dm1[1] + sv[2] * dm1[2]) : 0.0;
                const double Cc = on ? -2.0 * im * (sv[0] * dp1[0] + sv[1] * dp1[1] + sv[2] * dp1[2]) : 0.0;
                bool any_bad = false;
                const double x = pcr_solve(PCRW, nmax, m, t, Aa, B, Cc, on ? -g : 0.0, true, bad,
                                           it < md.shake_iter, &any_bad);
                if (!any_bad) break;
                if (it >= md.shake_iter) {
                    flags |= LB_ERR_CONSTRAINT;
                    break;
                }
                if (on) LAM[t] += x;
                __syncthreads();
            }
            // constrained positions and velocities (v = (r' - r) / h) of every bead
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const int i = grp + k * NG;
                if (!own[k]) continue;
                const double li = bnk[k] ? LAM[i] : 0.0, lm = bpk[k] ? LAM[i - 1] : 0.0;
                const double r_old[3] = {PX[i], PY[i], PZ[i]};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double di = bnk[k] ? SDV[c * nmax + i] : 0.0, dmi = bpk[k] ? SDV[c * nmax + i - 1] : 0.0;
                    r[k][c] += im * (li * di - lm * dmi);
                    v[k][c] = (Real)((r[k][c] - r_old[c]) * ih);
                }
            }
            __syncthreads();  // every read of the multipliers and of QX is done
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const int i = grp + k * NG;
                if (!own[k] || gl != 0) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    QX[c * nmax + i] = r[k][c];
                    VXV[c * nmax + i] = (double)v[k][c];
                }
            }
            __syncthreads();
            // RATTLE: (v'_t - v'_{t+1}) . s_t = 0 with v'_i = v_i + (mu_i s_i - mu_{i-1} s_{i-1})/m
            {
                double st[3] = {0.0, 0.0, 0.0}, sm[3] = {0.0, 0.0, 0.0}, sp[3] = {0.0, 0.0, 0.0};
                double rel = 0.0;
                auto bondvec = [&](int j, double* out) {  // r'_j - r'_{j+1}
                    const double pa[3] = {QX[j], QX[nmax + j], QX[2 * nmax + j]};
                    const double pb[3] = {QX[j + 1], QX[nmax + j + 1], QX[2 * nmax + j + 1]};
                    (void)separation_v<double, PERIODIC>(pa, pb, per, nd, out);
                };
                if (on) {
                    bondvec(t, st);
                    if (t > 0 && BN[t - 1]) bondvec(t - 1, sm);
                    if (t + 1 < m && BN[t + 1]) bondvec(t + 1, sp);
#pragma unroll
                    for (int c = 0; c < 3; ++c) rel += (VXV[c * nmax + t] - VXV[c * nmax + t + 1]) * st[c];
                }
                const double B = on ? 2.0 * im * (st[0] * st[0] + st[1] * st[1] + st[2] * st[2]) : 1.0;
                const double Aa = on ? -im * (st[0] * sm[0] + st[1] * sm[1] + st[2] * sm[2]) : 0.0;
                const double Cc = on ? -im * (st[0] * sp[0] + st[1] * sp[1] + st[2] * sp[2]) : 0.0;
                const double mu = pcr_solve(PCRW, nmax, m, t, Aa, B, Cc, on ? -rel : 0.0);
                if (t < nmax) LAM[t] = on ? mu : 0.0;
                __syncthreads();
#pragma unroll
                for (int k = 0; k < BPT; ++k) {
                    const int i = grp + k * NG;
                    if (!own[k]) continue;
                    double si[3] = {0.0, 0.0, 0.0}, sim[3] = {0.0, 0.0, 0.0};
                    if (bnk[k]) bondvec(i, si);
                    if (bpk[k]) bondvec(i - 1, sim);
                    const double mi = bnk[k] ? LAM[i] : 0.0, mm = bpk[k] ? LAM[i - 1] : 0.0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) v[k][c] = (Real)(VXV[c * nmax + i] + im * (mi * si[c] - mm * sim[c]));
                }
            }
        }
        int moved = 0;
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            if (!own[k]) continue;
            Real disp2 = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const Real dd = (Real)(r[k][c] - rref[k][c]);
                disp2 += dd * dd;
            }
            moved |= !(disp2 <= hs2);  // also catches a non-finite position
        }
        const int vb = sub & 1;
        const bool wave_moved = __ballot(moved) != 0ull;
        if ((tid & 63) == 0) vote[vb][wave] = wave_moved ? 1 : 0;
        __syncthreads();
        const uint4 vv = *(const uint4*)vote[vb];
        const bool any_moved = (vv.x | vv.y | vv.z | vv.w) != 0u;
        cur ^= 1;
        if (any_moved && sub + 1 < M) {
            ++builds;
            const double* NX = P + cur * 3 * nmax;
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const int i = grp + k * NG;
#pragma unroll
                for (int c = 0; c < 3; ++c) rref[k][c] = r[k][c];
                if (!own[k]) continue;
                cnt[k] = build_list<Real, G, PERIODIC>(i, n, bnk[k], bpk[k], r[k], NX, NX + nmax, NX + 2 * nmax,
                                                       per, nd, rl2, gl, lists + i, lstride);
            }
            __syncthreads();
            load_slots();
        }
    }

    // keep the lists for the next launch when they were (re)built in this one
    if (builds > 0) {
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int i = grp + k * NG;
            if (!own[k]) continue;
            const int gi = b0 + i;
            if (gl == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) a.b.rref[c * NT + gi] = rref[k][c];
                a.b.ncount[gi] = cnt[k];
            }
            if (a.list_in_lds) {
                const int m = cnt[k] < kNeighbourMax ? cnt[k] : kNeighbourMax;
                for (int q = gl; q < m; q += G) a.b.nlist[(size_t)q * NT + gi] = lists[i + q * lstride];
            }
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
            a.b.agg_at[gi] = lead ? R.pop_base + me : -1;
            a.b.agg_at[NT + gi] = R.S;
#pragma unroll
            for (int c = 0; c < 3; ++c) a.b.agg_f[c * NT + gi] = lead ? s[c] : Real(0);
        }
    }
    if (tid == 0) {
        dg[0] = acc[0];
        if (dg[1] < 0.0 && (int)acc[0] == n) dg[1] = (double)(step + 1);
        dg[2] = acc[1] / n;
        dg[3] = acc[2] / n;
        dg[4] = acc[3] / n;
        dg[5] = (double)(step + 1);
        dg[6] += (double)builds;
        if (builds > 0) dg[7] = 1.0;
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
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (bump_step && i == 0) st->step += 1;
    if (i >= b.ntot) return;
    // one round trip for everything a leader needs: where, stride, force
    const long long at = b.agg_at[i];
    const long long PS = b.agg_at[b.ntot + i];
    const Rl F[3] = {(Rl)b.agg_f[i], (Rl)b.agg_f[b.ntot + i], (Rl)b.agg_f[2 * b.ntot + i]};
    if (at < 0) return;
    typename C::T* __restrict__ base = dst + at;
    // S_p = -(w_p / c_s^2) Fbar . c_p with c_s^2 = 1/3
    auto source = [&](auto P) {
        constexpr int p = decltype(P)::value;
        Rl fc = 0;
        if constexpr (cx_of(p) != 0) fc += Rl(cx_of(p)) * F[0];
        if constexpr (cy_of(p) != 0) fc += Rl(cy_of(p)) * F[1];
        if constexpr (cz_of(p) != 0) fc += Rl(cz_of(p)) * F[2];
        return -Rl(3) * w_of<Rl>(p) * fc;
    };
    if constexpr (S == LB_STORE_F32 || S == LB_STORE_F64) {
        // full-precision storage: hardware float atomics without return (each node has one
        // leader, so no two threads add to one element and the result is deterministic)
        md_for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            if constexpr (p != 0) (void)unsafeAtomicAdd(&base[(long long)p * PS], source(P));
        });
    } else {
        // 16-bit storage: decode, add, re-encode; all 18 moving populations are read
        // before any is written
        Rl f[Q];
        md_for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            if constexpr (p != 0) f[p] = C::template load<p>(base[(long long)p * PS]);
        });
        md_for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            if constexpr (p != 0) base[(long long)p * PS] = C::template store<p>(f[p] + source(P));
        });
    }
}

__global__ void k_bump(RunState* st) { st->step += 1; }

// Observable record of the translocation analysis (Sec. III), one workgroup per replica,
// after the bead step and before the step counter moves: when (step + 1) is a multiple of
// obs_every, a row (step + 1, N_T, S_H = m gamma sum v.u, S_E = sum F_drive.v over beads on
// pore nodes, K = m/2 sum v^2, R_U^2, R_T^2, x of the centre of mass) is appended to the
// replica's record (rows beyond the capacity are counted, not kept).  FP64 sums in a fixed
// order; positions are taken relative to the pore centre, which keeps the second moments of
// the radii of gyration small.
template <class Real>
__global__ __launch_bounds__(256) void k_observe(const Replica* __restrict__ reps, BeadPtrs<Real> b,
                                                 const RunState* __restrict__ st, double mass_gamma,
                                                 double half_mass, double f_drive, int no_hydro) {
    __shared__ double red[16 * 12];
    const long long step = st->step;
    if ((step + 1) % b.obs_every != 0) return;
    const Replica& R = reps[blockIdx.x];
    const int n = R.n_beads;
    if (n == 0) return;
    const Geom GM = load_geom(R);
    const int b0 = R.bead0, NT = b.ntot;
    const double xmid = R.xmid;
    const double ref[3] = {xmid, 0.5 * R.ny, 0.5 * R.nz};
    // N_T, S_H, S_E, K, sum d (3), sum d^2, and over the translocated beads sum d (3), sum d^2
    double o[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int g = b0 + i;
        double r[3], v[3], u[3], d[3], d2 = 0.0, vu = 0.0, vv = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            r[c] = b.r[c * NT + g];
            v[c] = (double)b.v[c * NT + g];
            u[c] = no_hydro ? 0.0 : (double)b.u[c * NT + g];
            d[c] = r[c] - ref[c];
            d2 += d[c] * d[c];
            vu += v[c] * u[c];
            vv += v[c] * v[c];
        }
        bool pore = false;
#pragma unroll
        for (int w = 0; w < LB_MAX_WALLS; ++w) {
            if (w >= GM.n_walls) break;
            pore = pore || wall_pore_node<true>(GM, GM.wall[w], r);
        }
        const bool tr = r[0] > xmid;
        o[0] += tr ? 1.0 : 0.0;
        o[1] += mass_gamma * vu;
        o[2] += pore ? f_drive * v[0] : 0.0;
        o[3] += half_mass * vv;
        o[4] += d[0];
        o[5] += d[1];
        o[6] += d[2];
        o[7] += d2;
        if (tr) {
            o[8] += d[0];
            o[9] += d[1];
            o[10] += d[2];
            o[11] += d2;
        }
    }
    block_sums<Real>(o, 12, red);
    if (threadIdx.x != 0) return;
    double* rec = b.obs + (size_t)blockIdx.x * ((size_t)b.obs_cap + 1) * 8;
    const double cnt = rec[0];
    if (cnt < (double)b.obs_cap) {
        const double nT = o[0], nU = (double)n - o[0];
        double rT = 0.0, rU = 0.0;
        if (nT > 0) {
            const double c0 = o[8] / nT, c1 = o[9] / nT, c2 = o[10] / nT;
            rT = fmax(o[11] / nT - (c0 * c0 + c1 * c1 + c2 * c2), 0.0);
        }
        if (nU > 0) {
            const double c0 = (o[4] - o[8]) / nU, c1 = (o[5] - o[9]) / nU, c2 = (o[6] - o[10]) / nU;
            rU = fmax((o[7] - o[11]) / nU - (c0 * c0 + c1 * c1 + c2 * c2), 0.0);
        }
        double* row = rec + (size_t)(1 + (long long)cnt) * 8;
        row[0] = (double)(step + 1);
        row[1] = nT;
        row[2] = o[1];
        row[3] = o[2];
        row[4] = o[3];
        row[5] = rU;
        row[6] = rT;
        row[7] = ref[0] + o[4] / n;
    }
    rec[0] = cnt + 1.0;
}

// Trilinear stencil of a position: nodes floor(r_a) + {0, 1} per axis (periodic axes wrap,
// a node beyond a free-slip face is the face node) and the 1-D weights 1 - f, f.
__device__ __forceinline__ void trilinear_axes(const Replica& R, const double* r, int lo[3][2], double w1[3][2]) {
    const int n[3] = {R.nx, R.ny, R.nz};
    const int fs[3] = {R.fs[0], R.fs[1], R.fs[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double t = floor(r[a]);
        if (!(t >= -1e9 && t <= 1e9)) t = 0.0;  // non-finite or absurd
        const double fr = r[a] - t;
        w1[a][0] = 1.0 - fr;
        w1[a][1] = fr;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            int k = (int)t + s;
            if (!fs[a]) {
                k %= n[a];
                if (k < 0) k += n[a];
            } else {
                k = k < 0 ? 0 : (k > n[a] - 1 ? n[a] - 1 : k);
            }
            lo[a][s] = k;
        }
    }
}

// Step 1 with the trilinear stencil, one thread per bead: u_i = sum_c w_c u(x_c) over the 8
// surrounding nodes (u = 0 on solid ones), from the pre-collision populations; the
// start-of-step position is kept for the spread and the bead has no single node (-1).
template <class Real>
__global__ __launch_bounds__(256) void k_interp_tri(const Replica* __restrict__ reps, BeadPtrs<Real> b,
                                                    const void* cur, int storage) {
    // eight lanes a bead, lane c of the group owning stencil node c: the 8 x 19 population
    // reads of a bead are issued by 8 lanes at once instead of one after the other
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t >> 3, c = t & 7;
    if (i >= b.ntot) return;  // whole groups of eight leave together
    const int NT = b.ntot;
    const Replica& R = reps[b.rep_of[i]];
    const double r[3] = {b.r[i], b.r[NT + i], b.r[2 * NT + i]};
    int lo[3][2];
    double w1[3][2];
    trilinear_axes(R, r, lo, w1);
    const int g[3] = {lo[0][c & 1], lo[1][(c >> 1) & 1], lo[2][(c >> 2) & 1]};
    double part[3] = {0.0, 0.0, 0.0};
    if (!is_solid(R, g[0], g[1], g[2])) {
        const double w = w1[0][c & 1] * w1[1][(c >> 1) & 1] * w1[2][(c >> 2) & 1];
        Real uc[3];
        node_velocity<Real>(storage, R, cur, g, uc);
#pragma unroll
        for (int a = 0; a < 3; ++a) part[a] = w * (double)uc[a];
    }
    // the group's first lane adds the eight parts in stencil order (a solid node adds 0)
    double u[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] += __shfl(part[a], k, 8);
    if (c == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b.u[a * NT + i] = (Real)u[a];
            b.rs[a * NT + i] = r[a];
        }
        b.node[i] = -1;
    }
}

// Step 3 with the trilinear stencil, eight lanes a bead (FP32 and FP64 storage): -w_c (w_p /
// c_s^2) Fbar . c_p added to the post-collision populations of every fluid node of the
// start-of-step stencil.  Stencils of nearby beads share nodes, so the adds are atomic (their
// order, and so the last bits of FP32 sums, can differ between runs).  16-bit storage takes
// the fixed-point spread below.
template <int S>
__global__ __launch_bounds__(256) void k_spread_tri(const Replica* __restrict__ reps,
                                                    BeadPtrs<typename MDReal<S>::type> b,
                                                    typename Codec<S>::T* __restrict__ dst, RunState* st,
                                                    int bump_step) {
    using C = Codec<S>;
    using Rl = typename C::R;
    // eight lanes a bead, lane c adding to stencil node c
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t >> 3, c = t & 7;
    if (bump_step && t == 0) st->step += 1;
    if (i >= b.ntot) return;
    const int NT = b.ntot;
    const Replica& R = reps[b.rep_of[i]];
    const double r[3] = {b.rs[i], b.rs[NT + i], b.rs[2 * NT + i]};
    const Rl F[3] = {(Rl)b.fbar[i], (Rl)b.fbar[NT + i], (Rl)b.fbar[2 * NT + i]};
    int lo[3][2];
    double w1[3][2];
    trilinear_axes(R, r, lo, w1);
    const long long PS = R.S;  // population plane stride
    {
        const int g[3] = {lo[0][c & 1], lo[1][(c >> 1) & 1], lo[2][(c >> 2) & 1]};
        if (is_solid(R, g[0], g[1], g[2])) return;
        const Rl w = (Rl)(w1[0][c & 1] * w1[1][(c >> 1) & 1] * w1[2][(c >> 2) & 1]);
        typename C::T* base = dst + R.pop_base + g[0] + (long long)R.nx * (g[1] + (long long)R.ny * g[2]);
        md_for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            if constexpr (p != 0) {
                Rl fc = 0;
                if constexpr (cx_of(p) != 0) fc += Rl(cx_of(p)) * F[0];
                if constexpr (cy_of(p) != 0) fc += Rl(cy_of(p)) * F[1];
                if constexpr (cz_of(p) != 0) fc += Rl(cz_of(p)) * F[2];
                const Rl src = -Rl(3) * w_of<Rl>(p) * fc * w;
                (void)unsafeAtomicAdd(&base[(long long)p * PS], src);
            }
        });
    }
}

// Deterministic form of step 3 with the trilinear stencil.  Floating-point adds depend on
// their order, and the order of atomic adds changes from run to run; integer adds do not.
// Each contribution -w_c (w_p / c_s^2) Fbar . c_p is rounded once to a multiple of 2^-48
// (in FP64) and added as a 64-bit integer into a table entry of its node; a second pass adds
// each node's exact sums to its populations (one rounding each) and empties the entry.
// A contribution is at most 2^9 in magnitude (larger ones are dropped and flagged), so a
// node's signed 64-bit sum cannot overflow below 2^(63 - 48 - 9) = 64 contributions; a node
// collects one from each bead whose 8-node stencil holds it, a handful at WCA densities.
constexpr double kFxScale = 281474976710656.0;  // 2^48
constexpr double kFxLimit = 512.0;

// slot of a key: the splitmix64 finaliser (Steele, Lea and Flood, OOPSLA 2014) as a hash
__device__ __forceinline__ unsigned fx_hash(unsigned long long k, unsigned mask) {
    k ^= k >> 30;
    k *= 0xbf58476d1ce4e5b9ull;
    k ^= k >> 27;
    k *= 0x94d049bb133111ebull;
    k ^= k >> 31;
    return (unsigned)k & mask;
}

// Pass 1: the table entry of every fluid node of the start-of-step
// stencil (linear probing; the table holds at most 8 nodes a bead in 16 slots a bead, so a
// free slot is always found), then 18 integer atomic adds into it; eight lanes a bead.
template <class Real>
__global__ __launch_bounds__(64) void k_spread_tri_fx(const Replica* __restrict__ reps, BeadPtrs<Real> b,
                                                      RunState* st) {
    // eight lanes a bead, lane c inserting stencil node c (integer sums: the order of the
    // lanes' adds does not matter)
    const int lane8 = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = lane8 >> 3, c = lane8 & 7;
    if (i >= b.ntot) return;
    const int NT = b.ntot;
    const Replica& R = reps[b.rep_of[i]];
    const double r[3] = {b.rs[i], b.rs[NT + i], b.rs[2 * NT + i]};
    const double F[3] = {(double)b.fbar[i], (double)b.fbar[NT + i], (double)b.fbar[2 * NT + i]};
    int lo[3][2];
    double w1[3][2];
    trilinear_axes(R, r, lo, w1);
    const unsigned mask = b.hcap - 1;
    unsigned flags = 0;
    do {
        const int g[3] = {lo[0][c & 1], lo[1][(c >> 1) & 1], lo[2][(c >> 2) & 1]};
        if (is_solid(R, g[0], g[1], g[2])) break;
        const double w = w1[0][c & 1] * w1[1][(c >> 1) & 1] * w1[2][(c >> 2) & 1];
        const unsigned long long key =
            (unsigned long long)(R.pop_base + g[0] + (long long)R.nx * (g[1] + (long long)R.ny * g[2])) + 1ull;
        unsigned h = fx_hash(key, mask);
        bool found = false;
        for (unsigned t = 0; t <= mask; ++t) {
            const unsigned long long old = atomicCAS(&b.hkey[h], 0ull, key);
            if (old == 0ull) b.hrep[h] = b.rep_of[i];  // this thread opened the entry
            if (old == 0ull || old == key) {
                found = true;
                break;
            }
            h = (h + 1) & mask;
        }
        if (!found) {
            flags |= LB_ERR_NONFINITE;
            break;
        }
        md_for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            if constexpr (p != 0) {
                double fc = 0.0;
                if constexpr (cx_of(p) != 0) fc += cx_of(p) * F[0];
                if constexpr (cy_of(p) != 0) fc += cy_of(p) * F[1];
                if constexpr (cz_of(p) != 0) fc += cz_of(p) * F[2];
                const double src = -3.0 * w_of<double>(p) * fc * w;
                if (!(fabs(src) <= kFxLimit)) {
                    flags |= LB_ERR_NONFINITE;
                } else {
                    const long long q = (long long)rint(src * kFxScale);
                    (void)atomicAdd((unsigned long long*)&b.hsum[(size_t)(p - 1) * b.hcap + h], (unsigned long long)q);
                }
            }
        });
    } while (false);
    if (flags) atomicOr(&st->err, flags);
}

// Pass 2, one thread per table slot: adds an occupied entry's sums to the post-collision
// populations of its node (each node has one entry, so plain read-modify-writes) and empties
// the entry for the next step.
template <int S>
__global__ __launch_bounds__(256) void k_spread_fx_apply(const Replica* __restrict__ reps,
                                                         BeadPtrs<typename MDReal<S>::type> b,
                                                         typename Codec<S>::T* __restrict__ dst, RunState* st,
                                                         int bump_step) {
    using C = Codec<S>;
    using Rl = typename C::R;
    const unsigned h = blockIdx.x * blockDim.x + threadIdx.x;
    if (bump_step && h == 0) st->step += 1;
    if (h >= b.hcap) return;
    const unsigned long long key = b.hkey[h];
    if (key == 0ull) return;
    const long long PS = reps[b.hrep[h]].S;  // population plane stride
    typename C::T* __restrict__ base = dst + (long long)(key - 1ull);
    md_for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (p != 0) {
            long long* cell = &b.hsum[(size_t)(p - 1) * b.hcap + h];
            const long long q = *cell;
            if (q != 0) {
                const Rl add = (Rl)((double)q * (1.0 / kFxScale));
                base[(long long)p * PS] = C::template store<p>(C::template load<p>(base[(long long)p * PS]) + add);
                *cell = 0;
            }
        }
    });
    b.hkey[h] = 0ull;
}

// ---------------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------------
static int md_nmax(const Context& c) { return (c.max_beads + 63) / 64 * 64; }

static constexpr size_t kMDLdsBudget = 150 * 1024;
// the bead kernel's static LDS (block sums 512 B, rebuild vote 32 B) stays below this
static constexpr int kMDStaticLds = 2048;

static size_t md_base_lds(size_t nmax) { return nmax * (6 * sizeof(double) + sizeof(int) + 1); }
// SHAKE/RATTLE work area of rigid chains: 15 doubles per bead, always in LDS
static size_t md_rigid_lds(const Context& c, size_t nmax) { return c.md.rigid ? nmax * 15 * sizeof(double) : 0; }
static size_t md_list_lds(size_t nmax) { return nmax * kNeighbourMax * sizeof(unsigned short); }
static size_t md_noise_lds(const Context& c, size_t nmax) {
    return (size_t)c.md.M * 3 * nmax * (c.storage == LB_STORE_F64 ? sizeof(double) : sizeof(float));
}

// Verlet lists go to LDS when positions (two buffers), node/bond arrays and lists fit
static bool md_lists_in_lds(const Context& c) {
    const size_t nmax = (size_t)md_nmax(c);
    return md_base_lds(nmax) + md_rigid_lds(c, nmax) + md_list_lds(nmax) <= kMDLdsBudget;
}

// the per-step table of random forces, when several lanes share a bead and it fits
static bool md_noise_in_lds(const Context& c, int G) {
    const size_t nmax = (size_t)md_nmax(c);
    size_t b = md_base_lds(nmax) + md_rigid_lds(c, nmax) + md_noise_lds(c, nmax);
    if (md_lists_in_lds(c)) b += md_list_lds(nmax);
    return G > 1 && b <= kMDLdsBudget;
}

static size_t md_lds_bytes(const Context& c, int G) {
    const size_t nmax = (size_t)md_nmax(c);
    size_t b = md_base_lds(nmax) + md_rigid_lds(c, nmax);
    if (md_lists_in_lds(c)) b += md_list_lds(nmax);
    if (md_noise_in_lds(c, G)) b += md_noise_lds(c, nmax);
    return b;
}

int md_max_beads(bool rigid) {
    const size_t per = 6 * sizeof(double) + sizeof(int) + 1 + (rigid ? 15 * sizeof(double) : 0);
    const size_t nmax = (size_t)(160 * 1024 - kMDStaticLds) / per / 64 * 64;
    return (int)std::min<size_t>(nmax, 4096);
}

int md_default_lanes(int max_beads) {
    // lanes per bead: up to ~512 threads, so that each SIMD has two waves to interleave
    // (measured faster than one wave per SIMD for 100 beads, although the per-bead work
    // is repeated by every lane of a group); beyond 256 beads one lane per bead
    const int m = std::max(max_beads, 1);
    if (m <= 32) return 16;
    if (m <= 64) return 8;
    if (m <= 128) return 4;
    if (m <= 256) return 2;
    return 1;
}

bool md_lanes_valid(int lanes, int max_beads) {
    if (lanes == 1) return max_beads <= 4096;
    if (lanes == 2) return max_beads <= 512;
    return (lanes == 4 || lanes == 8 || lanes == 16) && (long long)lanes * max_beads <= 512;
}

template <class Real, int G, int BPT, bool PER, int MAXT, bool POLY>
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
    a.noise_in_lds = md_noise_in_lds(c, G) ? 1 : 0;
    const size_t lds = md_lds_bytes(c, G);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_md<Real, G, BPT, PER, MAXT, POLY>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024 - kMDStaticLds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_md<Real, G, BPT, PER, MAXT, POLY>), dim3((unsigned)c.reps.size()), dim3(block), lds, s, a,
                       c.storage);
    return hipGetLastError();
}

template <class Real, bool PER, bool POLY>
static hipError_t launch_md_g(const Context& c, const void* cur, int mode, hipStream_t s) {
    // G lanes per bead (the context's choice); with one lane per bead the 512-thread
    // bound up to 512 beads, the 1024-thread bound beyond, up to 4 beads per lane
    const int m = std::max(c.max_beads, 1);
    const int G = c.md_lanes > 0 ? c.md_lanes : md_default_lanes(m);
    if (!md_lanes_valid(G, m)) return hipErrorInvalidValue;
    auto blk = [](int t) { return std::min(1024, (t + 63) / 64 * 64); };
    switch (G) {
        case 16: return launch_md_t<Real, 16, 1, PER, 512, POLY>(c, cur, mode, blk(16 * m), s);
        case 8: return launch_md_t<Real, 8, 1, PER, 512, POLY>(c, cur, mode, blk(8 * m), s);
        case 4: return launch_md_t<Real, 4, 1, PER, 512, POLY>(c, cur, mode, blk(4 * m), s);
        case 2:
            // two lanes per bead: up to 256 beads in the 512-thread bound, up to 512 in the
            // 1024-thread one
            if (2 * m <= 512) return launch_md_t<Real, 2, 1, PER, 512, POLY>(c, cur, mode, blk(2 * m), s);
            return launch_md_t<Real, 2, 1, PER, 1024, POLY>(c, cur, mode, blk(2 * m), s);
        default: break;
    }
    if (m <= 512) return launch_md_t<Real, 1, 1, PER, 512, POLY>(c, cur, mode, blk(m), s);
    if (m <= 1024) return launch_md_t<Real, 1, 1, PER, 1024, POLY>(c, cur, mode, blk(m), s);
    if (m <= 2048) return launch_md_t<Real, 1, 2, PER, 1024, POLY>(c, cur, mode, 1024, s);
    if (m <= 3072) return launch_md_t<Real, 1, 3, PER, 1024, POLY>(c, cur, mode, 1024, s);
    if (m <= 4096) return launch_md_t<Real, 1, 4, PER, 1024, POLY>(c, cur, mode, 1024, s);
    return hipErrorInvalidValue;
}

template <class Real>
static hipError_t launch_md_r(const Context& c, const void* cur, int mode, hipStream_t s) {
    bool any_periodic = false;
    for (const Replica& R : c.reps)
        if (R.n_beads > 0 && (!R.fs[0] || !R.fs[1] || !R.fs[2])) any_periodic = true;
    if (c.md.rigid || c.md.kappa_phi != 0.0)
        return any_periodic ? launch_md_g<Real, true, true>(c, cur, mode, s)
                            : launch_md_g<Real, false, true>(c, cur, mode, s);
    return any_periodic ? launch_md_g<Real, true, false>(c, cur, mode, s)
                        : launch_md_g<Real, false, false>(c, cur, mode, s);
}

hipError_t launch_md(const Context& c, const void* cur, int mode, hipStream_t s) {
    if (c.storage == LB_STORE_F64) return launch_md_r<double>(c, cur, mode, s);
    return launch_md_r<float>(c, cur, mode, s);
}

template <int S>
static hipError_t launch_spread_t(const Context& c, void* dst, bool bump, hipStream_t s) {
    using Real = typename MDReal<S>::type;
    const BeadPtrs<Real> b = *(const BeadPtrs<Real>*)c.bead_ptrs;
    // 64 threads a block: each leader's 18 read-modify-writes miss the caches when the
    // sweep streamed the populations past them, and more compute units keep more of
    // these misses in flight
    const int grid = (c.ntot_beads + 63) / 64;
    hipLaunchKernelGGL((k_spread<S>), dim3(grid > 0 ? grid : 1), dim3(64), 0, s, c.d_reps, b,
                       (typename Codec<S>::T*)dst, c.d_state, bump ? 1 : 0);
    return hipGetLastError();
}

template <int S>
static hipError_t launch_spread_tri_t(const Context& c, void* dst, bool bump, hipStream_t s) {
    using Real = typename MDReal<S>::type;
    const BeadPtrs<Real> b = *(const BeadPtrs<Real>*)c.bead_ptrs;
    // eight lanes a bead in 64-thread blocks, as for the nearest-node spread
    const int grid = (8 * c.ntot_beads + 63) / 64;
    hipLaunchKernelGGL((k_spread_tri<S>), dim3(grid > 0 ? grid : 1), dim3(64), 0, s, c.d_reps, b,
                       (typename Codec<S>::T*)dst, c.d_state, bump ? 1 : 0);
    return hipGetLastError();
}

template <class Real>
static hipError_t launch_interp_tri_t(const Context& c, const void* cur, hipStream_t s) {
    const BeadPtrs<Real> b = *(const BeadPtrs<Real>*)c.bead_ptrs;
    // eight lanes a bead in 64-thread blocks: each bead's 8 x 19 population reads may miss
    // the caches, and more compute units keep more misses in flight
    const int grid = (8 * c.ntot_beads + 63) / 64;
    hipLaunchKernelGGL((k_interp_tri<Real>), dim3(grid > 0 ? grid : 1), dim3(64), 0, s, c.d_reps, b, cur,
                       c.storage);
    return hipGetLastError();
}

hipError_t launch_interp_trilinear(const Context& c, const void* cur, hipStream_t s) {
    if (c.ntot_beads == 0) return hipSuccess;
    return c.storage == LB_STORE_F64 ? launch_interp_tri_t<double>(c, cur, s)
                                     : launch_interp_tri_t<float>(c, cur, s);
}

template <int S>
static hipError_t launch_spread_fx_t(const Context& c, void* dst, bool bump, hipStream_t s) {
    using Real = typename MDReal<S>::type;
    const BeadPtrs<Real> b = *(const BeadPtrs<Real>*)c.bead_ptrs;
    const int grid = (8 * c.ntot_beads + 63) / 64;  // eight lanes a bead
    hipLaunchKernelGGL((k_spread_tri_fx<Real>), dim3(grid > 0 ? grid : 1), dim3(64), 0, s, c.d_reps, b, c.d_state);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_spread_fx_apply<S>), dim3((b.hcap + 255) / 256), dim3(256), 0, s, c.d_reps, b,
                       (typename Codec<S>::T*)dst, c.d_state, bump ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_spread(const Context& c, void* dst, bool bump, hipStream_t s) {
    // the trilinear spread in fixed point when asked for reproducible results, and always in
    // 16-bit storage: there a floating-point add into one element is a compare-and-swap loop on
    // its 32-bit word, and the integer atomics and one read-modify-write per node took 23 us
    // against 44 us on 128x64x64 (N = 100)
    const bool half = c.storage == LB_STORE_F16DEV || c.storage == LB_STORE_BF16DEV;
    if (c.md.stencil == LB_STENCIL_TRILINEAR && (c.deterministic || half)) {
        switch (c.storage) {
            case LB_STORE_F64: return launch_spread_fx_t<LB_STORE_F64>(c, dst, bump, s);
            case LB_STORE_F32: return launch_spread_fx_t<LB_STORE_F32>(c, dst, bump, s);
            case LB_STORE_F16DEV: return launch_spread_fx_t<LB_STORE_F16DEV>(c, dst, bump, s);
            case LB_STORE_BF16DEV: return launch_spread_fx_t<LB_STORE_BF16DEV>(c, dst, bump, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (c.md.stencil == LB_STENCIL_TRILINEAR) {
        switch (c.storage) {
            case LB_STORE_F64: return launch_spread_tri_t<LB_STORE_F64>(c, dst, bump, s);
            case LB_STORE_F32: return launch_spread_tri_t<LB_STORE_F32>(c, dst, bump, s);
            default: return hipErrorInvalidValue;  // 16-bit storage took the fixed-point path
        }
    }
    switch (c.storage) {
        case LB_STORE_F64: return launch_spread_t<LB_STORE_F64>(c, dst, bump, s);
        case LB_STORE_F32: return launch_spread_t<LB_STORE_F32>(c, dst, bump, s);
        case LB_STORE_F16DEV: return launch_spread_t<LB_STORE_F16DEV>(c, dst, bump, s);
        case LB_STORE_BF16DEV: return launch_spread_t<LB_STORE_BF16DEV>(c, dst, bump, s);
        default: return hipErrorInvalidValue;
    }
}

template <class Real>
static hipError_t launch_observe_t(const Context& c, bool no_hydro, hipStream_t s) {
    const BeadPtrs<Real> b = *(const BeadPtrs<Real>*)c.bead_ptrs;
    hipLaunchKernelGGL((k_observe<Real>), dim3((unsigned)c.reps.size()), dim3(256), 0, s, c.d_reps, b, c.d_state,
                       c.md.mass * c.md.gamma, 0.5 * c.md.mass, c.md.f_drive, no_hydro ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_observe(const Context& c, bool no_hydro, hipStream_t s) {
    if (c.obs_every <= 0 || c.ntot_beads == 0) return hipSuccess;
    return c.storage == LB_STORE_F64 ? launch_observe_t<double>(c, no_hydro, s)
                                     : launch_observe_t<float>(c, no_hydro, s);
}

hipError_t launch_bump(const Context& c, hipStream_t s) {
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(1), 0, s, c.d_state);
    return hipGetLastError();
}

}  // namespace lbmd
