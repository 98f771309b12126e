// lb_kernels.hip -- lattice kernels (gfx950).
//
// k_stream_collide: one LB time step (arXiv:0710.1272 Sec. II, Eq. lbe with F_p = 0;
// the source S_p is added afterwards by the spread kernel) in pull form.  Each thread
// owns one node: it gathers the 19 post-collision populations that stream into the
// node (periodic wrap, specular free-slip faces, half-way bounce-back on solid nodes),
// forms rho and j (Eqs. dens, vel), relaxes towards f_eq (f_eq eq.) with
// omega = 1/tau, and writes its own 19 post-collision values, coalesced and
// non-temporal.  Per replica the populations form a [19][V] block with x fastest;
// 16-bit storage keeps s_p (f_p - w_p rho0).  HBM traffic per fluid node is
// 19 loads + 19 stores of the storage type, the kernel's roofline.
#include <type_traits>
#include <utility>

#include "lbmd_internal.hpp"

namespace lbmd {

template <class F, int... Ps>
__device__ __forceinline__ void for_pops_impl(F&& f, std::integer_sequence<int, Ps...>) {
    (f(std::integral_constant<int, Ps>{}), ...);
}
template <class F>
__device__ __forceinline__ void for_pops(F&& f) {
    for_pops_impl(f, std::make_integer_sequence<int, Q>{});
}

// Blocks are dealt round-robin to the 8 XCDs.  Tile order options:
//   C < 0: XCD j takes one contiguous eighth of the tiles (best for one big box);
//   C = 0: the hardware order;
//   C > 0: XCD j takes the chunks j, j+8, j+16, ... of C consecutive tiles, locality
//          with balance when the work per tile is uneven (many small replicas); the
//          partial super-chunk at the end keeps its order.
__device__ __forceinline__ int xcd_tile(int b, int G, int C) {
    if (C < 0) {
        const int per = G >> 3, rem = G & 7, j = b & 7;
        return j * per + (j < rem ? j : rem) + (b >> 3);
    }
    if (C == 0) return b;
    const int S = 8 * C;
    if (b >= (G / S) * S) return b;
    const int j = b & 7, l = b >> 3;
    return ((l / C) * 8 + j) * C + (l % C);
}

__device__ __forceinline__ int replica_of_tile(const int* __restrict__ prefix, int n_reps, int tile) {
    int lo = 0, hi = n_reps - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Solidity of the 27 nodes (x+dx, y+dy, z+dz), dx, dy, dz in {-1, 0, 1}, as bit
// 9(dx+1) + 3(dy+1) + (dz+1): a neighbour is solid when its x plane is a wall plane and its
// (y, z) lies outside that wall's pore.
__device__ __forceinline__ unsigned solid_neighbours(const Replica& R, int x, int y, int z) {
    unsigned solid27 = 0u;
#pragma unroll
    for (int k = 0; k < LB_MAX_WALLS; ++k) {
        if (k >= R.n_walls) break;
        const int* w = R.wall[k];
        unsigned bx = 0, by = 0, bz = 0;
#pragma unroll
        for (int d = -1; d <= 1; ++d) {
            bx |= (unsigned)(x + d >= w[0] && x + d <= w[1]) << (d + 1);
            by |= (unsigned)(y + d >= w[2] && y + d <= w[3]) << (d + 1);
            bz |= (unsigned)(z + d >= w[4] && z + d <= w[5]) << (d + 1);
        }
        // pore membership of (y+dy, z+dz) for the 9 combinations, bit 3(dy+1) + (dz+1)
        unsigned m = 0;
        if (pore_open(w)) {
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dz = 0; dz < 3; ++dz)
                    m |= (((by >> dy) & (bz >> dz)) & 1u) << (3 * dy + dz);
        }
        const unsigned closed = ~m & 0x1FFu;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) solid27 |= (0u - ((bx >> dx) & 1u)) & (closed << (9 * dx));
    }
    return solid27;
}

// whether x lies within one plane of a wall (only such nodes have solid sources)
__device__ __forceinline__ bool in_wall_zone(const Replica& R, int x) {
    bool zone = false;
#pragma unroll
    for (int k = 0; k < LB_MAX_WALLS; ++k) {
        if (k >= R.n_walls) break;
        zone = zone || (x >= R.wall[k][0] - 1 && x <= R.wall[k][1] + 1);
    }
    return zone;
}

enum GatherKind { G_INTERIOR = 0, G_FAST = 1, G_WALL_PLANE = 2, G_WALL = 3, G_GENERIC = 4 };

// Element `node` of a population block that starts at the wave-uniform pointer bp.  The byte
// offset is formed in 32 bits (a replica's population block holds at most 4 GiB, which
// lb_validate_config enforces), so the load takes the scalar-base plus 32-bit-offset form
// and the address costs one vector instruction instead of a 64-bit multiply-add.
template <class T>
__device__ __forceinline__ T ld32(const T* __restrict__ bp, int node) {
    return *(const T*)((const char*)bp + (unsigned)node * (unsigned)sizeof(T));
}

// Incoming populations of one lane of the flattened mapping (64 consecutive nodes
// per wave, possibly spanning rows), as stored numbers (Codec::load_raw).
//  G_GENERIC:    any lane (full resolver, used by waves touching a y/z face);
//  G_WALL:       y and z interior, lanes may neighbour a wall and its pore (solid test per
//                source over the 27 neighbours);
//  G_WALL_PLANE: y and z interior, lanes may neighbour a wall but lie at least two nodes from
//                its pore in y or z, so that a source is solid exactly when its x plane is a
//                wall plane: only populations with c_x != 0 can bounce, on two per-lane bits;
//  G_FAST:       y and z interior, no wall within one node (only x faces need care);
//  G_INTERIOR:   no lane on any face or within one node of a wall (no test at all).
// Outside G_GENERIC each population is read from its own block at a 32-bit offset; a
// free-slip x face (the reflected population at the node itself) and a solid source (the
// node's own population opp(p), half-way bounce-back) are loads of their own, taken only
// by the lanes that need them.
// RAW: f receives the stored elements themselves (decoded later by the caller), so that no
// conversion sits between the loads of two nodes gathered one after the other.
template <int S, int KIND, bool RAW = false>
__device__ __forceinline__ void gather19(
    const Replica& R, const typename Codec<S>::T* __restrict__ src, int idx, int x, int y, int z,
    std::conditional_t<RAW, typename Codec<S>::T, typename Codec<S>::R>* f) {
    using C = Codec<S>;
    using T = typename C::T;
    auto cv = [](T v) {
        if constexpr (RAW) return v;
        else return C::load_raw(v);
    };
    const long long PS = R.S;  // population plane stride
    const int nx = R.nx, nxy = R.nx * R.ny;
    const T* __restrict__ base = src + R.pop_base;
    if constexpr (KIND == G_GENERIC) {
        for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            int q;
            const int node = pull_source<p>(R, x, y, z, &q);
            // q differs from p only by reflections or reversal, which keep the weight
            // class, so the codec scale of p applies to slot q
            f[p] = cv(base[(long long)q * PS + node]);
        });
        return;
    }
    // per-wall 3-bit masks: bit (d+1) set when x+d is a wall plane / y+d, z+d in the pore.
    // 16-bit storage (half the bytes per node, so the sweep is closer to issue-bound) folds
    // them once into the solidity of the 27 neighbours (x+dx, y+dy, z+dz), bit
    // 9(dx+1) + 3(dy+1) + (dz+1), and tests one bit per population; measured slower for
    // FP32 storage, which tests the wall masks per population
    constexpr bool kMask27 = C::deviation;
    unsigned mx[LB_MAX_WALLS] = {0u, 0u}, mp[LB_MAX_WALLS] = {0u, 0u};
    unsigned solid27 = 0u;
    if constexpr (KIND == G_WALL) {
        if constexpr (kMask27) {
            solid27 = solid_neighbours(R, x, y, z);
        } else {
#pragma unroll
            for (int k = 0; k < LB_MAX_WALLS; ++k) {
                if (k >= R.n_walls) break;
                const int* w = R.wall[k];
                unsigned bx = 0, by = 0, bz = 0;
#pragma unroll
                for (int d = -1; d <= 1; ++d) {
                    bx |= (unsigned)(x + d >= w[0] && x + d <= w[1]) << (d + 1);
                    by |= (unsigned)(y + d >= w[2] && y + d <= w[3]) << (d + 1);
                    bz |= (unsigned)(z + d >= w[4] && z + d <= w[5]) << (d + 1);
                }
                // pore membership of (y+dy, z+dz) for the 9 combinations, bit 3*(dy+1)+(dz+1)
                unsigned m = 0;
                if (pore_open(w)) {
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                        for (int dz = 0; dz < 3; ++dz)
                            m |= (((by >> dy) & (bz >> dz)) & 1u) << (3 * dy + dz);
                }
                mx[k] = bx;
                mp[k] = m;
            }
        }
    }
    // G_WALL_PLANE: whether the planes x - 1 and x + 1 are wall planes (a fluid node far from
    // the pores is not on one itself, so its c_x = 0 sources are fluid)
    bool solid_m = false, solid_p = false;
    if constexpr (KIND == G_WALL_PLANE) {
#pragma unroll
        for (int k = 0; k < LB_MAX_WALLS; ++k) {
            if (k >= R.n_walls) break;
            solid_m = solid_m || (x - 1 >= R.wall[k][0] && x - 1 <= R.wall[k][1]);
            solid_p = solid_p || (x + 1 >= R.wall[k][0] && x + 1 <= R.wall[k][1]);
        }
    }
    const bool xlo = x == 0, xhi = x == nx - 1, fsx = R.fs[0] != 0;
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        constexpr int cx = cx_of(p), cy = cy_of(p), cz = cz_of(p);
        int node = idx - (cx + cy * nx + cz * nxy);
        // at an x face the source row's node x itself (free slip, fixed below) or the
        // periodic image
        if constexpr (KIND != G_INTERIOR && cx == 1) {
            if (xlo) node += fsx ? 1 : nx;
        }
        if constexpr (KIND != G_INTERIOR && cx == -1) {
            if (xhi) node -= fsx ? 1 : nx;
        }
        f[p] = cv(ld32(base + (long long)p * PS, node));
        if constexpr (KIND == G_WALL && p != 0) {
            // source offset -c: neighbour bit 9(1 - c_x) + 3(1 - c_y) + (1 - c_z), or bit
            // (1 - c) of each wall's masks
            bool solid = false;
            if constexpr (kMask27) {
                constexpr int bit = 9 * (1 - cx) + 3 * (1 - cy) + (1 - cz);
                solid = (solid27 >> bit) & 1u;
            } else {
#pragma unroll
                for (int k = 0; k < LB_MAX_WALLS; ++k) {
                    if (k >= R.n_walls) break;
                    bool inx = (mx[k] >> (1 - cx)) & 1u;
                    bool inpore = (mp[k] >> (3 * (1 - cy) + (1 - cz))) & 1u;
                    solid = solid || (inx && !inpore);
                }
            }
            // half-way bounce-back: the node's own population opp(p) of the last collision
            if (solid) f[p] = cv(ld32(base + (long long)opp_of(p) * PS, idx));
        }
        if constexpr (KIND == G_WALL_PLANE && cx != 0) {
            if (cx == 1 ? solid_m : solid_p) f[p] = cv(ld32(base + (long long)opp_of(p) * PS, idx));
        }
    });
    if constexpr (KIND != G_INTERIOR) {
        // a free-slip x face: the populations arriving through it are those with c_x reflected,
        // from the node's own plane (one branch per face, taken by the lanes on it)
        if (fsx && xlo) {
            for_pops([&](auto P) {
                constexpr int p = decltype(P)::value;
                if constexpr (cx_of(p) == 1)
                    f[p] = cv(ld32(base + (long long)mirror_of(p, 0) * PS,
                                            idx - (cy_of(p) * nx + cz_of(p) * nxy)));
            });
        }
        if (fsx && xhi) {
            for_pops([&](auto P) {
                constexpr int p = decltype(P)::value;
                if constexpr (cx_of(p) == -1)
                    f[p] = cv(ld32(base + (long long)mirror_of(p, 0) * PS,
                                            idx - (cy_of(p) * nx + cz_of(p) * nxy)));
            });
        }
    }
}

// Whether (y, z) lies within one node of an open pore of a wall whose zone holds x (only then
// can a neighbour of a fluid node next to the wall lie in the pore).
__device__ __forceinline__ bool near_pore(const Replica& R, int x, int y, int z) {
    bool near = false;
#pragma unroll
    for (int k = 0; k < LB_MAX_WALLS; ++k) {
        if (k >= R.n_walls) break;
        const int* w = R.wall[k];
        near = near || (pore_open(w) && x >= w[0] - 1 && x <= w[1] + 1 && y >= w[2] - 1 && y <= w[3] + 1 &&
                        z >= w[4] - 1 && z <= w[5] + 1);
    }
    return near;
}

// Row-segment work units: one wave owns up to 64 consecutive x of one row (y, z) of
// one replica, so y, z and every face decision are uniform across the wave and a
// lane only has to care about its own x.  segs = ceil(nx / 64) units per row.
struct RowUnit {
    int y, z, x0;
    bool valid;
};

__device__ __forceinline__ RowUnit row_unit(const Replica& R, int unit) {
    RowUnit u;
    const int segs = (R.nx + 63) >> 6;
    const int rows = R.ny * R.nz;
    u.valid = unit < rows * segs;
    const int row = unit / segs;
    u.x0 = (unit - row * segs) << 6;
    u.z = row / R.ny;
    u.y = row - u.z * R.ny;
    return u;
}

// Incoming populations of one lane of a row unit.  Face handling is uniform (the wave's
// y and z, so the source population after a y or z reflection is uniform too); x faces
// are per lane.  WALL: the segment is within one node of a wall plane, so every source
// is tested for solidity (bounce-back); the pore test of a source depends only on
// (y - c_y, z - c_z) and is uniform.
template <int S, bool WALL>
__device__ __forceinline__ void gather_row(const Replica& R, const typename Codec<S>::T* __restrict__ src,
                                           int idx, int x, int y, int z, typename Codec<S>::R* f) {
    using C = Codec<S>;
    using T = typename C::T;
    const long long PS = R.S;  // population plane stride
    const int nx = R.nx, ny = R.ny, nz = R.nz, nxy = R.nx * R.ny;
    const T* __restrict__ base = src + R.pop_base;
    const bool xlo = x == 0, xhi = x == nx - 1, fsx = R.fs[0] != 0;
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        constexpr int cx = cx_of(p), cy = cy_of(p), cz = cz_of(p);
        int node = idx - (cx + cy * nx + cz * nxy);
        bool fy = false, fz = false;
        int sy = y - cy, sz = z - cz;
        if constexpr (cy != 0) {
            if (y == (cy > 0 ? 0 : ny - 1)) {
                if (R.fs[1]) { node += cy * nx; fy = true; sy = y; }
                else node += cy * nxy;
            }
        }
        if constexpr (cz != 0) {
            if (z == (cz > 0 ? 0 : nz - 1)) {
                if (R.fs[2]) { node += cz * nxy; fz = true; sz = z; }
                else node += cz * (long long)nxy * nz;
            }
        }
        if constexpr (cx == 1) {
            if (xlo) node += fsx ? 1 : nx;
        }
        if constexpr (cx == -1) {
            if (xhi) node -= fsx ? 1 : nx;
        }
        const int q = mirror_combo<p>(false, fy, fz);  // uniform over the wave
        f[p] = C::load_raw(ld32(base + (long long)q * PS, node));
        if constexpr (cx != 0) {
            // free slip: the population with c_x reflected as well, from that node
            if (fsx && (cx == 1 ? xlo : xhi)) {
                const int m = mirror_combo<p>(true, fy, fz);
                f[p] = C::load_raw(ld32(base + (long long)m * PS, node));
            }
        }
        if constexpr (WALL && p != 0) {
            // walls are at least two planes away from the x faces, so x - c_x is the
            // source plane of every lane that can see a wall
            bool solid = false;
#pragma unroll
            for (int k = 0; k < LB_MAX_WALLS; ++k) {
                if (k >= R.n_walls) break;
                const int* w = R.wall[k];
                const bool inpore = pore_open(w) && sy >= w[2] && sy <= w[3] && sz >= w[4] && sz <= w[5];
                solid = solid || (!inpore && x - cx >= w[0] && x - cx <= w[1]);
            }
            // half-way bounce-back: the node's own population opp(p) of the last collision
            if (solid) f[p] = C::load_raw(ld32(base + (long long)opp_of(p) * PS, idx));
        }
    });
}

// BGK relaxation of one node (Eq. lbe with the f_eq equation), in place on the stored numbers
// h_p = k_p (f_p - o_p) with k_p the codec's scale and o_p = w_p rho0 for deviation storage
// (k_p = 1, o_p = 0 for full storage); returns rho.  The opposite populations p, opp(p) are
// taken as pairs: their sum and difference give the moments, and they share |c.u| in f_eq:
// f_eq,p - o_p = w_p (b + rho (4.5 (c.u)^2 - 1.5 u^2) +- 3 rho c.u) with b = sum_p (f_p - o_p),
// that is rho - rho0 for deviation storage and rho for full storage.  The relaxation
// h*_p = (1 - omega) h_p + omega k_p (f_eq,p - o_p) keeps every scale in a constant.
template <int S>
__device__ __forceinline__ typename Codec<S>::R collide(typename Codec<S>::R* h,
                                                        typename Codec<S>::R omega,
                                                        typename Codec<S>::R rho0) {
    using C = Codec<S>;
    using Rl = typename C::R;
    // moments from the pair sums and differences (the o_p cancel in j: sum_p w_p c_p = 0)
    Rl m0 = h[0] * (Rl(1) / C::template kScale<0>), jx = 0, jy = 0, jz = 0;
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (p % 2 == 1) {
            constexpr Rl is = Rl(1) / C::template kScale<p>;  // opp(p) = p + 1 shares it
            const Rl sum = h[p] + h[p + 1], dif = h[p] - h[p + 1];
            m0 += sum * is;
            if constexpr (cx_of(p) != 0) jx += dif * Rl(cx_of(p) * is);
            if constexpr (cy_of(p) != 0) jy += dif * Rl(cy_of(p) * is);
            if constexpr (cz_of(p) != 0) jz += dif * Rl(cz_of(p) * is);
        }
    });
    // deviation storage: m0 = rho - rho0; full storage: m0 = rho
    const Rl rho = C::deviation ? rho0 + m0 : m0;
    Rl inv;
    if constexpr (sizeof(Rl) == 4) inv = __builtin_amdgcn_rcpf(rho);  // about 1 ulp
    else inv = Rl(1) / rho;
    const Rl ux = jx * inv, uy = jy * inv, uz = jz * inv;
    const Rl rus = rho * (Rl(1.5) * (ux * ux + uy * uy + uz * uz));
    const Rl r3 = Rl(3) * rho, r45 = Rl(4.5) * rho;
    const Rl om1 = Rl(1) - omega;
    // omega k_p w_p per weight class (k_p is a power of two near 1/w_p)
    const Rl cw0 = omega * (w_of<Rl>(0) * C::template kScale<0>);
    const Rl cw1 = omega * (w_of<Rl>(1) * C::template kScale<1>);
    const Rl cw7 = omega * (w_of<Rl>(7) * C::template kScale<7>);
    h[0] = om1 * h[0] + cw0 * (m0 - rus);
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (p % 2 == 1) {
            Rl cu = 0;
            if constexpr (cx_of(p) != 0) cu += Rl(cx_of(p)) * ux;
            if constexpr (cy_of(p) != 0) cu += Rl(cy_of(p)) * uy;
            if constexpr (cz_of(p) != 0) cu += Rl(cz_of(p)) * uz;
            const Rl e = m0 + ((r45 * cu) * cu - rus);  // b + rho (4.5 cu^2 - 1.5 u^2)
            const Rl t = r3 * cu;
            const Rl cw = p <= 6 ? cw1 : cw7;
            h[p] = om1 * h[p] + cw * (e + t);
            h[p + 1] = om1 * h[p + 1] + cw * (e - t);
        }
    });
    return rho;
}

// Thermal source F_p of Eq. lbe (the fluctuating LB that Sec. II adopts), added to the
// post-collision populations: F = phi Pi eta, eta_p = sqrt(w_p) xi_p with xi_p of zero
// mean and unit variance (sqrt(12) times a symmetric uniform from Philox words p of the
// counters (node, step, j, 2)), Pi x = x - w (sum x + 3 c . sum c x) (no density or
// momentum in the noise), phi^2 = (kT / c_s^2) (1 - gamma^2) rho.  Its covariance
// mu rho (1 - gamma^2) Pi W is what keeps the equilibrium fluctuations mu rho w_p of the
// populations through a BGK collision with rate omega = 1 - gamma.  f holds the codec's stored
// numbers, so the source of population p is added times its scale k_p.
template <class C, class Rl>
__device__ __forceinline__ void add_thermal(Rl* f, uint32_t node, uint32_t step, uint32_t k0, uint32_t k1,
                                            Rl phi) {
    Rl s0 = 0, sx = 0, sy = 0, sz = 0;
    U4 w{0u, 0u, 0u, 0u};
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (p % 4 == 0) w = philox4x32_10(U4{node, step, (uint32_t)(p / 4), 2u}, k0, k1);
        uint32_t word;
        if constexpr (p % 4 == 0) word = w.x;
        else if constexpr (p % 4 == 1) word = w.y;
        else if constexpr (p % 4 == 2) word = w.z;
        else word = w.w;
        // sqrt(12 w_p): 2 for the rest population, sqrt(2/3) and sqrt(1/3) for faces and edges
        constexpr int c2 = cx_of(p) * cx_of(p) + cy_of(p) * cy_of(p) + cz_of(p) * cz_of(p);
        constexpr double amp = c2 == 0 ? 2.0 : c2 == 1 ? 0.81649658092772603 : 0.57735026918962576;
        const Rl eta = Rl(amp) * symmetric_uniform<Rl>(word);
        s0 += eta;
        if constexpr (cx_of(p) != 0) sx += Rl(cx_of(p)) * eta;
        if constexpr (cy_of(p) != 0) sy += Rl(cy_of(p)) * eta;
        if constexpr (cz_of(p) != 0) sz += Rl(cz_of(p)) * eta;
        f[p] += (phi * C::template kScale<p>) * eta;
    });
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        Rl m = s0;
        if constexpr (cx_of(p) != 0) m += Rl(3 * cx_of(p)) * sx;
        if constexpr (cy_of(p) != 0) m += Rl(3 * cy_of(p)) * sy;
        if constexpr (cz_of(p) != 0) m += Rl(3 * cz_of(p)) * sz;
        f[p] -= phi * (w_of<Rl>(p) * C::template kScale<p>) * m;
    });
}

// Thread-to-node mappings of the lattice kernel.  MAP_SHIFTED is MAP_FLAT with every x-row
// rotated by the replica's x_shift, chosen on the host so that the planes within one node of a
// wall fall into as few 64-lane waves as possible: the other waves of a row then take the
// gather without solid tests (used when nx is a multiple of 64, so that waves are row segments).
// MAP_FLAT2: two nodes per lane, 64 apart (k_stream_collide_2n).
enum LatticeMapping { MAP_FLAT = 0, MAP_ROWS = 1, MAP_SHIFTED = 2, MAP_FLAT2 = 3 };

// Collision of one fluid node (Eq. lbe), the density check, and the thermal source F_p.
template <int S, bool TH>
__device__ __forceinline__ void relax_node(const Replica& R, typename Codec<S>::R* f, int idx,
                                           RunState* __restrict__ st) {
    using Rl = typename Codec<S>::R;
    const Rl rho = collide<S>(f, (Rl)R.omega, (Rl)R.rho0);
    if (!(rho > Rl(0)) || !(rho < Rl(1e30))) atomicOr(&st->err, LB_ERR_DENSITY);
    if constexpr (TH) {
        // the step counter does not move during a sweep with a thermal source
        const Rl phi = sqrt(fmax((Rl)R.noise_c * rho, Rl(0)));
        add_thermal<Codec<S>, Rl>(f, (uint32_t)idx, (uint32_t)st->step, R.seed_lo, R.seed_hi, phi);
    }
}

// The slots of a solid node: never read (a fluid node bounces back off its own slots, and the
// read-outs report zero there), but written with every sweep, the rest value w_p rho0 that
// lb_init leaves there, so that a store instruction of a wave covers whole cache lines.  A
// wave whose lanes skip their stores leaves partly written lines, which HBM completes with a
// read-modify-write: in 48-96 node rows, each crossing a wall, that cost the 16-bit sweep 40 %.
template <int S>
__device__ __forceinline__ void rest_slots(const Replica& R, typename Codec<S>::R* f) {
    using C = Codec<S>;
    using Rl = typename C::R;
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (C::deviation) f[p] = Rl(0);
        else f[p] = w_of<Rl>(p) * (Rl)R.rho0;
    });
}

template <int S, int BLOCK, bool NT, bool TH>
__global__ __launch_bounds__(BLOCK) void k_stream_collide(const Replica* __restrict__ reps,
                                                          const int* __restrict__ prefix,
                                                          int n_reps,
                                                          const typename Codec<S>::T* __restrict__ src,
                                                          typename Codec<S>::T* __restrict__ dst,
                                                          RunState* __restrict__ st, int bump_step,
                                                          int xcd_chunk, int mapping) {
    using C = Codec<S>;
    using Rl = typename C::R;
    if (bump_step && blockIdx.x == 0 && threadIdx.x == 0) st->step += 1;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, xcd_chunk);
    const int r = replica_of_tile(prefix, n_reps, tile);
    const Replica& R = reps[r];
    Rl f[Q];
    int idx;
    bool solid = false;
    if (mapping == MAP_ROWS) {
        // one wave per row segment: y, z and the face decisions are wave-uniform
        constexpr int W = BLOCK / 64;
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const RowUnit U = row_unit(R, (tile - prefix[r]) * W + wave);
        if (!U.valid) return;
        const int x = U.x0 + (threadIdx.x & 63);
        const int y = U.y, z = U.z;
        if (x >= R.nx) return;
        solid = is_solid(R, x, y, z);
        idx = x + R.nx * (y + R.ny * z);
        bool zone = false;
#pragma unroll
        for (int k = 0; k < LB_MAX_WALLS; ++k) {
            if (k >= R.n_walls) break;
            zone = zone || (U.x0 <= R.wall[k][1] + 1 && U.x0 + 63 >= R.wall[k][0] - 1);
        }
        if (!solid) {
            if (zone) gather_row<S, true>(R, src, idx, x, y, z, f);
            else gather_row<S, false>(R, src, idx, x, y, z, f);
        }
    } else {
        // 64 consecutive nodes per wave; waves that touch a y/z face take the general
        // resolver, waves next to a wall the solid-testing one
        const int n = (tile - prefix[r]) * BLOCK + threadIdx.x;
        const bool inside = n < R.V;
        bool active = inside;
        const uint32_t t = fdiv((uint32_t)n, R.div_nx);
        int x = n - (int)t * R.nx;
        if (mapping == MAP_SHIFTED) {
            x += R.x_shift;
            if (x >= R.nx) x -= R.nx;
        }
        idx = x + (int)t * R.nx;
        const uint32_t zz = fdiv(t, R.div_ny);
        const int y = (int)t - (int)zz * R.ny;
        const int z = (int)zz;
        bool face = false, zone = false, xface = false, pore = false;
        if (active) {
            if (is_solid(R, x, y, z)) active = false;
            face = y == 0 || y == R.ny - 1 || z == 0 || z == R.nz - 1;
            zone = in_wall_zone(R, x);
            xface = x == 0 || x == R.nx - 1;
            pore = near_pore(R, x, y, z);
        }
        face = face && active;
        zone = zone && active;
        xface = xface && active;
        pore = pore && active;
        const bool any_face = __ballot(face) != 0;
        const bool any_zone = __ballot(zone) != 0;
        const bool any_xface = __ballot(xface) != 0;
        const bool any_pore = __ballot(pore) != 0;
        if (!inside) return;
        solid = !active;
        if (active) {
            if (any_face) gather19<S, G_GENERIC>(R, src, idx, x, y, z, f);
            else if (any_pore) gather19<S, G_WALL>(R, src, idx, x, y, z, f);
            else if (any_zone) gather19<S, G_WALL_PLANE>(R, src, idx, x, y, z, f);
            else if (any_xface) gather19<S, G_FAST>(R, src, idx, x, y, z, f);
            else gather19<S, G_INTERIOR>(R, src, idx, x, y, z, f);
        }
    }

    if (solid) rest_slots<S>(R, f);
    else relax_node<S, TH>(R, f, idx, st);

    typename C::T* __restrict__ out = dst + R.pop_base + idx;
    const long long PS = R.S;  // population plane stride
    // non-temporal stores keep a box larger than the last-level cache from evicting the
    // next step's sources; a box that fits it is better left cached for the next sweep
    if constexpr (NT) {
        for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            __builtin_nontemporal_store(C::store_raw(f[p]), out + (long long)p * PS);
        });
    } else {
        for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            out[(long long)p * PS] = C::store_raw(f[p]);
        });
    }
}

template <int S, int KIND, class E>
__device__ __forceinline__ void gather_two(const Replica& R, const typename Codec<S>::T* __restrict__ src,
                                           const int* n, const int* x, const int* y, const int* z, E* f0,
                                           E* f1) {
    constexpr bool raw = !std::is_same_v<E, typename Codec<S>::R>;
    gather19<S, KIND, raw>(R, src, n[0], x[0], y[0], z[0], f0);
    gather19<S, KIND, raw>(R, src, n[1], x[1], y[1], z[1], f1);
}

// One LB step for two nodes per lane, 64 apart: a wave takes 128 consecutive nodes of a
// replica and every load still covers 64 consecutive elements.  Both nodes' 19 loads are
// issued before the first collision, so a wave keeps twice the bytes in flight while it
// computes (16-bit storage moves only 128 bytes per load).  Both gathers run for every lane:
// a solid node, or a lane past the end of the replica (which takes the last node), reads
// nodes of the box and its results are dropped; solid nodes store their rest slots.
template <int S, int BLOCK, bool NT, bool TH>
__global__ __launch_bounds__(BLOCK) void k_stream_collide_2n(const Replica* __restrict__ reps,
                                                             const int* __restrict__ prefix, int n_reps,
                                                             const typename Codec<S>::T* __restrict__ src,
                                                             typename Codec<S>::T* __restrict__ dst,
                                                             RunState* __restrict__ st, int bump_step,
                                                             int xcd_chunk) {
    using C = Codec<S>;
    using Rl = typename C::R;
    if (bump_step && blockIdx.x == 0 && threadIdx.x == 0) st->step += 1;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, xcd_chunk);
    const int r = replica_of_tile(prefix, n_reps, tile);
    const Replica& R = reps[r];
    const int first = (tile - prefix[r]) * (2 * BLOCK) + (threadIdx.x >> 6) * 128 + (threadIdx.x & 63);
    int n[2], x[2], y[2], z[2];
    bool act[2], in[2];
    bool face = false, zone = false, xface = false, pore = false;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        int m = first + 64 * k;
        in[k] = m < R.V;
        act[k] = in[k];
        if (!in[k]) m = R.V - 1;
        const uint32_t t = fdiv((uint32_t)m, R.div_nx);
        x[k] = m - (int)t * R.nx;
        const uint32_t zz = fdiv(t, R.div_ny);
        y[k] = (int)t - (int)zz * R.ny;
        z[k] = (int)zz;
        n[k] = m;
        // the gather kind covers every node the lane reads around, solid or not
        face = face || y[k] == 0 || y[k] == R.ny - 1 || z[k] == 0 || z[k] == R.nz - 1;
        zone = zone || in_wall_zone(R, x[k]);
        xface = xface || x[k] == 0 || x[k] == R.nx - 1;
        pore = pore || near_pore(R, x[k], y[k], z[k]);
        act[k] = act[k] && !is_solid(R, x[k], y[k], z[k]);
    }
    const bool any_face = __ballot(face) != 0;
    const bool any_zone = __ballot(zone) != 0;
    const bool any_xface = __ballot(xface) != 0;
    const bool any_pore = __ballot(pore) != 0;
    if (!in[0]) return;  // then the second node is outside too
    // 16-bit elements are gathered as stored and decoded after both nodes' loads are issued
    using E = std::conditional_t<C::deviation, typename C::T, Rl>;
    E g0[Q], g1[Q];
    if (any_face) gather_two<S, G_GENERIC>(R, src, n, x, y, z, g0, g1);
    else if (any_pore) gather_two<S, G_WALL>(R, src, n, x, y, z, g0, g1);
    else if (any_zone) gather_two<S, G_WALL_PLANE>(R, src, n, x, y, z, g0, g1);
    else if (any_xface) gather_two<S, G_FAST>(R, src, n, x, y, z, g0, g1);
    else gather_two<S, G_INTERIOR>(R, src, n, x, y, z, g0, g1);
    Rl f0[Q], f1[Q];
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (C::deviation) {
            f0[p] = C::load_raw(g0[p]);
            f1[p] = C::load_raw(g1[p]);
        } else {
            f0[p] = g0[p];
            f1[p] = g1[p];
        }
    });

    const long long PS = R.S;  // population plane stride
    typename C::T* __restrict__ out = dst + R.pop_base;
    auto finish = [&](Rl* f, int idx, bool fluid) {
        if (fluid) relax_node<S, TH>(R, f, idx, st);
        else rest_slots<S>(R, f);
        for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            if constexpr (NT) __builtin_nontemporal_store(C::store_raw(f[p]), out + (long long)p * PS + idx);
            else out[(long long)p * PS + idx] = C::store_raw(f[p]);
        });
    };
    finish(f0, n[0], act[0]);
    if (in[1]) finish(f1, n[1], act[1]);
}

// Same-pattern reference of the lattice kernel: every population of every node read at the
// kernel's pull address (the node index minus c_p's offset, wrapped into the replica; no faces,
// no solids, no arithmetic) and written unchanged to the node's own slot of the other buffer,
// in the kernel's tile order and store policy, one node per lane.  Its bandwidth bounds what
// the sweep's access pattern can reach.
template <int S, int BLOCK, bool NT>
__global__ __launch_bounds__(BLOCK) void k_pattern(const Replica* __restrict__ reps, const int* __restrict__ prefix,
                                                   int n_reps, const typename Codec<S>::T* __restrict__ src,
                                                   typename Codec<S>::T* __restrict__ dst, int xcd_chunk) {
    using T = typename Codec<S>::T;
    const int tile = xcd_tile(blockIdx.x, gridDim.x, xcd_chunk);
    const int r = replica_of_tile(prefix, n_reps, tile);
    const Replica& R = reps[r];
    const long long V = R.V, PS = R.S;
    const long long n = (long long)(tile - prefix[r]) * BLOCK + threadIdx.x;
    if (n >= V) return;
    const T* __restrict__ base = src + R.pop_base;
    T* __restrict__ out = dst + R.pop_base;
    const long long nx = R.nx, nxy = (long long)R.nx * R.ny;
    T v[Q];
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        long long s = n - (cx_of(p) + cy_of(p) * nx + cz_of(p) * nxy);
        if (s < 0) s += V;
        else if (s >= V) s -= V;
        v[p] = base[(long long)p * PS + s];
    });
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        if constexpr (NT) __builtin_nontemporal_store(v[p], out + (long long)p * PS + n);
        else out[(long long)p * PS + n] = v[p];
    });
}

// ---------------------------------------------------------------------------------
// Initial state: a post-collision buffer whose pull reproduces wanted pre-collision
// populations f0 (given, or f_eq of given rho/u, or w_p rho0).  Slot (s, q) holds
// f0 at the push target (x, p) of (s, q).
// ---------------------------------------------------------------------------------
// f_eq of Sec. II for all 19 populations (c_s^2 = 1/3), in FP64
__device__ __forceinline__ void feq19(double rho, double ux, double uy, double uz, double* feq) {
    const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        const double cu = cx_of(p) * ux + cy_of(p) * uy + cz_of(p) * uz;
        feq[p] = w_of<double>(p) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - usq);
    });
}

// element p of a register array without dynamic indexing
__device__ __forceinline__ double pick19(const double* a, int p) {
    double v = 0.0;
    for_pops([&](auto P) {
        constexpr int k = decltype(P)::value;
        v = (p == k) ? a[k] : v;
    });
    return v;
}

template <int S>
__global__ __launch_bounds__(256) void k_init(const Replica* __restrict__ reps, int r,
                                              typename Codec<S>::T* __restrict__ dst,
                                              const double* __restrict__ rho_in,
                                              const double* __restrict__ u_in,
                                              const double* __restrict__ pops_in) {
    using C = Codec<S>;
    const Replica& R = reps[r];
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= R.V) return;
    const long long V = R.V;  // the given fields are dense [19][V] / [3][V]
    const int sx = s % R.nx, sy = (s / R.nx) % R.ny, sz = s / (R.nx * R.ny);
    const bool solid = is_solid(R, sx, sy, sz);
    typename C::T* out = dst + R.pop_base + s;
    // the wanted pre-collision population p at node x
    auto wanted = [&](int p, int x) -> double {
        if (pops_in) return pops_in[(long long)p * V + x];
        const double rho = rho_in ? rho_in[x] : R.rho0;
        double feq[Q];
        if (u_in) feq19(rho, u_in[x], u_in[V + x], u_in[2 * V + x], feq);
        else feq19(rho, 0.0, 0.0, 0.0, feq);
        return pick19(feq, p);
    };
    for_pops([&](auto P) {
        constexpr int q = decltype(P)::value;
        double val = w_of<double>(q) * R.rho0;
        int p;
        if (!solid) {
            const int x = push_target<q>(R, sx, sy, sz, &p);
            val = wanted(p, x);
        }
        if constexpr (C::deviation) val -= w_of<double>(q) * R.rho0;
        out[(long long)q * R.S] = C::template store<q>((typename C::R)val);
    });
}

// ---------------------------------------------------------------------------------
// Pre-collision view of the current state (lb_moments): pull-gather of one node,
// decoded to FP64 full populations.
// ---------------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ void gather_f64(const Replica& R, const typename Codec<S>::T* __restrict__ src,
                                           int x, int y, int z, double* f) {
    using C = Codec<S>;
    const long long PS = R.S;  // population plane stride
    for_pops([&](auto P) {
        constexpr int p = decltype(P)::value;
        int q;
        const int node = pull_source<p>(R, x, y, z, &q);
        double v = (double)C::template load<p>(src[R.pop_base + (long long)q * PS + node]);
        if constexpr (C::deviation) v += w_of<double>(p) * R.rho0;
        f[p] = v;
    });
}

// mode 0: populations [19][count]; mode 1: rho, u_x, u_y, u_z [4][count]
template <int S>
__global__ __launch_bounds__(256) void k_gather(const Replica* __restrict__ reps, int r,
                                                const typename Codec<S>::T* __restrict__ src, int mode,
                                                long long node0, int count, double* __restrict__ out) {
    const Replica& R = reps[r];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const long long s = node0 + i;
    const int x = (int)(s % R.nx), y = (int)((s / R.nx) % R.ny), z = (int)(s / ((long long)R.nx * R.ny));
    double f[Q];
    if (is_solid(R, x, y, z)) {
        for_pops([&](auto P) { f[decltype(P)::value] = 0.0; });
    } else {
        gather_f64<S>(R, src, x, y, z, f);
    }
    if (mode == 0) {
        for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            out[(long long)p * count + i] = f[p];
        });
    } else {
        double rho = 0, jx = 0, jy = 0, jz = 0;
        for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            rho += f[p];
            jx += cx_of(p) * f[p];
            jy += cy_of(p) * f[p];
            jz += cz_of(p) * f[p];
        });
        const double inv = rho != 0.0 ? 1.0 / rho : 0.0;
        out[i] = rho;
        out[count + i] = jx * inv;
        out[2LL * count + i] = jy * inv;
        out[3LL * count + i] = jz * inv;
    }
}

// FP64 totals of rho and j over the fluid nodes of replica r (Eqs. dens, vel summed over the
// box): per-lane sums over a fixed sequence of 64-node chunks, wavefront butterfly, block
// tree, one partial per block; a second single-block pass adds the partials in a fixed order
// (deterministic for a given grid).
template <int S>
__global__ __launch_bounds__(256) void k_conserved_partial(const Replica R,
                                                           const typename Codec<S>::T* __restrict__ src,
                                                           double* __restrict__ partials) {
    using C = Codec<S>;
    using Rl = typename C::R;
    // 64 consecutive nodes per wave, dealt to the waves of the grid in a fixed order; each
    // wave takes the cheapest gather that covers its lanes, as the lattice kernel does
    double acc[4] = {0, 0, 0, 0};
    const int lane = threadIdx.x & 63;
    const long long chunks = (R.V + 63) / 64;
    for (long long ch = blockIdx.x * 4LL + (threadIdx.x >> 6); ch < chunks; ch += gridDim.x * 4LL) {
        const long long n = ch * 64 + lane;
        const bool inside = n < R.V;
        const int idx = inside ? (int)n : (int)(R.V - 1);
        const uint32_t t = fdiv((uint32_t)idx, R.div_nx);
        const int x = idx - (int)t * R.nx;
        const uint32_t zz = fdiv(t, R.div_ny);
        const int y = (int)t - (int)zz * R.ny;
        const int z = (int)zz;
        const bool fluid = inside && !is_solid(R, x, y, z);
        const bool any_face = __ballot(fluid && (y == 0 || y == R.ny - 1 || z == 0 || z == R.nz - 1)) != 0;
        const bool any_pore = __ballot(fluid && near_pore(R, x, y, z)) != 0;
        const bool any_zone = __ballot(fluid && in_wall_zone(R, x)) != 0;
        const bool any_xface = __ballot(fluid && (x == 0 || x == R.nx - 1)) != 0;
        if (!fluid) continue;
        Rl f[Q];
        if (any_face) gather19<S, G_GENERIC>(R, src, idx, x, y, z, f);
        else if (any_pore) gather19<S, G_WALL>(R, src, idx, x, y, z, f);
        else if (any_zone) gather19<S, G_WALL_PLANE>(R, src, idx, x, y, z, f);
        else if (any_xface) gather19<S, G_FAST>(R, src, idx, x, y, z, f);
        else gather19<S, G_INTERIOR>(R, src, idx, x, y, z, f);
        for_pops([&](auto P) {
            constexpr int p = decltype(P)::value;
            // the stored number decoded as Codec::load does, then the rest value added in FP64
            double v = (double)(f[p] * (Rl(1) / C::template kScale<p>));
            if constexpr (C::deviation) v += w_of<double>(p) * R.rho0;
            acc[0] += v;
            if constexpr (cx_of(p) != 0) acc[1] += cx_of(p) * v;
            if constexpr (cy_of(p) != 0) acc[2] += cy_of(p) * v;
            if constexpr (cz_of(p) != 0) acc[3] += cz_of(p) * v;
        });
    }
    __shared__ double red[4][256 / 64];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0;
        for (int w = 0; w < 256 / 64; ++w) v += red[threadIdx.x][w];
        partials[blockIdx.x * 4 + threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(256) void k_conserved_final(const double* __restrict__ partials, int nblk,
                                                         double* __restrict__ out4) {
    __shared__ double red[4][256];
    double acc[4] = {0, 0, 0, 0};
    // thread t adds partials t, t + 256, t + 512, ... in that order; eight rows are loaded
    // before they are added, so that their latencies overlap
    for (int b0 = threadIdx.x; b0 < nblk; b0 += 256 * 8) {
        double v[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + u * 256;
#pragma unroll
            for (int k = 0; k < 4; ++k) v[u][k] = b < nblk ? partials[b * 4 + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (b0 + u * 256 >= nblk) break;
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] += v[u][k];
        }
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int half = 128; half >= 1; half >>= 1) {
        if (threadIdx.x < half)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x < 4) out4[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------------
template <int S, int BLOCK, bool NT, bool TH>
static hipError_t launch_sc_n(const Context& c, const void* src, void* dst, bool bump, hipStream_t s) {
    using T = typename Codec<S>::T;
    if (c.lat.mapping == MAP_FLAT2) {
        if constexpr (BLOCK >= 128 && BLOCK <= 512) {
            hipLaunchKernelGGL((k_stream_collide_2n<S, BLOCK, NT, TH>), dim3(c.lat.total_tiles), dim3(BLOCK), 0, s,
                               c.d_reps, c.lat.d_prefix, (int)c.reps.size(), (const T*)src, (T*)dst, c.d_state,
                               bump ? 1 : 0, c.lat_chunk);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;  // two nodes per lane: blocks of 128 to 512 threads
        }
    }
    hipLaunchKernelGGL((k_stream_collide<S, BLOCK, NT, TH>), dim3(c.lat.total_tiles), dim3(BLOCK), 0, s,
                       c.d_reps, c.lat.d_prefix, (int)c.reps.size(), (const T*)src, (T*)dst, c.d_state,
                       bump ? 1 : 0, c.lat_chunk, c.lat.mapping);
    return hipGetLastError();
}

template <int S, int BLOCK, bool NT>
static hipError_t launch_pattern_n(const Context& c, const void* src, void* dst, hipStream_t s) {
    using T = typename Codec<S>::T;
    // the flat tile table of this block size (the rows mapping has other tiles)
    const LatticeLaunch* L = nullptr;
    for (const auto& l : c.lat_all)
        if (l.block == BLOCK && l.mapping == MAP_FLAT) L = &l;
    if (!L) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_pattern<S, BLOCK, NT>), dim3(L->total_tiles), dim3(BLOCK), 0, s, c.d_reps, L->d_prefix,
                       (int)c.reps.size(), (const T*)src, (T*)dst, c.lat_chunk);
    return hipGetLastError();
}

template <int S, int BLOCK>
static hipError_t launch_pattern_t(const Context& c, const void* src, void* dst, hipStream_t s) {
    return c.lat_nt ? launch_pattern_n<S, BLOCK, true>(c, src, dst, s) : launch_pattern_n<S, BLOCK, false>(c, src, dst, s);
}

template <int S>
static hipError_t launch_pattern_s(const Context& c, const void* src, void* dst, hipStream_t s) {
    switch (c.lat.block) {
        case 64: return launch_pattern_t<S, 64>(c, src, dst, s);
        case 128: return launch_pattern_t<S, 128>(c, src, dst, s);
        case 256: return launch_pattern_t<S, 256>(c, src, dst, s);
        case 512: return launch_pattern_t<S, 512>(c, src, dst, s);
        case 1024: return launch_pattern_t<S, 1024>(c, src, dst, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pattern(const Context& c, const void* src, void* dst, hipStream_t s) {
    switch (c.storage) {
        case LB_STORE_F64: return launch_pattern_s<LB_STORE_F64>(c, src, dst, s);
        case LB_STORE_F32: return launch_pattern_s<LB_STORE_F32>(c, src, dst, s);
        case LB_STORE_F16DEV: return launch_pattern_s<LB_STORE_F16DEV>(c, src, dst, s);
        case LB_STORE_BF16DEV: return launch_pattern_s<LB_STORE_BF16DEV>(c, src, dst, s);
        default: return hipErrorInvalidValue;
    }
}

template <int S, int BLOCK>
static hipError_t launch_sc_t(const Context& c, const void* src, void* dst, bool bump, hipStream_t s) {
    if (c.thermal) {
        // the thermal source reads the step counter, which must not move during the sweep
        if (bump) return hipErrorInvalidValue;
        return c.lat_nt ? launch_sc_n<S, BLOCK, true, true>(c, src, dst, false, s)
                        : launch_sc_n<S, BLOCK, false, true>(c, src, dst, false, s);
    }
    return c.lat_nt ? launch_sc_n<S, BLOCK, true, false>(c, src, dst, bump, s)
                    : launch_sc_n<S, BLOCK, false, false>(c, src, dst, bump, s);
}

template <int S>
static hipError_t launch_sc_s(const Context& c, const void* src, void* dst, bool bump, hipStream_t s) {
    switch (c.lat.block) {
        case 64: return launch_sc_t<S, 64>(c, src, dst, bump, s);
        case 128: return launch_sc_t<S, 128>(c, src, dst, bump, s);
        case 256: return launch_sc_t<S, 256>(c, src, dst, bump, s);
        case 512: return launch_sc_t<S, 512>(c, src, dst, bump, s);
        case 1024: return launch_sc_t<S, 1024>(c, src, dst, bump, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stream_collide(const Context& c, const void* src, void* dst, bool bump, hipStream_t s) {
    switch (c.storage) {
        case LB_STORE_F64: return launch_sc_s<LB_STORE_F64>(c, src, dst, bump, s);
        case LB_STORE_F32: return launch_sc_s<LB_STORE_F32>(c, src, dst, bump, s);
        case LB_STORE_F16DEV: return launch_sc_s<LB_STORE_F16DEV>(c, src, dst, bump, s);
        case LB_STORE_BF16DEV: return launch_sc_s<LB_STORE_BF16DEV>(c, src, dst, bump, s);
        default: return hipErrorInvalidValue;
    }
}

template <int S>
static hipError_t launch_init_t(const Context& c, int r, void* dst, const double* rho, const double* u,
                                const double* pops, hipStream_t s) {
    using T = typename Codec<S>::T;
    const int V = c.reps[r].V;
    hipLaunchKernelGGL((k_init<S>), dim3((V + 255) / 256), dim3(256), 0, s, c.d_reps, r, (T*)dst, rho, u,
                       pops);
    return hipGetLastError();
}

hipError_t launch_init(const Context& c, int r, void* dst, const double* rho, const double* u,
                       const double* pops, hipStream_t s) {
    switch (c.storage) {
        case LB_STORE_F64: return launch_init_t<LB_STORE_F64>(c, r, dst, rho, u, pops, s);
        case LB_STORE_F32: return launch_init_t<LB_STORE_F32>(c, r, dst, rho, u, pops, s);
        case LB_STORE_F16DEV: return launch_init_t<LB_STORE_F16DEV>(c, r, dst, rho, u, pops, s);
        case LB_STORE_BF16DEV: return launch_init_t<LB_STORE_BF16DEV>(c, r, dst, rho, u, pops, s);
        default: return hipErrorInvalidValue;
    }
}

template <int S>
static hipError_t launch_gather_t(const Context& c, int r, const void* src, int mode, long long node0,
                                  int count, double* out, hipStream_t s) {
    using T = typename Codec<S>::T;
    hipLaunchKernelGGL((k_gather<S>), dim3((count + 255) / 256), dim3(256), 0, s, c.d_reps, r,
                       (const T*)src, mode, node0, count, out);
    return hipGetLastError();
}

hipError_t launch_gather(const Context& c, int r, const void* src, int mode, long long node0, int count,
                         double* out, hipStream_t s) {
    switch (c.storage) {
        case LB_STORE_F64: return launch_gather_t<LB_STORE_F64>(c, r, src, mode, node0, count, out, s);
        case LB_STORE_F32: return launch_gather_t<LB_STORE_F32>(c, r, src, mode, node0, count, out, s);
        case LB_STORE_F16DEV: return launch_gather_t<LB_STORE_F16DEV>(c, r, src, mode, node0, count, out, s);
        case LB_STORE_BF16DEV: return launch_gather_t<LB_STORE_BF16DEV>(c, r, src, mode, node0, count, out, s);
        default: return hipErrorInvalidValue;
    }
}

template <int S>
static hipError_t launch_conserved_t(const Replica& R, const void* src, double* partials, int nblk, double* out4,
                                     hipStream_t s) {
    using T = typename Codec<S>::T;
    hipLaunchKernelGGL((k_conserved_partial<S>), dim3(nblk), dim3(256), 0, s, R, (const T*)src, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_conserved_final, dim3(1), dim3(256), 0, s, (const double*)partials, nblk, out4);
    return hipGetLastError();
}

hipError_t launch_conserved_desc(const Replica& R, int storage, const void* src, double* partials, int nblk,
                                 double* out4, hipStream_t s) {
    switch (storage) {
        case LB_STORE_F64: return launch_conserved_t<LB_STORE_F64>(R, src, partials, nblk, out4, s);
        case LB_STORE_F32: return launch_conserved_t<LB_STORE_F32>(R, src, partials, nblk, out4, s);
        case LB_STORE_F16DEV: return launch_conserved_t<LB_STORE_F16DEV>(R, src, partials, nblk, out4, s);
        case LB_STORE_BF16DEV: return launch_conserved_t<LB_STORE_BF16DEV>(R, src, partials, nblk, out4, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_conserved(const Context& c, int r, const void* src, double* out4, hipStream_t s) {
    // one block of partial sums per 4096 nodes (16 chunks of 64 nodes per wave), and at least
    // 2048 blocks (8192 waves) so that a small box still has loads in flight everywhere: a
    // 512^3 box took 2.6 ms with 2048 blocks and 1.8 ms with 32768
    const long long want = (c.reps[r].V + 4095) / 4096;
    const int nblk = (int)std::min<long long>(c.partial_blocks, std::max<long long>(2048, want));
    return launch_conserved_desc(c.reps[r], c.storage, src, c.d_partials, nblk, out4, s);
}

}  // namespace lbmd
