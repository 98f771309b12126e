// lbmd_device.hpp -- device-side building blocks of the coupled LB / bead library (gfx950).
//
// Lattice: D3Q19 (arXiv:0710.1272 Sec. II, "the standard three-dimensional 19-speed
// lattice"), weights 1/3, 1/18, 1/36, c_s^2 = 1/3, in the population order of lbmd.h.
// Storage codecs: FP64, FP32, and 16-bit deviations h_p = s_p (f_p - w_p rho0) with
// s_p = 2, 16, 32 (powers of two near 1/w_p, keeping FP16 away from subnormals).
// Geometry is analytic (box size, face types, walls with a pore); no per-node flags.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbmd.h"

namespace lbmd {

constexpr int Q = 19;

__host__ __device__ constexpr int cx_of(int p) {
    constexpr int t[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[p];
}
__host__ __device__ constexpr int cy_of(int p) {
    constexpr int t[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[p];
}
__host__ __device__ constexpr int cz_of(int p) {
    constexpr int t[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[p];
}
// population with velocity -c_p: pairs are (2k-1, 2k)
__host__ __device__ constexpr int opp_of(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }

__host__ __device__ constexpr int find_pop(int x, int y, int z) {
    for (int p = 0; p < Q; ++p)
        if (cx_of(p) == x && cy_of(p) == y && cz_of(p) == z) return p;
    return -1;
}
// population with component `axis` of c_p reversed (specular reflection)
__host__ __device__ constexpr int mirror_of(int p, int axis) {
    return axis == 0 ? find_pop(-cx_of(p), cy_of(p), cz_of(p))
         : axis == 1 ? find_pop(cx_of(p), -cy_of(p), cz_of(p))
                     : find_pop(cx_of(p), cy_of(p), -cz_of(p));
}
template <class R>
__host__ __device__ constexpr R w_of(int p) {
    return p == 0 ? R(1) / R(3) : (p <= 6 ? R(1) / R(18) : R(1) / R(36));
}
// 16-bit deviation scale (power of two)
__host__ __device__ constexpr float scale_of(int p) { return p == 0 ? 2.0f : (p <= 6 ? 16.0f : 32.0f); }

// ---------------------------------------------------------------------------------
// Storage codecs.
// ---------------------------------------------------------------------------------
template <int S>
struct Codec;

// load/store: the population (full, or its deviation from w_p rho0).  load_raw/store_raw: the
// stored number as such (16-bit: the scaled deviation s_p (f_p - w_p rho0)), which the lattice
// kernel collides in directly with the scales folded into its constants; kScale<P> is the
// factor between the two (1 for full storage).
template <>
struct Codec<LB_STORE_F64> {
    using T = double;
    using R = double;
    static constexpr bool deviation = false;
    template <int P>
    static constexpr R kScale = 1.0;
    template <int P>
    __device__ static R load(T v) { return v; }
    template <int P>
    __device__ static T store(R v) { return v; }
    __device__ static R load_raw(T v) { return v; }
    __device__ static T store_raw(R v) { return v; }
};

template <>
struct Codec<LB_STORE_F32> {
    using T = float;
    using R = float;
    static constexpr bool deviation = false;
    template <int P>
    static constexpr R kScale = 1.0f;
    template <int P>
    __device__ static R load(T v) { return v; }
    template <int P>
    __device__ static T store(R v) { return v; }
    __device__ static R load_raw(T v) { return v; }
    __device__ static T store_raw(R v) { return v; }
};

template <>
struct Codec<LB_STORE_F16DEV> {
    using T = _Float16;
    using R = float;
    static constexpr bool deviation = true;
    template <int P>
    static constexpr R kScale = scale_of(P);
    template <int P>
    __device__ static R load(T v) { return (float)v * (1.0f / scale_of(P)); }
    template <int P>
    __device__ static T store(R v) { return (_Float16)(v * scale_of(P)); }  // IEEE round-to-nearest-even
    __device__ static R load_raw(T v) { return (float)v; }
    __device__ static T store_raw(R v) { return (_Float16)v; }
};

template <>
struct Codec<LB_STORE_BF16DEV> {
    using T = uint16_t;
    using R = float;
    static constexpr bool deviation = true;
    template <int P>
    static constexpr R kScale = scale_of(P);
    __device__ static R load_raw(T v) { return __builtin_bit_cast(float, (uint32_t)v << 16); }
    // round to nearest even (one hardware conversion on gfx950); NaN stays a quiet NaN
    __device__ static T store_raw(R v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    template <int P>
    __device__ static R load(T v) { return load_raw(v) * (1.0f / scale_of(P)); }
    template <int P>
    __device__ static T store(R v) { return store_raw(v * scale_of(P)); }
};

// runtime-p wrappers (init / gather paths that are not performance critical)
template <int S, int P = 0>
__device__ inline typename Codec<S>::R load_rt(typename Codec<S>::T v, int p) {
    if constexpr (P == Q) {
        return 0;
    } else {
        if (p == P) return Codec<S>::template load<P>(v);
        return load_rt<S, P + 1>(v, p);
    }
}
template <int S, int P = 0>
__device__ inline typename Codec<S>::T store_rt(typename Codec<S>::R v, int p) {
    if constexpr (P == Q) {
        return typename Codec<S>::T(0);
    } else {
        if (p == P) return Codec<S>::template store<P>(v);
        return store_rt<S, P + 1>(v, p);
    }
}

// ---------------------------------------------------------------------------------
// Unsigned division by a run-time invariant (Granlund & Montgomery 1994, Fig. 4.1):
// q = (t + ((n - t) >> 1)) >> (l - 1), t = mulhi(m, n), l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1.  d = 1 is handled separately.
// ---------------------------------------------------------------------------------
struct FastDiv {
    uint32_t d, m, s;
};
inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f{d, 0u, 0u};
    if (d <= 1) return f;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
    f.s = l;
    return f;
}
__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f) {
    if (f.d <= 1) return n;
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t t = __umulhi(n, f.m);
#else
    uint32_t t = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
    return (t + ((n - t) >> 1)) >> (f.s - 1);
}

// ---------------------------------------------------------------------------------
// Replica descriptor: everything a kernel needs to know about one box.
// ---------------------------------------------------------------------------------
struct Replica {
    int nx, ny, nz, V;
    int S;              // population plane stride in elements (S >= V, see plane_stride)
    int fs[3];          // 1 if the axis has free-slip faces, 0 if periodic
    int n_walls;
    int wall[LB_MAX_WALLS][6];
    int wzone_lo, wzone_hi;  // x range within one node of any wall (lanes that need solid checks)
    int x_shift;        // shifted flat mapping: position n of a row holds x = (n + x_shift) mod nx
    long long pop_base; // element offset of this replica's [19][S] block
    int bead0, n_beads;
    uint32_t seed_lo, seed_hi;
    double omega, rho0;
    double noise_c;     // thermal source: phi^2 = noise_c rho (0 without one)
    double xmid;        // mid-plane of wall 0, for the translocation count
    FastDiv div_nx, div_ny;
};

__host__ __device__ inline bool pore_open(const int* w) { return w[2] <= w[3] && w[4] <= w[5]; }

// wall loops run over the compile-time maximum with a guard, so that the wall table
// is indexed by constants (no private-array indexing)
__host__ __device__ inline bool is_solid(const Replica& R, int x, int y, int z) {
    bool s = false;
#pragma unroll
    for (int k = 0; k < LB_MAX_WALLS; ++k) {
        if (k >= R.n_walls) break;
        const int* w = R.wall[k];
        bool inx = x >= w[0] && x <= w[1];
        bool pore = pore_open(w) && y >= w[2] && y <= w[3] && z >= w[4] && z <= w[5];
        s = s || (inx && !pore);
    }
    return s;
}

__host__ __device__ inline bool is_pore(const Replica& R, int x, int y, int z) {
    bool s = false;
#pragma unroll
    for (int k = 0; k < LB_MAX_WALLS; ++k) {
        if (k >= R.n_walls) break;
        const int* w = R.wall[k];
        s = s || (x >= w[0] && x <= w[1] && pore_open(w) && y >= w[2] && y <= w[3] && z >= w[4] &&
                  z <= w[5]);
    }
    return s;
}

// population P with the components flagged in (fx, fy, fz) reversed; all
// candidates are compile-time constants, the choice is a select tree
template <int P>
__host__ __device__ __forceinline__ int mirror_combo(bool fx, bool fy, bool fz) {
    constexpr int mx = mirror_of(P, 0), my = mirror_of(P, 1), mz = mirror_of(P, 2);
    constexpr int mxy = mirror_of(mx, 1), mxz = mirror_of(mx, 2), myz = mirror_of(my, 2);
    constexpr int mxyz = mirror_of(mxy, 2);
    return fx ? (fy ? (fz ? mxyz : mxy) : (fz ? mxz : mx)) : (fy ? (fz ? myz : my) : (fz ? mz : P));
}

// Face resolution of the pull source of population P at node (x,y,z): s = x - c_P; a periodic
// axis wraps, a free-slip axis keeps x_a and reflects component a.  No solidity test.  Returns
// the node index within the replica, its coordinates in sc[3] and the population stored there
// in *q.
template <int P>
__host__ __device__ __forceinline__ int pull_resolve(const Replica& R, int x, int y, int z, int* sc, int* q) {
    constexpr int cx = cx_of(P), cy = cy_of(P), cz = cz_of(P);
    int sx = x - cx, sy = y - cy, sz = z - cz;
    bool fx = false, fy = false, fz = false;
    if constexpr (cx != 0) {
        if (sx < 0 || sx >= R.nx) {
            if (R.fs[0]) { sx = x; fx = true; }
            else sx += sx < 0 ? R.nx : -R.nx;
        }
    }
    if constexpr (cy != 0) {
        if (sy < 0 || sy >= R.ny) {
            if (R.fs[1]) { sy = y; fy = true; }
            else sy += sy < 0 ? R.ny : -R.ny;
        }
    }
    if constexpr (cz != 0) {
        if (sz < 0 || sz >= R.nz) {
            if (R.fs[2]) { sz = z; fz = true; }
            else sz += sz < 0 ? R.nz : -R.nz;
        }
    }
    *q = mirror_combo<P>(fx, fy, fz);
    sc[0] = sx;
    sc[1] = sy;
    sc[2] = sz;
    return sx + R.nx * (sy + R.ny * sz);
}

// Pull resolver for a fluid node (x,y,z) and population P: where the value that
// arrives in slot (x,P) was stored after the previous collision.  The face-resolved
// source, or, when that source is solid, slot (x, opp(P)): the population bounced back.
// Returns the node index within the replica; *q receives the population.
template <int P>
__host__ __device__ __forceinline__ int pull_source(const Replica& R, int x, int y, int z, int* q) {
    int sc[3];
    const int s = pull_resolve<P>(R, x, y, z, sc, q);
    if (is_solid(R, sc[0], sc[1], sc[2])) {
        *q = opp_of(P);
        return x + R.nx * (y + R.ny * z);
    }
    return s;
}

// Face resolution of the push target of population QP leaving node (sx,sy,sz), the inverse of
// pull_resolve: t = s + c_QP, a periodic axis wraps, a free-slip axis keeps s_a and reflects
// component a.  No solidity test.  Returns the node index, its coordinates in tc[3] and the
// population that arrives there in *p.
template <int QP>
__host__ __device__ __forceinline__ int push_resolve(const Replica& R, int sx, int sy, int sz, int* tc, int* p) {
    constexpr int cx = cx_of(QP), cy = cy_of(QP), cz = cz_of(QP);
    int tx = sx + cx, ty = sy + cy, tz = sz + cz;
    bool fx = false, fy = false, fz = false;
    if constexpr (cx != 0) {
        if (tx < 0 || tx >= R.nx) {
            if (R.fs[0]) { tx = sx; fx = true; }
            else tx += tx < 0 ? R.nx : -R.nx;
        }
    }
    if constexpr (cy != 0) {
        if (ty < 0 || ty >= R.ny) {
            if (R.fs[1]) { ty = sy; fy = true; }
            else ty += ty < 0 ? R.ny : -R.ny;
        }
    }
    if constexpr (cz != 0) {
        if (tz < 0 || tz >= R.nz) {
            if (R.fs[2]) { tz = sz; fz = true; }
            else tz += tz < 0 ? R.nz : -R.nz;
        }
    }
    *p = mirror_combo<QP>(fx, fy, fz);
    tc[0] = tx;
    tc[1] = ty;
    tc[2] = tz;
    return tx + R.nx * (ty + R.ny * tz);
}

// Push resolver (inverse of pull_source): where population Q leaving fluid node s
// ends up, bounced back into (s, opp(Q)) when the face-resolved target is solid.  Used to
// build a post-collision buffer whose pull gives wanted populations.
template <int QP>
__host__ __device__ __forceinline__ int push_target(const Replica& R, int sx, int sy, int sz, int* p) {
    int tc[3];
    const int t = push_resolve<QP>(R, sx, sy, sz, tc, p);
    if (is_solid(R, tc[0], tc[1], tc[2])) {
        *p = opp_of(QP);
        return sx + R.nx * (sy + R.ny * sz);
    }
    return t;
}

// ---------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two 32x32->64
// multiplies with a Weyl-sequence key schedule.
// ---------------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};
__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        uint64_t a = (uint64_t)0xD2511F53u * c.x;
        uint64_t b = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = (uint32_t)(b >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)b;
        n.z = (uint32_t)(a >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)a;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}
// top 24 bits as a signed fraction in [-1/2, 1/2); exact in FP32
template <class R>
__host__ __device__ inline R centred_uniform(uint32_t r) {
    return (R)(int32_t)(r & 0xFFFFFF00u) * (R)(1.0 / 4294967296.0);
}
// top 24 bits k as (k + 1/2) / 2^24 - 1/2: symmetric about 0 in (-1/2, 1/2), variance
// (1 - 2^-48) / 12; one rounding in FP32, exact in FP64
template <class R>
__host__ __device__ inline R symmetric_uniform(uint32_t r) {
    return (R)(r >> 8) * (R)(1.0 / 16777216.0) + (R)(1.0 / 33554432.0 - 0.5);
}

// ---------------------------------------------------------------------------------
// Device-side run state and bead buffers.
// ---------------------------------------------------------------------------------
constexpr int kNeighbourMax = 64;  // Verlet-list capacity per bead

struct RunState {
    long long step;  // LB step counter (Philox counter word)
    unsigned err;    // error word, LB_ERR_* bits
    unsigned pad;
};

template <class Real>
struct BeadPtrs {
    double* r;          // [3][Ntot] positions (FP64 accumulation)
    Real* v;            // [3][Ntot]
    Real* u;            // [3][Ntot] interpolated fluid velocity
    Real* fbar;         // [3][Ntot] substep-averaged drag + random force
    int* node;          // [Ntot] nearest node (within the replica), -1 on solid
    unsigned char* bond_next;  // [Ntot] 1 if bead i and i+1 are bonded
    long long* agg_at;  // [2][Ntot]: element offset of population 0 at the node a bead leads
                        // (pop_base + node, else -1), and the replica's plane stride S
    Real* agg_f;        // [3][Ntot] summed Fbar of the beads sharing the node a bead leads
    int* rep_of;        // [Ntot] replica of each bead
    double* diag;       // [n_replicas][8]: N_T, t_done, com x,y,z, last step, list builds,
                        // stored lists valid (1) or not (0)
    unsigned short* nlist;  // [kNeighbourMax][Ntot] Verlet neighbours (index within the replica)
    int* ncount;        // [Ntot] number of neighbours; > kNeighbourMax means overflow
    double* rref;       // [3][Ntot] positions at the last list build (lists are kept across
                        // LB steps while diag[7] of the replica is 1)
    double* rs;         // [3][Ntot] start-of-step positions (trilinear stencil of the spread)
    double* obs;        // [n_replicas][obs_cap + 1][8] observable record (header row first)
    // deterministic trilinear spread: open-addressing table of the nodes the stencils touch
    unsigned long long* hkey;  // [hcap] element offset of the node's population 0, plus 1 (0: empty)
    int* hrep;                 // [hcap] replica of the node
    long long* hsum;           // [18][hcap] fixed-point sums of the moving populations' sources
    unsigned hcap;             // power of two, or 0 without the trilinear stencil
    int obs_every, obs_cap;
    int ntot;
};

}  // namespace lbmd
