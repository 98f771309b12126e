/*
 * lbmd_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of one coupled
 * lattice-Boltzmann / bead-dynamics time step, written directly from
 * Fyta, Melchionna, Kaxiras & Succi, "Coupling Lattice Boltzmann with Atomistic
 * Dynamics for the multiscale simulation of nano-biological flows"
 * (arXiv:0710.1272), Sec. II.  It exists to check the GPU library and nothing
 * else: only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with the
 * GPU library; the D3Q19 table, the boundary resolver, the force laws and the
 * Philox generator below are written out again here on purpose.
 *
 * Formulation: the literal PUSH form of the lattice Boltzmann equation (Eq. lbe):
 * every fluid node collides its own populations and sends each one along its
 * link c_p to the node x + c_p, through an explicit boundary resolver.  The GPU
 * library uses the opposite (pull) formulation.
 *
 * Readings of the paper that the paper leaves open (numbered as in the design
 * notes of the repository):
 *   - S_p carries minus the bead force (the fluid receives -Fbar), Sec. II S_p eq.
 *   - the spread force is the average of drag + random force over the M MD substeps;
 *   - nearest-grid-point node = floor(x + 1/2) per axis, used for both directions;
 *   - u = sum f c / rho of the pre-collision populations, S_p added after collision;
 *   - D3Q19 weights 1/3, 1/18, 1/36, c_s^2 = 1/3;
 *   - boundary rules: periodic wrap, specular free-slip at outer faces (plane at
 *     -1/2 and n-1/2), half-way bounce-back at solid nodes;
 *   - bead integrator: kick-drift (symplectic Euler) with explicit drag;
 *   - random force: uniform, centred, variance 2 m gamma kT / h per component,
 *     drawn from Philox4x32-10 (Salmon et al., SC'11) keyed by the replica seed;
 *   - WCA bead-bead repulsion, bonded neighbours excluded; harmonic bonds;
 *     WCA wall repulsion on the distance to the nearest solid surface;
 *   - thermal source F_p (the paper gives no formula and cites the fluctuating LB of
 *     Adhikari et al.): noise on every non-conserved mode of the collision with the
 *     covariance that keeps the populations at their equilibrium fluctuations
 *     <df_p df_q> = mu rho w_p delta_pq, mu = kT / c_s^2 (Duenweg, Schiller and Ladd's
 *     fluctuation-dissipation condition for one BGK relaxation rate); uniform variates
 *     of unit variance drawn from Philox keyed by the replica seed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* ---------------------------------------------------------------------------
 * D3Q19 velocity set (Sec. II: "the standard three-dimensional 19-speed
 * lattice").  Order: rest, 6 faces, 12 edges; opposite pairs are adjacent.
 * ------------------------------------------------------------------------- */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight(int p)
{
    /* "a set of weights normalized to unity" (Sec. II, f_eq eq.) */
    if (p == 0) return 1.0 / 3.0;
    if (p <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static const double CS2 = 1.0 / 3.0; /* squared lattice sound speed */

/* the population whose velocity is -c_p */
static int opposite(int p)
{
    for (int q = 0; q < Q; ++q)
        if (CV[q][0] == -CV[p][0] && CV[q][1] == -CV[p][1] && CV[q][2] == -CV[p][2]) return q;
    return -1;
}

/* the population whose velocity is c_p with component `axis` negated */
static int mirror(int p, int axis)
{
    int c[3] = {CV[p][0], CV[p][1], CV[p][2]};
    c[axis] = -c[axis];
    for (int q = 0; q < Q; ++q)
        if (CV[q][0] == c[0] && CV[q][1] == c[1] && CV[q][2] == c[2]) return q;
    return -1;
}

/* ---------------------------------------------------------------------------
 * Problem description.
 * ------------------------------------------------------------------------- */
typedef struct {
    int nx, ny, nz;
    int bc[3];       /* per axis: 0 = periodic, 1 = free-slip (specular) faces */
    int n_walls;     /* 0, 1 or 2 separating walls */
    int wall[2][6];  /* x0,x1: solid planes x0..x1; y0,y1,z0,z1: open pore (empty if y0>y1) */
    double tau;      /* BGK relaxation time, omega = 1/tau (Delta t = 1) */
    double rho0;     /* reference density */
    double kT;       /* temperature of the thermal source F_p; 0: F_p = 0 */
} ora_box;

typedef struct {
    int M;           /* MD substeps per LB step, Delta t_MD = 1/M */
    double mass, gamma, kT;
    double k_bond, r0;        /* harmonic bond k (r-r0)^2/2 */
    double eps, sigma;        /* bead-bead WCA */
    double eps_w, sigma_w;    /* bead-wall WCA */
    double f_drive;           /* pulling force magnitude inside the pore */
    int drive_sign;           /* +1: along +x, -1: along -x */
    int rigid;                /* 1: rigid bonds of length r0 (SHAKE/RATTLE), 0: harmonic bonds */
    double kappa_phi;         /* angular term kappa_phi phi^2 / 2 between consecutive bonds */
    double shake_tol;         /* rigid bonds: |s^2 - r0^2| <= shake_tol r0^2 */
    int shake_iter;           /* rigid bonds: most Newton iterations per substep */
    int stencil;              /* coupling stencil: 0 nearest node, 1 trilinear over the 8 surrounding nodes */
} ora_md;

enum { ORA_BEAD_IN_SOLID = 1, ORA_BEAD_OUTSIDE = 2, ORA_NONFINITE = 4, ORA_BOND_STRETCH = 8,
       ORA_CONSTRAINT = 32 };

static long node_index(const ora_box* b, int x, int y, int z)
{
    return (long)x + (long)b->nx * ((long)y + (long)b->ny * (long)z);
}

static int pore_open(const int* w) { return w[2] <= w[3] && w[4] <= w[5]; }

/* A node is solid when it lies inside a wall's x-range and outside that wall's
 * pore (Sec. III: a separating wall with a square hole at its centre). */
int ora_is_solid(const ora_box* b, int x, int y, int z)
{
    for (int k = 0; k < b->n_walls; ++k) {
        const int* w = b->wall[k];
        if (x < w[0] || x > w[1]) continue;
        if (pore_open(w) && y >= w[2] && y <= w[3] && z >= w[4] && z <= w[5]) continue;
        return 1;
    }
    return 0;
}

int ora_is_pore(const ora_box* b, int x, int y, int z)
{
    for (int k = 0; k < b->n_walls; ++k) {
        const int* w = b->wall[k];
        if (x >= w[0] && x <= w[1] && pore_open(w) && y >= w[2] && y <= w[3] && z >= w[4] &&
            z <= w[5])
            return 1;
    }
    return 0;
}

/* Push-form boundary resolver.  The population q leaving fluid node s travels
 * along c_q.  On a periodic axis it wraps; on a free-slip axis, leaving the box
 * reflects that velocity component and keeps the node coordinate; if it lands
 * on a solid node it returns to s reversed (half-way bounce-back). */
void ora_push_target(const ora_box* b, int sx, int sy, int sz, int q, int* out)
{
    int n[3] = {b->nx, b->ny, b->nz};
    int s[3] = {sx, sy, sz};
    int t[3];
    int p = q;
    for (int a = 0; a < 3; ++a) {
        t[a] = s[a] + CV[q][a];
        if (t[a] < 0 || t[a] >= n[a]) {
            if (b->bc[a] == 0) {
                t[a] = (t[a] + n[a]) % n[a];
            } else {
                t[a] = s[a];
                p = mirror(p, a);
            }
        }
    }
    if (ora_is_solid(b, t[0], t[1], t[2])) {
        t[0] = s[0];
        t[1] = s[1];
        t[2] = s[2];
        p = opposite(q);
    }
    out[0] = t[0];
    out[1] = t[1];
    out[2] = t[2];
    out[3] = p;
}

/* ---------------------------------------------------------------------------
 * Equilibrium (Sec. II, f_eq eq.):
 *   f_p^eq = w_p rho { 1 + u.c_p / cs^2 + [ (u.c_p)^2 - cs^2 u.u ] / (2 cs^4) }
 * ------------------------------------------------------------------------- */
void ora_feq(double rho, const double* u, double* feq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int p = 0; p < Q; ++p) {
        double cu = CV[p][0] * u[0] + CV[p][1] * u[1] + CV[p][2] * u[2];
        feq[p] = weight(p) * rho * (1.0 + cu / CS2 + (cu * cu - CS2 * uu) / (2.0 * CS2 * CS2));
    }
}

/* Density and momentum (Sec. II, Eqs. dens and vel). */
static void node_moments(const double* fp, double* rho, double* j)
{
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int p = 0; p < Q; ++p) {
        r += fp[p];
        jx += fp[p] * CV[p][0];
        jy += fp[p] * CV[p][1];
        jz += fp[p] * CV[p][2];
    }
    *rho = r;
    j[0] = jx;
    j[1] = jy;
    j[2] = jz;
}

void ora_philox(const uint32_t* ctr_in, const uint32_t* key_in, uint32_t* out);
static double sym_uniform(uint32_t r);

/* Thermal source F_p of Eq. lbe at one fluid node, for the BGK collision with the
 * single rate omega (gamma = 1 - omega is the factor by which the collision scales
 * every non-conserved mode).  Fluctuation-dissipation asks for noise of covariance
 *     <F_p F_q> = mu rho (1 - gamma^2) (Pi W)_pq,   W = diag(w),  mu = kT / c_s^2,
 * where Pi removes the conserved density and momentum parts (so that the collision
 * keeps conserving them):  (Pi x)_p = x_p - w_p (sum_q x_q + c_p . sum_q c_q x_q / c_s^2).
 * Drawn as F = phi Pi eta with eta_p = sqrt(w_p) xi_p and xi_p independent of zero mean
 * and unit variance (then Cov(Pi eta) = Pi W Pi^T = Pi W); phi = sqrt(mu rho (1-gamma^2)).
 * xi_p = sqrt(12) U_p, U_p the symmetric uniforms of Philox words 4k..4k+3 of counters
 * (node, step, k, 2), k = 0..4, key = the replica seed; rho = the pre-collision density. */
static void thermal_source(const ora_box* b, long node, double rho, uint32_t step, uint64_t seed, double* F)
{
    const double omega = 1.0 / b->tau, gamma = 1.0 - omega;
    const double mu = b->kT / CS2;
    const double phi = sqrt(mu * rho * (1.0 - gamma * gamma));
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    double eta[20];
    for (int k = 0; k < 5; ++k) {
        uint32_t ctr[4] = {(uint32_t)node, step, (uint32_t)k, 2u}, rnd[4];
        ora_philox(ctr, key, rnd);
        for (int a = 0; a < 4; ++a) eta[4 * k + a] = sqrt(12.0) * sym_uniform(rnd[a]);
    }
    double s0 = 0.0, s1[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < Q; ++p) {
        eta[p] *= sqrt(weight(p));
        s0 += eta[p];
        for (int a = 0; a < 3; ++a) s1[a] += CV[p][a] * eta[p];
    }
    for (int p = 0; p < Q; ++p) {
        const double cs = CV[p][0] * s1[0] + CV[p][1] * s1[1] + CV[p][2] * s1[2];
        F[p] = phi * (eta[p] - weight(p) * (s0 + cs / CS2));
    }
}

/* Lattice layout shared as a data format with the callers: population p of
 * node (x,y,z) lives at f[p*V + x + nx*(y + ny*z)].  Solid nodes hold zero. */

/* One LB time step, Eq. lbe with Delta t = 1:
 *   f_p(x + c_p, t+1) = f_p(x,t) - omega (f_p - f_p^eq)(x,t) + F_p(x,t) + S_p(x,t)
 * F_p: the thermal source above when b->kT > 0 (its random numbers indexed by `step`
 * and keyed by `seed`), else 0.  f: pre-collision populations at t (in), at t+1 (out).
 * S: source or NULL.  work: scratch of 19*V doubles. Returns the number of fluid
 * nodes whose density was not positive and finite. */
long ora_lb_step(const ora_box* b, double* f, double* work, const double* S, uint32_t step, uint64_t seed)
{
    const long V = (long)b->nx * b->ny * b->nz;
    const double omega = 1.0 / b->tau;
    long bad = 0;
    memset(work, 0, sizeof(double) * Q * (size_t)V);
#pragma omp parallel for reduction(+ : bad) schedule(static)
    for (int z = 0; z < b->nz; ++z) {
        for (int y = 0; y < b->ny; ++y) {
            for (int x = 0; x < b->nx; ++x) {
                if (ora_is_solid(b, x, y, z)) continue;
                long i = node_index(b, x, y, z);
                double fp[Q], feq[Q], rho, j[3], u[3];
                for (int p = 0; p < Q; ++p) fp[p] = f[(long)p * V + i];
                node_moments(fp, &rho, j);
                if (!(rho > 0.0) || !isfinite(rho)) ++bad;
                u[0] = j[0] / rho;
                u[1] = j[1] / rho;
                u[2] = j[2] / rho;
                ora_feq(rho, u, feq);
                double F[Q] = {0.0};
                if (b->kT > 0.0) thermal_source(b, i, rho, step, seed, F);
                for (int q = 0; q < Q; ++q) {
                    double post = fp[q] - omega * (fp[q] - feq[q]) + F[q];
                    if (S) post += S[(long)q * V + i];
                    int t[4];
                    ora_push_target(b, x, y, z, q, t);
                    work[(long)t[3] * V + node_index(b, t[0], t[1], t[2])] = post;
                }
            }
        }
    }
    memcpy(f, work, sizeof(double) * Q * (size_t)V);
    return bad;
}

/* Pure streaming of a source field (linear part of Eq. lbe): adds S_p(x),
 * carried along c_p through the same resolver, to f.  Used to check the two
 * halves of a coupled step separately. */
void ora_add_streamed_source(const ora_box* b, double* f, const double* S)
{
    const long V = (long)b->nx * b->ny * b->nz;
    for (int z = 0; z < b->nz; ++z)
        for (int y = 0; y < b->ny; ++y)
            for (int x = 0; x < b->nx; ++x) {
                if (ora_is_solid(b, x, y, z)) continue;
                long i = node_index(b, x, y, z);
                for (int q = 0; q < Q; ++q) {
                    double s = S[(long)q * V + i];
                    if (s == 0.0) continue;
                    int t[4];
                    ora_push_target(b, x, y, z, q, t);
                    f[(long)t[3] * V + node_index(b, t[0], t[1], t[2])] += s;
                }
            }
}

/* Local density and velocity of every node (Eqs. dens, vel); solid nodes give
 * rho = 0, u = 0.  u is stored [3][V]. */
void ora_fields(const ora_box* b, const double* f, double* rho, double* u)
{
    const long V = (long)b->nx * b->ny * b->nz;
    for (int z = 0; z < b->nz; ++z)
        for (int y = 0; y < b->ny; ++y)
            for (int x = 0; x < b->nx; ++x) {
                long i = node_index(b, x, y, z);
                if (ora_is_solid(b, x, y, z)) {
                    rho[i] = 0.0;
                    u[i] = u[V + i] = u[2 * V + i] = 0.0;
                    continue;
                }
                double fp[Q], r, j[3];
                for (int p = 0; p < Q; ++p) fp[p] = f[(long)p * V + i];
                node_moments(fp, &r, j);
                rho[i] = r;
                u[i] = j[0] / r;
                u[V + i] = j[1] / r;
                u[2 * V + i] = j[2] / r;
            }
}

/* Total mass and momentum over the fluid nodes, summed in node order. */
void ora_conserved(const ora_box* b, const double* f, double* out4)
{
    const long V = (long)b->nx * b->ny * b->nz;
    double m = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int z = 0; z < b->nz; ++z)
        for (int y = 0; y < b->ny; ++y)
            for (int x = 0; x < b->nx; ++x) {
                if (ora_is_solid(b, x, y, z)) continue;
                long i = node_index(b, x, y, z);
                double fp[Q], r, j[3];
                for (int p = 0; p < Q; ++p) fp[p] = f[(long)p * V + i];
                node_moments(fp, &r, j);
                m += r;
                jx += j[0];
                jy += j[1];
                jz += j[2];
            }
    out4[0] = m;
    out4[1] = jx;
    out4[2] = jy;
    out4[3] = jz;
}

/* ---------------------------------------------------------------------------
 * Philox4x32-10, from its publication: J. K. Salmon, M. A. Moraes, R. O. Dror,
 * D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11.
 * ------------------------------------------------------------------------- */
void ora_philox(const uint32_t* ctr_in, const uint32_t* key_in, uint32_t* out)
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* centred uniform in [-1/2, 1/2): the top 24 bits read as a signed fraction */
static double centred(uint32_t r)
{
    return (double)(int32_t)(r & 0xFFFFFF00u) * (1.0 / 4294967296.0);
}

/* symmetric uniform in (-1/2, 1/2): the top 24 bits as k, (k + 1/2) / 2^24 - 1/2; mean 0,
 * variance (1 - 2^-48) / 12 */
static double sym_uniform(uint32_t r)
{
    return ((double)(r >> 8) + 0.5) * (1.0 / 16777216.0) - 0.5;
}

/* ---------------------------------------------------------------------------
 * Bead <-> lattice transfer (Sec. II, coupling steps 1 and 3, Fig. 1).
 * ------------------------------------------------------------------------- */

/* nearest-grid-point node of a position: floor(r + 1/2) per axis, wrapped on a
 * periodic axis and clamped into the box on a free-slip axis */
static void ngp(const ora_box* b, const double* r, int* g)
{
    int n[3] = {b->nx, b->ny, b->nz};
    for (int a = 0; a < 3; ++a) {
        double t = floor(r[a] + 0.5);
        long k;
        if (b->bc[a] == 0) {
            k = (long)fmod(t, (double)n[a]);
            if (k < 0) k += n[a];
        } else {
            if (!(t >= 0.0)) t = 0.0; /* also catches NaN */
            if (t > n[a] - 1) t = n[a] - 1;
            k = (long)t;
        }
        g[a] = (int)k;
    }
}

/* Step 1, "interpolation of the velocity": u_i = u(x) at the bead's nearest
 * node, from the pre-collision populations; u_i = 0 when that node is solid,
 * in which case node[i] = -1. */
void ora_interp(const ora_box* b, const double* f, int n, const double* r, double* u, long* node)
{
    const long V = (long)b->nx * b->ny * b->nz;
    for (int i = 0; i < n; ++i) {
        int g[3];
        ngp(b, r + 3 * i, g);
        if (ora_is_solid(b, g[0], g[1], g[2])) {
            node[i] = -1;
            u[3 * i] = u[3 * i + 1] = u[3 * i + 2] = 0.0;
            continue;
        }
        long k = node_index(b, g[0], g[1], g[2]);
        double fp[Q], rho, j[3];
        for (int p = 0; p < Q; ++p) fp[p] = f[(long)p * V + k];
        node_moments(fp, &rho, j);
        node[i] = k;
        u[3 * i] = j[0] / rho;
        u[3 * i + 1] = j[1] / rho;
        u[3 * i + 2] = j[2] / rho;
    }
}

/* Trilinear stencil of a position, the flagged variant of steps 1 and 3 (the fluid
 * velocity taken from, and the force given back to, the nodes surrounding the bead): the
 * 8 nodes floor(r_a) + {0, 1} per axis with weights prod_a (1 - |r_a - x_a|), which sum to
 * one.  A periodic axis wraps the node index; on a free-slip axis a node outside the box
 * (index -1 or n, for a bead within half a node of a face) is the mirror image of the face
 * node across the face plane, i.e. the face node itself. */
static void trilinear_stencil(const ora_box* b, const double* r, int node[8][3], double wt[8])
{
    const int n[3] = {b->nx, b->ny, b->nz};
    int lo[3][2];
    double w1[3][2];
    for (int a = 0; a < 3; ++a) {
        double t = floor(r[a]);
        if (!(t >= -1e9 && t <= 1e9)) t = 0.0; /* non-finite positions */
        const double fr = r[a] - t;
        w1[a][0] = 1.0 - fr;
        w1[a][1] = fr;
        for (int s = 0; s < 2; ++s) {
            long k = (long)t + s;
            if (b->bc[a] == 0) {
                k %= n[a];
                if (k < 0) k += n[a];
            } else {
                if (k < 0) k = 0;
                if (k > n[a] - 1) k = n[a] - 1;
            }
            lo[a][s] = (int)k;
        }
    }
    for (int c = 0; c < 8; ++c) {
        const int sx = c & 1, sy = (c >> 1) & 1, sz = (c >> 2) & 1;
        node[c][0] = lo[0][sx];
        node[c][1] = lo[1][sy];
        node[c][2] = lo[2][sz];
        wt[c] = w1[0][sx] * w1[1][sy] * w1[2][sz];
    }
}

/* Step 1 with the trilinear stencil: u_i = sum_c wt_c u(x_c), u = j / rho at fluid nodes and
 * 0 at solid ones. */
void ora_interp_trilinear(const ora_box* b, const double* f, int n, const double* r, double* u)
{
    const long V = (long)b->nx * b->ny * b->nz;
    for (int i = 0; i < n; ++i) {
        int nd[8][3];
        double wt[8];
        trilinear_stencil(b, r + 3 * i, nd, wt);
        u[3 * i] = u[3 * i + 1] = u[3 * i + 2] = 0.0;
        for (int c = 0; c < 8; ++c) {
            if (ora_is_solid(b, nd[c][0], nd[c][1], nd[c][2])) continue;
            long k = node_index(b, nd[c][0], nd[c][1], nd[c][2]);
            double fp[Q], rho, j[3];
            for (int p = 0; p < Q; ++p) fp[p] = f[(long)p * V + k];
            node_moments(fp, &rho, j);
            for (int a = 0; a < 3; ++a) u[3 * i + a] += wt[c] * j[a] / rho;
        }
    }
}

/* Step 3 with the trilinear stencil: S_p(x_c) += -wt_c (w_p / cs^2) Fbar_i . c_p at every
 * fluid node x_c of the stencil of the start-of-step position r (shares on solid nodes
 * are dropped, as a nearest node on a solid node drops the whole force). */
void ora_spread_trilinear(const ora_box* b, int n, const double* r, const double* fbar, double* S)
{
    const long V = (long)b->nx * b->ny * b->nz;
    for (int i = 0; i < n; ++i) {
        int nd[8][3];
        double wt[8];
        trilinear_stencil(b, r + 3 * i, nd, wt);
        for (int c = 0; c < 8; ++c) {
            if (ora_is_solid(b, nd[c][0], nd[c][1], nd[c][2])) continue;
            long k = node_index(b, nd[c][0], nd[c][1], nd[c][2]);
            for (int p = 0; p < Q; ++p) {
                double fc = fbar[3 * i] * CV[p][0] + fbar[3 * i + 1] * CV[p][1] +
                            fbar[3 * i + 2] * CV[p][2];
                S[(long)p * V + k] += -wt[c] * (weight(p) / CS2) * fc;
            }
        }
    }
}

/* Step 3, "extrapolation of the forces" (S_p eq.):
 *   S_p(x) += -(w_p / cs^2) Fbar_i . c_p  for every bead whose node is x.
 * S is [19][V] and is accumulated into. */
void ora_spread(const ora_box* b, int n, const long* node, const double* fbar, double* S)
{
    const long V = (long)b->nx * b->ny * b->nz;
    for (int i = 0; i < n; ++i) {
        if (node[i] < 0) continue;
        for (int p = 0; p < Q; ++p) {
            double fc = fbar[3 * i] * CV[p][0] + fbar[3 * i + 1] * CV[p][1] +
                        fbar[3 * i + 2] * CV[p][2];
            S[(long)p * V + node[i]] += -(weight(p) / CS2) * fc;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Bead forces (Sec. II, Eq. force and the LJ potential).
 * ------------------------------------------------------------------------- */

/* WCA: 4 eps [(s/r)^12 - (s/r)^6] + eps for r < 2^(1/6) s, else 0 */
static double wca_energy(double r2, double eps, double sigma)
{
    double rc2 = pow(2.0, 1.0 / 3.0) * sigma * sigma;
    if (r2 >= rc2) return 0.0;
    double s6 = pow(sigma * sigma / r2, 3.0);
    return 4.0 * eps * (s6 * s6 - s6) + eps;
}

/* -(1/r) dV/dr, so that the force on the first particle is this times d */
static double wca_force_over_r(double r2, double eps, double sigma)
{
    double rc2 = pow(2.0, 1.0 / 3.0) * sigma * sigma;
    if (r2 >= rc2) return 0.0;
    double s6 = pow(sigma * sigma / r2, 3.0);
    return 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
}

/* displacement a - b with the minimum-image convention on periodic axes */
static void displacement(const ora_box* b, const double* ra, const double* rb, double* d)
{
    int n[3] = {b->nx, b->ny, b->nz};
    for (int a = 0; a < 3; ++a) {
        d[a] = ra[a] - rb[a];
        if (b->bc[a] == 0) d[a] -= n[a] * floor(d[a] / n[a] + 0.5);
    }
}

/* Distance from r to the nearest solid surface, and the vector from that
 * nearest surface point to r.  Solid node (i,j,k) occupies the unit cube
 * centred on it; a wall is the slab x0-1/2..x1+1/2 minus the pore prism,
 * written as four boxes.  Returns HUGE_VAL when there is no wall. */
double ora_wall_distance(const ora_box* b, const double* r_in, double* dvec)
{
    /* positions are kept unwrapped on periodic axes: fold them into the box first */
    int nn[3] = {b->nx, b->ny, b->nz};
    double r[3];
    for (int a = 0; a < 3; ++a)
        r[a] = b->bc[a] == 0 ? r_in[a] - nn[a] * floor((r_in[a] + 0.5) / nn[a]) : r_in[a];
    double best = HUGE_VAL;
    dvec[0] = dvec[1] = dvec[2] = 0.0;
    for (int k = 0; k < b->n_walls; ++k) {
        const int* w = b->wall[k];
        double lo[4][3], hi[4][3];
        int nb;
        double X0 = w[0] - 0.5, X1 = w[1] + 0.5;
        if (pore_open(w)) {
            double Y0 = w[2] - 0.5, Y1 = w[3] + 0.5, Z0 = w[4] - 0.5, Z1 = w[5] + 0.5;
            nb = 4;
            /* below the pore in y, above it in y, and the two pieces beside it in z */
            double L[4][3] = {{X0, -HUGE_VAL, -HUGE_VAL}, {X0, Y1, -HUGE_VAL}, {X0, Y0, -HUGE_VAL},
                              {X0, Y0, Z1}};
            double H[4][3] = {{X1, Y0, HUGE_VAL}, {X1, HUGE_VAL, HUGE_VAL}, {X1, Y1, Z0},
                              {X1, Y1, HUGE_VAL}};
            memcpy(lo, L, sizeof L);
            memcpy(hi, H, sizeof H);
        } else {
            nb = 1;
            lo[0][0] = X0; lo[0][1] = -HUGE_VAL; lo[0][2] = -HUGE_VAL;
            hi[0][0] = X1; hi[0][1] = HUGE_VAL;  hi[0][2] = HUGE_VAL;
        }
        for (int m = 0; m < nb; ++m) {
            double d[3], d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double c = r[a];
                if (c < lo[m][a]) c = lo[m][a];
                if (c > hi[m][a]) c = hi[m][a];
                d[a] = r[a] - c;
                d2 += d[a] * d[a];
            }
            double dist = sqrt(d2);
            if (dist < best) {
                best = dist;
                dvec[0] = d[0];
                dvec[1] = d[1];
                dvec[2] = d[2];
            }
        }
    }
    return best;
}

static int bonded_to_next(int i, int n_chains, const int* chain_len)
{
    /* true when bead i and bead i+1 belong to the same chain */
    int start = 0;
    for (int c = 0; c < n_chains; ++c) {
        int end = start + chain_len[c];
        if (i >= start && i < end) return i + 1 < end;
        start = end;
    }
    return 0;
}

/* Angular term of the angle-potential equation at bead i (chain neighbours i-1 and
 * i+1): phi is the angle between the consecutive bonds d1 = r_i - r_{i-1} and
 * d2 = r_{i+1} - r_i (0 for a straight chain), V = kappa_phi phi^2 / 2.  Adds -grad V to
 * F of the three beads and returns V.  With c = cos(phi) = d1.d2 / (|d1||d2|):
 * dV/dr_{i-1} = -kappa phi / sin(phi) * (-dc/dd1), dV/dr_{i+1} = ... (dc/dd2),
 * and bead i takes minus the sum; phi / sin(phi) -> 1 as phi -> 0. */
static double angle_term(const ora_box* b, const ora_md* md, const double* r, int i, double* F)
{
    double d1[3], d2[3];
    displacement(b, r + 3 * i, r + 3 * (i - 1), d1);
    displacement(b, r + 3 * (i + 1), r + 3 * i, d2);
    double l1 = sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);
    double l2 = sqrt(d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2]);
    double dot = d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2];
    double cr[3] = {d1[1] * d2[2] - d1[2] * d2[1], d1[2] * d2[0] - d1[0] * d2[2], d1[0] * d2[1] - d1[1] * d2[0]};
    double cross = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double phi = atan2(cross, dot);
    double s = cross / (l1 * l2);
    double phi_over_sin = s > 1e-8 ? phi / s : 1.0 + phi * phi / 6.0;
    double c = dot / (l1 * l2);
    double k = md->kappa_phi * phi_over_sin;
    for (int a = 0; a < 3; ++a) {
        double dc1 = d2[a] / (l1 * l2) - c * d1[a] / (l1 * l1); /* d cos / d d1 */
        double dc2 = d1[a] / (l1 * l2) - c * d2[a] / (l2 * l2); /* d cos / d d2 */
        double fa = -k * dc1;                                   /* force on i-1 */
        double fc = k * dc2;                                    /* force on i+1 */
        F[3 * (i - 1) + a] += fa;
        F[3 * (i + 1) + a] += fc;
        F[3 * i + a] -= fa + fc;
    }
    return 0.5 * md->kappa_phi * phi * phi;
}

/* Conservative forces at the given positions: harmonic bonds (when the bonds are
 * not rigid), the angular term, WCA between all non-bonded pairs, WCA against the
 * nearest solid surface and against the free-slip faces.  F is [n][3] and is
 * overwritten.  Returns flags. */
int ora_conservative_forces(const ora_box* b, const ora_md* md, int n, int n_chains,
                            const int* chain_len, const double* r, double* F)
{
    int flags = 0;
    int nn[3] = {b->nx, b->ny, b->nz};
    memset(F, 0, sizeof(double) * 3 * (size_t)n);
    /* angular term between consecutive bonds */
    if (md->kappa_phi != 0.0)
        for (int i = 1; i + 1 < n; ++i)
            if (bonded_to_next(i - 1, n_chains, chain_len) && bonded_to_next(i, n_chains, chain_len))
                angle_term(b, md, r, i, F);
    /* bonds (rigid bonds carry no potential: their forces are the constraint reactions) */
    for (int i = 0; i + 1 < n; ++i) {
        if (md->rigid || !bonded_to_next(i, n_chains, chain_len)) continue;
        double d[3];
        displacement(b, r + 3 * (i + 1), r + 3 * i, d); /* from i to i+1 */
        double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (len > 2.0 * md->r0) flags |= ORA_BOND_STRETCH;
        double coef = md->k_bond * (len - md->r0) / len; /* force on i along d */
        for (int a = 0; a < 3; ++a) {
            F[3 * i + a] += coef * d[a];
            F[3 * (i + 1) + a] -= coef * d[a];
        }
    }
    /* non-bonded WCA */
    for (int i = 0; i < n; ++i) {
        for (int j = i + 1; j < n; ++j) {
            if (j == i + 1 && bonded_to_next(i, n_chains, chain_len)) continue;
            double d[3];
            displacement(b, r + 3 * i, r + 3 * j, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double c = wca_force_over_r(r2, md->eps, md->sigma);
            for (int a = 0; a < 3; ++a) {
                F[3 * i + a] += c * d[a];
                F[3 * j + a] -= c * d[a];
            }
        }
    }
    /* walls and free-slip faces */
    for (int i = 0; i < n; ++i) {
        const double* ri = r + 3 * i;
        if (!isfinite(ri[0]) || !isfinite(ri[1]) || !isfinite(ri[2])) flags |= ORA_NONFINITE;
        if (b->n_walls > 0) {
            double dv[3];
            double dist = ora_wall_distance(b, ri, dv);
            if (dist == 0.0) {
                flags |= ORA_BEAD_IN_SOLID;
            } else {
                double c = wca_force_over_r(dist * dist, md->eps_w, md->sigma_w);
                for (int a = 0; a < 3; ++a) F[3 * i + a] += c * dv[a];
            }
        }
        for (int a = 0; a < 3; ++a) {
            if (b->bc[a] != 1) continue;
            double dlo = ri[a] + 0.5, dhi = (nn[a] - 0.5) - ri[a];
            if (dlo <= 0.0 || dhi <= 0.0) {
                flags |= ORA_BEAD_OUTSIDE;
                continue;
            }
            F[3 * i + a] += wca_force_over_r(dlo * dlo, md->eps_w, md->sigma_w) * dlo;
            F[3 * i + a] -= wca_force_over_r(dhi * dhi, md->eps_w, md->sigma_w) * dhi;
        }
    }
    return flags;
}

/* Potential energy of the same interactions (for finite-difference checks). */
double ora_potential_energy(const ora_box* b, const ora_md* md, int n, int n_chains,
                            const int* chain_len, const double* r)
{
    double E = 0.0;
    int nn[3] = {b->nx, b->ny, b->nz};
    if (md->kappa_phi != 0.0) {
        double* junk = (double*)calloc(3 * (size_t)n, sizeof(double));
        for (int i = 1; i + 1 < n; ++i)
            if (bonded_to_next(i - 1, n_chains, chain_len) && bonded_to_next(i, n_chains, chain_len))
                E += angle_term(b, md, r, i, junk);
        free(junk);
    }
    for (int i = 0; i + 1 < n; ++i) {
        if (md->rigid || !bonded_to_next(i, n_chains, chain_len)) continue;
        double d[3];
        displacement(b, r + 3 * (i + 1), r + 3 * i, d);
        double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        E += 0.5 * md->k_bond * (len - md->r0) * (len - md->r0);
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            if (j == i + 1 && bonded_to_next(i, n_chains, chain_len)) continue;
            double d[3];
            displacement(b, r + 3 * i, r + 3 * j, d);
            E += wca_energy(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], md->eps, md->sigma);
        }
    for (int i = 0; i < n; ++i) {
        const double* ri = r + 3 * i;
        if (b->n_walls > 0) {
            double dv[3];
            double dist = ora_wall_distance(b, ri, dv);
            if (dist > 0.0) E += wca_energy(dist * dist, md->eps_w, md->sigma_w);
        }
        for (int a = 0; a < 3; ++a) {
            if (b->bc[a] != 1) continue;
            double dlo = ri[a] + 0.5, dhi = (nn[a] - 0.5) - ri[a];
            if (dlo > 0.0) E += wca_energy(dlo * dlo, md->eps_w, md->sigma_w);
            if (dhi > 0.0) E += wca_energy(dhi * dhi, md->eps_w, md->sigma_w);
        }
    }
    return E;
}

/* Tridiagonal solve by the Thomas algorithm: a[k] x[k-1] + bd[k] x[k] + c[k] x[k+1] = d[k]
 * for k = 0..m-1 (a[0], c[m-1] unused).  The solution overwrites d; bd and c are clobbered. */
static void thomas(int m, const double* a, double* bd, double* c, double* d)
{
    for (int k = 1; k < m; ++k) {
        double w = a[k] / bd[k - 1];
        bd[k] -= w * c[k - 1];
        d[k] -= w * d[k - 1];
    }
    d[m - 1] /= bd[m - 1];
    for (int k = m - 2; k >= 0; --k) d[k] = (d[k] - c[k] * d[k + 1]) / bd[k];
}

/* Rigid bonds: the N-1 holonomic constraints of Sec. II, enforced on positions by
 * SHAKE and on velocities by RATTLE.  Bond k joins beads k and k+1 of one chain; the
 * rows of the other k are identities.
 * Positions: r'_i = u_i + (lam_k d_k - lam_{k-1} d_{k-1}) / m, with u the unconstrained
 * positions and d_k = r_k - r_{k+1} the bond vectors at the start of the substep; the
 * multipliers solve |s_k|^2 = r0^2, s_k = r'_k - r'_{k+1}, by Newton iterations (the
 * Jacobian is tridiagonal: dg_k/dlam_k = 4 s_k.d_k/m, dg_k/dlam_{k+-1} = -2 s_k.d_{k+-1}/m)
 * until every |s_k^2 - r0^2| <= shake_tol r0^2.
 * Velocities: v_i = (r'_i - r_i) / h, then v_i += (mu_k s_k - mu_{k-1} s_{k-1}) / m with
 * the mu solving (v_k - v_{k+1}) . s_k = 0 for every bond (one tridiagonal solve), so the
 * relative velocity of bonded beads is orthogonal to their separation.
 * u is replaced by r'; v receives the constrained velocities.  Returns ORA_CONSTRAINT if
 * the Newton iterations did not converge. */
int ora_shake_rattle(const ora_box* b, const ora_md* md, int n, int n_chains, const int* chain_len,
                     const double* r_old, double* u, double* v, double h)
{
    if (n < 2) {
        for (int i = 0; i < 3 * n; ++i) v[i] = (u[i] - r_old[i]) / h;
        return 0;
    }
    const int m = n - 1;
    const double im = 1.0 / md->mass, b2 = md->r0 * md->r0;
    double* d = (double*)calloc(3 * (size_t)m, sizeof(double));   /* reference bond vectors */
    double* sv = (double*)calloc(3 * (size_t)m, sizeof(double));  /* current bond vectors */
    double* lam = (double*)calloc((size_t)m, sizeof(double));
    double* A = (double*)calloc((size_t)m, sizeof(double));
    double* B = (double*)calloc((size_t)m, sizeof(double));
    double* Cc = (double*)calloc((size_t)m, sizeof(double));
    double* R = (double*)calloc((size_t)m, sizeof(double));
    double* r = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    int* on = (int*)calloc((size_t)m, sizeof(int));
    for (int k = 0; k < m; ++k) {
        on[k] = bonded_to_next(k, n_chains, chain_len);
        if (on[k]) displacement(b, r_old + 3 * k, r_old + 3 * (k + 1), d + 3 * k);
    }
    int flags = ORA_CONSTRAINT;
    for (int it = 0; it <= md->shake_iter; ++it) {
        /* positions for the current multipliers and the constraint residuals */
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                double x = u[3 * i + a];
                if (i < m && on[i]) x += im * lam[i] * d[3 * i + a];
                if (i > 0 && on[i - 1]) x -= im * lam[i - 1] * d[3 * (i - 1) + a];
                r[3 * i + a] = x;
            }
        double worst = 0.0;
        for (int k = 0; k < m; ++k) {
            if (!on[k]) continue;
            displacement(b, r + 3 * k, r + 3 * (k + 1), sv + 3 * k);
            double g = sv[3 * k] * sv[3 * k] + sv[3 * k + 1] * sv[3 * k + 1] + sv[3 * k + 2] * sv[3 * k + 2] - b2;
            worst = fmax(worst, fabs(g));
            R[k] = -g;
        }
        if (worst <= md->shake_tol * b2) {
            flags = 0;
            break;
        }
        if (it == md->shake_iter) break;
        for (int k = 0; k < m; ++k) {
            if (!on[k]) {
                A[k] = Cc[k] = 0.0;
                B[k] = 1.0;
                R[k] = 0.0;
                continue;
            }
            const double* sk = sv + 3 * k;
            B[k] = 4.0 * im * (sk[0] * d[3 * k] + sk[1] * d[3 * k + 1] + sk[2] * d[3 * k + 2]);
            A[k] = (k > 0 && on[k - 1])
                       ? -2.0 * im * (sk[0] * d[3 * (k - 1)] + sk[1] * d[3 * (k - 1) + 1] + sk[2] * d[3 * (k - 1) + 2])
                       : 0.0;
            Cc[k] = (k + 1 < m && on[k + 1])
                        ? -2.0 * im * (sk[0] * d[3 * (k + 1)] + sk[1] * d[3 * (k + 1) + 1] + sk[2] * d[3 * (k + 1) + 2])
                        : 0.0;
        }
        thomas(m, A, B, Cc, R);
        for (int k = 0; k < m; ++k) lam[k] += R[k];
    }
    for (int i = 0; i < 3 * n; ++i) {
        v[i] = (r[i] - r_old[i]) / h;
        u[i] = r[i];
    }
    /* RATTLE: relative velocities of bonded beads orthogonal to their separations */
    for (int k = 0; k < m; ++k) {
        if (!on[k]) {
            A[k] = Cc[k] = 0.0;
            B[k] = 1.0;
            R[k] = 0.0;
            continue;
        }
        displacement(b, r + 3 * k, r + 3 * (k + 1), sv + 3 * k);
        const double* sk = sv + 3 * k;
        double rel = 0.0;
        for (int a = 0; a < 3; ++a) rel += (v[3 * k + a] - v[3 * (k + 1) + a]) * sk[a];
        R[k] = -rel;
        B[k] = 2.0 * im * (sk[0] * sk[0] + sk[1] * sk[1] + sk[2] * sk[2]);
        A[k] = 0.0;
        Cc[k] = 0.0;
    }
    for (int k = 0; k < m; ++k) {
        if (!on[k]) continue;
        const double* sk = sv + 3 * k;
        if (k > 0 && on[k - 1])
            A[k] = -im * (sk[0] * sv[3 * (k - 1)] + sk[1] * sv[3 * (k - 1) + 1] + sk[2] * sv[3 * (k - 1) + 2]);
        if (k + 1 < m && on[k + 1])
            Cc[k] = -im * (sk[0] * sv[3 * (k + 1)] + sk[1] * sv[3 * (k + 1) + 1] + sk[2] * sv[3 * (k + 1) + 2]);
    }
    thomas(m, A, B, Cc, R);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            if (i < m && on[i]) v[3 * i + a] += im * R[i] * sv[3 * i + a];
            if (i > 0 && on[i - 1]) v[3 * i + a] -= im * R[i - 1] * sv[3 * (i - 1) + a];
        }
    free(d); free(sv); free(lam); free(A); free(B); free(Cc); free(R); free(r); free(on);
    return flags;
}

/* Step 2: M molecular-dynamics substeps of length h = 1/M with the fluid
 * velocity u_i frozen (Sec. II).  Per substep, every force is evaluated at the
 * positions of the start of the substep:
 *   F = F_bond + F_WCA + F_wall + F_drive + F_drag + F_r,
 *   F_drag = -m gamma (v - u_i)                 (drag eq.)
 *   F_r    = A (c0, c1, c2),  A = sqrt(24 m gamma kT / h), c uniform in [-1/2,1/2)
 *   F_drive = f_drive x-hat inside the pore (Sec. III)
 * then v += (h/m) F; r += h v, and with rigid bonds SHAKE/RATTLE (ora_shake_rattle)
 * on the new positions and velocities.  Fbar accumulates (F_drag + F_r)/M, the force
 * whose reaction the fluid receives (constraint reactions are internal).  Philox
 * counter = (bead, step, substep, 1), key = (seed low word, seed high word). Returns
 * error flags. */
int ora_md_substeps(const ora_box* b, const ora_md* md, int n, int n_chains, const int* chain_len,
                    double* r, double* v, const double* u, double* fbar, uint32_t step,
                    uint64_t seed)
{
    const int M = md->M;
    const double h = 1.0 / M;
    const double A = sqrt(24.0 * md->mass * md->gamma * md->kT / h);
    int flags = 0;
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double* r0 = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    for (int i = 0; i < 3 * n; ++i) fbar[i] = 0.0;
    for (int k = 0; k < M; ++k) {
        flags |= ora_conservative_forces(b, md, n, n_chains, chain_len, r, F);
        for (int i = 0; i < n; ++i) {
            int g[3];
            ngp(b, r + 3 * i, g);
            if (ora_is_pore(b, g[0], g[1], g[2])) F[3 * i] += md->drive_sign * md->f_drive;
            uint32_t ctr[4] = {(uint32_t)i, step, (uint32_t)k, 1u}, rnd[4];
            ora_philox(ctr, key, rnd);
            for (int a = 0; a < 3; ++a) {
                double drag = -md->mass * md->gamma * (v[3 * i + a] - u[3 * i + a]);
                double noise = A * centred(rnd[a]);
                F[3 * i + a] += drag + noise;
                fbar[3 * i + a] += (drag + noise) / M;
            }
        }
        if (md->rigid) memcpy(r0, r, sizeof(double) * 3 * (size_t)n);
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                v[3 * i + a] += h / md->mass * F[3 * i + a];
                r[3 * i + a] += h * v[3 * i + a];
            }
        if (md->rigid) flags |= ora_shake_rattle(b, md, n, n_chains, chain_len, r0, r, v, h);
    }
    free(F);
    free(r0);
    return flags;
}

/* Translocation coordinate: number of beads past the mid-plane of wall 0
 * (Sec. III "number of translocated beads"), and the centre of mass. */
int ora_transloc(const ora_box* b, int n, const double* r, double* com)
{
    double xmid = b->n_walls > 0 ? 0.5 * (b->wall[0][0] + b->wall[0][1]) : 0.5 * (b->nx - 1);
    int nt = 0;
    com[0] = com[1] = com[2] = 0.0;
    for (int i = 0; i < n; ++i) {
        if (r[3 * i] > xmid) ++nt;
        com[0] += r[3 * i];
        com[1] += r[3 * i + 1];
        com[2] += r[3 * i + 2];
    }
    if (n > 0) {
        com[0] /= n;
        com[1] /= n;
        com[2] /= n;
    }
    return nt;
}

/* Observables of the translocation analysis (Sec. III) for the state at the end of an LB
 * step; u holds the fluid velocity interpolated at each bead for that step (0 without a
 * solvent).  out[0] N_T (beads past the mid-plane of wall 0); out[1] S_H = m gamma sum_i
 * v_i . u_i, the work rate of the fluid on the chain (eq. Shydro; the drag's fluid part
 * m gamma u_i times v_i); out[2] S_E = sum_i F_drive,i . v_i (eq. Selec; the drive acts on
 * beads whose nearest node is a pore node); out[3] K = m/2 sum_i |v_i|^2; out[4], out[5] the
 * squared radii of gyration of the untranslocated (x <= mid-plane) and translocated beads,
 * sum |r_i - r_c|^2 / n over each part (0 for an empty part); out[6] x of the centre of
 * mass. */
void ora_observables(const ora_box* b, const ora_md* md, int n, const double* r, const double* v,
                     const double* u, double* out)
{
    const double xmid = b->n_walls > 0 ? 0.5 * (b->wall[0][0] + b->wall[0][1]) : 0.5 * (b->nx - 1);
    double com[3];
    int nt = ora_transloc(b, n, r, com);
    double sh = 0.0, se = 0.0, ke = 0.0;
    for (int i = 0; i < n; ++i) {
        int g[3];
        ngp(b, r + 3 * i, g);
        for (int a = 0; a < 3; ++a) {
            sh += v[3 * i + a] * u[3 * i + a];
            ke += v[3 * i + a] * v[3 * i + a];
        }
        if (ora_is_pore(b, g[0], g[1], g[2])) se += md->drive_sign * md->f_drive * v[3 * i];
    }
    /* radii of gyration: centre of each part first, then the mean squared distance */
    double rg2[2] = {0.0, 0.0};
    for (int part = 0; part < 2; ++part) {
        double c[3] = {0.0, 0.0, 0.0};
        int cnt = 0;
        for (int i = 0; i < n; ++i) {
            if ((r[3 * i] > xmid) != (part == 1)) continue;
            for (int a = 0; a < 3; ++a) c[a] += r[3 * i + a];
            ++cnt;
        }
        if (cnt == 0) continue;
        for (int a = 0; a < 3; ++a) c[a] /= cnt;
        double s2 = 0.0;
        for (int i = 0; i < n; ++i) {
            if ((r[3 * i] > xmid) != (part == 1)) continue;
            for (int a = 0; a < 3; ++a) s2 += (r[3 * i + a] - c[a]) * (r[3 * i + a] - c[a]);
        }
        rg2[part] = s2 / cnt;
    }
    out[0] = nt;
    out[1] = md->mass * md->gamma * sh;
    out[2] = se;
    out[3] = 0.5 * md->mass * ke;
    out[4] = rg2[0];
    out[5] = rg2[1];
    out[6] = com[0];
}

/* One coupled LB time step in the order of Sec. II:
 *   1. interpolate u(x) -> u_i at the beads' nodes;
 *   2. M MD substeps with u_i frozen;
 *   3. extrapolate Fbar_i -> S_p(x);
 *   4. advance the populations with S_p (Eq. lbe).
 * f: [19][V] pre-collision populations; S, work: [19][V] scratch.
 * u, fbar: [n][3]; node: [n]. Returns MD flags, plus 16 if the LB step met a
 * non-positive density. */
int ora_coupled_step(const ora_box* b, const ora_md* md, int n, int n_chains, const int* chain_len,
                     double* f, double* S, double* work, double* r, double* v, double* u,
                     double* fbar, long* node, uint32_t step, uint64_t seed)
{
    const long V = (long)b->nx * b->ny * b->nz;
    ora_interp(b, f, n, r, u, node);
    double* r_start = NULL;
    if (md->stencil == 1) {
        /* the trilinear stencil of the start-of-step positions, for both halves */
        ora_interp_trilinear(b, f, n, r, u);
        r_start = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        memcpy(r_start, r, sizeof(double) * 3 * (size_t)n);
    }
    int flags = ora_md_substeps(b, md, n, n_chains, chain_len, r, v, u, fbar, step, seed);
    memset(S, 0, sizeof(double) * Q * (size_t)V);
    if (md->stencil == 1) {
        ora_spread_trilinear(b, n, r_start, fbar, S);
        free(r_start);
    } else {
        ora_spread(b, n, node, fbar, S);
    }
    if (ora_lb_step(b, f, work, S, step, seed) > 0) flags |= 16;
    return flags;
}

/* the velocity table, weights and opposites, for table-identity tests */
void ora_lattice(int* c, double* w, int* opp)
{
    for (int p = 0; p < Q; ++p) {
        c[3 * p] = CV[p][0];
        c[3 * p + 1] = CV[p][1];
        c[3 * p + 2] = CV[p][2];
        w[p] = weight(p);
        opp[p] = opposite(p);
    }
}

double ora_cs2(void) { return CS2; }

/* number of threads the LB loop uses (1 without OpenMP) */
int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
