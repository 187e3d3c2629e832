/*
 * CPU oracle of the generalized lattice Boltzmann model (GLBM) of
 * Wang, Chen, Kang & Rahman, "Permeability prediction of organic shale with
 * generalized lattice Boltzmann model considering surface diffusion effect"
 * (arXiv:1601.00704), Sec. 2.3, Eq. (27)-(37).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness authority that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product never does.  It shares
 * no code, header, table or constant with the GPU path.
 *
 * It is written for a reader with the paper beside it, not for speed:
 *   - populations f_i are stored as plain values (no shift), one plane per
 *     direction, f[i * N + node], node = (z * ny + y) * nx + x;
 *   - one step is "collide, then stream" exactly as Eq. (29) reads: the
 *     post-collision value at x is pushed to x + e_i;
 *   - the moments are Eq. (32)-(35), the drag force Eq. (27) with K -> K_app
 *     (Eq. 28), the equilibrium Eq. (30) and the forcing term Eq. (31);
 *   - observables are summed in one fixed serial order, so results do not
 *     depend on the thread count.
 *
 * Arithmetic: FP64 by default.  The same source compiled with REF_LONG_DOUBLE
 * runs in x87 extended precision (64-bit significand).  Plain storage of f
 * loses digits to cancellation when the small velocity part of f is summed
 * out of values near w_i (about 1e-17 absolute per population); the extended
 * build moves that floor about 2000x lower and serves as the reference for
 * tight FP64 parity.
 *
 * Readings of the paper taken here (the paper is silent or garbled):
 *   - lattice units dx = dt = c = 1, c_s^2 = 1/3, nu = (tau - 1/2) / 3, and the
 *     effective viscosity equals nu;
 *   - the standard D2Q9 and D3Q19 velocity sets and weights;
 *   - Eq. (31)'s last term carries 1/eps, i.e. -(3 / (eps c^2)) (u . F); with
 *     the printed form the forcing term would create mass where eps < 1;
 *   - Eq. (28) is read as F = -(eps nu / K_app) u + eps G;
 *   - walls use halfway bounce-back; a node of class 255 is a solid wall node;
 *     open faces are periodic.
 *
 * Optional storage emulation (store_mode 1-5, see store_round) rounds every
 * stored value as a reduced-precision store would, to study what it can
 * reach.  Mode 0 is the plain oracle.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 19
#define WALL_CLASS 255

#ifdef REF_LONG_DOUBLE
typedef long double real;
#define SQRT sqrtl
#else
typedef double real;
#define SQRT sqrt
#endif

typedef struct {
    int q;
    int e[MAXQ][3];
    real w[MAXQ];
    int opp[MAXQ];
} lattice_t;

/* D2Q9: rest (4/9), 4 axis (1/9), 4 diagonal (1/36).
 * D3Q19: rest (1/3), 6 faces (1/18), 12 edges (1/36). */
static int make_lattice(int q, lattice_t* L)
{
    memset(L, 0, sizeof(*L));
    L->q = q;
    if (q == 9) {
        static const int e2[9][2] = { { 0, 0 }, { 1, 0 }, { 0, 1 }, { -1, 0 }, { 0, -1 },
                                      { 1, 1 }, { -1, 1 }, { -1, -1 }, { 1, -1 } };
        for (int i = 0; i < 9; ++i) {
            L->e[i][0] = e2[i][0];
            L->e[i][1] = e2[i][1];
            L->e[i][2] = 0;
            int s = abs(e2[i][0]) + abs(e2[i][1]);
            L->w[i] = s == 0 ? (real)4 / 9 : (s == 1 ? (real)1 / 9 : (real)1 / 36);
        }
    } else if (q == 19) {
        int n = 0;
        L->w[n++] = (real)1 / 3;
        for (int a = 0; a < 3; ++a)
            for (int s = -1; s <= 1; s += 2) {
                L->e[n][a] = s;
                L->w[n++] = (real)1 / 18;
            }
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b)
                for (int sa = -1; sa <= 1; sa += 2)
                    for (int sb = -1; sb <= 1; sb += 2) {
                        L->e[n][a] = sa;
                        L->e[n][b] = sb;
                        L->w[n++] = (real)1 / 36;
                    }
    } else {
        return -1;
    }
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] && L->e[j][2] == -L->e[i][2])
                L->opp[i] = j;
    return 0;
}

/* Velocity set, weights and opposites, for the tests. e: q*3 ints. */
int ref_lattice(int q, int32_t* e, double* w, int32_t* opp)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) e[3 * i + a] = L.e[i][a];
        w[i] = (double)L.w[i];
        opp[i] = L.opp[i];
    }
    return 0;
}

static real store_round(real f, real w, int mode, int scale_log2, real rho_x);

/* Nearest float16 value of x (ties to even), +-inf past 65504. */
static double round_half(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    double a = fabs(x);
    int e;
    frexp(a, &e);           /* a = m 2^e, m in [0.5, 1): unit exponent e - 1 */
    int ue = e - 1;
    if (ue < -14) ue = -14; /* subnormals: fixed quantum 2^-24 */
    double quantum = ldexp(1.0, ue - 10);
    double r = nearbyint(a / quantum) * quantum; /* default rounding mode: ties to even */
    if (r > 65504.0) r = INFINITY;
    return x < 0 ? -r : r;
}

/* round_half of every element of x (n values) into out, for the tests. */
int ref_round_half(int64_t n, const double* x, double* out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = round_half(x[k]);
    return 0;
}

/* Storage rounding of one value (store_round below), for the tests. */
double ref_store_round(double f, double w, int mode, int scale_log2, double rho_x)
{
    return (double)store_round((real)f, (real)w, mode, scale_log2, (real)rho_x);
}

/* mode 1: (f - w) through float; mode 2: (f - w) 2^s through float16;
 * mode 3: (f - w rho_x) 2^s through float16 with rho_x - 1 through float,
 * rho_x the density of the node the value leaves; mode 4: the same through
 * float32; mode 5: as mode 3 with rho_x - 1 stored as (rho_x - 1) 2^10
 * through float16 (a variant of the FP16 local-density form, kept for the
 * precision study). */
static real store_round(real f, real w, int mode, int scale_log2, real rho_x)
{
    if (mode == 1) return (real)(float)(f - w) + w;
    if (mode == 2) {
        double s = ldexp(1.0, scale_log2);
        return (real)(round_half((double)((f - w) * s)) / s) + w;
    }
    if (mode == 3) {
        double s = ldexp(1.0, scale_log2);
        real r32 = 1 + (real)(float)(rho_x - 1);
        return (real)(round_half((double)((f - w * r32) * s)) / s) + w * r32;
    }
    if (mode == 5) {
        double s = ldexp(1.0, scale_log2);
        real r16 = 1 + (real)(round_half((double)((rho_x - 1) * 1024.0)) / 1024.0);
        return (real)(round_half((double)((f - w * r16) * s)) / s) + w * r16;
    }
    if (mode == 4) {
        real r32 = 1 + (real)(float)(rho_x - 1);
        return (real)(float)(f - w * r32) + w * r32;
    }
    return f;
}

typedef struct {
    real rho, u[3], F[3];
} node_state;

/*
 * Moments of one node (Eq. 32-35) and its total body force (Eq. 27/28):
 *   rho = sum_i f_i                                                  (Eq. 32)
 *   rho v = sum_i f_i e_i + (dt/2) eps rho G                         (Eq. 35)
 *   u = v / (c0 + sqrt(c0^2 + c1 |v|))                               (Eq. 34)
 *   c0 = (1 + eps (dt/2) nu / K) / 2,  c1 = eps (dt/2) F_eps / sqrt(K)  (Eq. 36-37)
 *   F = -eps nu u / K - eps F_eps |u| u / sqrt(K) + eps G            (Eq. 27)
 * with kinv = 1/K (0 for an open pore).  Eq. (34) is the root of Eq. (33),
 * rho u = sum_i f_i e_i + (dt/2) rho F, with F taken at u.
 */
static void node_moments(const lattice_t* L, const real* fi, real eps, real kinv, real feps, real nu,
                         const real* G, node_state* s)
{
    real rho = 0, j[3] = { 0, 0, 0 };
    for (int i = 0; i < L->q; ++i) {
        rho += fi[i];
        for (int a = 0; a < 3; ++a) j[a] += fi[i] * L->e[i][a];
    }
    real v[3];
    for (int a = 0; a < 3; ++a) v[a] = j[a] / rho + (real)0.5 * eps * G[a];
    real vmag = SQRT(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    real c0 = (real)0.5 * (1 + eps * (real)0.5 * nu * kinv);
    real c1 = eps * (real)0.5 * feps * SQRT(kinv);
    real den = c0 + SQRT(c0 * c0 + c1 * vmag);
    for (int a = 0; a < 3; ++a) s->u[a] = v[a] / den;
    real umag = SQRT(s->u[0] * s->u[0] + s->u[1] * s->u[1] + s->u[2] * s->u[2]);
    for (int a = 0; a < 3; ++a)
        s->F[a] = -eps * nu * kinv * s->u[a] - eps * feps * SQRT(kinv) * umag * s->u[a] + eps * G[a];
    s->rho = rho;
}

/* Equilibrium, Eq. (30), direction i, c = 1. */
static real f_eq(const lattice_t* L, int i, real rho, const real* u, real eps)
{
    real eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
    real uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return L->w[i] * rho * (1 + 3 * eu + 9 / (2 * eps) * eu * eu - 3 / (2 * eps) * uu);
}

/* Forcing term, Eq. (31) with 1/eps on its last term, direction i, c = 1. */
static real f_force(const lattice_t* L, int i, real rho, const real* u, const real* F, real eps,
                    real tau)
{
    real eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
    real eF = L->e[i][0] * F[0] + L->e[i][1] * F[1] + L->e[i][2] * F[2];
    real uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    return L->w[i] * rho * (1 - 1 / (2 * tau)) * (3 * eF + 9 / eps * eu * eF - 3 / eps * uF);
}

static void load_G(const double* G, real* g)
{
    for (int a = 0; a < 3; ++a) g[a] = (real)G[a];
}

/* Single-node collision for the tests: fout_i = f_i - (f_i - feq_i)/tau + F_i. */
int ref_collide_node(int q, const double* f, double eps, double kinv, double feps, double tau,
                     const double* G, double* fout, double* rho_u_F /* 7 doubles */)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    real fi[MAXQ], g[3];
    for (int i = 0; i < q; ++i) fi[i] = f[i];
    load_G(G, g);
    node_state s;
    real nu = ((real)tau - (real)0.5) / 3;
    node_moments(&L, fi, eps, kinv, feps, nu, g, &s);
    for (int i = 0; i < q; ++i)
        fout[i] = (double)(fi[i] - (fi[i] - f_eq(&L, i, s.rho, s.u, eps)) / tau +
                           f_force(&L, i, s.rho, s.u, s.F, eps, tau));
    if (rho_u_F) {
        rho_u_F[0] = (double)s.rho;
        for (int a = 0; a < 3; ++a) {
            rho_u_F[1 + a] = (double)s.u[a];
            rho_u_F[4 + a] = (double)s.F[a];
        }
    }
    return 0;
}

/* Equilibrium and forcing vectors of one node, for the tests. */
int ref_feq_force(int q, double rho, const double* u, const double* F, double eps, double tau,
                  double* feq, double* fi)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    real ur[3], Fr[3];
    for (int a = 0; a < 3; ++a) { ur[a] = u[a]; Fr[a] = F[a]; }
    for (int i = 0; i < q; ++i) {
        feq[i] = (double)f_eq(&L, i, rho, ur, eps);
        fi[i] = (double)f_force(&L, i, rho, ur, Fr, eps, tau);
    }
    return 0;
}

typedef struct {
    int nx, ny, nz;
    unsigned walls; /* bit 0: x-, 1: x+, 2: y-, 3: y+, 4: z-, 5: z+ */
} grid_t;

/*
 * Pressure-driven runs (the inlet / outlet pressures of the paper's Tab. 4 and
 * Tab. 7) with the local apparent permeability at the local pressure (Eq. 18-19).
 *   axis      0: none; 1, 2, 3: pressure faces normal to x, y, z.  The face
 *             c_a = 0 is held at density rho_in, the face c_a = n_a - 1 at
 *             rho_out; populations leaving through them are lost and those
 *             entering are rebuilt (fill_pressure_faces).
 *   k_const, k_kn, k_surf, lang_b   per class, in lattice units (K / dx^2):
 *             K(P) = k_const + k_kn / P + k_surf / (P (1 + lang_b P)), which is
 *             Eq. (18) (K_0 + eta D_K / P) plus the surface term of Eq. (19)
 *             with the ideal-gas density; k_const = +inf marks an open pore.
 *             NULL: the constant K of the class table.
 *   p_in, p_out  physical pressures of the two faces.  The lattice density
 *             carries the pressure of Eq. (26) (c_s^2 rho), so the local
 *             physical pressure is its affine image
 *             P(x) = p_out + (rho(x) - rho_out) (p_in - p_out) / (rho_in - rho_out).
 */
typedef struct {
    int axis;
    double rho_in, rho_out;
    const double *k_const, *k_kn, *k_surf, *lang_b;
    double p_in, p_out;
} ref_pressure;

/*
 * Target of the move x -> x + e_i.  Returns 1 and the (periodically wrapped)
 * target node if the move streams; 0 if it is reflected because it crosses a
 * wall face or lands on a wall node (halfway bounce-back); 2 if it leaves the
 * domain through a pressure face.
 */
static int stream_target(const grid_t* g, const lattice_t* L, const uint8_t* cls, int paxis, int x, int y,
                         int z, int i, int64_t* tn)
{
    int c[3] = { x + L->e[i][0], y + L->e[i][1], z + L->e[i][2] };
    int n[3] = { g->nx, g->ny, g->nz };
    for (int a = 0; a < 3; ++a) {
        if (a == paxis - 1 && (c[a] < 0 || c[a] >= n[a])) return 2;
        if (c[a] < 0) {
            if (g->walls & (1u << (2 * a))) return 0;
            c[a] += n[a];
        } else if (c[a] >= n[a]) {
            if (g->walls & (1u << (2 * a + 1))) return 0;
            c[a] -= n[a];
        }
    }
    int64_t t = ((int64_t)c[2] * g->ny + c[1]) * g->nx + c[0];
    if (cls[t] == WALL_CLASS) return 0;
    *tn = t;
    return 1;
}

typedef struct {
    lattice_t L;
    grid_t g;
    int64_t N;
    real tau, nu, G[3];
    const uint8_t* cls;
    const double *eps, *kinv, *feps;
    int store_mode, scale_log2;
    const ref_pressure* pr; /* NULL: no pressure faces, constant K */
} problem_t;

/* 1/K of class c at a node of density rho: the class table's constant K, or in
 * a pressure-driven run with per-class K(P) the value at the local pressure. */
static real local_kinv(const problem_t* P, int c, real rho)
{
    const ref_pressure* pr = P->pr;
    if (!pr || !pr->k_const) return P->kinv[c];
    if (isinf(pr->k_const[c])) return 0;
    const real pl = (real)pr->p_out + (rho - (real)pr->rho_out) * ((real)pr->p_in - (real)pr->p_out) /
                                          ((real)pr->rho_in - (real)pr->rho_out);
    const real k = (real)pr->k_const[c] + (real)pr->k_kn[c] / pl +
                   (real)pr->k_surf[c] / (pl * (1 + (real)pr->lang_b[c] * pl));
    return 1 / k;
}

/*
 * Zou-He (non-equilibrium bounce-back) density condition on the pressure
 * faces.  At a fluid node of the face c_a = 0, with n the unit normal into
 * the domain (+a) and rho_f = rho_in, the populations with e_i . n > 0 come
 * from outside and are rebuilt from the known ones: the normal momentum
 * follows from the imposed density,
 *     j_n = rho_f - sum_{e.n = 0} f - 2 sum_{e.n < 0} f,
 * the tangential momentum is set to zero, and the non-equilibrium parts of
 * opposite populations are equal:
 *     f_i = f_opp(i) + 6 w_i (e_i . n) j_n - sum_t (e_i . t) N_t,
 *     N_t = sum_{e.n = 0} f e_t / sum_{e.n > 0} (e . t)^2
 * over the tangential axes t.  The face c_a = n_a - 1 is the same with
 * n = -a and rho_out.  Applied to every state, so that a state always
 * satisfies the face densities (Zou & He, Phys. Fluids 9, 1997).
 */
static void fill_pressure_faces(const problem_t* P, real* f)
{
    if (!P->pr || !P->pr->axis) return;
    const lattice_t* L = &P->L;
    const int q = L->q, a = P->pr->axis - 1;
    const int n3[3] = { P->g.nx, P->g.ny, P->g.nz };
    const int64_t N = P->N;
    for (int z = 0; z < n3[2]; ++z)
        for (int y = 0; y < n3[1]; ++y)
            for (int x = 0; x < n3[0]; ++x) {
                const int c[3] = { x, y, z };
                const int64_t n = ((int64_t)z * n3[1] + y) * n3[0] + x;
                if (P->cls[n] == WALL_CLASS) continue;
                for (int side = 0; side < 2; ++side) {
                    if (c[a] != (side == 0 ? 0 : n3[a] - 1)) continue;
                    const int sgn = side == 0 ? 1 : -1;
                    const real rho_f = side == 0 ? (real)P->pr->rho_in : (real)P->pr->rho_out;
                    real s0 = 0, sneg = 0, nt[3] = { 0, 0, 0 }, den[3] = { 0, 0, 0 };
                    for (int i = 0; i < q; ++i) {
                        const int en = sgn * L->e[i][a];
                        const real fi = f[i * N + n];
                        if (en == 0) {
                            s0 += fi;
                            for (int t = 0; t < 3; ++t)
                                if (t != a) nt[t] += fi * L->e[i][t];
                        } else if (en < 0) {
                            sneg += fi;
                        } else {
                            for (int t = 0; t < 3; ++t)
                                if (t != a) den[t] += (real)(L->e[i][t] * L->e[i][t]);
                        }
                    }
                    const real jn = rho_f - s0 - 2 * sneg;
                    for (int t = 0; t < 3; ++t) nt[t] = den[t] > 0 ? nt[t] / den[t] : 0;
                    for (int i = 0; i < q; ++i) {
                        const int en = sgn * L->e[i][a];
                        if (en <= 0) continue;
                        real v = f[L->opp[i] * N + n] + 6 * L->w[i] * en * jn;
                        for (int t = 0; t < 3; ++t)
                            if (t != a) v -= L->e[i][t] * nt[t];
                        f[i * N + n] = v;
                    }
                }
            }
}

static int make_problem(problem_t* P, int q, int nx, int ny, int nz, unsigned walls, double tau,
                        const double* G, const uint8_t* cls, const double* eps_t, const double* kinv_t,
                        const double* feps_t, int store_mode, int scale_log2, const ref_pressure* pr)
{
    if (make_lattice(q, &P->L)) return -1;
    P->pr = (pr && pr->axis) ? pr : NULL;
    if (P->pr) {
        const int a = pr->axis - 1;
        const int n3[3] = { nx, ny, nz };
        if (a < 0 || a > 2 || n3[a] < 2 || ((walls >> (2 * a)) & 3u) || !(pr->rho_in != pr->rho_out)) return -1;
    }
    P->g.nx = nx; P->g.ny = ny; P->g.nz = nz; P->g.walls = walls;
    P->N = (int64_t)nx * ny * nz;
    P->tau = tau;
    P->nu = (P->tau - (real)0.5) / 3;
    load_G(G, P->G);
    P->cls = cls; P->eps = eps_t; P->kinv = kinv_t; P->feps = feps_t;
    P->store_mode = store_mode; P->scale_log2 = scale_log2;
    return 0;
}

/*
 * One time step, Eq. (29): collide at every fluid node, then push each
 * post-collision value to x + e_i, or reflect it into the opposite direction
 * at x where the move is blocked.  Wall-node slots of fout are zero.
 */
static void step(const problem_t* P, const real* f, real* fout)
{
    const lattice_t* L = &P->L;
    const int q = L->q, nx = P->g.nx, ny = P->g.ny, nz = P->g.nz;
    const int64_t N = P->N;
    for (int64_t k = 0; k < (int64_t)q * N; ++k) fout[k] = 0;
#pragma omp parallel for collapse(2) schedule(static) if (N >= 16384)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t n = ((int64_t)z * ny + y) * nx + x;
                const int c = P->cls[n];
                if (c == WALL_CLASS) continue;
                const real eps = P->eps[c];
                real fi[MAXQ];
                for (int i = 0; i < q; ++i) fi[i] = f[i * N + n];
                real rho = 0;
                for (int i = 0; i < q; ++i) rho += fi[i];
                node_state s;
                node_moments(L, fi, eps, local_kinv(P, c, rho), P->feps[c], P->nu, P->G, &s);
                for (int i = 0; i < q; ++i) {
                    real fs = fi[i] - (fi[i] - f_eq(L, i, s.rho, s.u, eps)) / P->tau +
                              f_force(L, i, s.rho, s.u, s.F, eps, P->tau);
                    int64_t t;
                    const int m = stream_target(&P->g, L, P->cls, P->pr ? P->pr->axis : 0, x, y, z, i, &t);
                    if (m == 1)
                        fout[i * N + t] = store_round(fs, L->w[i], P->store_mode, P->scale_log2, s.rho);
                    else if (m == 0)
                        fout[L->opp[i] * N + n] =
                            store_round(fs, L->w[L->opp[i]], P->store_mode, P->scale_log2, s.rho);
                }
            }
    fill_pressure_faces(P, fout);
}

/* Density and velocity (Eq. 32-34) at every node; wall nodes get zeros. */
static void fields(const problem_t* P, const real* f, double* rho, double* u)
{
    const lattice_t* L = &P->L;
    const int64_t N = P->N;
#pragma omp parallel for schedule(static) if (N >= 16384)
    for (int64_t n = 0; n < N; ++n) {
        const int c = P->cls[n];
        if (c == WALL_CLASS) {
            rho[n] = 0;
            u[n] = u[N + n] = u[2 * N + n] = 0;
            continue;
        }
        real fi[MAXQ];
        for (int i = 0; i < L->q; ++i) fi[i] = f[i * N + n];
        real r = 0;
        for (int i = 0; i < L->q; ++i) r += fi[i];
        node_state s;
        node_moments(L, fi, P->eps[c], local_kinv(P, c, r), P->feps[c], P->nu, P->G, &s);
        rho[n] = (double)s.rho;
        u[n] = (double)s.u[0];
        u[N + n] = (double)s.u[1];
        u[2 * N + n] = (double)s.u[2];
    }
}

/* r = ||u - u_prev|| / (dsteps ||u||) over fluid nodes, summed in node order. */
static double residual(const problem_t* P, const double* u, const double* up, int64_t dsteps)
{
    const int64_t N = P->N;
    long double sd = 0, su = 0;
    for (int64_t n = 0; n < N; ++n) {
        if (P->cls[n] == WALL_CLASS) continue;
        for (int a = 0; a < 3; ++a) {
            long double d = (long double)u[a * N + n] - up[a * N + n];
            sd += d * d;
            su += (long double)u[a * N + n] * u[a * N + n];
        }
    }
    return (double)(sqrtl(sd) / ((long double)dsteps * sqrtl(su)));
}

/*
 * Iterate the state f (q * N doubles, in/out) for up to nsteps steps.  With
 * check_every > 0 the residual is evaluated every check_every steps
 * (hist[k] = r after (k+1) * check_every steps, inf if ||u|| = 0) and, if
 * tol > 0, the run stops at the first check with r <= tol.  On return
 * rho (N) and u (3N) hold the fields of the final state.  The state is held
 * in the build's arithmetic type for the whole run.  Returns the number of
 * steps taken, or < 0 on error.
 */
int64_t ref_solve(int q, int nx, int ny, int nz, unsigned walls, double tau, const double* G,
                  const uint8_t* cls, const double* eps_t, const double* kinv_t, const double* feps_t,
                  double* f, int64_t nsteps, int check_every, double tol, int store_mode, int scale_log2,
                  double* rho, double* u, double* hist, int64_t hist_cap, const ref_pressure* pr)
{
    problem_t P;
    if (make_problem(&P, q, nx, ny, nz, walls, tau, G, cls, eps_t, kinv_t, feps_t, store_mode,
                     scale_log2, pr))
        return -1;
    const int64_t N = P.N, QN = (int64_t)q * N;
    real* a = (real*)malloc((size_t)QN * sizeof(real));
    real* b = (real*)malloc((size_t)QN * sizeof(real));
    double* up = (double*)malloc((size_t)(3 * N) * sizeof(double));
    if (!a || !b || !up) {
        free(a); free(b); free(up);
        return -2;
    }
    for (int64_t k = 0; k < QN; ++k) a[k] = f[k];
    fill_pressure_faces(&P, a);
    fields(&P, a, rho, up);
    int64_t s = 0, nh = 0;
    while (s < nsteps) {
        step(&P, a, b);
        real* t = a; a = b; b = t;
        ++s;
        if (check_every > 0 && s % check_every == 0) {
            fields(&P, a, rho, u);
            double r = residual(&P, u, up, check_every);
            if (nh < hist_cap) hist[nh] = r;
            ++nh;
            memcpy(up, u, (size_t)(3 * N) * sizeof(double));
            if (tol > 0 && r <= tol) break;
        }
    }
    fields(&P, a, rho, u);
    for (int64_t k = 0; k < QN; ++k) f[k] = (double)a[k];
    free(a); free(b); free(up);
    return s;
}

/* One step from f to fout (both q * N doubles), for the tests. */
int ref_step(int q, int nx, int ny, int nz, unsigned walls, double tau, const double* G,
             const uint8_t* cls, const double* eps_t, const double* kinv_t, const double* feps_t,
             const double* f, double* fout, int store_mode, int scale_log2, const ref_pressure* pr)
{
    problem_t P;
    if (make_problem(&P, q, nx, ny, nz, walls, tau, G, cls, eps_t, kinv_t, feps_t, store_mode,
                     scale_log2, pr))
        return -1;
    const int64_t QN = (int64_t)q * P.N;
    real* a = (real*)malloc((size_t)QN * sizeof(real));
    real* b = (real*)malloc((size_t)QN * sizeof(real));
    if (!a || !b) { free(a); free(b); return -2; }
    for (int64_t k = 0; k < QN; ++k) a[k] = f[k];
    fill_pressure_faces(&P, a);
    step(&P, a, b);
    for (int64_t k = 0; k < QN; ++k) fout[k] = (double)b[k];
    free(a); free(b);
    return 0;
}

/* Density and velocity of the state f, for the tests. rho: N, u: 3N (planes). */
int ref_fields(int q, int nx, int ny, int nz, unsigned walls, double tau, const double* G, const uint8_t* cls,
               const double* eps_t, const double* kinv_t, const double* feps_t, const double* f,
               double* rho, double* u, const ref_pressure* pr)
{
    problem_t P;
    if (make_problem(&P, q, nx, ny, nz, walls, tau, G, cls, eps_t, kinv_t, feps_t, 0, 0, pr)) return -1;
    const int64_t QN = (int64_t)q * P.N;
    real* a = (real*)malloc((size_t)QN * sizeof(real));
    if (!a) return -2;
    for (int64_t k = 0; k < QN; ++k) a[k] = f[k];
    fill_pressure_faces(&P, a);
    fields(&P, a, rho, u);
    free(a);
    return 0;
}

/* Rest state f_i = w_i rho0 everywhere. */
int ref_init_rest(int q, int64_t N, double rho0, double* f)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    for (int i = 0; i < q; ++i)
        for (int64_t n = 0; n < N; ++n) f[i * N + n] = (double)(L.w[i] * rho0);
    return 0;
}

/* Equilibrium Eq. (30) of given (rho, u) at every fluid node (wall nodes: zero). */
int ref_init_fields(int q, int nx, int ny, int nz, const uint8_t* cls, const double* eps_t,
                    const double* rho, const double* u, double* f)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t n = 0; n < N; ++n) {
        const int c = cls[n];
        real un[3] = { u[n], u[N + n], u[2 * N + n] };
        for (int i = 0; i < q; ++i)
            f[i * N + n] = c == WALL_CLASS ? 0.0 : (double)f_eq(&L, i, rho[n], un, eps_t[c]);
    }
    return 0;
}

/* OpenMP threads a parallel region of the oracle uses. */
int ref_num_threads(void) { return omp_get_max_threads(); }

/* Set the OpenMP thread count of later parallel regions (for timing at one thread). */
int ref_set_threads(int n)
{
    if (n < 1) return -1;
    omp_set_num_threads(n);
    return 0;
}
