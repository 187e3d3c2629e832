// HIP kernels of the GLBM sweep for gfx950 (MI355X).
//
// The state of an instance is q population deviations d_i = f_i - w_i per node
// (rho0 = 1) in one of several storage types, in node blocks or planes
// (glbm_internal.h); node = (z * ny + y) * nx + x indexes the class map, the
// density plane and the snapshot, pidx() the populations.  One time step of the
// generalized lattice Boltzmann equation (Eq. 29 of arXiv:1601.00704) is one
// launch of k_sweep: every thread pulls the q post-collision values that stream
// into its node (periodic wrap, or halfway bounce-back at wall faces and wall
// nodes), evaluates the moments (Eq. 32-35), the Brinkman-Forchheimer force
// (Eq. 27-28), the porous equilibrium (Eq. 30) and the forcing term (Eq. 31,
// with the 1/eps that keeps it mass-conserving), relaxes, and writes its own q
// values to the other buffer.  The kernel is bound by HBM bandwidth: it reads
// q values and one class byte and writes q values per node, with the per-class
// constants (eps, 1/eps, c0, drag) in LDS, indexed by the class byte.
//
// k_observe evaluates the same moments on the current state and reduces, per
// tile and in FP64, the residual terms |u - u_snap|^2 and |u|^2, the velocity
// sum (Darcy flux) and a non-finite count; k_finalize sums the tiles of each
// instance in a fixed order, so results are deterministic.
#include "glbm_internal.h"
#include "glbm.h"

#include <hip/hip_fp16.h>

#include <type_traits>

namespace glbm {
namespace {

// ---------------------------------------------------------------- lattices --
// D2Q9: rest, +x, +y, -x, -y, then the diagonals (+,+), (-,+), (-,-), (+,-).
// D3Q19: rest, the 6 faces in +/- pairs (x, y, z), then the 12 edges in
// opposite pairs.  Weights: D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36.
template <int Q> struct Lat;
template <> struct Lat<9> {
    static constexpr int D = 2;
    static constexpr int ex(int i) { constexpr int a[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}; return a[i]; }
    static constexpr int ey(int i) { constexpr int a[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1}; return a[i]; }
    static constexpr int ez(int) { return 0; }
    static constexpr int opp(int i) { constexpr int a[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6}; return a[i]; }
    static constexpr double w(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
};
template <> struct Lat<19> {
    static constexpr int D = 3;
    static constexpr int ex(int i) {
        constexpr int a[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        return a[i];
    }
    static constexpr int ey(int i) {
        constexpr int a[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        return a[i];
    }
    static constexpr int ez(int i) {
        constexpr int a[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        return a[i];
    }
    static constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
    static constexpr double w(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
};

// Boundary modes (Config::bc): 0 periodic, 1 face walls, 2 face walls and wall
// nodes, 3 pressure faces, 4 pressure faces and wall nodes.
constexpr bool face_walls(int bc) { return bc == 1 || bc == 2; }
constexpr bool wall_nodes(int bc) { return bc == 2 || bc == 4; }
constexpr bool pressure_faces(int bc) { return bc >= 3; }

// ----------------------------------------------------------------- storage --
template <int STORE> struct St;
// kRho: the stored value is relative to w_i rho(x) of the node that wrote it,
// whose rho - 1 sits in a float plane after the q population planes.
template <> struct St<GLBM_STORE_F64> {
    static constexpr bool kRho = false;
    using S = double;
    using T = double;
    __device__ static T dec(S s, float) { return s; }
    __device__ static S enc(T d, float) { return d; }
};
template <> struct St<GLBM_STORE_F32> {
    static constexpr bool kRho = false;
    using S = float;
    using T = float;
    __device__ static T dec(S s, float) { return s; }
    __device__ static S enc(T d, float) { return d; }
};
template <> struct St<GLBM_STORE_F16DEV> {
    static constexpr bool kRho = false;
    using S = uint16_t;
    using T = float;
    __device__ static T dec(S s, float inv_scale) { return __half2float(__ushort_as_half(s)) * inv_scale; }
    __device__ static S enc(T d, float scale) { return __half_as_ushort(__float2half_rn(d * scale)); }
};
template <> struct St<GLBM_STORE_F16LOC> : St<GLBM_STORE_F16DEV> {
    static constexpr bool kRho = true;
};
template <> struct St<GLBM_STORE_F32LOC> : St<GLBM_STORE_F32> {
    static constexpr bool kRho = true;
};

// The float plane of rho - 1 of a kRho buffer (after the q planes).
template <int STORE>
__device__ __forceinline__ const float* rho_plane(const typename St<STORE>::S* base, int q, int stride)
{
    return reinterpret_cast<const float*>(base + (size_t)q * stride);
}
template <int STORE>
__device__ __forceinline__ float* rho_plane(typename St<STORE>::S* base, int q, int stride)
{
    return reinterpret_cast<float*>(base + (size_t)q * stride);
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Map them so that
// each XCD walks a contiguous range of tiles: x-neighbouring tiles share the
// cache lines their shifted reads straddle, and those then meet in one L2.
__device__ __forceinline__ int xcd_tile(int bid, int G)
{
    const int q = G >> 3, r = G & 7, x = bid & 7, k = bid >> 3;
    return x * q + min(x, r) + k;
}

template <typename T> __device__ __forceinline__ bool finite(T v) { return isfinite(v); }

// 1 / x: in FP32 the hardware reciprocal refined by one Newton step (within
// an ulp or two of the rounded quotient, without the full division sequence);
// in FP64 the correctly rounded division.
template <typename T> __device__ __forceinline__ T recip(T x)
{
    if constexpr (sizeof(T) == 4) {
        const float r = __builtin_amdgcn_rcpf(x);
        return r * __builtin_fmaf(-x, r, 2.0f);
    } else {
        return T(1) / x;
    }
}

// Element i of a uniform base, addressed by a 32-bit unsigned byte offset
// (base + zero-extended offset: one vector instruction per access instead of
// a sign extension and a 64-bit add).  Valid while i * sizeof(V) < 2^32,
// which the host's size check guarantees for a population buffer.  The FP16
// stores (planes) are bound by vector instructions and use it; the FP32 and
// FP64 stores keep 64-bit per-lane addresses, which measured faster there.
template <typename V> __device__ __forceinline__ V* elem(V* base, uint32_t i)
{
    using B = typename std::conditional<std::is_const<V>::value, const char, char>::type;
    return reinterpret_cast<V*>(reinterpret_cast<B*>(base) + i * uint32_t(sizeof(V)));
}

// Element index of population i of node n (layout: glbm_internal.h).  For
// node blocks, ((n >> 12) q + i) 4096 + (n & 4095) written as n plus whole
// blocks: one shift and one shift-add per node (q - 1 = 8 is a power of two
// for D2Q9), the i term a constant.
template <int Q, int STORE> __device__ __forceinline__ int pidx(int i, int n, int stride)
{
    if constexpr (node_blocks(STORE))
        return n + (n >> kBlkLog2) * ((Q - 1) << kBlkLog2) + (i << kBlkLog2);
    else
        return i * stride + n;
}

// Instance constants in the compute type (FP32 copies made on the host).
template <typename T> __device__ __forceinline__ T inst_g(const InstDev& I, int a)
{
    if constexpr (sizeof(T) == 4) return I.gf[a]; else return I.g[a];
}
template <typename T> __device__ __forceinline__ T inst_omega(const InstDev& I)
{
    if constexpr (sizeof(T) == 4) return I.omegaf; else return I.omega;
}
template <typename T> __device__ __forceinline__ T inst_cforce(const InstDev& I)
{
    if constexpr (sizeof(T) == 4) return I.cforcef; else return I.cforce;
}

// Zou-He rule on a pressure face (bc 3 and 4).  On entry d holds the deviations
// f_i - w_i of the known populations (for a kRho store: local parts, with the
// source densities in r) and zeros for the directions entering through the
// face.  With n the unit normal into the domain (side * the axis) and the face
// density rho_f: j_n = (rho_f - 1) - sum_{e.n = 0} d - 2 sum_{e.n < 0} d, and
// for every entering direction d_i = d_opp(i) + 6 w_i j_n - sum_t e_i,t N_t,
// N_t = sum_{e.n = 0} d e_t / 2 (tangential momentum zero; both lattices have
// two entering directions with e_t = +-1 for each tangential axis t).  On exit
// a kRho store holds deviations with source density 1 (r = 0).
template <int Q, bool RHO, typename T>
__device__ __forceinline__ void fill_face(T (&d)[Q], T (&r)[Q], const InstDev& I, int side)
{
    using L = Lat<Q>;
    const int a = I.paxis;
    if constexpr (RHO) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            d[i] += T(L::w(i)) * r[i];
            r[i] = T(0);
        }
    }
    T s0 = 0, sneg = 0, nt[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int e[3] = {L::ex(i), L::ey(i), L::ez(i)};
        const int en = side * (a == 0 ? e[0] : (a == 1 ? e[1] : e[2]));
        if (en == 0) {
            s0 += d[i];
#pragma unroll
            for (int t = 0; t < L::D; ++t)
                if (e[t]) nt[t] += (t == a) ? T(0) : (e[t] > 0 ? d[i] : -d[i]);
        } else if (en < 0) {
            sneg += d[i];
        }
    }
    const T drf = side > 0 ? T(sizeof(T) == 4 ? I.drinf : I.drin) : T(sizeof(T) == 4 ? I.droutf : I.drout);
    const T jn = drf - s0 - T(2) * sneg;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int e[3] = {L::ex(i), L::ey(i), L::ez(i)};
        const int en = side * (a == 0 ? e[0] : (a == 1 ? e[1] : e[2]));
        if (en <= 0) continue;
        T v = d[L::opp(i)] + T(6.0 * L::w(i)) * jn;
#pragma unroll
        for (int t = 0; t < L::D; ++t)
            if (e[t] && t != a) v -= (e[t] > 0 ? T(0.5) : T(-0.5)) * nt[t];
        d[i] = v;
    }
}

// Pull the q post-collision values that stream into node (x, y, z).
// For a kRho store, d[i] receives the stored part (f_i - w_i rho_s) and r[i]
// the density deviation rho_s - 1 of the source node s; otherwise d[i] is the
// full deviation f_i - w_i and r is not touched.
template <int Q, int STORE, int BC>
__device__ __forceinline__ void gather(typename St<STORE>::T (&d)[Q], typename St<STORE>::T (&r)[Q],
                                       const typename St<STORE>::S* __restrict__ src,
                                       const uint8_t* __restrict__ cls, const InstDev& I, int x, int y, int z,
                                       int n, bool nt_aligned = false)
{
    using L = Lat<Q>;
    using S = St<STORE>;
    using SV = typename S::S;
    // Full 64-bit per-lane addresses: measured faster here than a uniform plane
    // base with a 32-bit per-lane offset, although the latter needs fewer
    // instructions.
    const int nx = I.nx, ny = I.ny, nz = I.nz, stride = I.stride;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
    // pressure faces: side = +1 on the inlet face (coordinate 0), -1 on the
    // outlet face (n - 1), 0 elsewhere; directions entering through the face
    // (side * e_a > 0) are rebuilt below instead of pulled
    int side = 0;
    if constexpr (pressure_faces(BC)) {
        const int a = I.paxis;
        const int ca = a == 0 ? x : (a == 1 ? y : z), na = a == 0 ? nx : (a == 1 ? ny : nz);
        side = ca == 0 ? 1 : (ca == na - 1 ? -1 : 0);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ex = L::ex(i), ey = L::ey(i), ez = L::ez(i);
        if constexpr (pressure_faces(BC)) {
            const int ea = I.paxis == 0 ? ex : (I.paxis == 1 ? ey : ez);
            if (side * ea > 0) {
                d[i] = 0;
                if constexpr (S::kRho) r[i] = 0;
                continue;
            }
        }
        const int sx = ex > 0 ? xm : (ex < 0 ? xp : x);
        const int sy = ey > 0 ? ym : (ey < 0 ? yp : y);
        const int sz = ez > 0 ? zm : (ez < 0 ? zp : z);
        const int sn = (sz * ny + sy) * nx + sx;
        int idx;
        if constexpr (node_blocks(STORE))
            idx = pidx<Q, STORE>(i, sn, stride);
        else
            idx = i * stride + sn;
        int node = sn;
        if constexpr (face_walls(BC) || wall_nodes(BC)) {
            const uint32_t w = I.walls;
            bool blocked = false;
            if constexpr (face_walls(BC)) {
                if (ex > 0) blocked |= (x == 0) && (w & 1u);
                if (ex < 0) blocked |= (x == nx - 1) && (w & 2u);
                if (ey > 0) blocked |= (y == 0) && (w & 4u);
                if (ey < 0) blocked |= (y == ny - 1) && (w & 8u);
                if (ez > 0) blocked |= (z == 0) && (w & 16u);
                if (ez < 0) blocked |= (z == nz - 1) && (w & 32u);
            }
            if (wall_nodes(BC) && i != 0) blocked |= cls[sn] == kWallClass;
            if (blocked) {
                if constexpr (node_blocks(STORE))
                    idx = pidx<Q, STORE>(L::opp(i), n, stride);
                else
                    idx = L::opp(i) * stride + n;
                node = n;
            }
        }
        // planes without an x shift are read by exactly one wavefront per cache line
        const SV* at;
        if constexpr (node_blocks(STORE))
            at = src + idx;
        else
            at = elem(src, uint32_t(idx));
        const SV raw = (ex == 0 && nt_aligned) ? __builtin_nontemporal_load(at) : *at;
        d[i] = S::dec(raw, I.inv_scale);
        if constexpr (S::kRho) r[i] = *elem(rho_plane<STORE>(src, Q, stride), uint32_t(node));
    }
    if constexpr (pressure_faces(BC))
        if (side != 0) fill_face<Q, S::kRho>(d, r, I, side);
}

// Local form of a kRho node: drho = sum_i (w_i r_i + d_i), and d becomes
// e_i = f_i - w_i rho(x) = d_i + w_i (r_i - drho): only differences of
// neighbouring densities are formed, never the full density part.
template <int Q, typename T>
__device__ __forceinline__ T localize(T (&d)[Q], const T (&r)[Q])
{
    using L = Lat<Q>;
    T a = T(L::w(0)) * r[0], b = d[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        a += T(L::w(i)) * r[i];
        b += d[i];
    }
    const T drho = a + b;
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] += T(L::w(i)) * (r[i] - drho);
    return drho;
}

// A leading direction of an opposite pair (the one whose first non-zero
// component is positive).
template <int Q> __host__ __device__ constexpr bool lead(int i)
{
    using L = Lat<Q>;
    return L::ex(i) > 0 || (L::ex(i) == 0 && (L::ey(i) > 0 || (L::ey(i) == 0 && L::ez(i) > 0)));
}

// a . b over the first D components.
template <int D, typename T> __device__ __forceinline__ T dot(const T (&a)[3], const T (&b)[3])
{
    T s = a[0] * b[0];
#pragma unroll
    for (int k = 1; k < D; ++k) s += a[k] * b[k];
    return s;
}

// e_i . v over the non-zero components of e_i (each is +1 or -1).
template <int Q, typename T> __device__ __forceinline__ T edot(int i, const T (&v)[3])
{
    using L = Lat<Q>;
    const int e[3] = {L::ex(i), L::ey(i), L::ez(i)};
    T s = 0;
    bool seen = false;
#pragma unroll
    for (int a = 0; a < L::D; ++a) {
        if (!e[a]) continue;
        const T t = e[a] > 0 ? v[a] : -v[a];
        s = seen ? s + t : t;
        seen = true;
    }
    return s;
}

// Moments and force of one node: Eq. (32)-(35) and (27)-(28) on deviations.
// PRES (pressure faces): the class's K is K(P) at the node's pressure
// P = p0 + (rho - 1) p1, with K(P) = A + (B + C / (1 + b P)) / P (Eq. 18-19).
template <int Q, typename T, bool FORCH, bool PRES = false> struct Node {
    T drho, rho, u[3], F[3];
    __device__ __forceinline__ void moments(const T (&d)[Q], const T* tab, const T g[3], const InstDev& I)
    {
        T dr = d[0];
#pragma unroll
        for (int i = 1; i < Q; ++i) dr += d[i];
        moments_with(d, dr, tab, g, I);
    }
    // d: deviations (or local parts e_i, whose momentum is the same), dr: rho - 1
    __device__ __forceinline__ void moments_with(const T (&d)[Q], T dr, const T* tab, const T g[3], const InstDev& I)
    {
        using L = Lat<Q>;
        constexpr int D = L::D;
        // Opposite populations share their density part w_i drho; summing the
        // momentum as differences of opposite pairs cancels it exactly (each
        // difference of two close values is exact in floating point) before
        // anything is rounded.  Each sum starts from its first term, and a
        // 2-D lattice never touches the z components (IEEE arithmetic cannot
        // drop a 0 * x or a 0 + x on its own).
        T j[3] = {0, 0, 0};
        bool seen[3] = {false, false, false};
        drho = dr;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int o = L::opp(i);
            if (!lead<Q>(i)) continue;
            const T diff = d[i] - d[o];
            const int e[3] = {L::ex(i), L::ey(i), L::ez(i)};
#pragma unroll
            for (int a = 0; a < D; ++a) {
                if (!e[a]) continue;
                const T t = e[a] > 0 ? diff : -diff;
                j[a] = seen[a] ? j[a] + t : t;
                seen[a] = true;
            }
        }
        rho = T(1) + drho;
        const T irho = recip(rho);
        const T eps = tab[TAB_EPS];
        T v[3];
#pragma unroll
        for (int a = 0; a < D; ++a) v[a] = j[a] * irho + T(0.5) * eps * g[a];
        if constexpr (PRES) {
            const bool f32 = sizeof(T) == 4;
            const T P = T(f32 ? I.p0f : I.p0) + dr * T(f32 ? I.p1f : I.p1);
            const T K = tab[TAB_PA] + recip(P) * (tab[TAB_PB] + tab[TAB_PC] * recip(T(1) + tab[TAB_PBL] * P));
            const T drag = eps * T(f32 ? I.nuf : I.nu) * tab[TAB_POPEN] * recip(K);   // eps nu / K
            const T h = recip(T(1) + T(0.5) * drag);                                  // 1 / (2 c0), Eq. (36)
#pragma unroll
            for (int a = 0; a < D; ++a) {
                u[a] = v[a] * h;
                F[a] = eps * g[a] - drag * u[a];
            }
        } else if (FORCH) {
            const T c0 = tab[TAB_C0], c1 = tab[TAB_C1];
            const T vm = sqrt(dot<D>(v, v));
            const T den = T(1) / (c0 + sqrt(c0 * c0 + c1 * vm));
#pragma unroll
            for (int a = 0; a < D; ++a) u[a] = v[a] * den;
            const T um = sqrt(dot<D>(u, u));
            const T drag = tab[TAB_DRAG] + tab[TAB_FORCH] * um;
#pragma unroll
            for (int a = 0; a < D; ++a) F[a] = eps * g[a] - drag * u[a];
        } else {
            const T h = tab[TAB_INV_2C0], drag = tab[TAB_DRAG];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                u[a] = v[a] * h;
                F[a] = eps * g[a] - drag * u[a];
            }
        }
#pragma unroll
        for (int a = D; a < 3; ++a) u[a] = F[a] = T(0);
    }
};

// 1 - sum of the weights as rounded to T (exactly representable: a sum of a
// few floats computed in double).
template <int Q, typename T> __device__ __forceinline__ T weight_defect()
{
    double sw = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) sw += double(T(Lat<Q>::w(i)));
    return T(1.0 - sw);
}

// Relax towards Eq. (30) and add Eq. (31).
//   LOCAL = false: deviations d_i = f_i - w_i in and out.
//   LOCAL = true (kRho stores): local parts e_i = f_i - w_i rho(x) in and out,
//     e*_i = (1 - omega) e_i + omega w_i rho teq_i + F_i.
// For a pair of opposite directions, omega times the equilibrium plus the
// forcing term splits into a part even in e_i (shared) and an odd part (sign
// flipped), so each pair is evaluated once:
//   even  P = w rho [e.u (omega k1 e.u + cforce k2 e.F) + C0]   (+ omega w drho
//         for deviations), k1 = 4.5 / eps, k2 = 9 / eps,
//         C0 = -(1.5 omega u.u + 3 cforce u.F) / eps;
//   odd   D = 3 w rho (omega e.u + cforce e.F).
// The rest direction takes what closes the zeroth moments (sum_i feq_i = rho,
// sum_i F_i = 0): minus twice the sum of the pairs' even parts, the very
// values added to the moving directions, so that rounded weights cannot
// create or destroy mass; in the local form it also takes drho times the
// defect 1 - sum w of the rounded weights, so that the values leaving the
// node, w_i drho + e*_i, carry exactly its mass.
template <int Q, typename T, bool LOCAL, typename NodeT>
__device__ __forceinline__ void relax(T (&d)[Q], const NodeT& s, const T* tab, T omega, T cforce)
{
    using L = Lat<Q>;
    const T ieps = tab[TAB_INV_EPS];
    constexpr int DIM = L::D;
    const T uu = dot<DIM>(s.u, s.u);
    const T uF = dot<DIM>(s.u, s.F);
    const T ok1 = omega * T(4.5) * ieps, ck2 = cforce * T(9) * ieps;
    const T C0 = -(T(1.5) * omega * uu + T(3) * cforce * uF) * ieps;
    const T omw = T(1) - omega;
    T sum = T(0);
    bool first = true;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (!lead<Q>(i)) continue;
        const int o = L::opp(i);
        const T eu = edot<Q>(i, s.u);
        const T eF = edot<Q>(i, s.F);
        const T w = T(L::w(i));
        const T wr = w * s.rho;
        const T even = eu * (ok1 * eu + ck2 * eF) + C0;
        const T P = LOCAL ? wr * even : omega * (w * s.drho) + wr * even;
        const T D = T(3) * wr * (omega * eu + cforce * eF);
        d[i] = omw * d[i] + P + D;
        d[o] = omw * d[o] + P - D;
        sum = first ? P : sum + P;
        first = false;
    }
    if (LOCAL)
        d[0] = omw * d[0] - T(2) * sum + weight_defect<Q, T>() * s.drho;
    else
        d[0] = omw * d[0] + omega * s.drho - T(2) * sum;
}

// Columns of the class table a kernel reads (pressure faces and Forchheimer use all).
template <int BC, bool FORCH> constexpr int tab_cols() { return (FORCH || pressure_faces(BC)) ? kTabW : 4; }

template <int Q, typename T, int NT>
__device__ __forceinline__ void load_table(T* lds, const Args& a, int inst)
{
    const T* gt = static_cast<const T*>(a.tab) + (size_t)inst * kClasses * kTabW;
    for (int k = threadIdx.x; k < kClasses * NT; k += kBlock) lds[k] = gt[(k / NT) * kTabW + (k % NT)];
    __syncthreads();
}

// ---------------------------------------------------------------- the sweep --
// U consecutive slots of a thread (U = 1 in use; the loads of all U slots are
// issued before the first node is collided).  NTS: nontemporal population
// stores.  It is a template parameter so that the two store forms stay
// separate code: as a run-time branch over otherwise identical stores, the
// optimizer merges them and drops the nontemporal hint.
// Collide one node (moments, Eq. 32-37; relaxation towards Eq. 30 with the
// forcing of Eq. 31) and write its q post-collision values (and, for a kRho
// store, its density) to the other buffer.  d and r hold what gather()
// returned for the node; ct is its row of the class table.
// The collision of one node: d (and r) as gather() returned them become the
// node's q post-collision values in the store's form; for a kRho store the
// return value is the node's density deviation (what its density plane
// receives), otherwise 0.
template <int Q, int STORE, int BC, bool FORCH>
__device__ __forceinline__ typename St<STORE>::T collide_node(typename St<STORE>::T (&d)[Q],
                                                              typename St<STORE>::T (&r)[Q],
                                                              const typename St<STORE>::T* ct, const InstDev& I,
                                                              const typename St<STORE>::T (&g)[3],
                                                              typename St<STORE>::T omega, typename St<STORE>::T cforce)
{
    using SS = St<STORE>;
    using T = typename SS::T;
    Node<Q, T, FORCH, pressure_faces(BC)> s;
    T dr = T(0);
    if constexpr (SS::kRho) {
        // local form; collision conserves mass, so the node writes its
        // density and the parts relative to it
        dr = localize<Q, T>(d, r);
        s.moments_with(d, dr, ct, g, I);
        relax<Q, T, true>(d, s, ct, omega, cforce);
    } else if constexpr (STORE == GLBM_STORE_F32) {
        // FP32 deviations d_i = f_i - w_i collide in the local form: the
        // node's own density part w_i drho is split off with a fused
        // multiply-add (the product is not rounded), the collision works
        // on the small parts, and one more fused multiply-add puts the
        // density back.  Each stored value then carries a single rounding
        // at the scale of the density deviation instead of several, which
        // is what keeps the residual falling below 1e-8 on shale maps.
        using L = Lat<Q>;
        T dr = d[0];
#pragma unroll
        for (int i = 1; i < Q; ++i) dr += d[i];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = __builtin_fmaf(-T(L::w(i)), dr, d[i]);
        s.moments_with(d, dr, ct, g, I);
        relax<Q, T, true>(d, s, ct, omega, cforce);
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = __builtin_fmaf(T(L::w(i)), dr, d[i]);
    } else {
        s.moments(d, ct, g, I);
        relax<Q, T, false>(d, s, ct, omega, cforce);
    }
    return dr;
}

template <int Q, int STORE, int BC, bool FORCH, bool NTS>
__device__ __forceinline__ void collide_store(typename St<STORE>::T (&d)[Q], typename St<STORE>::T (&r)[Q], int n,
                                              const typename St<STORE>::T* ct, const InstDev& I,
                                              const typename St<STORE>::T (&g)[3], typename St<STORE>::T omega,
                                              typename St<STORE>::T cforce, typename St<STORE>::S* __restrict__ dst)
{
    using SS = St<STORE>;
    const typename SS::T dr = collide_node<Q, STORE, BC, FORCH>(d, r, ct, I, g, omega, cforce);
    if constexpr (SS::kRho) {
        if constexpr (node_blocks(STORE))
            rho_plane<STORE>(dst, Q, I.stride)[n] = dr;
        else
            *elem(rho_plane<STORE>(dst, Q, I.stride), uint32_t(n)) = dr;
    }
    if constexpr (node_blocks(STORE)) {
        if constexpr (NTS) {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                __builtin_nontemporal_store(SS::enc(d[i], I.scale), dst + pidx<Q, STORE>(i, n, 0));
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) dst[pidx<Q, STORE>(i, n, 0)] = SS::enc(d[i], I.scale);
        }
    } else {
        // plane base uniform, one 32-bit byte offset shared by the q stores
        if constexpr (NTS) {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                __builtin_nontemporal_store(SS::enc(d[i], I.scale), elem(dst + (size_t)i * I.stride, uint32_t(n)));
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) *elem(dst + (size_t)i * I.stride, uint32_t(n)) = SS::enc(d[i], I.scale);
        }
    }
}

template <int U, int Q, int STORE, int BC, bool FORCH, bool NTS>
__device__ __forceinline__ void sweep_slots(const Args& a, const Tile& t, const InstDev& I, int sl0,
                                            const typename St<STORE>::T* __restrict__ tb, int tw,
                                            const typename St<STORE>::S* __restrict__ src,
                                            typename St<STORE>::S* __restrict__ dst, const uint8_t* __restrict__ cls)
{
    using SS = St<STORE>;
    using T = typename SS::T;
    const T g[3] = {inst_g<T>(I, 0), inst_g<T>(I, 1), inst_g<T>(I, 2)};
    const T omega = inst_omega<T>(I), cforce = inst_cforce<T>(I);
    const bool nt_load = (a.cache & 2) != 0;
    const int twm = (1 << a.tw_log2) - 1;
    const int z = t.z0;
    int n[U], c[U];
    bool ok[U];
    T d[U][Q], r[U][Q];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int slot = (sl0 + u) * kBlock + threadIdx.x;
        const int x = t.x0 + (slot & twm);
        const int y = t.y0 + (slot >> a.tw_log2);
        ok[u] = x < I.nx && y < I.ny;
        n[u] = ok[u] ? (z * I.ny + y) * I.nx + x : 0;
        c[u] = ok[u] ? cls[n[u]] : 0;
        if (wall_nodes(BC) && c[u] == kWallClass) ok[u] = false;
        if (ok[u]) gather<Q, STORE, BC>(d[u], r[u], src, cls, I, x, y, z, n[u], nt_load);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (!ok[u]) continue;
        collide_store<Q, STORE, BC, FORCH, NTS>(d[u], r[u], n[u], tb + c[u] * tw, I, g, omega, cforce, dst);
    }
}

template <int Q, int STORE, int BC, bool FORCH>
__device__ __forceinline__ void sweep_tile(const Args& a, const Tile& t, const InstDev& I,
                                           const typename St<STORE>::T* __restrict__ tb, int tw)
{
    using S = typename St<STORE>::S;
    const int sel = (a.parity + I.par) & 1;
    const S* __restrict__ src = static_cast<const S*>(a.buf[sel]) + I.pop_off;
    S* __restrict__ dst = static_cast<S*>(a.buf[sel ^ 1]) + I.pop_off;
    const uint8_t* __restrict__ cls = a.cls + I.cls_off;
    if (a.cache & 1) {
        for (int sl = 0; sl < a.nslot; ++sl) sweep_slots<1, Q, STORE, BC, FORCH, true>(a, t, I, sl, tb, tw, src, dst, cls);
    } else {
        for (int sl = 0; sl < a.nslot; ++sl) sweep_slots<1, Q, STORE, BC, FORCH, false>(a, t, I, sl, tb, tw, src, dst, cls);
    }
}

// One time step of one tile.  Policy bits of a.cache: 0 nontemporal stores,
// 1 nontemporal loads of x-aligned planes, 2 plain workgroup order (no XCD
// grouping), 3 per-class constants read through the L1 cache instead of being
// staged in LDS.  The best setting depends on the layout and the map, and
// glbm_autotune picks it; on the 4096^2 FP32 map (k_sweep9, 6 waves per
// SIMD) it is 256 x 1 tiles with all four bits set (about 6.3 TB/s of
// algorithmic bytes).
template <int Q, int STORE, int BC, bool FORCH> __device__ __forceinline__ void sweep_block(const Args& a)
{
    using T = typename St<STORE>::T;
    constexpr int NT = tab_cols<BC, FORCH>();
    __shared__ T tab[kClasses * NT];

    const int tid = (a.cache & 4) ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
    const Tile t = a.tiles[tid];
    if (!a.active[t.inst]) return;
    const InstDev& I = a.inst[t.inst];
    if (a.cache & 8) {
        const T* gt = static_cast<const T*>(a.tab) + (size_t)t.inst * kClasses * kTabW;
        sweep_tile<Q, STORE, BC, FORCH>(a, t, I, gt, kTabW);
    } else {
        load_table<Q, T, NT>(tab, a, t.inst);
        sweep_tile<Q, STORE, BC, FORCH>(a, t, I, tab, NT);
    }
}

template <int Q, int STORE, int BC, bool FORCH> __global__ __launch_bounds__(kBlock) void k_sweep(Args a)
{
    sweep_block<Q, STORE, BC, FORCH>(a);
}

// D3Q19 with a cap of W waves per SIMD.  With 19 read and 19 write streams per
// wave, fewer waves in flight than the register count allows measured faster
// for the FP32 and FP64 stores (4 waves: 1.4 % faster than 5, 2.7 % faster
// than 8 on the 256^3 map); the FP16 stores, which issue more instructions
// per byte, run best with 5 or more.
template <int STORE, int BC, bool FORCH, int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, W))) void k_sweep19(Args a)
{
    sweep_block<19, STORE, BC, FORCH>(a);
}
template <int STORE> constexpr int waves19()
{
    return (STORE == GLBM_STORE_F16DEV || STORE == GLBM_STORE_F16LOC) ? 5 : 4;
}

// D2Q9 with the node-block stores (FP64, FP32, FP32LOC), capped at 6 waves per
// SIMD.  On the 4096^2 map, FP32 with the class constants read through L1
// measured 0.1951 ms against 0.2023 uncapped (best uncapped tile: 0.2018);
// FP32LOC -2.7 %, the FP32 batch -1.7 %, FP64 unchanged; caps of 4, 5 and 7
// were slower than 6.  The FP16 stores run 6 % slower capped and use k_sweep.
template <int STORE, int BC, bool FORCH, int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, W))) void k_sweep9(Args a)
{
    sweep_block<9, STORE, BC, FORCH>(a);
}
constexpr int kWaves9 = 6;

// ---------------------------------------------------- LDS-staged FP16 sweep --
// D2Q9 with an FP16 store on periodic instances whose nx is a multiple of 8,
// tiles of at most kStW x kStH nodes.  A workgroup first copies into LDS, for
// each of the nine planes, the rows its nodes pull from (the tile shifted by
// -e_i, with one 8-half chunk more on each side, wrapped periodically) and,
// for F16LOC, the density rows y0 - 1 .. y0 + th, all with 16-byte loads;
// every node then reads its nine values and source densities from LDS.  That
// replaces nine 2-byte and nine 4-byte loads per node, which kept the address
// unit busy for 85 % of the plain kernel's cycles, by about two 16-byte loads.
// The arithmetic and the stores are those of k_sweep (collide_store), so the
// results are bitwise equal.
constexpr int kStW = 256;                  // widest staged tile
constexpr int kStH = 4;                    // most rows
constexpr int kStPad = 8;                  // halo: one 8-half chunk on each side
constexpr int kStRow = kStW + 2 * kStPad;  // staged columns per row
// e_y + 1 of the D2Q9 directions, two bits per direction
constexpr uint32_t pack9(bool y)
{
    uint32_t v = 0;
    for (int i = 0; i < 9; ++i) v |= uint32_t((y ? Lat<9>::ey(i) : Lat<9>::ex(i)) + 1) << (2 * i);
    return v;
}
constexpr uint32_t kEy9 = pack9(true);

template <int STORE, bool FORCH, bool NTS>
__device__ __forceinline__ void sweep_staged_tile(const Args& a, const Tile& t, const InstDev& I, const float* tb,
                                                  int tcols, uint16_t (*sp)[kStH][kStRow],
                                                  float (*srho)[kStRow])
{
    using SS = St<STORE>;
    using S = typename SS::S;
    using T = typename SS::T;
    using L = Lat<9>;
    typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
    const int twl = a.tw_log2, tw = 1 << twl, th = (a.nslot * kBlock) >> twl;
    const int nx = I.nx, ny = I.ny;
    const int sel = (a.parity + I.par) & 1;
    const S* __restrict__ src = static_cast<const S*>(a.buf[sel]) + I.pop_off;
    S* __restrict__ dst = static_cast<S*>(a.buf[sel ^ 1]) + I.pop_off;
    const uint8_t* __restrict__ cls = a.cls + I.cls_off;
    // populations: plane i, staged row rr <- grid row y0 + rr - e_y(i), staged
    // column 8 cc .. 8 cc + 7 <- grid columns x0 - 8 + 8 cc .. (wrapped).  Each
    // staged row is one wavefront (lane = chunk cc, cc < tw / 8 + 2 <= 34), so the
    // index arithmetic is shifts and masks; th is 1, 2 or 4.  Rows and chunks that
    // no node of the tile reads (past the grid's last row or column) are skipped,
    // which keeps every source index within one period of the grid.
    const int thl = th == 4 ? 2 : (th == 2 ? 1 : 0);
    const int cpr = (tw >> 3) + 2;
    for (int row = threadIdx.x >> 6; row < 9 * th; row += kBlock >> 6) {
        const int cc = threadIdx.x & 63;
        const int i = row >> thl, rr = row & (th - 1);
        int gx = t.x0 - kStPad + 8 * cc;
        if (cc < cpr && gx <= nx && t.y0 + rr < ny) {
            int gy = t.y0 + rr - (int((kEy9 >> (2 * i)) & 3u) - 1);
            gy += gy < 0 ? ny : (gy >= ny ? -ny : 0);
            gx += gx < 0 ? nx : (gx >= nx ? -nx : 0);
            const S* p = src + (size_t)i * I.stride + (size_t)gy * nx + gx;
            *reinterpret_cast<u32x4v*>(&sp[i][rr][8 * cc]) = *reinterpret_cast<const u32x4v*>(p);
        }
    }
    if constexpr (SS::kRho) {
        // density rows y0 - 1 .. y0 + th, columns x0 - 8 .. x0 + tw + 7, four floats a
        // load: two staged rows per pass of 128 lanes (cc < tw / 4 + 4 <= 68)
        const float* rp = rho_plane<STORE>(src, 9, I.stride);
        const int cpr4 = (tw >> 2) + 4;
        for (int rr = threadIdx.x >> 7; rr < th + 2; rr += kBlock >> 7) {
            const int cc = threadIdx.x & 127;
            int gy = t.y0 - 1 + rr, gx = t.x0 - kStPad + 4 * cc;
            if (cc < cpr4 && gx <= nx && gy <= ny) {
                gy += gy < 0 ? ny : (gy >= ny ? -ny : 0);
                gx += gx < 0 ? nx : (gx >= nx ? -nx : 0);
                *reinterpret_cast<u32x4v*>(&srho[rr][4 * cc]) =
                    *reinterpret_cast<const u32x4v*>(rp + (size_t)gy * nx + gx);
            }
        }
    }
    __syncthreads();
    const T g[3] = {inst_g<T>(I, 0), inst_g<T>(I, 1), inst_g<T>(I, 2)};
    const T omega = inst_omega<T>(I), cforce = inst_cforce<T>(I);
    for (int sl = 0; sl < a.nslot; ++sl) {
        const int slot = sl * kBlock + threadIdx.x;
        const int lx = slot & (tw - 1), ry = slot >> twl;
        const int x = t.x0 + lx, y = t.y0 + ry;
        if (x >= nx || y >= ny) continue;
        const int n = y * nx + x;
        T d[9], r[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int col = lx + kStPad - L::ex(i);
            d[i] = SS::dec(sp[i][ry][col], I.inv_scale);
            if constexpr (SS::kRho) r[i] = srho[ry + 1 - L::ey(i)][col];
        }
        collide_store<9, STORE, 0, FORCH, NTS>(d, r, n, tb + cls[n] * tcols, I, g, omega, cforce, dst);
    }
}

template <int STORE, bool FORCH>
__global__ __launch_bounds__(kBlock) void k_sweep9h(Args a)
{
    constexpr int NT = tab_cols<0, FORCH>();
    __shared__ float tab[kClasses * NT];
    __shared__ __align__(16) uint16_t sp[9][kStH][kStRow];
    __shared__ __align__(16) float srho[St<STORE>::kRho ? kStH + 2 : 1][kStRow];
    const int tid = (a.cache & 4) ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
    const Tile t = a.tiles[tid];
    if (!a.active[t.inst]) return;
    const InstDev& I = a.inst[t.inst];
    const float* tb;
    int tcols;
    if (a.cache & 8) {
        tb = static_cast<const float*>(a.tab) + (size_t)t.inst * kClasses * kTabW;
        tcols = kTabW;
    } else {
        load_table<9, float, NT>(tab, a, t.inst);   // ends with a barrier before tab is read
        tb = tab;
        tcols = NT;
    }
    if (a.cache & 1) sweep_staged_tile<STORE, FORCH, true>(a, t, I, tb, tcols, sp, srho);
    else sweep_staged_tile<STORE, FORCH, false>(a, t, I, tb, tcols, sp, srho);
}

// ------------------------------------------------ paired-node FP16 sweep --
// D2Q9 with an FP16 store on periodic instances whose nx is even, tiles at
// least 128 nodes wide and a whole number of 512-node groups.  Each lane owns
// two x-adjacent nodes (x even), so a wavefront covers 128 consecutive nodes
// of one row.  Per plane the lane reads the pair's source values as one
// 4-byte word; for the planes shifted along x, the value that falls outside
// the pair (x - 1 or x + 2) is the neighbouring lane's word, fetched with a
// DPP wavefront shift, and read from memory only at the wavefront's ends and
// at the grid's periodic seam.  For F16LOC the three density rows a pair
// pulls from are read as 8-byte pairs the same way (three loads serve all
// nine directions of both nodes).  The two nodes collide exactly as in
// k_sweep and are written back as 4-byte words (plus one 8-byte density
// pair), so the results are bitwise equal to the plain sweep's.
__device__ __forceinline__ uint32_t from_lane_below(uint32_t v)
{
    // lane l receives lane l - 1's value (lane 0 receives 0)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t from_lane_above(uint32_t v)
{
    // lane l receives lane l + 1's value (lane 63 receives 0)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);
}

template <int STORE, bool FORCH, bool NTS>
__device__ __forceinline__ void sweep_pair_tile(const Args& a, const Tile& t, const InstDev& I, const float* tb,
                                                int tcols)
{
    using SS = St<STORE>;
    using S = typename SS::S;
    using T = typename SS::T;
    using L = Lat<9>;
    const int twl = a.tw_log2, hwl = twl - 1;  // pairs per tile row: 2^hwl
    const int nx = I.nx, ny = I.ny;
    const int lane = threadIdx.x & 63;
    const int sel = (a.parity + I.par) & 1;
    const S* __restrict__ src = static_cast<const S*>(a.buf[sel]) + I.pop_off;
    S* __restrict__ dst = static_cast<S*>(a.buf[sel ^ 1]) + I.pop_off;
    const uint8_t* __restrict__ cls = a.cls + I.cls_off;
    const T g[3] = {inst_g<T>(I, 0), inst_g<T>(I, 1), inst_g<T>(I, 2)};
    const T omega = inst_omega<T>(I), cforce = inst_cforce<T>(I);
    for (int it = 0; it < (a.nslot >> 1); ++it) {
        const int s = it * kBlock + threadIdx.x;
        const int x = t.x0 + 2 * (s & ((1 << hwl) - 1)), y = t.y0 + (s >> hwl);
        if (y >= ny) continue;  // whole wavefronts: a wavefront covers one tile row
        const bool on = x < nx;
        // every lane reads at a valid address (lanes past the grid's last
        // column read its first pair and store nothing), so that the
        // wavefront shifts below see defined values in every lane
        const int xc = on ? x : 0;
        const bool left_ok = lane != 0 && xc != 0;        // lane l - 1 holds x - 2, x - 1
        const bool right_ok = lane != 63 && xc + 2 < nx;  // lane l + 1 holds x + 2, x + 3
        const int xl = xc == 0 ? nx - 1 : xc - 1, xr = xc + 2 == nx ? 0 : xc + 2;
        const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        // all loads first (the class bytes, the words, the density pairs, and
        // the few values past the wavefront's ends), then the wavefront
        // shifts: no load waits on another
        const uint32_t cc = *reinterpret_cast<const uint16_t*>(cls + (y * nx + xc));
        const S* plane[9];
        uint32_t w[9], el[9], er[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int ey = L::ey(i);
            const int sy = ey > 0 ? ym : (ey < 0 ? yp : y);
            plane[i] = src + (size_t)i * I.stride + (size_t)sy * nx;
            w[i] = *reinterpret_cast<const uint32_t*>(plane[i] + xc);  // source values at xc, xc + 1
            el[i] = 0u;
            er[i] = 0u;
        }
        const float* rrow[3];
        float2 rv[3];
        float fl[3] = {0.f, 0.f, 0.f}, fr[3] = {0.f, 0.f, 0.f};
        if constexpr (SS::kRho) {
            const float* rp = rho_plane<STORE>(src, 9, I.stride);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                rrow[k] = rp + (size_t)(k == 0 ? ym : (k == 1 ? y : yp)) * nx;
                rv[k] = *reinterpret_cast<const float2*>(rrow[k] + xc);
            }
        }
        if (!left_ok) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (L::ex(i) > 0) el[i] = plane[i][xl];
            if constexpr (SS::kRho) {
#pragma unroll
                for (int k = 0; k < 3; ++k) fl[k] = rrow[k][xl];
            }
        }
        if (!right_ok) {
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (L::ex(i) < 0) er[i] = plane[i][xr];
            if constexpr (SS::kRho) {
#pragma unroll
                for (int k = 0; k < 3; ++k) fr[k] = rrow[k][xr];
            }
        }
        T da[9], db[9], ra[9], rb[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int ex = L::ex(i);
            uint32_t lo = w[i] & 0xffffu, hi = w[i] >> 16;
            if (ex > 0) {
                // node x pulls x - 1: the high half of the word below
                const uint32_t v = from_lane_below(w[i]) >> 16;
                hi = lo;
                lo = left_ok ? v : el[i];
            } else if (ex < 0) {
                // node x + 1 pulls x + 2: the low half of the word above
                const uint32_t v = from_lane_above(w[i]) & 0xffffu;
                lo = hi;
                hi = right_ok ? v : er[i];
            }
            da[i] = SS::dec(S(lo), I.inv_scale);
            db[i] = SS::dec(S(hi), I.inv_scale);
        }
        if constexpr (SS::kRho) {
            float rl[3], r0[3], r1[3], rr[3];  // per source row: x - 1, x, x + 1, x + 2
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float below = __uint_as_float(from_lane_below(__float_as_uint(rv[k].y)));
                const float above = __uint_as_float(from_lane_above(__float_as_uint(rv[k].x)));
                rl[k] = left_ok ? below : fl[k];
                r0[k] = rv[k].x;
                r1[k] = rv[k].y;
                rr[k] = right_ok ? above : fr[k];
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int ex = L::ex(i), ey = L::ey(i);
                const int k = ey > 0 ? 0 : (ey < 0 ? 2 : 1);
                ra[i] = ex > 0 ? rl[k] : (ex < 0 ? r1[k] : r0[k]);
                rb[i] = ex > 0 ? r0[k] : (ex < 0 ? rr[k] : r1[k]);
            }
        }
        if (!on) continue;
        const int n = y * nx + x;
        const T dra = collide_node<9, STORE, 0, FORCH>(da, ra, tb + (cc & 0xffu) * tcols, I, g, omega, cforce);
        const T drb = collide_node<9, STORE, 0, FORCH>(db, rb, tb + (cc >> 8) * tcols, I, g, omega, cforce);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const uint32_t v = uint32_t(SS::enc(da[i], I.scale)) | (uint32_t(SS::enc(db[i], I.scale)) << 16);
            uint32_t* at = reinterpret_cast<uint32_t*>(dst + (size_t)i * I.stride + n);
            if constexpr (NTS) __builtin_nontemporal_store(v, at);
            else *at = v;
        }
        if constexpr (SS::kRho) {
            typedef float f32x2 __attribute__((ext_vector_type(2)));
            f32x2* at = reinterpret_cast<f32x2*>(rho_plane<STORE>(dst, 9, I.stride) + n);
            const f32x2 v = {dra, drb};
            if constexpr (NTS) __builtin_nontemporal_store(v, at);
            else *at = v;
        }
    }
}

template <int STORE, bool FORCH>
__global__ __launch_bounds__(kBlock) void k_sweep9p(Args a)
{
    constexpr int NT = tab_cols<0, FORCH>();
    __shared__ float tab[kClasses * NT];
    const int tid = (a.cache & 4) ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
    const Tile t = a.tiles[tid];
    if (!a.active[t.inst]) return;
    const InstDev& I = a.inst[t.inst];
    const float* tb;
    int tcols;
    if (a.cache & 8) {
        tb = static_cast<const float*>(a.tab) + (size_t)t.inst * kClasses * kTabW;
        tcols = kTabW;
    } else {
        load_table<9, float, NT>(tab, a, t.inst);   // ends with a barrier before tab is read
        tb = tab;
        tcols = NT;
    }
    if (a.cache & 1) sweep_pair_tile<STORE, FORCH, true>(a, t, I, tb, tcols);
    else sweep_pair_tile<STORE, FORCH, false>(a, t, I, tb, tcols);
}

// --------------------------------------------- two steps per launch (D2Q9) --
// Temporal blocking on periodic D2Q9 instances.  A workgroup owns a TW x TH
// tile and advances it two time steps in one launch:
//   1. every node of the tile grown by one node on each side is swept from the
//      source buffer as in a single-step sweep (pull, collide); its q values,
//      encoded as the store would hold them, and for a kRho store its density
//      deviation, are kept in LDS, not written back;
//   2. every node of the tile pulls those values from LDS, decodes them as a
//      load from the store would, collides again and writes the result to the
//      other buffer.
// The nodes of the one-node rim are computed by the neighbouring tiles as
// well (redundantly: (TW + 2)(TH + 2) / (TW TH) - 1 of the collisions), but the
// intermediate state never travels through HBM, so one launch moves about the
// bytes of one plain sweep for two steps.  The arithmetic is that of
// collide_node, and step 2 sees exactly the values a load of the store would
// return, so the result is bitwise equal to two single-step launches.  The
// state then sits in the buffer a single step would have written, so the
// host issues these launches in pairs (four steps between state reads).
template <int TW, int TH> struct TbShape {
    static constexpr int kRW = TW + 2, kRH = TH + 2, kRegion = kRW * kRH;
};

// Step 2's pull of node (x, y), at (lx, ly) in the tile, from the grown tile in
// LDS, with the boundary rules of gather(): directions entering through a
// pressure face are left to fill_face, and a pull that a face wall or a wall
// node blocks takes the node's own opposite value.  c1 holds the classes of
// the grown tile (step 2 takes its nodes' classes from there too, instead of
// a second read of the class map).
template <int STORE, int BC, int TW, int TH>
__device__ __forceinline__ void pull_tb(typename St<STORE>::T (&d)[9], typename St<STORE>::T (&r)[9],
                                        const typename St<STORE>::S (*f1)[TbShape<TW, TH>::kRegion],
                                        const float* __restrict__ rho1, const uint8_t* __restrict__ c1,
                                        const InstDev& I, int x, int y, int lx, int ly)
{
    using SS = St<STORE>;
    using T = typename SS::T;
    using L = Lat<9>;
    using Sh = TbShape<TW, TH>;
    const int own = (ly + 1) * Sh::kRW + (lx + 1);
    int side = 0;
    if constexpr (pressure_faces(BC)) {
        const int ca = I.paxis == 0 ? x : y, na = I.paxis == 0 ? I.nx : I.ny;
        side = ca == 0 ? 1 : (ca == na - 1 ? -1 : 0);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ex = L::ex(i), ey = L::ey(i);
        if constexpr (pressure_faces(BC)) {
            const int ea = I.paxis == 0 ? ex : (I.paxis == 1 ? ey : 0);
            if (side * ea > 0) {
                d[i] = T(0);
                r[i] = T(0);
                continue;
            }
        }
        int e = (ly + 1 - ey) * Sh::kRW + (lx + 1 - ex);
        int j = i;
        if constexpr (face_walls(BC) || wall_nodes(BC)) {
            const uint32_t w = I.walls;
            bool blocked = false;
            if constexpr (face_walls(BC)) {
                if (ex > 0) blocked |= (x == 0) && (w & 1u);
                if (ex < 0) blocked |= (x == I.nx - 1) && (w & 2u);
                if (ey > 0) blocked |= (y == 0) && (w & 4u);
                if (ey < 0) blocked |= (y == I.ny - 1) && (w & 8u);
            }
            if (wall_nodes(BC) && i != 0) blocked |= c1[e] == kWallClass;
            if (blocked) {
                e = own;
                j = L::opp(i);
            }
        }
        d[i] = SS::dec(f1[j][e], I.inv_scale);
        if constexpr (SS::kRho) r[i] = rho1[e];
        else r[i] = T(0);
    }
    if constexpr (pressure_faces(BC))
        if (side != 0) fill_face<9, SS::kRho>(d, r, I, side);
}

template <int STORE, int BC, bool FORCH, bool NTS, int TW, int TH>
__device__ __forceinline__ void sweep_tb_tile(const Args& a, const Tile& t, const InstDev& I,
                                              const typename St<STORE>::T* __restrict__ tb, int tcols,
                                              typename St<STORE>::S (*f1)[TbShape<TW, TH>::kRegion],
                                              float* __restrict__ rho1, uint8_t* __restrict__ c1)
{
    using SS = St<STORE>;
    using S = typename SS::S;
    using T = typename SS::T;
    using Sh = TbShape<TW, TH>;
    const int nx = I.nx, ny = I.ny;
    const int sel = (a.parity + I.par) & 1;
    const S* __restrict__ src = static_cast<const S*>(a.buf[sel]) + I.pop_off;
    S* __restrict__ dst = static_cast<S*>(a.buf[sel ^ 1]) + I.pop_off;
    const uint8_t* __restrict__ cls = a.cls + I.cls_off;
    const T g[3] = {inst_g<T>(I, 0), inst_g<T>(I, 1), inst_g<T>(I, 2)};
    const T omega = inst_omega<T>(I), cforce = inst_cforce<T>(I);
    const bool nt_load = (a.cache & 2) != 0;
    // step 1 over the grown tile (coordinates wrapped onto the grid; beyond a
    // face wall or a pressure face the wrapped rim nodes are computed but never
    // pulled, since those pulls are blocked or rebuilt)
    for (int e = threadIdx.x; e < Sh::kRegion; e += kBlock) {
        const int ry = e / Sh::kRW, rx = e - ry * Sh::kRW;
        int x = t.x0 - 1 + rx, y = t.y0 - 1 + ry;
        x += x < 0 ? nx : 0;
        y += y < 0 ? ny : 0;
        if (x >= nx) x -= nx;
        if (x >= nx) x %= nx;  // grids narrower than the tile
        if (y >= ny) y -= ny;
        if (y >= ny) y %= ny;
        const int n = y * nx + x;
        const int c = cls[n];
        c1[e] = uint8_t(c);
        if (wall_nodes(BC) && c == kWallClass) continue;  // never swept, never pulled from
        T d[9], r[9];
        gather<9, STORE, BC>(d, r, src, cls, I, x, y, 0, n, nt_load);
        const T dr = collide_node<9, STORE, BC, FORCH>(d, r, tb + c * tcols, I, g, omega, cforce);
#pragma unroll
        for (int i = 0; i < 9; ++i) f1[i][e] = SS::enc(d[i], I.scale);
        if constexpr (SS::kRho) rho1[e] = dr;
    }
    __syncthreads();
    // step 2 over the tile, pulling from the grown tile in LDS
    for (int s = threadIdx.x; s < TW * TH; s += kBlock) {
        const int ly = s / TW, lx = s - ly * TW;
        const int x = t.x0 + lx, y = t.y0 + ly;
        if (x >= nx || y >= ny) continue;
        const int n = y * nx + x;
        const int c = c1[(ly + 1) * Sh::kRW + lx + 1];
        if (wall_nodes(BC) && c == kWallClass) continue;
        T d[9], r[9];
        pull_tb<STORE, BC, TW, TH>(d, r, f1, rho1, c1, I, x, y, lx, ly);
        collide_store<9, STORE, BC, FORCH, NTS>(d, r, n, tb + c * tcols, I, g, omega, cforce, dst);
    }
}

template <int STORE, int BC, bool FORCH, int TW, int TH>
__global__ __launch_bounds__(kBlock) void k_sweep9tb(Args a)
{
    using SS = St<STORE>;
    using T = typename SS::T;
    using Sh = TbShape<TW, TH>;
    constexpr int NT = tab_cols<BC, FORCH>();
    __shared__ T tab[kClasses * NT];
    __shared__ typename SS::S f1[9][Sh::kRegion];
    __shared__ float rho1[SS::kRho ? Sh::kRegion : 1];
    __shared__ uint8_t c1[Sh::kRegion];
    const int tid = (a.cache & 4) ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
    const Tile t = a.tiles[tid];
    if (!a.active[t.inst]) return;
    const InstDev& I = a.inst[t.inst];
    const T* tb;
    int tcols;
    if (a.cache & 8) {
        tb = static_cast<const T*>(a.tab) + (size_t)t.inst * kClasses * kTabW;
        tcols = kTabW;
    } else {
        load_table<9, T, NT>(tab, a, t.inst);   // ends with a barrier before tab is read
        tb = tab;
        tcols = NT;
    }
    if (a.cache & 1) sweep_tb_tile<STORE, BC, FORCH, true, TW, TH>(a, t, I, tb, tcols, f1, rho1, c1);
    else sweep_tb_tile<STORE, BC, FORCH, false, TW, TH>(a, t, I, tb, tcols, f1, rho1, c1);
}

// ------------------------------------------------------------ observations --
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum kN doubles over the 256 threads of a block in a fixed order; result in thread 0.
template <int kN> __device__ __forceinline__ void block_sum(double (&v)[kN], double* lds)
{
#pragma unroll
    for (int k = 0; k < kN; ++k) v[k] = wave_sum(v[k]);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < kN; ++k) lds[wave * kN + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < kN; ++k) v[k] = lds[k] + lds[kN + k] + lds[2 * kN + k] + lds[3 * kN + k];
}

// mode bit 0: store u into the snapshot; bit 1: accumulate |u - u_snap|^2.
template <int Q, int STORE, int BC, bool FORCH>
__device__ __forceinline__ void observe_tile(const Args& a, const Tile& t, const InstDev& I, int tid, int mode,
                                             const typename St<STORE>::T* __restrict__ tb, int tw, double* red)
{
    using SS = St<STORE>;
    using S = typename SS::S;
    using T = typename SS::T;
    const int sel = (a.parity + I.par) & 1;
    const S* __restrict__ src = static_cast<const S*>(a.buf[sel]) + I.pop_off;
    const uint8_t* __restrict__ cls = a.cls + I.cls_off;
    T* __restrict__ snap = static_cast<T*>(a.snap) + I.snap_off;
    const int N = I.nx * I.ny * I.nz;
    const T g[3] = {inst_g<T>(I, 0), inst_g<T>(I, 1), inst_g<T>(I, 2)};
    const int twm = (1 << a.tw_log2) - 1;
    const int z = t.z0;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // P_SD .. P_BAD, then the count for P_FAST

    for (int sl = 0; sl < a.nslot; ++sl) {
        const int slot = sl * kBlock + threadIdx.x;
        const int x = t.x0 + (slot & twm);
        const int y = t.y0 + (slot >> a.tw_log2);
        if (x >= I.nx || y >= I.ny) continue;
        const int n = (z * I.ny + y) * I.nx + x;
        const int c = cls[n];
        if (wall_nodes(BC) && c == kWallClass) continue;
        T d[Q], rr[Q];
        gather<Q, STORE, BC>(d, rr, src, cls, I, x, y, z, n);
        Node<Q, T, FORCH, pressure_faces(BC)> s;
        if constexpr (SS::kRho) {
            const T dr = localize<Q, T>(d, rr);
            s.moments_with(d, dr, tb + c * tw, g, I);
        } else {
            s.moments(d, tb + c * tw, g, I);
        }
        if (mode & 2) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double du = double(s.u[k]) - double(snap[k * N + n]);
                acc[P_SD] += du * du;
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            acc[P_SU] += double(s.u[k]) * double(s.u[k]);
            acc[P_UX + k] += double(s.u[k]);
        }
        if (!(finite(s.drho) && finite(s.u[0]) && finite(s.u[1]) && finite(s.u[2]))) acc[P_BAD] += 1.0;
        const double u2 = double(s.u[0]) * double(s.u[0]) + double(s.u[1]) * double(s.u[1]) +
                          double(s.u[2]) * double(s.u[2]);
        if (u2 > kUMax * kUMax) acc[6] += 1.0;
        if (mode & 1)
#pragma unroll
            for (int k = 0; k < 3; ++k) snap[k * N + n] = s.u[k];
    }
    block_sum<7>(acc, red);
    if (threadIdx.x == 0) {
        double* p = a.part + (size_t)tid * kPartW;
#pragma unroll
        for (int k = 0; k < 6; ++k) p[k] = acc[k];
        p[P_FAST_T] = acc[6];
    }
}

// mode bit 0: store u into the snapshot; bit 1: accumulate |u - u_snap|^2.
template <int Q, int STORE, int BC, bool FORCH>
__global__ __launch_bounds__(kBlock) void k_observe(Args a, int mode, int all)
{
    using T = typename St<STORE>::T;
    constexpr int NT = tab_cols<BC, FORCH>();
    __shared__ T tab[kClasses * NT];
    __shared__ double red[4 * 7];

    const int tid = (a.cache & 4) ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
    const Tile t = a.tiles[tid];
    if (!all && !a.active[t.inst]) return;
    const InstDev& I = a.inst[t.inst];
    if (a.cache & 8) {
        const T* gt = static_cast<const T*>(a.tab) + (size_t)t.inst * kClasses * kTabW;
        observe_tile<Q, STORE, BC, FORCH>(a, t, I, tid, mode, gt, kTabW, red);
    } else {
        load_table<Q, T, NT>(tab, a, t.inst);
        observe_tile<Q, STORE, BC, FORCH>(a, t, I, tid, mode, tab, NT, red);
    }
}

// One 1024-thread workgroup per instance sums its tile partials.  They are
// read as one flat array of doubles, so that a wavefront's loads are
// contiguous: thread t adds component t % 8 of tiles t / 8, t / 8 + 128, ...
// (eight loads in flight), then a fixed-order tree over the threads that hold
// the same component.  The order depends only on the tile count, so results
// are deterministic and equal between a batch and a single-instance run.
constexpr int kFinBlock = 1024;
constexpr int kFinTiles = kFinBlock / kPartW;   // tiles per pass
__global__ __launch_bounds__(kFinBlock) void k_finalize(Args a, double tol, int with_r, int count_check, int all)
{
    static_assert(kFinBlock % kPartW == 0, "a thread keeps one component");
    __shared__ double red[kFinBlock];
    const int inst = blockIdx.x;
    if (!all && !a.active[inst]) return;
    const InstDev& I = a.inst[inst];
    const int k = threadIdx.x % kPartW, t0 = threadIdx.x / kPartW;
    double acc = 0.0;
    if ((k < 6 || k == P_FAST_T) && t0 < I.ntiles) {
        // element (t0 + kFinTiles * j) * kPartW + k of the instance's partials
        const double* p = a.part + (size_t)I.tile0 * kPartW + threadIdx.x;
        const int nj = (I.ntiles - 1 - t0) / kFinTiles + 1;
        int j = 0;
        for (; j + 8 <= nj; j += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(j + u) * kFinBlock];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; j < nj; ++j) acc += p[(size_t)j * kFinBlock];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kFinBlock / 2; s >= kPartW; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double out[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) out[c] = red[c];
        double* res = a.res + (size_t)inst * kResW;
#pragma unroll
        for (int c = 0; c < 6; ++c) res[c] = out[c];
        res[P_FAST] = red[P_FAST_T];
        if (with_r) {
            const double r = sqrt(out[P_SD]) / (double(a.dsteps[inst]) * sqrt(out[P_SU]));
            res[P_R] = (out[P_SU] > 0.0) ? r : INFINITY;
            if (out[P_BAD] > 0.0) res[P_R] = NAN;
            if (tol > 0.0 && res[P_R] <= tol) a.active[inst] = 0;
        }
        if (count_check) res[P_NCHK] += 1.0;
    }
}

// Streaming copy with nontemporal 16-byte loads and stores, one element per
// lane and one grid covering the whole range: the memory pattern of a sweep
// without its gathers or arithmetic, as a practical bandwidth ceiling for this
// GPU.  (Measured on a 1 GiB copy: 6.5 TB/s this way; a grid-stride loop over
// 65,536 or fewer workgroups, with one or four loads in flight per lane,
// reached 4.3-5.9 TB/s.)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                     size_t n, size_t base)
{
    const size_t i = base + blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void k_zero(uint32_t* p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Equilibrium of (rho, u) written so that the next pull reads it back as f(x).
// A double source holds rho; a float source holds rho - 1, so that a small
// density deviation is not rounded against 1 before it reaches the kernel.
template <int Q, int STORE, int BC, typename R>
__global__ __launch_bounds__(kBlock) void k_set_fields(Args a, int inst, const R* rho_in, const R* u_in)
{
    constexpr bool kDrho = sizeof(R) == 4;
    using SS = St<STORE>;
    using S = typename SS::S;
    using T = typename SS::T;
    using L = Lat<Q>;
    const InstDev& I = a.inst[inst];
    const Tile t = a.tiles[I.tile0 + blockIdx.x];
    const T* tabg = static_cast<const T*>(a.tab) + (size_t)inst * kClasses * kTabW;
    const int sel = (a.parity + I.par) & 1;
    S* __restrict__ dst = static_cast<S*>(a.buf[sel]) + I.pop_off;
    const uint8_t* __restrict__ cls = a.cls + I.cls_off;
    const int N = I.nx * I.ny * I.nz;
    const int twm = (1 << a.tw_log2) - 1;
    const int z = t.z0;
    for (int sl = 0; sl < a.nslot; ++sl) {
        const int slot = sl * kBlock + threadIdx.x;
        const int x = t.x0 + (slot & twm);
        const int y = t.y0 + (slot >> a.tw_log2);
        if (x >= I.nx || y >= I.ny) continue;
        const int n = (z * I.ny + y) * I.nx + x;
        const int c = cls[n];
        if (c == kWallClass) continue;
        const auto drho_at = [&](int m) { return kDrho ? T(rho_in[m]) : T(rho_in[m] - R(1)); };
        const T drn = drho_at(n);
        const T rho = T(1) + drn;
        const T u[3] = {T(u_in[n]), T(u_in[N + n]), T(u_in[2 * N + n])};
        if (SS::kRho) rho_plane<STORE>(dst, Q, I.stride)[n] = drn;
        const T ieps = tabg[c * kTabW + TAB_INV_EPS];
        const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const T eu = T(L::ex(i)) * u[0] + T(L::ey(i)) * u[1] + T(L::ez(i)) * u[2];
            const T dq = T(L::w(i)) * (drn + rho * (T(3) * eu + T(4.5) * ieps * eu * eu - T(1.5) * ieps * uu));
            // destination slot: the pull of direction i at n reads plane i at n - e_i
            // when that move is open, else plane opp(i) at n itself.
            const int ex = L::ex(i), ey = L::ey(i), ez = L::ez(i);
            int sx = x - ex, sy = y - ey, sz = z - ez;
            bool blocked = false;
            if (sx < 0) { blocked |= (I.walls & 1u) != 0; sx += I.nx; }
            if (sx >= I.nx) { blocked |= (I.walls & 2u) != 0; sx -= I.nx; }
            if (sy < 0) { blocked |= (I.walls & 4u) != 0; sy += I.ny; }
            if (sy >= I.ny) { blocked |= (I.walls & 8u) != 0; sy -= I.ny; }
            if (sz < 0) { blocked |= (I.walls & 16u) != 0; sz += I.nz; }
            if (sz >= I.nz) { blocked |= (I.walls & 32u) != 0; sz -= I.nz; }
            const int sn = (sz * I.ny + sy) * I.nx + sx;
            if (wall_nodes(BC) && !blocked && i != 0) blocked = cls[sn] == kWallClass;
            const int idx = blocked ? pidx<Q, STORE>(L::opp(i), n, I.stride) : pidx<Q, STORE>(i, sn, I.stride);
            // a kRho value is decoded with the density of the node whose slot it occupies
            const T dr = SS::kRho ? drho_at(blocked ? n : sn) : T(0);
            dst[idx] = SS::enc(dq - T(L::w(i)) * dr, I.scale);
        }
    }
}

template <int Q, int STORE, int BC, bool FORCH>
__global__ __launch_bounds__(kBlock) void k_get_fields(Args a, int inst, double* rho_out, double* u_out,
                                                        double* pops)
{
    using SS = St<STORE>;
    using S = typename SS::S;
    using T = typename SS::T;
    using L = Lat<Q>;
    const InstDev& I = a.inst[inst];
    const Tile t = a.tiles[I.tile0 + blockIdx.x];
    const T* tabg = static_cast<const T*>(a.tab) + (size_t)inst * kClasses * kTabW;
    const int sel = (a.parity + I.par) & 1;
    const S* __restrict__ src = static_cast<const S*>(a.buf[sel]) + I.pop_off;
    const uint8_t* __restrict__ cls = a.cls + I.cls_off;
    const int N = I.nx * I.ny * I.nz;
    const T g[3] = {inst_g<T>(I, 0), inst_g<T>(I, 1), inst_g<T>(I, 2)};
    const int twm = (1 << a.tw_log2) - 1;
    const int z = t.z0;
    for (int sl = 0; sl < a.nslot; ++sl) {
        const int slot = sl * kBlock + threadIdx.x;
        const int x = t.x0 + (slot & twm);
        const int y = t.y0 + (slot >> a.tw_log2);
        if (x >= I.nx || y >= I.ny) continue;
        const int n = (z * I.ny + y) * I.nx + x;
        const int c = cls[n];
        if (c == kWallClass) {
            if (rho_out) rho_out[n] = 0.0;
            if (u_out) u_out[n] = u_out[N + n] = u_out[2 * N + n] = 0.0;
            if (pops)
                for (int i = 0; i < Q; ++i) pops[(size_t)i * N + n] = 0.0;
            continue;
        }
        T d[Q], rr[Q];
        gather<Q, STORE, BC>(d, rr, src, cls, I, x, y, z, n);
        T ct[kTabW];
#pragma unroll
        for (int k = 0; k < kTabW; ++k) ct[k] = tabg[c * kTabW + k];
        Node<Q, T, FORCH, pressure_faces(BC)> s;
        if constexpr (SS::kRho) {
            const T dr = localize<Q, T>(d, rr);
            s.moments_with(d, dr, ct, g, I);
#pragma unroll
            for (int i = 0; i < Q; ++i) d[i] += T(L::w(i)) * dr;  // back to f_i - w_i for the readback
        } else {
            s.moments(d, ct, g, I);
        }
        if (rho_out) rho_out[n] = 1.0 + double(s.drho);
        if (u_out)
            for (int k = 0; k < 3; ++k) u_out[k * N + n] = double(s.u[k]);
        if (pops)
#pragma unroll
            for (int i = 0; i < Q; ++i) pops[(size_t)i * N + n] = L::w(i) + double(d[i]);
    }
}

// -------------------------------------------------------------- dispatch --
template <int Q, int STORE, int BC, bool FORCH> struct SweepK {
    static hipError_t go(const Args& a, hipStream_t s)
    {
        if constexpr (Q == 9 && !node_blocks(STORE) && BC == 0) {
            if (a.staged) {
                hipLaunchKernelGGL((k_sweep9h<STORE, FORCH>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
                return hipGetLastError();
            }
            if (a.paired) {
                hipLaunchKernelGGL((k_sweep9p<STORE, FORCH>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
                return hipGetLastError();
            }
        }
        if constexpr (Q == 19)
            hipLaunchKernelGGL((k_sweep19<STORE, BC, FORCH, waves19<STORE>()>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
        else if constexpr (node_blocks(STORE))
            hipLaunchKernelGGL((k_sweep9<STORE, BC, FORCH, kWaves9>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_sweep<Q, STORE, BC, FORCH>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
};
template <int Q, int STORE, int BC, bool FORCH> struct ObserveK {
    static hipError_t go(const Args& a, hipStream_t s, int mode, int all)
    {
        hipLaunchKernelGGL((k_observe<Q, STORE, BC, FORCH>), dim3(a.ntiles), dim3(kBlock), 0, s, a, mode, all);
        return hipGetLastError();
    }
};
template <int Q, int STORE, int BC, bool FORCH> struct GetFieldsK {
    static hipError_t go(const Args& a, hipStream_t s, int inst, int ntiles, double* rho, double* u, double* p)
    {
        hipLaunchKernelGGL((k_get_fields<Q, STORE, BC, FORCH>), dim3(ntiles), dim3(kBlock), 0, s, a, inst, rho, u,
                           p);
        return hipGetLastError();
    }
};

template <template <int, int, int, bool> class K, typename... A>
hipError_t dispatch(const Config& c, A... args)
{
#define GLBM_CASE(QQ, SS, BB, FF)                                                          \
    if (c.q == QQ && c.store == SS && c.bc == BB && c.forch == FF) return K<QQ, SS, BB, FF>::go(args...);
#define GLBM_F(QQ, SS, BB) GLBM_CASE(QQ, SS, BB, false) GLBM_CASE(QQ, SS, BB, true)
#define GLBM_B(QQ, SS)                                                                      \
    GLBM_F(QQ, SS, 0) GLBM_F(QQ, SS, 1) GLBM_F(QQ, SS, 2) GLBM_CASE(QQ, SS, 3, false) GLBM_CASE(QQ, SS, 4, false)
#define GLBM_S(QQ)                                                                                 \
    GLBM_B(QQ, GLBM_STORE_F64) GLBM_B(QQ, GLBM_STORE_F32) GLBM_B(QQ, GLBM_STORE_F16DEV)              \
    GLBM_B(QQ, GLBM_STORE_F16LOC) GLBM_B(QQ, GLBM_STORE_F32LOC)
    GLBM_S(9)
    GLBM_S(19)
#undef GLBM_S
#undef GLBM_B
#undef GLBM_F
#undef GLBM_CASE
    return hipErrorInvalidValue;
}

template <int Q, int STORE, int BC, typename R>
hipError_t set_fields_go(const Args& a, hipStream_t s, int inst, int ntiles, const R* rho, const R* u)
{
    hipLaunchKernelGGL((k_set_fields<Q, STORE, BC, R>), dim3(ntiles), dim3(kBlock), 0, s, a, inst, rho, u);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep(const Config& c, const Args& a, hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    return dispatch<SweepK>(c, a, s);
}

bool tb_applies(const Config& c, int tw_log2, int th)
{
    if (c.q != 9) return false;
    const int tw = 1 << tw_log2;
    const bool small = (tw == 64 && (th == 4 || th == 8)) || (tw == 128 && th == 4);
    const bool large = (tw == 64 && th == 16) || (tw == 128 && th == 8) || (tw == 256 && th == 4);
    if (c.bc == 3 || c.bc == 4)  // pressure faces (no Forchheimer classes there)
        return !c.forch && small && (c.store == GLBM_STORE_F64 || c.store == GLBM_STORE_F32);
    if (c.bc != 0) return false;
    switch (c.store) {
    case GLBM_STORE_F32:
    case GLBM_STORE_F32LOC:
    case GLBM_STORE_F16LOC: return small || large;
    case GLBM_STORE_F64: return small;  // 72 bytes of LDS per grown-tile node
    default: return false;
    }
}

hipError_t launch_sweep_tb(const Config& c, const Args& a, hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    const int tw = 1 << a.tw_log2, th = (a.nslot * kBlock) >> a.tw_log2;
    if (!tb_applies(c, a.tw_log2, th)) return hipErrorInvalidValue;
#define GLBM_TB_ST(ST, W, H)                                                                         \
    if (c.store == ST) {                                                                             \
        if (c.forch)                                                                                 \
            hipLaunchKernelGGL((k_sweep9tb<ST, 0, true, W, H>), dim3(a.ntiles), dim3(kBlock), 0, s, a);  \
        else                                                                                         \
            hipLaunchKernelGGL((k_sweep9tb<ST, 0, false, W, H>), dim3(a.ntiles), dim3(kBlock), 0, s, a); \
        return hipGetLastError();                                                                    \
    }
#define GLBM_TB_P(ST, W, H)                                                                          \
    if (c.store == ST) {                                                                             \
        if (c.bc == 3)                                                                               \
            hipLaunchKernelGGL((k_sweep9tb<ST, 3, false, W, H>), dim3(a.ntiles), dim3(kBlock), 0, s, a); \
        else                                                                                         \
            hipLaunchKernelGGL((k_sweep9tb<ST, 4, false, W, H>), dim3(a.ntiles), dim3(kBlock), 0, s, a); \
        return hipGetLastError();                                                                    \
    }
#define GLBM_TB(W, H)                                                                                \
    if (tw == W && th == H) {                                                                        \
        GLBM_TB_ST(GLBM_STORE_F32, W, H)                                                             \
        GLBM_TB_ST(GLBM_STORE_F32LOC, W, H)                                                          \
        GLBM_TB_ST(GLBM_STORE_F16LOC, W, H)                                                          \
        return hipErrorInvalidValue;                                                                 \
    }
#define GLBM_TB64(W, H)                                                                              \
    if (tw == W && th == H) {                                                                        \
        if (c.bc != 0) {                                                                             \
            GLBM_TB_P(GLBM_STORE_F32, W, H)                                                          \
            GLBM_TB_P(GLBM_STORE_F64, W, H)                                                          \
            return hipErrorInvalidValue;                                                             \
        }                                                                                            \
        GLBM_TB_ST(GLBM_STORE_F32, W, H)                                                             \
        GLBM_TB_ST(GLBM_STORE_F32LOC, W, H)                                                          \
        GLBM_TB_ST(GLBM_STORE_F16LOC, W, H)                                                          \
        GLBM_TB_ST(GLBM_STORE_F64, W, H)                                                             \
        return hipErrorInvalidValue;                                                                 \
    }
    GLBM_TB64(64, 4) GLBM_TB64(64, 8) GLBM_TB64(128, 4) GLBM_TB(64, 16) GLBM_TB(128, 8) GLBM_TB(256, 4)
#undef GLBM_TB64
#undef GLBM_TB_P
#undef GLBM_TB_ST
#undef GLBM_TB
    return hipErrorInvalidValue;
}

hipError_t launch_observe(const Config& c, const Args& a, int mode, hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    return dispatch<ObserveK>(c, a, s, mode & 3, (mode & 4) ? 1 : 0);
}

hipError_t launch_finalize(const Args& a, int n_inst, double tol, int with_r, int count_check, hipStream_t s)
{
    const int all = with_r ? 0 : 1;
    hipLaunchKernelGGL(k_finalize, dim3(n_inst), dim3(kFinBlock), 0, s, a, tol, with_r, count_check, all);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    // at most 2^30 workgroups per launch (the grid's x dimension is below 2^31)
    const size_t per_launch = size_t(1) << 38;  // elements: 2^30 workgroups x 256
    for (size_t base = 0; base < n; base += per_launch) {
        const size_t cnt = std::min(per_launch, n - base);
        hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                           static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n, base);
    }
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint32_t*>(p), n);
    return hipGetLastError();
}

hipError_t launch_set_fields(const Config& c, const Args& a, int inst, int ntiles, const void* rho,
                             const void* u, int src_is_double, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
#define GLBM_SF(QQ, SS, BB)                                                                              \
    if (c.q == QQ && c.store == SS && c.bc == BB)                                                        \
        return src_is_double                                                                             \
                   ? set_fields_go<QQ, SS, BB, double>(a, s, inst, ntiles, static_cast<const double*>(rho), \
                                                       static_cast<const double*>(u))                     \
                   : set_fields_go<QQ, SS, BB, float>(a, s, inst, ntiles, static_cast<const float*>(rho),   \
                                                      static_cast<const float*>(u));
#define GLBM_SF_B(QQ, SS) GLBM_SF(QQ, SS, 0) GLBM_SF(QQ, SS, 1) GLBM_SF(QQ, SS, 2) GLBM_SF(QQ, SS, 3) GLBM_SF(QQ, SS, 4)
#define GLBM_SF_S(QQ)                                                                              \
    GLBM_SF_B(QQ, GLBM_STORE_F64) GLBM_SF_B(QQ, GLBM_STORE_F32) GLBM_SF_B(QQ, GLBM_STORE_F16DEV)     \
    GLBM_SF_B(QQ, GLBM_STORE_F16LOC) GLBM_SF_B(QQ, GLBM_STORE_F32LOC)
    GLBM_SF_S(9)
    GLBM_SF_S(19)
#undef GLBM_SF_S
#undef GLBM_SF_B
#undef GLBM_SF
    return hipErrorInvalidValue;
}

hipError_t launch_get_fields(const Config& c, const Args& a, int inst, int ntiles, double* rho, double* u,
                             double* pops, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    return dispatch<GetFieldsK>(c, a, s, inst, ntiles, rho, u, pops);
}

}  // namespace glbm
