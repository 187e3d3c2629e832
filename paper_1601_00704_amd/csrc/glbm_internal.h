// Internal declarations shared by the HIP kernels and the host side of libglbm.
// Not part of the public ABI (include/glbm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glbm.h"

namespace glbm {

constexpr int kBlock = 256;         // threads per workgroup (4 wavefronts)
constexpr int kMinTileW = 64;       // a wavefront covers 64 consecutive x
constexpr int kMaxTileW = 1024;
constexpr int kClasses = 256;
constexpr int kWallClass = 255;
constexpr int kTabW = 8;            // constants per class in the device table
constexpr int kPartW = 8;           // doubles per tile partial (slots below)
constexpr int kResW = 16;           // doubles per instance result (slots below)

// Per-class constants (index into a row of kTabW values).
enum TabSlot {
    TAB_EPS = 0,        // eps
    TAB_INV_EPS = 1,    // 1 / eps
    TAB_INV_2C0 = 2,    // 1 / (2 c0), Eq. (36)
    TAB_DRAG = 3,       // eps nu / K
    TAB_C0 = 4,         // c0, Eq. (36)
    TAB_C1 = 5,         // c1, Eq. (37)
    TAB_FORCH = 6,      // eps F_eps / sqrt(K)
    // pressure-driven instances (bc 3, 4): K(P) = A + (B + C / (1 + b P)) / P, 1/K scaled by OPEN
    TAB_PA = 2,         // A (K_0 / dx^2; 1 for an open pore)
    TAB_PB = 3,         // B (eta D_K / dx^2)
    TAB_PC = 4,         // C (surface-diffusion coefficient / dx^2)
    TAB_PBL = 5,        // b (Langmuir, 1 / pressure unit)
    TAB_POPEN = 6,      // 0 for an open pore (no drag), 1 otherwise
};

// Per-tile / per-instance reduction record (doubles).
enum PartSlot {
    P_SD = 0,    // sum |u - u_snap|^2
    P_SU = 1,    // sum |u|^2
    P_UX = 2,    // sum u_x
    P_UY = 3,
    P_UZ = 4,
    P_BAD = 5,   // count of non-finite nodes
    P_R = 6,     // residual (instance record only)
    P_NCHK = 7,  // checks done (instance record only)
    P_FAST = 8,  // count of nodes with |u| > kUMax, the instability guard (instance record)
    P_FAST_T = 6,  // the same count in a tile partial (whose slot 6 holds no residual)
};

// Instability guard: a check that sees a node velocity above this (lattice
// units; the sound speed is 1/sqrt(3)) ends glbm_step_n with GLBM_EUNSTABLE,
// since the equilibrium of Eq. (30) holds only at low Mach numbers.
constexpr double kUMax = 0.1;

// Population layout.  FP64 and FP32 stores keep the q values of kBlk
// consecutive nodes together, as q runs of kBlk elements (node blocks): the
// 2q streams of a sweep then stay within a few hundred KiB of each other,
// which measured 2-7 % faster than q whole-lattice planes.  The FP16 stores,
// bound by instructions rather than bytes, measured faster with planes
// (element i * stride + node).
constexpr int kBlkLog2 = 12;
constexpr int kBlk = 1 << kBlkLog2;
constexpr bool node_blocks(int store) { return store != GLBM_STORE_F16DEV && store != GLBM_STORE_F16LOC; }

// Device-side instance descriptor.
struct InstDev {
    int64_t pop_off;     // element offset of plane 0 of this instance in each buffer
    int64_t cls_off;     // byte offset of the class map
    int64_t snap_off;    // element offset of the u snapshot (3 planes of N)
    int32_t stride;      // elements per population plane (node blocks: padded to whole blocks); the
                         // FP32 density plane of the local-density stores starts at q * stride
    int32_t nx, ny, nz;
    uint32_t walls;      // face bits
    int32_t par;         // parity offset: state buffer = (g + par) & 1 at global step g
    int32_t tile0, ntiles;  // range of this instance in the tile list
    double g[3];
    double omega;        // 1 / tau
    double cforce;       // 1 - 1 / (2 tau)
    double nu;
    float scale, inv_scale;  // FP16 deviation scale 2^s and 2^-s
    float gf[3];             // g, omega and cforce rounded to float (FP32 kernels)
    float omegaf, cforcef;
    // pressure faces (bc 3, 4): axis 0..2, face densities as rho - 1, and the local
    // pressure P = p0 + (rho - 1) p1 (double, and float copies)
    int32_t paxis;
    double drin, drout, p0, p1;
    float drinf, droutf, p0f, p1f, nuf;
};

struct Tile {
    int32_t inst, x0, y0, z0;
};

// Everything a kernel launch needs (passed by value).
struct Args {
    const Tile* tiles;
    const InstDev* inst;
    const uint8_t* cls;
    void* buf[2];          // population buffers A, B
    const void* tab;       // per instance kTabW * kClasses values of the compute type
    void* snap;            // u snapshots (compute type)
    double* part;          // per tile kPartW doubles
    double* res;           // per instance kPartW doubles
    int32_t* active;       // per instance flag
    const int32_t* dsteps; // per instance steps since the snapshot
    int32_t ntiles;
    int32_t parity;        // g & 1
    int32_t tw_log2;       // tile width 2^tw_log2 nodes along x (64 .. 1024)
    int32_t nslot;         // tile nodes / kBlock: nodes each thread visits
    int32_t cache;         // bit 0: nontemporal population stores; bit 1: nontemporal loads of x-aligned planes
    int32_t staged;        // D2Q9 FP16 sweep with LDS-staged rows (k_sweep9h)
    int32_t paired;        // D2Q9 FP16 sweep with two x-adjacent nodes per lane (k_sweep9p)
};

// Kernel configuration of a context.
struct Config {
    int q;        // 9 or 19
    int store;    // GLBM_STORE_*
    int bc;       // 0 periodic only, 1 face walls, 2 face walls + wall nodes, 3 pressure faces, 4 pressure faces + wall nodes
    bool forch;   // any F_eps > 0
};

// Host launchers (glbm_kernels.hip).
hipError_t launch_sweep(const Config& c, const Args& a, hipStream_t s);
// two time steps per launch (D2Q9, FP32 node blocks, periodic; tiles 64 x 4/8/16,
// 128 x 4/8, 256 x 4): reads the buffer of a.parity, writes the other one
bool tb_applies(const Config& c, int tw_log2, int th);
hipError_t launch_sweep_tb(const Config& c, const Args& a, hipStream_t s);
// mode bit 0: update snapshot; bit 1: accumulate residual terms
hipError_t launch_observe(const Config& c, const Args& a, int mode, hipStream_t s);
// tol > 0: deactivate converged instances; with_r: compute r from S_d, S_u
hipError_t launch_finalize(const Args& a, int n_inst, double tol, int with_r, int count_check,
                           hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
// Write the equilibrium of (rho, u) of instance `inst` (device arrays): src_is_double = 1 reads
// rho as double, 0 reads rho - 1 as float; u is 3 planes of N of the same type
hipError_t launch_set_fields(const Config& c, const Args& a, int inst, int ntiles, const void* rho,
                             const void* u, int src_is_double, hipStream_t s);
// Density, velocity (double, N and 3N) and optionally populations (double, q*N) of instance `inst`
hipError_t launch_get_fields(const Config& c, const Args& a, int inst, int ntiles, double* rho, double* u,
                             double* pops, hipStream_t s);

// Warm-start coupling kernels (glbm_cnn.hip).
hipError_t launch_cnn_features(const uint8_t* cls, long long n, const float* table, uint16_t* x, hipStream_t s);
hipError_t launch_cnn_targets(const double* rho, const double* u, const uint8_t* cls, long long n, double rs,
                              double us, float* target, uint8_t* mask, hipStream_t s);
hipError_t launch_cnn_apply(const float* y, long long n, double rs, double us, float* drho, float* u, hipStream_t s);

// Error message of the calling thread (glbm_api.cpp).
void set_error(const char* msg);

}  // namespace glbm
