// lbm_internal.h -- declarations shared by the kernels (lbm_kernels.hip) and
// the C ABI implementation (lbm_api.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lbm.h"

namespace lbm {

// Kernel flavours of the fused step (one source, selected at compile time).
enum Mode : int {
    MODE_STEP = 0,     // advance: write post-collision populations
    MODE_CHECK = 1,    // advance and accumulate FP64 block sums for the check
    MODE_MOMENTS = 2,  // no advance: write rho_1, rho_2, u_F of the current state
    MODE_REDUCE = 3,   // no advance: FP64 block sums only
};

// Population storage.  Fluid sites have slot indices k; kGroup consecutive
// slots form a group.  A buffer has two halves, directions 0 .. kSplit - 1
// and kSplit .. 18 (each opposite pair inside one half).  In its half, the
// component pair (f^1_i, f^2_i) of direction i (i - kSplit in the second
// half) of slot k is pair number
//   ((k / kGroup) * kHalfDirs + i_half) * kGroup + k % kGroup,
// so the directions of a group lie in two short runs of memory, and a run
// of kGroup slots of one direction is contiguous.
constexpr int kGroup = 32;
constexpr int kHalfDirs = 11;
constexpr int kSplit = 11;

// Per-block partial sums written by MODE_CHECK / MODE_REDUCE:
// [rho1, rho2, rho uF_x, rho uF_y, rho uF_z, non-finite count, 0, 0].
constexpr int kPartialStride = 8;

// Everything a step launch needs, by value.  Physical parameters are kept
// in double; each kernel converts them to its compute type.
struct StepLaunch {
    const void *src;
    void *dst;
    const int32_t *idx;     // compact population index of each lattice site, -1 where solid
    const int32_t *itab;    // index tiles of the step (launch_index_tiles) for this tile shape
    const int32_t *wstart;  // work list bounds: per tile column (ty ntx + tx) nz + 1 entries
    const uint16_t *wpos;   // work list entries: tile positions ly tile_x + lx of fluid sites
    int nx, ny, nz;
    int64_t ngroups;        // slot groups per buffer half (fluid sites' groups plus padding)
    int tile_x, tile_y, zchunk;
    int ntx, nty, nzc;      // tiles in x, y and chunks in z
    // Work items of the launch, 4 ints each (tile x, tile y, first and end
    // plane), one per block; null: every column cut into chunks of zchunk
    // planes (ntx nty nzc blocks)
    const int32_t *btab;
    int nblk;
    double tau0, tau1, G, gx, gy, gz, wall0, wall1, ref0, ref1;
    double tau_crit;        // 32/16-bit storage: sites with tau_mix below it form P_ab in FP64
    int eq_kind, force_kind, wall_kind;
    double *partials;       // kPartialStride doubles per block
    double *out_rho0, *out_rho1, *out_u;  // MODE_MOMENTS outputs (N, N, 3N)
};

// Launches one fused step (or moments / reduce pass) of precision prec.
hipError_t launch_step(int prec, Mode mode, const StepLaunch &L, hipStream_t s);
// Sums nblocks partials (fixed order) into out[kPartialStride] on the device.
hipError_t launch_finalize(const double *partials, int nblocks, double *out, hipStream_t s);
// Index tiles of the step for tiles of tx x ty sites: per tile column
// (ty ntx + tx) and plane, the (tx + 4)(ty + 4) sites around the tile (a
// periodic ring of two) row by row, each as the byte offset of its
// population pairs (pair_bytes each) within a buffer half, all bits set
// where solid; ntx nty nz (tx + 4)(ty + 4) entries.
hipError_t launch_index_tiles(const int32_t *idx, int32_t *itab, int nx, int ny, int nz, int tx, int ty, int pair_bytes,
                              hipStream_t s);
// Per-site link mask: bit 0 = site solid, bit i = site - c_i solid (periodic).
hipError_t launch_links(const uint8_t *solid, uint32_t *links, int nx, int ny, int nz, hipStream_t s);
// Restart field checks (N sites; u 3N or null): out[0] += fluid sites,
// out[1] = min(out[1], lowest fluid site with invalid densities), out[2] =
// min(out[2], lowest with a non-finite velocity); the caller sets out to
// {0, N, N} first.
hipError_t launch_check_fields(const uint32_t *links, const double *rho0, const double *rho1, const double *u,
                               int64_t N, unsigned long long *out, hipStream_t s);
// Internal state from fields: f*_j(x) = f_j(x + c_j) if that site is fluid,
// else f_opp(j)(x), with f = f_eq from rho (2N), u (3N or null), plus the
// strain's non-equilibrium part when pi (6N, launch_strain) is given; with
// acc (6N, launch_accel) u is u_F and component a takes u_F - acc_a / 2.
// Populations of fluid site s are at slot idx[s].
hipError_t launch_init_fields(int prec, void *dst, const uint32_t *links, const int32_t *idx, const double *rho0,
                              const double *rho1, const double *u, const double *pi, const double *acc, int nx,
                              int ny, int nz, int64_t ngroups, int eq_kind, const double ref[2], hipStream_t s);
// F_a / rho_a of each component (6N) from the densities: Eqs. (7) and (11)
// with the wall densities wall0, wall1 (W2 when wall_kind is 1), plus g.
hipError_t launch_accel(const uint32_t *links, const double *rho0, const double *rho1, double G, double wall0,
                        double wall1, int wall_kind, const double g[3], int nx, int ny, int nz, double *acc,
                        hipStream_t s);
// Pi / rho of the warm start's non-equilibrium part (6N: xx, yy, zz, xy, xz,
// yz) from the velocity field's strain; zero on solid sites.
hipError_t launch_strain(const uint32_t *links, const double *rho0, const double *rho1, const double *u, double tau0,
                         double tau1, int nx, int ny, int nz, double *pi, hipStream_t s);
// FP64 distance sums [sum d ra^2, sum ra^2, sum |d u|^2, sum |u|^2,
// sum ra_prev^2, sum |u_prev|^2] as block partials (nblocks blocks of 256
// threads).
hipError_t launch_residual(const double *ra, const double *u, const double *ra_prev, const double *u_prev, int64_t N,
                           int nblocks, double *partials, hipStream_t s);
// Internal state from ABI populations (inverse of the pull).
hipError_t launch_set_pops(int prec, void *dst, const uint32_t *links, const int32_t *idx, const double *f, int nx,
                           int ny, int nz, int64_t ngroups, const double ref[2], hipStream_t s);
// ABI populations from the internal state (the pull); solid sites read 0.
hipError_t launch_get_pops(int prec, const void *src, const uint32_t *links, const int32_t *idx, double *f, int nx,
                           int ny, int nz, int64_t ngroups, const double ref[2], hipStream_t s);
// Batched launches over many domains: a descriptor per domain (the typed
// kernel arguments, built by fill_batch_desc from a StepLaunch) and a work list
// of (domain, tile) pairs; flip swaps each descriptor's (src, dst).
size_t batch_desc_size(int prec);
void fill_batch_desc(int prec, const StepLaunch &L, void *out);
// hi: some domain uses the FP64 flux below tau_crit (the HI instances).
hipError_t launch_batch(int prec, Mode mode, bool hi, int tx, int ty, const void *descs, const int2 *work, int nwork,
                        int flip, hipStream_t s);

// Tile shapes the step kernel is compiled for.
bool tile_supported(int tx, int ty);
// Resident blocks per compute unit of the plain step kernel (0 if unknown).
int step_blocks_per_cu(int prec, int tx, int ty);

}  // namespace lbm
