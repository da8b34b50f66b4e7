// lbm_api.hip -- the C ABI declared in include/lbm.h: context lifecycle,
// argument validation, launch configuration, the periodic FP64 mass check,
// and the population / field exchange calls.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm_internal.h"

struct lbm_ctx {
    lbm_params p;               // copy; borrowed pointers cleared
    int64_t N = 0, ngroups = 0, nfluid = 0;
    size_t esz = 0;
    void *f[2] = {nullptr, nullptr};
    int cur = 0;
    uint32_t *links = nullptr;   // per-site link mask (set-up and exchange kernels)
    int32_t *idx = nullptr;      // compact population index per site, -1 where solid
    int32_t *itab = nullptr;     // index tiles of the step for the context's tile shape
    int32_t *wstart = nullptr;   // work lists of the step: bounds per tile column and plane
    int32_t *btab = nullptr;     // balanced work items of the step (4 ints each), or null
    int nblk = 0;                // their number
    uint16_t *wpos = nullptr;    // work list entries (tile positions of fluid sites)
    double *partials = nullptr;
    double *red_dev = nullptr;
    double *red_host = nullptr;   // pinned
    double *stage = nullptr;      // 5N doubles, allocated on first use
    double *warm = nullptr;       // 12N doubles of a strain restart, allocated on first use
    double *snap = nullptr;       // 4N doubles: rho1 and u_F of the last lbm_residual (first use)
    bool snap_valid = false;      // false: the snapshot is cleared before the next residual
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    double mass0[2] = {0, 0};
    double ref[2] = {0, 0};       // shift references of 16-bit storage (0 for FP32 / FP64)
    bool ref_set = false;
    int64_t steps_done = 0;
    int tile_x = 0, tile_y = 0, zchunk = 0, ntx = 0, nty = 0, nzc = 0;
    // replayable graphs of kGraphSteps plain steps, one per starting buffer
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    bool graphs_off = false;
    std::string err;
};

struct lbm_batch {
    std::vector<lbm_ctx *> ctx;
    int prec = 0, tile_x = 0, tile_y = 0;
    bool hi = false;                // some domain forms the flux in FP64 below its tau_crit
    hipStream_t stream = nullptr;
    size_t desc_size = 0;
    std::vector<char> descs_host;
    void *descs_dev = nullptr;
    int2 *work_dev = nullptr;
    int nwork = 0;
    std::vector<int> zchunk, nzc;   // per domain: the batch's z-chunk and chunk count
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graphs_off = false;
    std::string err;
};

namespace {

// Work memory of lbm_reduce_noalloc: the per-block partial sums of one
// reduction (kPartialStride doubles per block, at most kScratchBlocks
// blocks) followed by their total.  One copy per GPU, held until the process
// ends; host code reaches it only through the address that
// hipGetSymbolAddress gives for the current device (scratch_ptr).
constexpr int kScratchBlocks = 16384;
constexpr size_t kScratchDoubles = (size_t)(kScratchBlocks + 1) * lbm::kPartialStride;
__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::vector<double *> g_scratch_ptr;   // device address of scratch, per device (nullptr: not looked up yet)

// Looks up the device address of scratch on the current device, once per
// device.  Returns hipSuccess and leaves it in g_scratch_ptr[dev].
hipError_t scratch_setup(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (g_scratch_ptr[dev]) return hipSuccess;
    double *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
    return hipSuccess;
}

double *scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return dev < (int)g_scratch_ptr.size() ? g_scratch_ptr[dev] : nullptr;
}

// Plain steps per captured graph (even, so a replay returns to the buffer it
// started from).
constexpr int kGraphSteps = 16;

std::string g_init_error = "no error";

int fail(lbm_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    else g_init_error = msg;
    return code;
}

int bfail(lbm_batch *b, int code, const std::string &msg) {
    if (b) b->err = msg;
    else g_init_error = msg;
    return code;
}

#define HIPCHK(c, expr)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((c), LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t storage_bytes(int prec) {
    switch (prec) {
    case LBM_FP64: return 8;
    case LBM_FP32: return 4;
    case LBM_FP16S:
    case LBM_BF16S: return 2;
    default: return 0;
    }
}

double default_mass_tol(int prec) {
    switch (prec) {
    case LBM_FP64: return 1e-9;
    case LBM_FP32: return 1e-3;
    default: return 1e-1;
    }
}

int device_cus() {
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

// Fixed cost of a plane in units of pull jobs, per thread of the block
// (measured on the 256^3 packed spheres, FP32 and FP16S at 64 x 16:
// 0, 0.25, 0.5, 1, 2, 4 -> 1 is fastest, 3-4 % below uniform chunks).
constexpr double kPlaneFixed = 1.0;

// Work items of balanced cost for one launch of the step (4 ints each: tile
// x, tile y, first plane, end plane).  A block's time grows with the pull
// jobs of its planes (fluid sites plus the ring of the tile) and a fixed
// part per plane (barrier, index tile, moments in LDS), plus a start-up of
// about three planes (pulled one at a time before the pipeline runs).
// Each tile column is cut greedily into z-ranges of cost at most T (at
// least four planes each), T the smallest for which the items fit in one
// round of resident blocks; so dense columns get more, shorter items than
// sparse ones and the blocks finish together.  Items are ordered by their
// ordinal within the column, then tile row and column, so that the range
// of items one XCD receives (xcd_remap) are neighbours.
std::vector<int32_t> balance_items(const std::vector<int32_t> &wstart, int ntx, int nty, int nz, int tx, int ty,
                                   int64_t resident) {
    const int ncol = ntx * nty;
    const double ring = 2.0 * (tx + 2) + 2.0 * ty, fixed = kPlaneFixed * tx * ty;
    std::vector<double> cost((size_t)ncol * nz);
    double total = 0.0;
    for (int col = 0; col < ncol; ++col)
        for (int z = 0; z < nz; ++z) {
            const size_t w = (size_t)col * (nz + 1) + z;
            const double v = (double)(wstart[w + 1] - wstart[w]) + ring + fixed;
            cost[(size_t)col * nz + z] = v;
            total += v;
        }
    const double startup = 3.0 * total / ((double)ncol * nz);
    const int minp = std::min(4, nz);
    struct Item { int k, col, z0, z1; };
    auto cut = [&](double T, std::vector<Item> *out) {
        int64_t items = 0;
        for (int col = 0; col < ncol; ++col) {
            const double *cc = cost.data() + (size_t)col * nz;
            for (int z = 0, k = 0; z < nz; ++k) {
                double c = startup;
                int z1 = z;
                while (z1 < nz && (z1 - z < minp || c + cc[z1] <= T)) c += cc[z1++];
                if (nz - z1 < minp) z1 = nz;   // no short tail item
                if (out) out->push_back(Item{k, col, z, z1});
                ++items;
                z = z1;
            }
        }
        return items;
    };
    double hi = startup;
    for (int col = 0; col < ncol; ++col) {
        double s = startup;
        for (int z = 0; z < nz; ++z) s += cost[(size_t)col * nz + z];
        hi = std::max(hi, s);
    }
    double lo = 0.0;
    if (cut(hi, nullptr) <= resident)
        for (int it = 0; it < 60; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (cut(mid, nullptr) <= resident) hi = mid;
            else lo = mid;
        }
    std::vector<Item> items;
    cut(hi, &items);
    std::stable_sort(items.begin(), items.end(), [&](const Item &a, const Item &b) {
        return a.k != b.k ? a.k < b.k : a.col < b.col;
    });
    std::vector<int32_t> tab;
    tab.reserve(items.size() * 4);
    for (const Item &it : items) {
        tab.push_back(it.col % ntx);
        tab.push_back(it.col / ntx);
        tab.push_back(it.z0);
        tab.push_back(it.z1);
    }
    return tab;
}

// Launch shape of the step.  fluid: the fraction of fluid sites.
void choose_launch(lbm_ctx *c, double fluid) {
    const lbm_params &p = c->p;
    int tx = p.tile_x, ty = p.tile_y;
    if (tx == 0 || ty == 0) {
        // Wider tiles pull a smaller ring of neighbour densities per site.
        // At 32 and 16 bits the 64 x 16 block (1024 threads, one per CU) is
        // taken where a plane's expected jobs (fluid sites plus the 164
        // ring positions) fit in one pass, else 64 x 8; FP64 (two waves per
        // SIMD, 256-thread tiles only) runs as 32 x 8.
        const bool narrow = p.prec != LBM_FP64;
        if (narrow && p.nx >= 48 && p.ny >= 32 && fluid * 1024.0 + 164.0 <= 1024.0) { tx = 64; ty = 16; }
        else if (narrow && p.nx >= 48 && p.ny >= 16) { tx = 64; ty = 8; }
        else if (p.nx >= 24) { tx = 32; ty = 8; }
        else if (p.nx >= 12) { tx = 16; ty = 16; }
        else { tx = 8; ty = 32; }
    }
    c->tile_x = tx;
    c->tile_y = ty;
    c->ntx = (p.nx + tx - 1) / tx;
    c->nty = (p.ny + ty - 1) / ty;
    int zc = p.zchunk;
    if (zc <= 0) {
        // One round of resident blocks: as many z-chunks as fit beside the
        // tile columns at the kernel's occupancy, each as deep as that
        // allows (fewer chunks re-pull fewer boundary planes).
        const int64_t resident = (int64_t)std::max(lbm::step_blocks_per_cu(p.prec, tx, ty), 1) * device_cus();
        const int64_t xy = (int64_t)c->ntx * c->nty;
        const int64_t chunks = std::max<int64_t>(resident / xy, 1);
        zc = (int)((p.nz + chunks - 1) / chunks);
        if (zc < 4) zc = 4;
    }
    if (zc > p.nz) zc = p.nz;
    c->zchunk = zc;
    c->nzc = (p.nz + zc - 1) / zc;
}

lbm::StepLaunch make_launch(const lbm_ctx *c, const void *src, void *dst) {
    const lbm_params &p = c->p;
    lbm::StepLaunch L{};
    L.src = src;
    L.dst = dst;
    L.idx = c->idx;
    L.itab = c->itab;
    L.wstart = c->wstart;
    L.wpos = c->wpos;
    L.nx = p.nx; L.ny = p.ny; L.nz = p.nz;
    L.ngroups = c->ngroups;
    L.tile_x = c->tile_x; L.tile_y = c->tile_y; L.zchunk = c->zchunk;
    L.ntx = c->ntx; L.nty = c->nty; L.nzc = c->nzc;
    L.btab = c->btab;
    L.nblk = c->nblk;
    L.tau0 = p.tau[0]; L.tau1 = p.tau[1]; L.G = p.G;
    L.gx = p.g[0]; L.gy = p.g[1]; L.gz = p.g[2];
    L.wall0 = p.rho_s < 0 ? -p.rho_s : 0.0;   // rho^s_1 = -rho^s Theta(-rho^s)
    L.wall1 = p.rho_s > 0 ? p.rho_s : 0.0;    // rho^s_2 =  rho^s Theta(rho^s)
    L.ref0 = c->ref[0];
    L.ref1 = c->ref[1];
    L.tau_crit = p.tau_crit;
    L.eq_kind = p.eq_kind; L.force_kind = p.force_kind; L.wall_kind = p.wall_kind;
    L.partials = c->partials;
    return L;
}

int nblocks(const lbm_ctx *c) { return c->btab ? c->nblk : c->ntx * c->nty * c->nzc; }

// FP64 sums of the current state into c->red_host (synchronizes).
int measure(lbm_ctx *c, double *rho0, double *rho1, double *u) {
    lbm::StepLaunch L = make_launch(c, c->f[c->cur], nullptr);
    L.out_rho0 = rho0; L.out_rho1 = rho1; L.out_u = u;
    HIPCHK(c, lbm::launch_step(c->p.prec, lbm::MODE_MOMENTS, L, c->stream));
    HIPCHK(c, lbm::launch_finalize(c->partials, nblocks(c), c->red_dev, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->red_host, c->red_dev, sizeof(double) * lbm::kPartialStride,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int ensure_stage(lbm_ctx *c) {
    if (c->stage) return LBM_OK;
    if (hipMalloc(&c->stage, sizeof(double) * 5 * (size_t)c->N) != hipSuccess) {
        c->stage = nullptr;
        (void)hipGetLastError();
        return fail(c, LBM_ENOMEM, "cannot allocate the 5N-double staging buffer");
    }
    return LBM_OK;
}

int validate_fields(lbm_ctx *c, const uint8_t *solid_h, const double *r0, const double *r1, const double *u,
                    int64_t *nfluid) {
    int64_t nf = 0;
    for (int64_t s = 0; s < c->N; ++s) {
        if (solid_h && solid_h[s]) continue;
        ++nf;
        const double a = r0[s], b = r1[s];
        if (!std::isfinite(a) || !std::isfinite(b) || a < 0 || b < 0 || a + b <= 0) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "invalid densities at fluid site %lld: rho1=%g rho2=%g (need >= 0, sum > 0)",
                          (long long)s, a, b);
            return fail(c, LBM_EINVAL, buf);
        }
        if (u && !(std::isfinite(u[s]) && std::isfinite(u[c->N + s]) && std::isfinite(u[2 * c->N + s])))
            return fail(c, LBM_EINVAL, "non-finite initial velocity");
    }
    if (nf == 0) return fail(c, LBM_EINVAL, "the lattice has no fluid site");
    *nfluid = nf;
    return LBM_OK;
}

// Checks the staged fields (c->stage: rho1, rho2 and, with has_u, u_F) on
// the device: the verdicts and messages of validate_fields.  Sets
// c->nfluid.  Synchronizes the stream.
int check_staged_fields(lbm_ctx *c, bool has_u) {
    const unsigned long long N = (unsigned long long)c->N;
    unsigned long long init[3] = {0ull, N, N}, res[3] = {0ull, N, N};
    auto *out = reinterpret_cast<unsigned long long *>(c->red_dev);   // kPartialStride doubles: room for 3
    HIPCHK(c, hipMemcpyAsync(out, init, sizeof init, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, lbm::launch_check_fields(c->links, c->stage, c->stage + c->N, has_u ? c->stage + 2 * c->N : nullptr,
                                       c->N, out, c->stream));
    HIPCHK(c, hipMemcpyAsync(res, out, sizeof res, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (res[1] < N && res[1] <= res[2]) {
        double a = 0.0, b = 0.0;
        HIPCHK(c, hipMemcpy(&a, c->stage + res[1], sizeof(double), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(&b, c->stage + c->N + res[1], sizeof(double), hipMemcpyDeviceToHost));
        char buf[160];
        std::snprintf(buf, sizeof buf, "invalid densities at fluid site %lld: rho1=%g rho2=%g (need >= 0, sum > 0)",
                      (long long)res[1], a, b);
        return fail(c, LBM_EINVAL, buf);
    }
    if (res[2] < N) return fail(c, LBM_EINVAL, "non-finite initial velocity");
    if (res[0] == 0) return fail(c, LBM_EINVAL, "the lattice has no fluid site");
    c->nfluid = (int64_t)res[0];
    return LBM_OK;
}

// Sets the state from the staged fields: their equilibrium, plus (strain,
// with u_F) the non-equilibrium part that the velocity field's strain
// implies and the force shift; then records the masses.
int staged_to_state(lbm_ctx *c, bool has_u, bool strain) {
    // Warm start from u_F: the strain's flux Pi / rho (6N) and each
    // component's force per unit density (6N) in one work buffer, kept for
    // later restarts.
    double *pi = nullptr, *acc = nullptr;
    hipError_t e = hipSuccess;
    if (strain && has_u) {
        if (!c->warm && hipMalloc(&c->warm, 12 * sizeof(double) * (size_t)c->N) != hipSuccess) {
            c->warm = nullptr;
            (void)hipGetLastError();
            return fail(c, LBM_ENOMEM, "cannot allocate the 12N-double warm-start buffer");
        }
        pi = c->warm;
        acc = c->warm + 6 * c->N;
        const double wall0 = c->p.rho_s < 0 ? -c->p.rho_s : 0.0, wall1 = c->p.rho_s > 0 ? c->p.rho_s : 0.0;
        e = lbm::launch_strain(c->links, c->stage, c->stage + c->N, c->stage + 2 * c->N, c->p.tau[0], c->p.tau[1],
                               c->p.nx, c->p.ny, c->p.nz, pi, c->stream);
        if (e == hipSuccess)
            e = lbm::launch_accel(c->links, c->stage, c->stage + c->N, c->p.G, wall0, wall1, c->p.wall_kind, c->p.g,
                                  c->p.nx, c->p.ny, c->p.nz, acc, c->stream);
    }
    if (e == hipSuccess)
        e = lbm::launch_init_fields(c->p.prec, c->f[c->cur], c->links, c->idx, c->stage, c->stage + c->N,
                                    has_u ? c->stage + 2 * c->N : nullptr, pi, acc, c->p.nx, c->p.ny, c->p.nz,
                                    c->ngroups, c->p.eq_kind, c->ref, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, std::string("init_fields: ") + hipGetErrorString(e));
    c->snap_valid = false;
    int rc = measure(c, nullptr, nullptr, nullptr);
    if (rc) return rc;
    c->mass0[0] = c->red_host[0];
    c->mass0[1] = c->red_host[1];
    return LBM_OK;
}

// Loads fields into the state.  The first load (lbm_init) checks them on
// the host, where it also forms the 16-bit shift references from the mean
// densities; a restart stages them as they are (device inputs device to
// device) and checks them on the device.
int load_fields(lbm_ctx *c, const double *r0, const double *r1, const double *u, int on_device, bool strain = false) {
    const size_t NB = sizeof(double) * (size_t)c->N;
    int rc = ensure_stage(c);
    if (rc) return rc;
    if (c->ref_set) {
        // device inputs may come from work on other streams
        if (on_device) HIPCHK(c, hipDeviceSynchronize());
        const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        HIPCHK(c, hipMemcpyAsync(c->stage, r0, NB, kind, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->stage + c->N, r1, NB, kind, c->stream));
        if (u) HIPCHK(c, hipMemcpyAsync(c->stage + 2 * c->N, u, 3 * NB, kind, c->stream));
        rc = check_staged_fields(c, u != nullptr);
        if (rc) return rc;
        return staged_to_state(c, u != nullptr, strain);
    }
    std::vector<double> h0, h1, hu;
    std::vector<uint8_t> hs;
    const double *vr0 = r0, *vr1 = r1, *vu = u;
    if (on_device) {
        h0.resize(c->N); h1.resize(c->N);
        HIPCHK(c, hipMemcpy(h0.data(), r0, NB, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(h1.data(), r1, NB, hipMemcpyDeviceToHost));
        vr0 = h0.data(); vr1 = h1.data();
        if (u) {
            hu.resize(3 * c->N);
            HIPCHK(c, hipMemcpy(hu.data(), u, 3 * NB, hipMemcpyDeviceToHost));
            vu = hu.data();
        }
    }
    // solid mask back from the links (bit 0)
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<uint32_t> lk(c->N);
    HIPCHK(c, hipMemcpy(lk.data(), c->links, sizeof(uint32_t) * c->N, hipMemcpyDeviceToHost));
    hs.resize(c->N);
    for (int64_t s = 0; s < c->N; ++s) hs[s] = (uint8_t)(lk[s] & 1u);
    int64_t nf = 0;
    rc = validate_fields(c, hs.data(), vr0, vr1, vu, &nf);
    if (rc) return rc;
    c->nfluid = nf;
    // 16-bit storage: shift by w_i * rho_ref[a]; default = the mean initial density of the
    // component over fluid sites (the deviations stay small where a component is in its usual phase).
    const bool shifted = c->p.prec == LBM_FP16S || c->p.prec == LBM_BF16S;
    for (int a = 0; a < 2; ++a) {
        const double *r = a == 0 ? vr0 : vr1;
        double mean = 0.0;
        for (int64_t s = 0; s < c->N; ++s)
            if (!hs[s]) mean += r[s];
        mean /= (double)nf;
        const double want = c->p.rho_ref[a];
        c->ref[a] = !shifted ? 0.0 : (want > 0 ? want : (want < 0 ? 0.0 : mean));
    }
    c->ref_set = true;
    HIPCHK(c, hipMemcpyAsync(c->stage, vr0, NB, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->stage + c->N, vr1, NB, hipMemcpyHostToDevice, c->stream));
    if (vu) HIPCHK(c, hipMemcpyAsync(c->stage + 2 * c->N, vu, 3 * NB, hipMemcpyHostToDevice, c->stream));
    return staged_to_state(c, vu != nullptr, strain);
}

// Order of the positions (ly tx + lx) of a tile plane in storage: its two
// leftmost and two rightmost columns first, each top to bottom, then the
// rows without them.  A neighbouring tile's ring pulls read the column next
// to the edge (for the directions pointing into this tile) as well as the
// edge column itself, so both are contiguous (row by row they would be one
// site per row).
void tile_order(int tx, int ty, std::vector<int> &order) {
    order.clear();
    std::vector<int> cols;
    for (int c : {0, 1, tx - 2, tx - 1})
        if (c >= 0 && c < tx && std::find(cols.begin(), cols.end(), c) == cols.end()) cols.push_back(c);
    for (int c : cols)
        for (int ly = 0; ly < ty; ++ly) order.push_back(ly * tx + c);
    for (int ly = 0; ly < ty; ++ly)
        for (int lx = 0; lx < tx; ++lx)
            if (std::find(cols.begin(), cols.end(), lx) == cols.end()) order.push_back(ly * tx + lx);
}

// Slots of the fluid sites: z plane by plane, and within a plane tile by
// tile (the step's x-y tiles) in tile_order, so that the sites one block
// updates in a plane are contiguous.  Each tile plane's run starts on a
// multiple of align slots (a slot group): no group, hence no memory line, is
// written by two blocks.  Returns the slots used (fluid sites plus the
// unused slots between runs).
int64_t build_index(const uint8_t *solid, int nx, int ny, int nz, int tx, int ty, int align, std::vector<int32_t> &idx) {
    const int64_t N = (int64_t)nx * ny * nz;
    idx.assign((size_t)N, -1);
    int64_t k = 0;
    const int ntx = (nx + tx - 1) / tx, nty = (ny + ty - 1) / ty;
    std::vector<int> order;
    tile_order(tx, ty, order);
    auto segment = [&](int bx, int by, int z) {
        for (int q : order) {
            const int x = bx * tx + q % tx, y = by * ty + q / tx;
            if (x >= nx || y >= ny) continue;
            const int64_t s = x + (int64_t)nx * (y + (int64_t)ny * z);
            if (!solid || !solid[s]) idx[(size_t)s] = (int32_t)k++;
        }
        k = (k + align - 1) / align * align;   // the next segment starts a slot group
    };
    // Plane by plane: the blocks of one z-chunk march through neighbouring
    // memory at any one time (2-4 % faster than column by column).
    for (int z = 0; z < nz; ++z)
        for (int by = 0; by < nty; ++by)
            for (int bx = 0; bx < ntx; ++bx) segment(bx, by, z);
    return k;
}

// Work lists of the step: per tile column and z plane, the tile positions
// (ly tx + lx) of the plane's fluid sites in storage order.  In tiles that
// reach past the lattice edge, the positions beyond it stand for their
// periodic images (pulled for their densities, not stored).
void build_work(const uint8_t *solid, int nx, int ny, int nz, int tx, int ty, std::vector<int32_t> &wstart,
                std::vector<uint16_t> &wpos) {
    const int ntx = (nx + tx - 1) / tx, nty = (ny + ty - 1) / ty;
    std::vector<int> order;
    tile_order(tx, ty, order);
    wstart.assign((size_t)ntx * nty * (nz + 1), 0);
    wpos.clear();
    for (int by = 0; by < nty; ++by)
        for (int bx = 0; bx < ntx; ++bx) {
            const size_t col = (size_t)(by * ntx + bx) * (nz + 1);
            for (int z = 0; z < nz; ++z) {
                wstart[col + z] = (int32_t)wpos.size();
                for (int q : order) {
                    const int lx = q % tx, ly = q / tx;
                    const int x = (bx * tx + lx) % nx, y = (by * ty + ly) % ny;
                    const int64_t s = x + (int64_t)nx * (y + (int64_t)ny * z);
                    if (!solid || !solid[s]) wpos.push_back((uint16_t)q);
                }
            }
            wstart[col + nz] = (int32_t)wpos.size();
        }
}

void release(lbm_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (void *q : {c->f[0], c->f[1], (void *)c->links, (void *)c->idx, (void *)c->itab, (void *)c->wstart, (void *)c->btab, (void *)c->wpos,
                    (void *)c->partials, (void *)c->red_dev, (void *)c->stage, (void *)c->warm, (void *)c->snap})
        if (q) (void)hipFree(q);
    if (c->red_host) (void)hipHostFree(c->red_host);
    for (int k = 0; k < 2; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    }
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // namespace

extern "C" {

int lbm_init(const lbm_params *pin, lbm_ctx **out) {
    if (!out) return fail(nullptr, LBM_EINVAL, "lbm_init: out is NULL");
    *out = nullptr;
    if (!pin) return fail(nullptr, LBM_EINVAL, "lbm_init: params is NULL");
    const lbm_params &p = *pin;
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return fail(nullptr, LBM_EINVAL, "lattice dimensions must be >= 1");
    const size_t esz = storage_bytes(p.prec);
    if (!esz) return fail(nullptr, LBM_EINVAL, "unknown precision");
    for (int k = 0; k < 2; ++k)
        if (!(p.tau[k] > 0.5) || !std::isfinite(p.tau[k]))
            return fail(nullptr, LBM_EINVAL, "tau must be finite and > 1/2 (nu > 0)");
    if (!std::isfinite(p.G) || !std::isfinite(p.g[0]) || !std::isfinite(p.g[1]) || !std::isfinite(p.g[2]) ||
        !std::isfinite(p.rho_s))
        return fail(nullptr, LBM_EINVAL, "G, g and rho_s must be finite");
    if (p.eq_kind != 0 && p.eq_kind != 1) return fail(nullptr, LBM_EINVAL, "eq_kind must be 0 or 1");
    if (p.force_kind != 0 && p.force_kind != 1) return fail(nullptr, LBM_EINVAL, "force_kind must be 0 or 1");
    if (p.wall_kind != 0 && p.wall_kind != 1) return fail(nullptr, LBM_EINVAL, "wall_kind must be 0 or 1");
    if (p.check_every < 0) return fail(nullptr, LBM_EINVAL, "check_every must be >= 0");
    if (!(p.mass_tol >= 0) || !std::isfinite(p.rho_ref[0]) || !std::isfinite(p.rho_ref[1]))
        return fail(nullptr, LBM_EINVAL, "mass_tol must be >= 0 and rho_ref finite");
    if (!(p.tau_crit >= 0) || !std::isfinite(p.tau_crit))
        return fail(nullptr, LBM_EINVAL, "tau_crit must be finite and >= 0");
    if (!p.rho_init[0] || !p.rho_init[1]) return fail(nullptr, LBM_EINVAL, "rho_init pointers are NULL");
    if ((p.tile_x || p.tile_y) && !lbm::tile_supported(p.tile_x, p.tile_y))
        return fail(nullptr, LBM_EINVAL, "unsupported tile (64x4, 32x8, 16x16, 8x32, 64x8, 32x16 or 64x16)");

    // The FP64 step with 512-thread blocks gives results that differ from
    // run to run; it is refused until that is understood.
    if (p.prec == LBM_FP64 && p.tile_x * p.tile_y > 256)
        return fail(nullptr, LBM_EINVAL, "fp64 takes the 256-thread tiles only (64x4, 32x8, 16x16, 8x32)");
    if (p.zchunk < 0) return fail(nullptr, LBM_EINVAL, "zchunk must be >= 0");

    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_ENOMEM, "cannot allocate the context");
    c->p = p;
    c->p.solid = nullptr;
    c->p.rho_init[0] = c->p.rho_init[1] = nullptr;
    c->p.u_init = nullptr;
    if (c->p.mass_tol == 0) c->p.mass_tol = default_mass_tol(p.prec);
    c->N = (int64_t)p.nx * p.ny * p.nz;
    c->esz = esz;
    // Site indices are 32-bit (and the index map is read through a buffer
    // resource of 4 N bytes).
    if (c->N >= (int64_t)1 << 30) {
        int rc = fail(nullptr, LBM_EINVAL, "lattice too large: at most 2^30 sites");
        delete c;
        return rc;
    }

    auto bail = [&](int rc) {
        g_init_error = c->err;
        release(c);
        return rc;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(c, LBM_EDEVICE, "no HIP device"));
    {   // the allocation-free reduction's work memory on this device
        const hipError_t e = scratch_setup(c->device);
        if (e != hipSuccess)
            return bail(fail(c, LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)));
    }
    if (p.stream) c->stream = static_cast<hipStream_t>(p.stream);
    else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(c, LBM_EDEVICE, "hipStreamCreate failed"));
        c->own_stream = true;
    }

    // Solid mask on the host, the compact index of the fluid sites.
    std::vector<uint8_t> solid_h;
    if (p.solid) {
        solid_h.resize((size_t)c->N);
        if (!p.inputs_on_device) std::memcpy(solid_h.data(), p.solid, (size_t)c->N);
        else if (hipMemcpy(solid_h.data(), p.solid, c->N, hipMemcpyDeviceToHost) != hipSuccess)
            return bail(fail(c, LBM_EDEVICE, "cannot read the solid mask"));
    }
    {
        int64_t nsolid = 0;
        for (uint8_t v : solid_h) nsolid += v != 0;
        choose_launch(c, 1.0 - (double)nsolid / (double)c->N);
    }
    std::vector<int32_t> idx_h;
    const int64_t nfl = build_index(p.solid ? solid_h.data() : nullptr, p.nx, p.ny, p.nz, c->tile_x, c->tile_y,
                                    lbm::kGroup, idx_h);
    if (nfl == 0) return bail(fail(c, LBM_EINVAL, "the lattice has no fluid site"));
    // Groups of slots per buffer half, with 13 spare groups so that the two
    // halves do not start at offsets equal modulo large powers of two.
    c->ngroups = (nfl + lbm::kGroup - 1) / lbm::kGroup + 13;
    const uint64_t half_bytes = (uint64_t)c->ngroups * lbm::kHalfDirs * lbm::kGroup * 2 * esz;
    // The step addresses a buffer half with 32-bit byte offsets.
    if (half_bytes >= (1ull << 32))
        return bail(fail(c, LBM_EINVAL, "lattice too large: a half of the population storage must stay below 4 GiB"));

    const size_t fbytes = (size_t)(2 * half_bytes);
    for (int k = 0; k < 2; ++k) {
        if (hipMalloc(&c->f[k], fbytes) != hipSuccess) {
            c->f[k] = nullptr;
            return bail(fail(c, LBM_ENOMEM, "cannot allocate the population buffers"));
        }
        if (hipMemsetAsync(c->f[k], 0, fbytes, c->stream) != hipSuccess)
            return bail(fail(c, LBM_EDEVICE, "hipMemset failed"));
    }
    if (hipMalloc(&c->links, sizeof(uint32_t) * c->N) != hipSuccess ||
        hipMalloc(&c->idx, sizeof(int32_t) * c->N) != hipSuccess ||
        hipMalloc(&c->red_dev, sizeof(double) * lbm::kPartialStride) != hipSuccess ||
        hipHostMalloc(&c->red_host, sizeof(double) * lbm::kPartialStride, hipHostMallocDefault) != hipSuccess)
        return bail(fail(c, LBM_ENOMEM, "cannot allocate the link mask, index or reduction buffers"));
    if (hipMemcpy(c->idx, idx_h.data(), sizeof(int32_t) * c->N, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(c, LBM_EDEVICE, "cannot upload the site index"));
    if (p.prec != LBM_FP64) {
        // The 32/16-bit step reads a tile column's index tiles with 32-bit
        // offsets (the FP64 step gathers from the lattice index instead).
        const int64_t per = (int64_t)(c->tile_x + 4) * (c->tile_y + 4);
        if ((uint64_t)p.nz * (uint64_t)per * 4u >= (1ull << 32))
            return bail(fail(c, LBM_EINVAL, "lattice too long in z for the step's index tiles"));
        const size_t ib = sizeof(int32_t) * (size_t)c->ntx * c->nty * p.nz * per;
        if (hipMalloc(&c->itab, ib) != hipSuccess) {
            c->itab = nullptr;
            return bail(fail(c, LBM_ENOMEM, "cannot allocate the index tiles"));
        }
        hipError_t e = lbm::launch_index_tiles(c->idx, c->itab, p.nx, p.ny, p.nz, c->tile_x, c->tile_y,
                                               (int)(2 * esz), c->stream);
        if (e != hipSuccess) return bail(fail(c, LBM_EDEVICE, std::string("index tiles: ") + hipGetErrorString(e)));
    }
    {
        std::vector<int32_t> ws;
        std::vector<uint16_t> wp;
        build_work(p.solid ? solid_h.data() : nullptr, p.nx, p.ny, p.nz, c->tile_x, c->tile_y, ws, wp);
        if (hipMalloc(&c->wstart, sizeof(int32_t) * ws.size()) != hipSuccess ||
            hipMalloc(&c->wpos, sizeof(uint16_t) * std::max<size_t>(wp.size(), 1)) != hipSuccess)
            return bail(fail(c, LBM_ENOMEM, "cannot allocate the work lists"));
        if (hipMemcpy(c->wstart, ws.data(), sizeof(int32_t) * ws.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->wpos, wp.data(), sizeof(uint16_t) * wp.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(c, LBM_EDEVICE, "cannot upload the work lists"));
        if (p.zchunk == 0) {   // default z-chunks: balanced work items
            const int64_t resident =
                (int64_t)std::max(lbm::step_blocks_per_cu(p.prec, c->tile_x, c->tile_y), 1) * device_cus();
            std::vector<int32_t> items = balance_items(ws, c->ntx, c->nty, p.nz, c->tile_x, c->tile_y, resident);
            c->nblk = (int)(items.size() / 4);
            if (hipMalloc(&c->btab, sizeof(int32_t) * items.size()) != hipSuccess)
                return bail(fail(c, LBM_ENOMEM, "cannot allocate the work items"));
            if (hipMemcpy(c->btab, items.data(), sizeof(int32_t) * items.size(), hipMemcpyHostToDevice) != hipSuccess)
                return bail(fail(c, LBM_EDEVICE, "cannot upload the work items"));
        }
    }
    // Partial sums of the checks: one slot per block of the step, or of a
    // batch (uniform chunks), whichever is more.
    if (hipMalloc(&c->partials, sizeof(double) * lbm::kPartialStride *
                                    std::max<int64_t>(nblocks(c), (int64_t)c->ntx * c->nty * c->nzc)) != hipSuccess)
        return bail(fail(c, LBM_ENOMEM, "cannot allocate the reduction buffers"));

    // Solid mask -> link mask.
    uint8_t *solid_d = nullptr;
    if (p.solid) {
        if (hipMalloc(&solid_d, c->N) != hipSuccess) return bail(fail(c, LBM_ENOMEM, "cannot stage the solid mask"));
        hipError_t e = hipMemcpyAsync(solid_d, solid_h.data(), c->N, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = lbm::launch_links(solid_d, c->links, p.nx, p.ny, p.nz, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        (void)hipFree(solid_d);
        if (e != hipSuccess) return bail(fail(c, LBM_EDEVICE, std::string("link mask: ") + hipGetErrorString(e)));
    } else {
        hipError_t e = lbm::launch_links(nullptr, c->links, p.nx, p.ny, p.nz, c->stream);
        if (e != hipSuccess) return bail(fail(c, LBM_EDEVICE, std::string("link mask: ") + hipGetErrorString(e)));
    }
    int rc = load_fields(c, p.rho_init[0], p.rho_init[1], p.u_init, p.inputs_on_device);
    if (rc) return bail(rc);
    *out = c;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Checks the FP64 sums of a MODE_CHECK step (already finalized into
// c->red_dev and copied to c->red_host, stream synchronized).
int evaluate_check(lbm_ctx *c) {
    const double *r = c->red_host;
    char buf[200];
    if (r[5] != 0.0 || !std::isfinite(r[0]) || !std::isfinite(r[1])) {
        std::snprintf(buf, sizeof buf, "non-finite state at step %lld (%g sites)", (long long)c->steps_done - 1, r[5]);
        return fail(c, LBM_ENONFINITE, buf);
    }
    for (int a = 0; a < 2; ++a) {
        const double ref = c->mass0[a];
        const double drift = std::fabs(r[a] - ref) / (ref > 0 ? ref : 1.0);
        if (drift > c->p.mass_tol) {
            std::snprintf(buf, sizeof buf, "component %d mass drift %.3e > %.3e at step %lld", a + 1, drift,
                          c->p.mass_tol, (long long)c->steps_done - 1);
            return fail(c, LBM_EMASSDRIFT, buf);
        }
    }
    return LBM_OK;
}

int64_t plain_steps_before_check(int64_t done, int every) {
    if (every <= 0) return INT64_MAX;
    return every - 1 - done % every;
}

// Discards the captured step graphs (they are captured again on next use).
void drop_ctx_graphs(lbm_ctx *c) {
    for (int k = 0; k < 2; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
        c->gexec[k] = nullptr;
        c->graph[k] = nullptr;
    }
}

// Captures kGraphSteps plain steps starting from buffer `parity`.
bool capture_ctx_graph(lbm_ctx *c, int parity) {
    if (c->graphs_off) return false;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        c->graphs_off = true;
        return false;
    }
    hipError_t e = hipSuccess;
    int cur = parity;
    for (int j = 0; j < kGraphSteps && e == hipSuccess; ++j) {
        lbm::StepLaunch L = make_launch(c, c->f[cur], c->f[1 - cur]);
        e = lbm::launch_step(c->p.prec, lbm::MODE_STEP, L, c->stream);
        cur = 1 - cur;
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g ||
        hipGraphInstantiate(&c->gexec[parity], g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        c->gexec[parity] = nullptr;
        c->graphs_off = true;
        return false;
    }
    c->graph[parity] = g;
    return true;
}

}  // namespace

extern "C" {

int lbm_step(lbm_ctx *c, int64_t n) {
    if (!c) return fail(nullptr, LBM_EINVAL, "lbm_step: NULL context");
    if (n < 0) return fail(c, LBM_EINVAL, "lbm_step: n < 0");
    HIPCHK(c, hipSetDevice(c->device));
    int64_t k = 0;
    while (k < n) {
        int64_t plain = std::min(n - k, plain_steps_before_check(c->steps_done, c->p.check_every));
        // runs of plain steps: replay the captured graph where it fits
        while (plain >= kGraphSteps && (c->gexec[c->cur] || capture_ctx_graph(c, c->cur))) {
            HIPCHK(c, hipGraphLaunch(c->gexec[c->cur], c->stream));
            c->steps_done += kGraphSteps;
            k += kGraphSteps;
            plain -= kGraphSteps;
        }
        for (; plain > 0; --plain, ++k) {
            lbm::StepLaunch L = make_launch(c, c->f[c->cur], c->f[1 - c->cur]);
            HIPCHK(c, lbm::launch_step(c->p.prec, lbm::MODE_STEP, L, c->stream));
            c->cur = 1 - c->cur;
            c->steps_done++;
        }
        if (k < n) {  // a check step
            lbm::StepLaunch L = make_launch(c, c->f[c->cur], c->f[1 - c->cur]);
            HIPCHK(c, lbm::launch_step(c->p.prec, lbm::MODE_CHECK, L, c->stream));
            c->cur = 1 - c->cur;
            c->steps_done++;
            k++;
            HIPCHK(c, lbm::launch_finalize(c->partials, nblocks(c), c->red_dev, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->red_host, c->red_dev, sizeof(double) * lbm::kPartialStride,
                                     hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            int rc = evaluate_check(c);
            if (rc) return rc;
        }
    }
    return LBM_OK;
}

int lbm_moments(lbm_ctx *c, double *rho1, double *rho2, double *uF, int on_device) {
    if (!c) return fail(nullptr, LBM_EINVAL, "lbm_moments: NULL context");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t NB = sizeof(double) * (size_t)c->N;
    if (on_device) {
        // solid sites are not written by the kernel: they report 0
        if (rho1) HIPCHK(c, hipMemsetAsync(rho1, 0, NB, c->stream));
        if (rho2) HIPCHK(c, hipMemsetAsync(rho2, 0, NB, c->stream));
        if (uF) HIPCHK(c, hipMemsetAsync(uF, 0, 3 * NB, c->stream));
        return measure(c, rho1, rho2, uF);
    }
    int rc = ensure_stage(c);
    if (rc) return rc;
    double *d0 = rho1 ? c->stage : nullptr, *d1 = rho2 ? c->stage + c->N : nullptr;
    double *du = uF ? c->stage + 2 * c->N : nullptr;
    if (d0) HIPCHK(c, hipMemsetAsync(d0, 0, NB, c->stream));
    if (d1) HIPCHK(c, hipMemsetAsync(d1, 0, NB, c->stream));
    if (du) HIPCHK(c, hipMemsetAsync(du, 0, 3 * NB, c->stream));
    rc = measure(c, d0, d1, du);
    if (rc) return rc;
    if (rho1) HIPCHK(c, hipMemcpy(rho1, d0, NB, hipMemcpyDeviceToHost));
    if (rho2) HIPCHK(c, hipMemcpy(rho2, d1, NB, hipMemcpyDeviceToHost));
    if (uF) HIPCHK(c, hipMemcpy(uF, du, 3 * NB, hipMemcpyDeviceToHost));
    return LBM_OK;
}

int lbm_reduce(lbm_ctx *c, double out[5]) {
    if (!c || !out) return fail(c, LBM_EINVAL, "lbm_reduce: NULL argument");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = measure(c, nullptr, nullptr, nullptr);
    if (rc) return rc;
    for (int k = 0; k < 5; ++k) out[k] = c->red_host[k];
    return LBM_OK;
}

int lbm_reduce_noalloc(lbm_ctx *c, double *out_dev) {
    if (!c || !out_dev) return fail(c, LBM_EINVAL, "lbm_reduce_noalloc: NULL argument");
    const int nb = nblocks(c);
    if (nb > kScratchBlocks) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "lbm_reduce_noalloc: the step runs %d blocks, more than the %d its work memory holds",
                      nb, kScratchBlocks);
        return fail(c, LBM_EINVAL, buf);
    }
    HIPCHK(c, hipSetDevice(c->device));
    double *ws = scratch_ptr(c->device);
    if (!ws) return fail(c, LBM_EDEVICE, "lbm_reduce_noalloc: work memory of this device not set up");
    double *total = ws + (size_t)kScratchBlocks * lbm::kPartialStride;
    // Every block writes its own partial sums and the total is overwritten
    // whole, so nothing needs clearing between calls.
    lbm::StepLaunch L = make_launch(c, c->f[c->cur], nullptr);
    L.partials = ws;
    HIPCHK(c, lbm::launch_step(c->p.prec, lbm::MODE_MOMENTS, L, c->stream));
    HIPCHK(c, lbm::launch_finalize(ws, nb, total, c->stream));
    HIPCHK(c, hipMemcpyAsync(out_dev, total, sizeof(double) * 5, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

int lbm_get_populations(lbm_ctx *c, double *f, int on_device) {
    if (!c || !f) return fail(c, LBM_EINVAL, "lbm_get_populations: NULL argument");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t bytes = sizeof(double) * 38 * (size_t)c->N;
    double *dst = f;
    if (!on_device && hipMalloc(&dst, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, LBM_ENOMEM, "cannot allocate the population staging buffer");
    }
    hipError_t e = lbm::launch_get_pops(c->p.prec, c->f[c->cur], c->links, c->idx, dst, c->p.nx, c->p.ny, c->p.nz, c->ngroups,
                                        c->ref, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && !on_device) e = hipMemcpy(f, dst, bytes, hipMemcpyDeviceToHost);
    if (!on_device) (void)hipFree(dst);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, std::string("get_populations: ") + hipGetErrorString(e));
    return LBM_OK;
}

int lbm_set_populations(lbm_ctx *c, const double *f, int on_device) {
    if (!c || !f) return fail(c, LBM_EINVAL, "lbm_set_populations: NULL argument");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t bytes = sizeof(double) * 38 * (size_t)c->N;
    double *src = const_cast<double *>(f);
    if (!on_device) {
        if (hipMalloc(&src, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, LBM_ENOMEM, "cannot allocate the population staging buffer");
        }
        if (hipMemcpy(src, f, bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(src);
            return fail(c, LBM_EDEVICE, "set_populations: copy failed");
        }
    }
    auto encode = [&]() {
        hipError_t e = lbm::launch_set_pops(c->p.prec, c->f[c->cur], c->links, c->idx, src, c->p.nx, c->p.ny, c->p.nz,
                                            c->ngroups, c->ref, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        return e;
    };
    hipError_t e = encode();
    int rc = LBM_OK;
    const bool shifted = c->p.prec == LBM_FP16S || c->p.prec == LBM_BF16S;
    if (e == hipSuccess && shifted && (c->p.rho_ref[0] == 0 || c->p.rho_ref[1] == 0)) {
        // A default shift reference is the mean density of the state the
        // context holds: recompute it for the resumed state (the context may
        // have been created from placeholder fields) and encode again.
        rc = measure(c, nullptr, nullptr, nullptr);
        if (rc == LBM_OK) {
            double ref[2] = {c->ref[0], c->ref[1]};
            for (int a = 0; a < 2; ++a)
                if (c->p.rho_ref[a] == 0) ref[a] = c->red_host[a] / (double)c->nfluid;
            if (ref[0] != c->ref[0] || ref[1] != c->ref[1]) {
                c->ref[0] = ref[0];
                c->ref[1] = ref[1];
                drop_ctx_graphs(c);   // the captured steps carry the old reference
                e = encode();
            }
        }
    }
    if (!on_device) (void)hipFree(src);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, std::string("set_populations: ") + hipGetErrorString(e));
    if (rc) return rc;
    c->snap_valid = false;
    // The periodic check compares against the masses of the resumed state.
    rc = measure(c, nullptr, nullptr, nullptr);
    if (rc) return rc;
    c->mass0[0] = c->red_host[0];
    c->mass0[1] = c->red_host[1];
    return LBM_OK;
}

int lbm_set_fields(lbm_ctx *c, const double *rho1, const double *rho2, const double *u, int on_device) {
    if (!c || !rho1 || !rho2) return fail(c, LBM_EINVAL, "lbm_set_fields: NULL argument");
    HIPCHK(c, hipSetDevice(c->device));
    return load_fields(c, rho1, rho2, u, on_device);
}

int lbm_set_fields_strain(lbm_ctx *c, const double *rho1, const double *rho2, const double *u, int on_device) {
    if (!c || !rho1 || !rho2 || !u) return fail(c, LBM_EINVAL, "lbm_set_fields_strain: NULL argument");
    HIPCHK(c, hipSetDevice(c->device));
    return load_fields(c, rho1, rho2, u, on_device, true);
}

namespace {

// Distance sums of the current state (rho1, u_F) against (ra_prev, u_prev)
// (device, N and 3N) into c->red_host; the current fields are left in the
// staging buffer (rho1 at [0, N), u_F at [2N, 5N)).
int distance_sums(lbm_ctx *c, const double *ra_prev, const double *u_prev) {
    const size_t NB = sizeof(double) * (size_t)c->N;
    double *ra = c->stage, *u = c->stage + 2 * c->N;
    HIPCHK(c, hipMemsetAsync(ra, 0, NB, c->stream));
    HIPCHK(c, hipMemsetAsync(u, 0, 3 * NB, c->stream));
    lbm::StepLaunch L = make_launch(c, c->f[c->cur], nullptr);
    L.out_rho0 = ra;
    L.out_u = u;
    HIPCHK(c, lbm::launch_step(c->p.prec, lbm::MODE_MOMENTS, L, c->stream));
    const int nb = std::min<int64_t>(nblocks(c), std::max<int64_t>(1, (c->N + 255) / 256));
    HIPCHK(c, lbm::launch_residual(ra, u, ra_prev, u_prev, c->N, nb, c->partials, c->stream));
    HIPCHK(c, lbm::launch_finalize(c->partials, nb, c->red_dev, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->red_host, c->red_dev, sizeof(double) * lbm::kPartialStride, hipMemcpyDeviceToHost,
                             c->stream));
    return LBM_OK;
}

double rel_norm(double diff2, double norm2) {
    if (norm2 > 0) return std::sqrt(diff2 / norm2);
    return diff2 > 0 ? HUGE_VAL : 0.0;
}

}  // namespace

int lbm_residual(lbm_ctx *c, double out[2]) {
    if (!c || !out) return fail(c, LBM_EINVAL, "lbm_residual: NULL argument");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = ensure_stage(c);
    if (rc) return rc;
    const size_t NB = sizeof(double) * (size_t)c->N;
    if (!c->snap) {
        if (hipMalloc(&c->snap, 4 * NB) != hipSuccess) {
            c->snap = nullptr;
            (void)hipGetLastError();
            return fail(c, LBM_ENOMEM, "cannot allocate the 4N-double residual snapshot");
        }
        c->snap_valid = false;
    }
    if (!c->snap_valid) HIPCHK(c, hipMemsetAsync(c->snap, 0, 4 * NB, c->stream));
    rc = distance_sums(c, c->snap, c->snap + c->N);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->snap, c->stage, NB, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->snap + c->N, c->stage + 2 * c->N, 3 * NB, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->snap_valid = true;
    const double *r = c->red_host;
    if (!std::isfinite(r[0] + r[1] + r[2] + r[3])) return fail(c, LBM_ENONFINITE, "lbm_residual: non-finite fields");
    out[0] = rel_norm(r[2], r[3]);
    out[1] = rel_norm(r[0], r[1]);
    return LBM_OK;
}

int lbm_distance(lbm_ctx *c, const double *rho1, const double *u, int on_device, double out[2]) {
    if (!c || !rho1 || !u || !out) return fail(c, LBM_EINVAL, "lbm_distance: NULL argument");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = ensure_stage(c);
    if (rc) return rc;
    const size_t NB = sizeof(double) * (size_t)c->N;
    double *tmp = nullptr;
    const double *ra_ref = rho1, *u_ref = u;
    if (!on_device) {
        if (hipMalloc(&tmp, 4 * NB) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, LBM_ENOMEM, "lbm_distance: cannot allocate the 4N-double staging buffer");
        }
        if (hipMemcpyAsync(tmp, rho1, NB, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(tmp + c->N, u, 3 * NB, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
            (void)hipStreamSynchronize(c->stream);
            (void)hipFree(tmp);
            return fail(c, LBM_EDEVICE, "lbm_distance: copy failed");
        }
        ra_ref = tmp;
        u_ref = tmp + c->N;
    }
    rc = distance_sums(c, ra_ref, u_ref);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (tmp) (void)hipFree(tmp);
    if (rc) return rc;
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, std::string("lbm_distance: ") + hipGetErrorString(e));
    const double *r = c->red_host;
    if (!std::isfinite(r[0] + r[2] + r[4] + r[5])) return fail(c, LBM_ENONFINITE, "lbm_distance: non-finite fields");
    out[0] = rel_norm(r[2], r[5]);
    out[1] = rel_norm(r[0], r[4]);
    return LBM_OK;
}

int lbm_info(const lbm_ctx *c, lbm_info_t *out) {
    if (!c || !out) return LBM_EINVAL;
    out->n_sites = c->N;
    out->n_fluid = c->nfluid;
    out->steps_done = c->steps_done;
    out->bytes_per_lu = (int32_t)(2 * 2 * 19 * c->esz);
    out->tile_x = c->tile_x;
    out->tile_y = c->tile_y;
    out->zchunk = c->btab ? 0 : c->zchunk;   // 0: balanced work items of varying depth
    out->blocks = nblocks(c);
    out->mass0[0] = c->mass0[0];
    out->mass0[1] = c->mass0[1];
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : g_init_error.c_str(); }

void lbm_free(lbm_ctx *c) { release(c); }

// ---------------------------------------------------------------------------
// Batches of contexts stepped by one launch per step.
// ---------------------------------------------------------------------------

int lbm_batch_create(lbm_ctx *const *ctxs, int32_t n, lbm_batch **out) {
    if (!out) return bfail(nullptr, LBM_EINVAL, "lbm_batch_create: out is NULL");
    *out = nullptr;
    if (!ctxs || n < 1) return bfail(nullptr, LBM_EINVAL, "lbm_batch_create: no contexts");
    for (int d = 0; d < n; ++d) {
        if (!ctxs[d]) return bfail(nullptr, LBM_EINVAL, "lbm_batch_create: NULL context");
        if (ctxs[d]->p.prec != ctxs[0]->p.prec || ctxs[d]->tile_x != ctxs[0]->tile_x ||
            ctxs[d]->tile_y != ctxs[0]->tile_y || ctxs[d]->device != ctxs[0]->device)
            return bfail(nullptr, LBM_EINVAL, "lbm_batch_create: contexts differ in precision, tile or device");
        for (int e = 0; e < d; ++e)
            if (ctxs[e] == ctxs[d]) return bfail(nullptr, LBM_EINVAL, "lbm_batch_create: a context appears twice");
    }
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(nullptr, LBM_ENOMEM, "cannot allocate the batch");
    b->ctx.assign(ctxs, ctxs + n);
    b->prec = ctxs[0]->p.prec;
    b->tile_x = ctxs[0]->tile_x;
    b->tile_y = ctxs[0]->tile_y;
    for (int d = 0; d < n; ++d) b->hi = b->hi || ctxs[d]->p.tau_crit > 0;
    b->desc_size = lbm::batch_desc_size(b->prec);
    b->descs_host.resize(b->desc_size * n);
    // Z-chunks of the batch.  A context's own z-chunk fills the GPU with
    // that one domain; a batch that fills it several times over runs
    // deeper chunks (at least 16 planes: fewer boundary planes re-pulled),
    // never more blocks per domain than the context's own, so each keeps
    // its partial-sum slots.
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctxs[0]->device) != hipSuccess || cus <= 0)
            cus = 256;
        const int64_t resident =
            (int64_t)std::max(lbm::step_blocks_per_cu(b->prec, b->tile_x, b->tile_y), 1) * cus;
        b->zchunk.resize(n);
        b->nzc.resize(n);
        int64_t deep = 0;
        for (int d = 0; d < n; ++d) {
            const lbm_ctx *c = ctxs[d];
            b->zchunk[d] = std::max(c->zchunk, std::min(16, c->p.nz));
            b->nzc[d] = (c->p.nz + b->zchunk[d] - 1) / b->zchunk[d];
            deep += (int64_t)c->ntx * c->nty * b->nzc[d];
        }
        if (deep < resident)
            for (int d = 0; d < n; ++d) {
                b->zchunk[d] = ctxs[d]->zchunk;
                b->nzc[d] = ctxs[d]->nzc;
            }
    }
    auto bblocks = [&](int d) { return ctxs[d]->ntx * ctxs[d]->nty * b->nzc[d]; };
    // Work list: every tile of every domain, domain by domain, the largest
    // domains first so that their long columns of work start early.
    std::vector<int> order(n);
    for (int d = 0; d < n; ++d) order[d] = d;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return bblocks(x) > bblocks(y); });
    std::vector<int2> work;
    for (int d : order)
        for (int k = 0; k < bblocks(d); ++k) work.push_back(make_int2(d, k));
    b->nwork = (int)work.size();
    auto bail = [&](int rc) {
        g_init_error = b->err;
        lbm_batch_free(b);
        return rc;
    };
    if (hipSetDevice(ctxs[0]->device) != hipSuccess ||
        hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(bfail(b, LBM_EDEVICE, "cannot create the batch stream"));
    if (hipMalloc(&b->descs_dev, b->descs_host.size()) != hipSuccess ||
        hipMalloc(&b->work_dev, sizeof(int2) * work.size()) != hipSuccess)
        return bail(bfail(b, LBM_ENOMEM, "cannot allocate the batch tables"));
    if (hipMemcpy(b->work_dev, work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice) != hipSuccess)
        return bail(bfail(b, LBM_EDEVICE, "cannot upload the work list"));
    *out = b;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Descriptors from each context's current buffers (an even step reads f[cur]).
int upload_descs(lbm_batch *b) {
    for (size_t d = 0; d < b->ctx.size(); ++d) {
        lbm_ctx *c = b->ctx[d];
        lbm::StepLaunch L = make_launch(c, c->f[c->cur], c->f[1 - c->cur]);
        L.zchunk = b->zchunk[d];   // a batch cuts every domain into uniform chunks
        L.nzc = b->nzc[d];
        L.btab = nullptr;
        lbm::fill_batch_desc(b->prec, L, b->descs_host.data() + d * b->desc_size);
    }
    if (hipMemcpyAsync(b->descs_dev, b->descs_host.data(), b->descs_host.size(), hipMemcpyHostToDevice, b->stream) !=
        hipSuccess)
        return bfail(b, LBM_EDEVICE, "cannot upload the batch descriptors");
    return LBM_OK;
}

bool capture_batch_graph(lbm_batch *b) {
    if (b->graphs_off) return false;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        b->graphs_off = true;
        return false;
    }
    hipError_t e = hipSuccess;
    for (int j = 0; j < kGraphSteps && e == hipSuccess; ++j)
        e = lbm::launch_batch(b->prec, lbm::MODE_STEP, b->hi, b->tile_x, b->tile_y, b->descs_dev, b->work_dev, b->nwork,
                              j & 1, b->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g || hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        b->gexec = nullptr;
        b->graphs_off = true;
        return false;
    }
    b->graph = g;
    return true;
}

}  // namespace

extern "C" {

int lbm_batch_step(lbm_batch *b, int64_t n) {
    if (!b) return bfail(nullptr, LBM_EINVAL, "lbm_batch_step: NULL batch");
    if (n < 0) return bfail(b, LBM_EINVAL, "lbm_batch_step: n < 0");
    if (hipSetDevice(b->ctx[0]->device) != hipSuccess) return bfail(b, LBM_EDEVICE, "hipSetDevice failed");
    for (lbm_ctx *c : b->ctx)
        if (hipStreamSynchronize(c->stream) != hipSuccess) return bfail(b, LBM_EDEVICE, "context stream failed");
    int rc = upload_descs(b);
    if (rc) return rc;
    int flip = 0;   // parity of the steps done since the descriptors were built
    auto advance = [&](int64_t m) {
        for (lbm_ctx *c : b->ctx) {
            c->steps_done += m;
            if (m & 1) c->cur = 1 - c->cur;
        }
    };
    int64_t k = 0;
    while (k < n) {
        int64_t plain = n - k;
        for (lbm_ctx *c : b->ctx) plain = std::min(plain, plain_steps_before_check(c->steps_done, c->p.check_every));
        if (plain >= kGraphSteps + flip) {
            if (flip) {  // align to an even step before replaying
                if (lbm::launch_batch(b->prec, lbm::MODE_STEP, b->hi, b->tile_x, b->tile_y, b->descs_dev, b->work_dev,
                                      b->nwork, 1, b->stream) != hipSuccess)
                    return bfail(b, LBM_EDEVICE, "batch launch failed");
                advance(1);
                flip = 0;
                ++k;
                --plain;
            }
            while (plain >= kGraphSteps && (b->gexec || capture_batch_graph(b))) {
                if (hipGraphLaunch(b->gexec, b->stream) != hipSuccess) return bfail(b, LBM_EDEVICE, "graph launch failed");
                advance(kGraphSteps);
                k += kGraphSteps;
                plain -= kGraphSteps;
            }
        }
        for (; plain > 0; --plain, ++k) {
            if (lbm::launch_batch(b->prec, lbm::MODE_STEP, b->hi, b->tile_x, b->tile_y, b->descs_dev, b->work_dev, b->nwork,
                                  flip, b->stream) != hipSuccess)
                return bfail(b, LBM_EDEVICE, "batch launch failed");
            advance(1);
            flip ^= 1;
        }
        if (k < n) {  // a check step for at least one domain
            if (lbm::launch_batch(b->prec, lbm::MODE_CHECK, b->hi, b->tile_x, b->tile_y, b->descs_dev, b->work_dev, b->nwork,
                                  flip, b->stream) != hipSuccess)
                return bfail(b, LBM_EDEVICE, "batch launch failed");
            std::vector<lbm_ctx *> due;
            for (lbm_ctx *c : b->ctx)
                if (c->p.check_every > 0 && (c->steps_done + 1) % c->p.check_every == 0) due.push_back(c);
            advance(1);
            flip ^= 1;
            ++k;
            for (size_t d = 0; d < b->ctx.size(); ++d) {
                lbm_ctx *c = b->ctx[d];
                if (std::find(due.begin(), due.end(), c) == due.end()) continue;
                const int nb = c->ntx * c->nty * b->nzc[d];   // the batch's blocks of this domain
                if (lbm::launch_finalize(c->partials, nb, c->red_dev, b->stream) != hipSuccess ||
                    hipMemcpyAsync(c->red_host, c->red_dev, sizeof(double) * lbm::kPartialStride,
                                   hipMemcpyDeviceToHost, b->stream) != hipSuccess)
                    return bfail(b, LBM_EDEVICE, "batch check failed");
            }
            if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, LBM_EDEVICE, "batch stream failed");
            for (size_t d = 0; d < b->ctx.size(); ++d) {
                lbm_ctx *c = b->ctx[d];
                if (std::find(due.begin(), due.end(), c) == due.end()) continue;
                int r = evaluate_check(c);
                if (r) return bfail(b, r, "domain " + std::to_string(d) + ": " + c->err);
            }
        }
    }
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, LBM_EDEVICE, "batch stream failed");
    return LBM_OK;
}

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : g_init_error.c_str(); }

void lbm_batch_free(lbm_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->descs_dev) (void)hipFree(b->descs_dev);
    if (b->work_dev) (void)hipFree(b->work_dev);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"
