// lbm_kernels.hip -- gfx950 kernels of the two-component Shan-Chen D3Q19 step
// (Otomo et al., arXiv:1711.03254, Section 2, Eqs. 1-11).
//
// Storage: populations exist for fluid sites only.  Each fluid site has a
// compact index k (the host numbers them tile column by tile column, z
// plane by plane, so that a block's sites are contiguous); the plane of
// direction i holds, for every k, the pair (f^1_i, f^2_i) of the two
// components, which a pull reads from the same source site.  The
// buffer a step reads holds the post-collision populations f*(x, t-1) of
// the previous step; the step pulls f_i(x, t) = f*_i(x - c_i) (or, when
// x - c_i is solid, the reversed population f*_opp(i)(x): halfway
// bounce-back), collides and writes f*(x, t) at x into the other buffer.
//
// The Shan-Chen force at x needs the densities of the 18 neighbours at time
// t, which exist only after those neighbours have pulled.  A block owns an
// x-y tile of TX x TY columns and marches along z through a chunk of planes;
// for every plane it pulls the tile and its one-site ring, sums the
// densities into an LDS ring buffer of four planes, and collides the plane
// behind once the plane ahead is known.  The compact indices of the tile
// and a ring of two sites are staged in LDS too (six planes: the three a
// pull reads, the three the force's wall term of the plane behind may
// still read while the next tile is staged), so each pull finds its 18
// sources (or the wall) there.  The ring's pulls are the only
// redundant work; no density array goes to HBM.

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "lbm_internal.h"

namespace lbm {
namespace {

// ---------------------------------------------------------------------------
// D3Q19 in the ABI order (rest; +x -x +y -y +z -z; xy, xz, yz diagonals).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int cx_of(int i) {
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
           : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cy_of(int i) {
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
           : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int cz_of(int i) {
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
           : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr int opp_of(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double w_of(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Compile-time loop: f(integral_constant<int, 0>) ... f(integral_constant<int, N-1>).
template <int... Is, class F>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, Is...>, F &&f) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F &&f) {
    sfor_impl(std::make_integer_sequence<int, N>{}, f);
}

// ---------------------------------------------------------------------------
// Storage codecs.  16-bit formats hold the deviation f_i - w_i rho_ref[a].
// ---------------------------------------------------------------------------
// C is the arithmetic type; R the type a pulled population is held in until
// its moments are taken: FP16 values are widened as they arrive (fewer
// registers live across the pull than with the packed halves and their
// conversions), BF16 values when they are used (widening is a shift).
template <typename S> struct Codec;
template <> struct Codec<double> {
    using C = double;
    using R = double;
    static constexpr bool shifted = false;
    __device__ static double ld(double v) { return v; }
    __device__ static double st(double v) { return v; }
};
template <> struct Codec<float> {
    using C = float;
    using R = float;
    static constexpr bool shifted = false;
    __device__ static float ld(float v) { return v; }
    __device__ static float st(float v) { return v; }
};
template <> struct Codec<__half> {
    using C = float;
    using R = float;
    static constexpr bool shifted = true;
    __device__ static float ld(__half v) { return __half2float(v); }
    __device__ static __half st(float v) { return __float2half_rn(v); }
};
template <> struct Codec<__hip_bfloat16> {
    using C = float;
    using R = __hip_bfloat16;
    static constexpr bool shifted = true;
    __device__ static float ld(__hip_bfloat16 v) { return __bfloat162float(v); }
    __device__ static __hip_bfloat16 st(float v) { return __float2bfloat16(v); }
};

// A held population as the arithmetic type.
template <typename S>
__device__ __forceinline__ typename Codec<S>::C held(typename Codec<S>::R v) {
    if constexpr (std::is_same_v<typename Codec<S>::R, typename Codec<S>::C>) return v;
    else return Codec<S>::ld(v);
}

template <typename S>
struct KArgs {
    using C = typename Codec<S>::C;
    const S *src;
    S *dst;
    const int32_t *idx;     // compact index of each lattice site, -1 where solid (FP64 step)
    const int32_t *itab;    // index tiles of the step per tile column and plane (index_tiles_kernel)
    const int32_t *wstart;  // work list bounds per tile column and plane
    const uint16_t *wpos;   // work list entries: tile positions of the fluid sites
    int nx, ny, nz, ntx, nty, zchunk;
    const int32_t *btab;    // per block: tile x, tile y, first and end plane (null: uniform z-chunks)
    uint32_t half_bytes;    // bytes of one buffer half (directions 0-10 or 11-18)
    C tau0, tau1, G, gx, gy, gz, wall0, wall1, ref0, ref1;
    C tau_crit;             // sites with tau_mix below it form P_ab in FP64 (32/16-bit storage)
    int eq_kind, force_kind, wall_kind;
    double *partials;
    double *out_rho0, *out_rho1, *out_u;
    int64_t n_sites;
};

// Read-only tables of a launch, addressed as constant memory so that uniform
// reads of them go through the scalar unit.
typedef __attribute__((address_space(4))) const int32_t cint32;

__device__ __forceinline__ int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Raw buffer access.  A population pair (f^1_i, f^2_i) of the two
// components moves in one access.  Two buffer resources cover a buffer, one
// per half (directions 0-10 and 11-18, each opposite pair within one); the
// 32-bit lane offset selects the slot (group_off) and the scalar or
// immediate offset the direction (kGroup pairs per direction run).  Every
// access issued is in bounds (lanes without work are masked off), so the
// range check never applies.
constexpr int kRsrcWord3 = 0x00020000;   // gfx9 raw (unswizzled) buffer
constexpr int kNonTemporal = 2;          // cache policy of the population stores

// Byte offset of slot k within a buffer half, and the offset of direction i
// (its run within the group) for pairs of pb bytes.
__host__ __device__ constexpr uint32_t group_off(uint32_t k, uint32_t pb) {
    return ((k / kGroup) * (uint32_t)(kHalfDirs * kGroup) + k % kGroup) * pb;
}
__host__ __device__ constexpr uint32_t dir_off(int i, uint32_t pb) {
    return (uint32_t)(i < kSplit ? i : i - kSplit) * (uint32_t)kGroup * pb;
}
// Index tiles hold group_off of each site as a 32-bit pattern and this value
// where the site is solid: all bits set, which no offset takes (offsets are
// multiples of the pair size and a half stays below 4 GiB).  Offsets of 2 GiB
// and more read as negative ints, so a site is solid exactly when its entry
// equals kSolidOff, never when it is merely negative.
constexpr int kSolidOff = -1;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t half_rsrc(const void *base, int h, uint32_t half_bytes) {
    char *p = const_cast<char *>(static_cast<const char *>(base)) + (h ? (size_t)half_bytes : 0);
    return __builtin_amdgcn_make_buffer_rsrc(p, 0, (int)half_bytes, kRsrcWord3);
}

// Loads the pair at byte offset v + s of a half.  The loaded vector is
// reinterpreted as a whole (an integer or a struct) before it is split:
// extracting its elements one by one lets the compiler narrow the load to
// its first element.
struct U64Pair {
    uint64_t a, b;
};
template <typename S>
__device__ __forceinline__ void pair_load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, typename Codec<S>::R &a,
                                          typename Codec<S>::R &b) {
    if constexpr (std::is_same_v<S, float>) {
        const uint64_t x = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
        a = __builtin_bit_cast(float, (uint32_t)(x & 0xffffffffu));
        b = __builtin_bit_cast(float, (uint32_t)(x >> 32));
    } else if constexpr (std::is_same_v<S, double>) {
        const U64Pair x = __builtin_bit_cast(U64Pair, __builtin_amdgcn_raw_buffer_load_b128(r, v, s, 0));
        a = __builtin_bit_cast(double, x.a);
        b = __builtin_bit_cast(double, x.b);
    } else {
        const uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0);
        const S lo = __builtin_bit_cast(S, (unsigned short)(x & 0xffffu));
        const S hi = __builtin_bit_cast(S, (unsigned short)(x >> 16));
        if constexpr (std::is_same_v<typename Codec<S>::R, S>) {
            a = lo;
            b = hi;
        } else {
            a = Codec<S>::ld(lo);
            b = Codec<S>::ld(hi);
        }
    }
}

// Write-once streaming store of a post-collision pair (read again only in
// the next step, so it should not displace reused lines).
template <typename S>
__device__ __forceinline__ void pair_store(S a, S b, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    if constexpr (std::is_same_v<S, float>) {
        const uint64_t x = (uint64_t)__builtin_bit_cast(uint32_t, a) | ((uint64_t)__builtin_bit_cast(uint32_t, b) << 32);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v, s, kNonTemporal);
    } else if constexpr (std::is_same_v<S, double>) {
        const U64Pair x{__builtin_bit_cast(uint64_t, a), __builtin_bit_cast(uint64_t, b)};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), r, v, s, kNonTemporal);
    } else {
        const uint32_t x = (uint32_t)__builtin_bit_cast(unsigned short, a) |
                           ((uint32_t)__builtin_bit_cast(unsigned short, b) << 16);
        __builtin_amdgcn_raw_buffer_store_b32(x, r, v, s, kNonTemporal);
    }
}

// Eq. (4) and the second moments of one component's pulled populations:
// everything the regularized collision needs from them.  xx .. yz hold the
// second moments relative to the equilibrium of Eq. (3) at rest,
// P_ab = sum_i c_ia c_ib f_i - rho T0 delta_ab: the non-equilibrium flux that
// Eq. (10) projects, plus the equilibrium's own velocity terms (none for the
// printed Eq. 3).
template <typename C>
struct Moments {
    C r, jx, jy, jz, xx, yy, zz, xy, xz, yz;
};

// Second moments -> P_ab (the diagonal loses rho T0).
template <typename C>
__device__ __forceinline__ void to_flux(Moments<C> &m) {
    const C rt = m.r * C(1.0 / 3.0);
    m.xx = m.xx - rt;
    m.yy = m.yy - rt;
    m.zz = m.zz - rt;
}

// Adds s * v to an accumulator for a compile-time sign s in {-1, 0, 1}.
// Accumulators start at -0, which the compiler drops from the first sum.
template <int SGN, typename C> __device__ __forceinline__ void acc_signed(C &acc, C v) {
    if constexpr (SGN > 0) acc += v;
    if constexpr (SGN < 0) acc -= v;
}

// The moments from the sums s = f_i + f_opp(i) and differences
// d = f_i - f_opp(i) of the nine opposite pairs: c_i c_i is even under
// c -> -c and c_i odd, so each pair enters the second moments through s and
// the first through d.  For the shifted 16-bit storage (values
// f_i - w_i rho_ref) the shift is added back to the moments: sum_i w_i = 1,
// sum_i w_i c_i = 0 and sum_i w_i c_i c_i = T0 I.
template <typename S>
__device__ __forceinline__ Moments<typename Codec<S>::C> moments_of(const typename Codec<S>::R (&raw)[19],
                                                                   typename Codec<S>::C ref) {
    using C = typename Codec<S>::C;
    const C z = C(-0.0);
    Moments<C> m{z, z, z, z, z, z, z, z, z, z};
    m.r = held<S>(raw[0]);
    sfor<9>([&](auto K) {
        constexpr int i = 2 * K + 1;
        constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
        const C p = held<S>(raw[i]), q = held<S>(raw[i + 1]);
        const C s = p + q, d = p - q;
        m.r += s;
        acc_signed<X>(m.jx, d);
        acc_signed<Y>(m.jy, d);
        acc_signed<Z>(m.jz, d);
        acc_signed<X * X>(m.xx, s);
        acc_signed<Y * Y>(m.yy, s);
        acc_signed<Z * Z>(m.zz, s);
        acc_signed<X * Y>(m.xy, s);
        acc_signed<X * Z>(m.xz, s);
        acc_signed<Y * Z>(m.yz, s);
    });
    if constexpr (Codec<S>::shifted) {
        const C t = C(1.0 / 3.0) * ref;
        m.r += ref;
        m.xx += t;
        m.yy += t;
        m.zz += t;
    }
    to_flux(m);
    return m;
}

// The density alone, summed in exactly the order of moments_of: a site's
// density is the same bits whether a block pulls it as a tile site or as a
// ring site of a neighbouring tile.
template <typename S>
__device__ __forceinline__ typename Codec<S>::C density_of(const typename Codec<S>::R (&raw)[19],
                                                           typename Codec<S>::C ref) {
    using C = typename Codec<S>::C;
    C r = held<S>(raw[0]);
    sfor<9>([&](auto K) {
        constexpr int i = 2 * K + 1;
        r += held<S>(raw[i]) + held<S>(raw[i + 1]);
    });
    if constexpr (Codec<S>::shifted) r += ref;
    return r;
}

// 1 / x: the hardware reciprocal in single precision (1 ulp), a correctly
// rounded division in double precision.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// s1 * a + s2 * b + s3 * c for compile-time signs in {-1, 0, 1}.
template <int S1, int S2, int S3, typename C> __device__ __forceinline__ C dot_signed(C a, C b, C c) {
    C r = C(-0.0);
    acc_signed<S1>(r, a);
    acc_signed<S2>(r, b);
    acc_signed<S3>(r, c);
    return r;
}

// Everything the collision of one component needs, per site.
template <typename C>
struct CompState {
    C rho;            // rho_a
    C Fx, Fy, Fz;     // F^a (Shan-Chen plus body force)
    const Moments<C> *m;
    C ref;            // shift of the 16-bit storage (0 otherwise)
};

// Eqs. (3), (9), (10) for one component: f*_i = w_i [rho P_i +
// 4.5 (c_i c_i : X - T0 tr X) + 1.5 c_i . F] with X = (1 - 1/tau) Pi_neq +
// guo (u_F F + F u_F), P_i = 1 + 3 cu + 4.5 cu^3 - 4.5 cu u^2 (R2 adds
// 4.5 cu^2 - 1.5 u^2; r2 is 1 for R2, else 0).  Each opposite pair shares
// the part E even under c -> -c and the odd part O:
// f*_i = w (E + O), f*_opp(i) = w (E - O), with P_i split the same way
// (peven, podd per pair).  A component keeps only X, tr X, F and rho; each
// pair's terms are formed from them where the pair is stored (fewer live
// registers than holding all weighted terms), with only the non-zero
// components of c_i.  16-bit storage subtracts w_i ref here.
template <typename C>
struct Relaxed {
    C xx, yy, zz, xy, xz, yz, tr;   // X and its trace
    C Fx, Fy, Fz, rho, ref;
};

template <typename C>
__device__ __forceinline__ Relaxed<C> relax(C rho, C Fx, C Fy, C Fz, const Moments<C> &m, C ux, C uy, C uz, C r2,
                                            C keep, C guo, C ref) {
    // X: the non-equilibrium flux of Eq. (10) relaxed by 1 - 1/tau, plus the
    // second-order forcing part.
    const C ru = r2 * rho;
    const C g2 = C(2) * guo;
    Relaxed<C> x;
    x.xx = keep * (m.xx - ru * ux * ux) + g2 * ux * Fx;
    x.yy = keep * (m.yy - ru * uy * uy) + g2 * uy * Fy;
    x.zz = keep * (m.zz - ru * uz * uz) + g2 * uz * Fz;
    x.xy = keep * (m.xy - ru * ux * uy) + guo * (ux * Fy + Fx * uy);
    x.xz = keep * (m.xz - ru * ux * uz) + guo * (ux * Fz + Fx * uz);
    x.yz = keep * (m.yz - ru * uy * uz) + guo * (uy * Fz + Fy * uz);
    x.tr = x.xx + x.yy + x.zz;
    x.Fx = Fx;
    x.Fy = Fy;
    x.Fz = Fz;
    x.rho = rho;
    x.ref = ref;
    return x;
}

// f*_0 (w_0 = 1/3, c = 0).
template <typename C>
__device__ __forceinline__ C collide_rest(const Relaxed<C> &x, C pe0) {
    return C(1.0 / 3.0) * (x.rho * pe0 - x.ref) - C(0.5) * x.tr;
}

// f*_i and f*_opp(i) of the opposite pair k (odd member i = 2k + 1).
template <int k, typename C>
__device__ __forceinline__ void collide_pair(const Relaxed<C> &x, C podd, C peven, C &plus, C &minus) {
    constexpr int i = 2 * k + 1;
    constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
    const C t = C(1.0 / 3.0) * x.tr;
    C ew, ow;   // w E and w O
    if constexpr (i <= 6) {
        const C Xaa = X != 0 ? x.xx : (Y != 0 ? x.yy : x.zz);
        const C ref18 = x.ref * C(1.0 / 18.0);
        const C A = C(0.25) * (Xaa - t) - ref18;
        const C Fa = (X != 0 ? x.Fx : (Y != 0 ? x.Fy : x.Fz)) * C(1.0 / 12.0);
        const C r18 = x.rho * C(1.0 / 18.0);
        ew = r18 * peven + A;
        ow = r18 * podd + Fa;   // c_a = +1 for the odd member
    } else {
        const C Xaa = X != 0 ? x.xx : x.yy;
        const C Xbb = Z != 0 ? x.zz : x.yy;
        const C Xab = (X != 0 && Y != 0) ? x.xy : (X != 0 ? x.xz : x.yz);
        const C ref36 = x.ref * C(1.0 / 36.0);
        const C D = C(0.125) * (Xaa + Xbb - t) - ref36;
        const C Q = C(0.25) * Xab;
        constexpr int sg = X * Y + X * Z + Y * Z;   // product of the two non-zero components
        const C F36x = x.Fx * C(1.0 / 24.0), F36y = x.Fy * C(1.0 / 24.0), F36z = x.Fz * C(1.0 / 24.0);
        const C r36 = x.rho * C(1.0 / 36.0);
        ew = r36 * peven + (sg > 0 ? D + Q : D - Q);
        ow = r36 * podd + dot_signed<X, Y, Z>(F36x, F36y, F36z);
    }
    plus = ew + ow;
    minus = ew - ow;
}

// The collision of both components of a site (Eqs. 3, 5-6, 9, 10 and the
// forcing term), in two parts: collide_prepare relaxes the second moments
// (Eqs. 5-6 with p = rho_1 / rho: tau_mix is linear in p, so
// 1/tau = rho / (rho_1 tau_1 + rho_2 tau_2)); collide_emit forms the 19
// pairs and stores them at byte offset vo of each plane of the destination.
template <typename C>
struct SiteCollide {
    Relaxed<C> x0, x1;
    C ux, uy, uz, usq, pe0, r2;
};

template <typename S, typename C>
__device__ __forceinline__ SiteCollide<C> collide_prepare(const KArgs<S> &a, const C (&rho)[2], const C (&Fx)[2],
                                                          const C (&Fy)[2], const C (&Fz)[2], const Moments<C> (&m)[2],
                                                          C ux, C uy, C uz, C sref0, C sref1) {
    SiteCollide<C> sc;
    const C rho_t = rho[0] + rho[1];
    sc.usq = ux * ux + uy * uy + uz * uz;
    const C omega = rho_t * recip(rho[0] * a.tau0 + rho[1] * a.tau1);
    const C keep = C(1) - omega;
    const C guo = a.force_kind == 0 ? C(1) - C(0.5) * omega : C(0);
    sc.r2 = a.eq_kind == 1 ? C(1) : C(0);
    sc.pe0 = C(1) - sc.r2 * C(1.5) * sc.usq;
    sc.x0 = relax(rho[0], Fx[0], Fy[0], Fz[0], m[0], ux, uy, uz, sc.r2, keep, guo, sref0);
    sc.x1 = relax(rho[1], Fx[1], Fy[1], Fz[1], m[1], ux, uy, uz, sc.r2, keep, guo, sref1);
    sc.ux = ux;
    sc.uy = uy;
    sc.uz = uz;
    return sc;
}

template <typename S, typename C>
__device__ __forceinline__ void collide_emit(const SiteCollide<C> &sc, __amdgpu_buffer_rsrc_t dstA,
                                             __amdgpu_buffer_rsrc_t dstB, uint32_t vo) {
    auto put = [&](auto I, C v0, C v1) {
        constexpr int i = I;
        pair_store<S>(Codec<S>::st(v0), Codec<S>::st(v1), i < kSplit ? dstA : dstB, vo, dir_off(i, 2 * sizeof(S)));
    };
    put(std::integral_constant<int, 0>{}, collide_rest(sc.x0, sc.pe0), collide_rest(sc.x1, sc.pe0));
    sfor<9>([&](auto K) {
        constexpr int k = K;
        constexpr int i = 2 * k + 1;
        // The even and odd parts of P_i, shared by the two components.
        const C cu = dot_signed<cx_of(i), cy_of(i), cz_of(i)>(sc.ux, sc.uy, sc.uz);
        const C podd = cu * (C(3) + C(4.5) * (cu * cu - sc.usq));
        const C peven = sc.pe0 + sc.r2 * C(4.5) * cu * cu;
        C p0, m0, p1, m1;
        collide_pair<k>(sc.x0, podd, peven, p0, m0);
        collide_pair<k>(sc.x1, podd, peven, p1, m1);
        put(std::integral_constant<int, 2 * k + 1>{}, p0, p1);
        put(std::integral_constant<int, 2 * k + 2>{}, m0, m1);
    });
}

// ---------------------------------------------------------------------------
// The fused step.
// ---------------------------------------------------------------------------
// Consecutive block ids are dispatched to different XCDs in turn; remap so
// that each XCD receives a contiguous range of work items (neighbouring tiles
// then share its L2).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int per = nblocks >> 3;
    return b < (per << 3) ? (b & 7) * per + (b >> 3) : b;
}

// One block's work: work item b of the domain described by a (a tile
// column and a range of z planes, block_item); partial sums (MODE_CHECK /
// MODE_MOMENTS) go to a.partials[slot].
//
// Per plane: the tile's fluid sites are taken from the plane's work list
// (lane j gets the j-th fluid site, so lanes are busy only where there is
// fluid and whole waves idle on solid), the ring sites by the highest
// lanes.  Their pulls are issued together; the interior keeps only the ten
// moments per component of its site (the regularized collision rebuilds f*
// from them and the force), the ring only its densities.  The collision of
// a plane waits for the next plane's densities (one barrier per plane).
// The tile column and z-range of work item b: from the launch's table of
// balanced items (uniform reads through the scalar unit), else column
// b mod (ntx nty), chunk of zchunk planes b / (ntx nty).
template <typename S>
__device__ __forceinline__ void block_item(const KArgs<S> &a, int b, int &tx, int &ty, int &z0, int &z1) {
    if (a.btab) {
        const cint32 *t = (const cint32 *)(a.btab + 4 * b);
        tx = t[0];
        ty = t[1];
        z0 = t[2];
        z1 = t[3];
    } else {
        tx = b % a.ntx;
        b /= a.ntx;
        ty = b % a.nty;
        z0 = (b / a.nty) * a.zchunk;
        z1 = min(z0 + a.zchunk, a.nz);
    }
}

template <typename S, int TX, int TY, int MODE>
__device__ __forceinline__ void step_body(const KArgs<S> &a, int b, int slot) {
    static_assert(sizeof(S) == 8, "the 32- and 16-bit storage forms use step_body_pipe");
    using C = typename Codec<S>::C;
    constexpr int NT = TX * TY;
    constexpr int RW = TX + 2, RH = TY + 2;     // density tile with its ring
    constexpr int HW = TX + 4, HH = TY + 4;     // index tile with a ring of two
    constexpr int NE = (HW * HH + NT - 1) / NT; // index-tile entries per thread
    constexpr int NR = 2 * RW + 2 * TY;         // ring sites of the tile
    static_assert(NR <= NT, "the ring must fit in the block");

    // Densities of both components per site, side by side: one LDS access
    // moves a neighbour's pair.
    struct alignas(2 * sizeof(C)) PsiPair { C a, b; };
    __shared__ PsiPair psi[4][RH][RW];
    // byte offset (group_off) of each site's population pairs, kSolidOff where solid
    __shared__ int kid[6][HH][HW];
    __shared__ double red[NT / 64][6];

    int tx, ty, z0, z1;
    block_item(a, b, tx, ty, z0, z1);

    const int tid = threadIdx.x;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
    const uint32_t hb = a.half_bytes;
    constexpr uint32_t PB = 2 * sizeof(S);      // bytes of a component pair
    constexpr uint32_t DS = kGroup * PB;        // from one direction's run to the next

    // This thread's ring site in density-tile coordinates (rr, rc): the
    // rows above and below the tile, then its left and right columns; ring
    // index rt counts down from the last thread, so that the ring falls on
    // the waves the work list leaves idle first.
    const int rt = NT - 1 - tid;
    const bool has_ring = rt < NR;
    int rr = 0, rc = 0;
    if (rt < RW) { rr = 0; rc = rt; }
    else if (rt < 2 * RW) { rr = RH - 1; rc = rt - RW; }
    else if (rt < 2 * RW + TY) { rr = 1 + rt - 2 * RW; rc = 0; }
    else if (rt < NR) { rr = 1 + rt - 2 * RW - TY; rc = RW - 1; }
    // The site this thread owns for the solid test of the density tile.
    const int tly = tid / TX, tlx = tid % TX;

    // Work lists: per tile column and plane z, entries wstart[col (nz + 1) + z]
    // to wstart[... + z + 1] of wpos, the tile positions (ly TX + lx) of the
    // plane's fluid sites in storage order (positions beyond the lattice edge
    // stand for their periodic images and are pulled but not stored).
    // The bounds are uniform and read through the scalar unit (the constant
    // address space: they do not change during the launch), so waiting for
    // them does not wait for the vector stores still in flight.
    const cint32 *ws = (const cint32 *)(a.wstart + (size_t)(ty * a.ntx + tx) * (nz + 1));
    auto fetch_work = [&](int zq, int &cnt, int &pos) {
        const int zz = wrap(zq, nz);
        const int w0 = ws[zz];
        cnt = ws[zz + 1] - w0;
        pos = tid < cnt ? (int)a.wpos[w0 + tid] : 0;
    };

    // The index-tile entries this thread stages, gathered from the lattice
    // index (at 32 x 8 tiles the precomputed per-column tiles hold 1.69
    // entries per site that neighbouring tiles no longer share through L2;
    // the gather is 1.4 % faster here): their lattice (x, y).
    uint32_t exy[NE];
    bool eok[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const int e = tid + j * NT;
        eok[j] = e < HW * HH;
        const int er = e / HW, ec = e % HW;
        exy[j] = (uint32_t)wrap(tx * TX - 2 + ec, nx) + (uint32_t)nx * (uint32_t)wrap(ty * TY - 2 + er, ny);
    }
    const __amdgpu_buffer_rsrc_t ridx = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t *>(a.idx), 0, (int)(4u * (uint32_t)a.n_sites), kRsrcWord3);
    auto fetch_idx = [&](int zq, int (&v)[NE]) {
        const uint32_t zo = (uint32_t)wrap(zq, nz) * nxy * 4u;
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            v[j] = -1;
            if (eok[j]) v[j] = (int)__builtin_amdgcn_raw_buffer_load_b32(ridx, exy[j] * 4u, zo, 0);
        }
    };
    auto store_idx = [&](int q, const int (&v)[NE]) {
#pragma unroll
        for (int j = 0; j < NE; ++j)
            if (eok[j]) (&kid[q][0][0])[tid + j * NT] = v[j] >= 0 ? (int)group_off((uint32_t)v[j], PB) : kSolidOff;
    };

    const __amdgpu_buffer_rsrc_t srcA = half_rsrc(a.src, 0, hb), srcB = half_rsrc(a.src, 1, hb);

    // Pull of the site at index-tile position (hr, hc) whose populations sit
    // at byte offset self, planes zw - 1, zw, zw + 1 in index slots qm, q0,
    // qp: f_i = f*_i(x - c_i), or f*_opp(i)(x) when x - c_i is solid.  Both
    // members of an opposite pair are addressed from the odd member's plane
    // (the scalar offset), so the bounce-back is a select of lane offsets.
    using R = typename Codec<S>::R;
    auto issue = [&](int hr, int hc, int qm, int q0, int qp, uint32_t self, R (&raw)[2][19]) {
        const uint32_t self_p = self + DS;
        sfor<19>([&](auto I) {
            constexpr int i = I;
            constexpr int lo = i == 0 ? 0 : ((i & 1) ? i : i - 1);
            const uint32_t soff = dir_off(lo, PB);
            uint32_t off;
            if constexpr (i == 0) {
                off = self;
            } else {
                constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
                const int q = Z == 0 ? q0 : (Z > 0 ? qm : qp);   // plane zw - Z
                const int nb = kid[q][hr - Y][hc - X];
                if constexpr (i == lo) off = nb != kSolidOff ? (uint32_t)nb : self_p;
                else off = nb != kSolidOff ? (uint32_t)nb + DS : self;
            }
            pair_load<S>(lo < kSplit ? srcA : srcB, off, soff, raw[0][i], raw[1][i]);
        });
    };

    Moments<C> mc[2], mn[2];     // moments of the plane to collide / of the next plane
#pragma unroll
    for (int d = 0; d < 2; ++d) mn[d] = Moments<C>{C(0), C(0), C(0), C(0), C(0), C(0), C(0), C(0), C(0), C(0)};
    // this lane's work-list site of the plane to collide (c) / of the next plane (n)
    bool fluid_c = false, fluid_n = false;
    int kc = 0, kn = 0;          // byte offsets (group_off) of its populations
    int pc = 0, pn = 0;          // tile positions ly TX + lx
    int wcnt = 0, wpos = 0;      // work list of the plane to pull next (prefetched)
    const C ref0 = a.ref0, ref1 = a.ref1;

    // Pulls plane zw (z0 - 1 <= zw <= z1, unwrapped) into density slot
    // lslot; the interior's moments go to mn.  Index slot of plane p:
    // (p - z0 + 2) mod 6; the tile of plane zw + 2 is staged on the way.
    // Lane j pulls the plane's j-th fluid site (work-list entry j) and its
    // own ring position, both in one round trip.
    auto load_plane = [&](int zw, int lslot, bool keep) {
        const int qw = zw - z0 + 2;
        const int qm = (qw + 5) % 6, q0 = qw % 6, qp = (qw + 1) % 6;
        const int cnt = wcnt;
        const int pos_here = wpos;
        const int lx = wpos % TX, ly = wpos / TX;
        int vnext[NE];
        fetch_idx(zw + 2, vnext);
        fetch_work(zw + 1, wcnt, wpos);
        fluid_n = tid < cnt;
        pn = pos_here;
        // (A job list with a second pass for the ring, as the 32/16-bit
        // step runs, gave run-to-run differences in the FP64 step with
        // 512-thread blocks; this form does not.)
        const bool fi = tid < cnt;
        const int si = fi ? kid[q0][ly + 2][lx + 2] : kSolidOff;
        const int sr = has_ring ? kid[q0][rr + 1][rc + 1] : kSolidOff;
        const bool fr = sr != kSolidOff;
        kn = si;
        R ri[2][19], rg[2][19];
        if (fi) issue(ly + 2, lx + 2, qm, q0, qp, (uint32_t)si, ri);
        if (fr) issue(rr + 1, rc + 1, qm, q0, qp, (uint32_t)sr, rg);
        __builtin_amdgcn_sched_barrier(0);
        if (fi) {
            C r0, r1;
            if (keep) {
                mn[0] = moments_of<S>(ri[0], ref0);
                mn[1] = moments_of<S>(ri[1], ref1);
                r0 = mn[0].r;
                r1 = mn[1].r;
            } else {
                r0 = density_of<S>(ri[0], ref0);
                r1 = density_of<S>(ri[1], ref1);
            }
            psi[lslot][ly + 1][lx + 1] = PsiPair{r0, r1};
        }
        if (has_ring) {
            C q0v = a.wall0, q1v = a.wall1;
            if (fr) {
                q0v = density_of<S>(rg[0], ref0);
                q1v = density_of<S>(rg[1], ref1);
            }
            psi[lslot][rr][rc] = PsiPair{q0v, q1v};
        }
        if (kid[q0][tly + 2][tlx + 2] == kSolidOff) {   // solid site of the tile: the wall densities
            psi[lslot][tly + 1][tlx + 1] = PsiPair{a.wall0, a.wall1};
        }
        store_idx((qw + 2) % 6, vnext);
    };

    double acc[6] = {0, 0, 0, 0, 0, 0};

    {   // index tiles of planes z0 - 2, z0 - 1, z0
        int v[NE];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            fetch_idx(z0 - 2 + q, v);
            store_idx(q, v);
        }
    }
    fetch_work(z0 - 1, wcnt, wpos);
    __syncthreads();
    load_plane(z0 - 1, 0, false);
    __syncthreads();
    load_plane(z0, 1, true);
    mc[0] = mn[0];
    mc[1] = mn[1];
    fluid_c = fluid_n;
    kc = kn;
    pc = pn;
    __syncthreads();

    const __amdgpu_buffer_rsrc_t dstA = half_rsrc(a.dst, 0, hb), dstB = half_rsrc(a.dst, 1, hb);

    for (int z = z0; z < z1; ++z) {
        const int sm = (z - z0) & 3, s0 = (z - z0 + 1) & 3, sp = (z - z0 + 2) & 3;
        load_plane(z + 1, sp, true);
        __syncthreads();

        const int lx = pc % TX, ly = pc / TX;
        const bool inside = tx * TX + lx < nx && ty * TY + ly < ny;   // not a periodic image
        if (inside && fluid_c) {
            const C rho[2] = {mc[0].r, mc[1].r};

            // Eqs. (7), (11): sum_i w_i c_i psi'(x + c_i) from the LDS planes.
            const C nz0 = C(-0.0);
            C n0x = nz0, n0y = nz0, n0z = nz0, n1x = nz0, n1y = nz0, n1z = nz0;
            sfor<19>([&](auto I) {
                constexpr int i = I;
                if constexpr (i > 0) {
                    constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
                    constexpr C wx = C(X * w_of(i)), wy = C(Y * w_of(i)), wz = C(Z * w_of(i));
                    const int sl = Z == 0 ? s0 : (Z > 0 ? sp : sm);
                    const PsiPair pp = psi[sl][ly + 1 + Y][lx + 1 + X];
                    const C p0 = pp.a, p1 = pp.b;
                    if constexpr (X != 0) { n0x += wx * p0; n1x += wx * p1; }
                    if constexpr (Y != 0) { n0y += wy * p0; n1y += wy * p1; }
                    if constexpr (Z != 0) { n0z += wz * p0; n1z += wz * p1; }
                }
            });
            // Force on component 0 from component 1 and vice versa, plus body force.
            C Fx[2], Fy[2], Fz[2];
            Fx[0] = rho[0] * (a.G * n1x + a.gx);
            Fy[0] = rho[0] * (a.G * n1y + a.gy);
            Fz[0] = rho[0] * (a.G * n1z + a.gz);
            Fx[1] = rho[1] * (a.G * n0x + a.gx);
            Fy[1] = rho[1] * (a.G * n0y + a.gy);
            Fz[1] = rho[1] * (a.G * n0z + a.gz);
            if (a.wall_kind == 1) {
                // Momentum-balanced walls: the wall part of the force on
                // component a is G rho_a rho^s_b S with S = sum of w_i c_i over
                // the solid neighbours x + c_i; each component gives up its
                // share rho_a / rho of the sum over both components.
                C Sx = C(-0.0), Sy = C(-0.0), Sz = C(-0.0);
                sfor<19>([&](auto I) {
                    constexpr int i = I;
                    if constexpr (i > 0) {
                        constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
                        const int q = ((z + Z) - z0 + 2) % 6;   // index slot of plane z + Z
                        const C sol = kid[q][ly + 2 + Y][lx + 2 + X] == kSolidOff ? C(w_of(i)) : C(0);
                        if constexpr (X != 0) Sx += C(X) * sol;
                        if constexpr (Y != 0) Sy += C(Y) * sol;
                        if constexpr (Z != 0) Sz += C(Z) * sol;
                    }
                });
                const C net = a.G * (rho[0] * a.wall1 + rho[1] * a.wall0);
                const C inv_t = recip(rho[0] + rho[1]);
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    const C share = rho[d] * inv_t * net;
                    Fx[d] -= share * Sx;
                    Fy[d] -= share * Sy;
                    Fz[d] -= share * Sz;
                }
            }

            // Eq. (8): u_F = (j_1 + j_2 + F / 2) / rho.
            const C rho_t = rho[0] + rho[1];
            const C inv = recip(rho_t);
            const C ux = (mc[0].jx + mc[1].jx + C(0.5) * (Fx[0] + Fx[1])) * inv;
            const C uy = (mc[0].jy + mc[1].jy + C(0.5) * (Fy[0] + Fy[1])) * inv;
            const C uz = (mc[0].jz + mc[1].jz + C(0.5) * (Fz[0] + Fz[1])) * inv;

            if constexpr (MODE == MODE_CHECK || MODE == MODE_MOMENTS) {
                const bool ok = isfinite(rho[0]) && isfinite(rho[1]) && isfinite(ux) && isfinite(uy) && isfinite(uz);
                acc[0] += (double)rho[0];
                acc[1] += (double)rho[1];
                acc[2] += (double)rho_t * (double)ux;
                acc[3] += (double)rho_t * (double)uy;
                acc[4] += (double)rho_t * (double)uz;
                acc[5] += ok ? 0.0 : 1.0;
            }
            if constexpr (MODE == MODE_MOMENTS) {
                const uint32_t s = (uint32_t)(tx * TX + lx) + (uint32_t)nx * (uint32_t)(ty * TY + ly) + (uint32_t)z * nxy;
                if (a.out_rho0) a.out_rho0[s] = (double)rho[0];
                if (a.out_rho1) a.out_rho1[s] = (double)rho[1];
                if (a.out_u) {
                    a.out_u[s] = (double)ux;
                    a.out_u[(size_t)a.n_sites + s] = (double)uy;
                    a.out_u[2 * (size_t)a.n_sites + s] = (double)uz;
                }
            }

            if constexpr (MODE == MODE_STEP || MODE == MODE_CHECK) {
                const C sref0 = Codec<S>::shifted ? ref0 : C(0), sref1 = Codec<S>::shifted ? ref1 : C(0);
                collide_emit<S>(collide_prepare(a, rho, Fx, Fy, Fz, mc, ux, uy, uz, sref0, sref1), dstA, dstB,
                                (uint32_t)kc);
            }
        }

        mc[0] = mn[0];
        mc[1] = mn[1];
        fluid_c = fluid_n;
        kc = kn;
        pc = pn;
    }

    if constexpr (MODE == MODE_CHECK || MODE == MODE_MOMENTS) {
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double v = acc[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) red[wv][k] = v;
        }
        __syncthreads();
        if (tid < 6) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NT / 64; ++q) s += red[q][tid];
            a.partials[(size_t)slot * kPartialStride + tid] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// The fused step at 32- and 16-bit storage, software-pipelined along z.
// ---------------------------------------------------------------------------
// A pulled opposite-pair member as loaded: both components' values of one
// direction, 64 bits at FP32, 32 bits (two halves) at 16 bits.  Held packed
// until its moments are taken, so a plane's pulls occupy 38 registers at
// FP32 and 19 at 16 bits while they are in flight.
template <typename S> struct Held;
template <> struct Held<float> { using T = uint64_t; };
template <> struct Held<__half> { using T = uint32_t; };
template <> struct Held<__hip_bfloat16> { using T = uint32_t; };

template <typename S>
__device__ __forceinline__ typename Held<S>::T held_load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    if constexpr (std::is_same_v<S, float>)
        return __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
    else
        return __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0);
}

// Component D (0 or 1) of a held pair, as FP32.
template <typename S, int D>
__device__ __forceinline__ float held_comp(typename Held<S>::T x) {
    if constexpr (std::is_same_v<S, float>) {
        return __builtin_bit_cast(float, (uint32_t)(D == 0 ? x : x >> 32));
    } else if constexpr (std::is_same_v<S, __half>) {
        return __half2float(__builtin_bit_cast(__half, (unsigned short)(D == 0 ? x & 0xffffu : x >> 16)));
    } else {
        return __builtin_bit_cast(float, D == 0 ? x << 16 : x & 0xffff0000u);
    }
}

// Eq. (4) of component D of a held pull (density and momentum), summed in
// the order of moments_of (the pair sums and differences of the nine
// opposite pairs), with the 16-bit shift added back to the density.
template <typename S, int D>
__device__ __forceinline__ void held_density_momentum(const typename Held<S>::T (&raw)[19], float ref,
                                                      Moments<float> &m) {
    m.r = held_comp<S, D>(raw[0]);
    m.jx = m.jy = m.jz = -0.0f;
    sfor<9>([&](auto K) {
        constexpr int i = 2 * K + 1;
        constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
        const float p = held_comp<S, D>(raw[i]), q = held_comp<S, D>(raw[i + 1]);
        const float s = p + q, d = p - q;
        m.r += s;
        acc_signed<X>(m.jx, d);
        acc_signed<Y>(m.jy, d);
        acc_signed<Z>(m.jz, d);
    });
    if constexpr (Codec<S>::shifted) m.r += ref;
}

// The second moments of component D of a held pull as P_ab (FP32), from the
// same pair sums; m.r must hold the component's density.
template <typename S, int D>
__device__ __forceinline__ void held_flux(const typename Held<S>::T (&raw)[19], float ref, Moments<float> &m) {
    m.xx = m.yy = m.zz = m.xy = m.xz = m.yz = -0.0f;
    sfor<9>([&](auto K) {
        constexpr int i = 2 * K + 1;
        constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
        const float s = held_comp<S, D>(raw[i]) + held_comp<S, D>(raw[i + 1]);
        acc_signed<X * X>(m.xx, s);
        acc_signed<Y * Y>(m.yy, s);
        acc_signed<Z * Z>(m.zz, s);
        acc_signed<X * Y>(m.xy, s);
        acc_signed<X * Z>(m.xz, s);
        acc_signed<Y * Z>(m.yz, s);
    });
    if constexpr (Codec<S>::shifted) {
        const float t = (1.0f / 3.0f) * ref;
        m.xx += t;
        m.yy += t;
        m.zz += t;
    }
    to_flux(m);
}

// The density of component D alone, in the same order (same bits).
template <typename S, int D>
__device__ __forceinline__ float held_density(const typename Held<S>::T (&raw)[19], float ref) {
    float r = held_comp<S, D>(raw[0]);
    sfor<9>([&](auto K) {
        constexpr int i = 2 * K + 1;
        r += held_comp<S, D>(raw[i]) + held_comp<S, D>(raw[i + 1]);
    });
    if constexpr (Codec<S>::shifted) r += ref;
    return r;
}

// P_ab of component D accumulated in FP64 and rounded once to FP32: for
// sites whose relaxation time is near 1/2 (low viscosity), where the viscous
// stress is a small difference of sums of size rho / 3 and FP32 sums would
// lose most of its digits.  P_ab = sum_i (c_ia c_ib - T0 delta_ab) f_i, so a
// storage shift w_i rho_ref drops out (sum_i w_i (c c - T0 I) = 0) and the
// 16-bit deviations enter as they are.
template <typename S, int D>
__device__ __forceinline__ void held_flux_fp64(const typename Held<S>::T (&raw)[19], Moments<float> &m) {
    double r = (double)held_comp<S, D>(raw[0]);
    double xx = 0, yy = 0, zz = 0, xy = 0, xz = 0, yz = 0;
    sfor<9>([&](auto K) {
        constexpr int i = 2 * K + 1;
        constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
        const double s = (double)held_comp<S, D>(raw[i]) + (double)held_comp<S, D>(raw[i + 1]);
        r += s;
        acc_signed<X * X>(xx, s);
        acc_signed<Y * Y>(yy, s);
        acc_signed<Z * Z>(zz, s);
        acc_signed<X * Y>(xy, s);
        acc_signed<X * Z>(xz, s);
        acc_signed<Y * Z>(yz, s);
    });
    const double rt = r * (1.0 / 3.0);
    m.xx = (float)(xx - rt);
    m.yy = (float)(yy - rt);
    m.zz = (float)(zz - rt);
    m.xy = (float)xy;
    m.xz = (float)xz;
    m.yz = (float)yz;
}


// What the collision of a site needs from its pulled populations besides
// the densities (which the LDS plane holds): the mixture momentum j_1 + j_2
// and each component's second moments.
struct SiteMoments {
    float jx, jy, jz;
    Moments<float> m[2];   // only the second moments (xx .. yz) are used
};

// One block's work at 32- and 16-bit storage: as step_body, but with the
// pulls of plane z + 2 issued before the collision of plane z, so that the
// next plane's loads are in flight while the collision computes and stores.
// Iteration z:
//   D  issue the pulls of plane z + 2 (one job per lane), the index tile of
//      plane z + 4 and this lane's work-list entry of plane z + 3;
//   E  collide plane z and store;
//   A  consume the pulls of plane z + 2: moments of its sites, densities of
//      the plane and its ring into LDS; ring jobs beyond one pass (dense
//      tiles only) are pulled here, one round trip each; stage the index
//      tile of plane z + 4;
//   B  barrier.
// LDS slots: densities of planes z - 1 .. z + 2 (four: E of plane z reads
// z - 1 .. z + 1 while a faster wave's A writes z + 2), index tiles of
// planes z - 1 .. z + 4 (six); each slot is rewritten only after a barrier
// that follows its last read.
template <typename S, int TX, int TY, int MODE, bool HI>
__device__ __forceinline__ void step_body_pipe(const KArgs<S> &a, int b, int slot) {
    using C = float;
    using H = typename Held<S>::T;
    constexpr int NT = TX * TY;
    constexpr int RW = TX + 2, RH = TY + 2;     // density tile with its ring
    constexpr int HW = TX + 4, HH = TY + 4;     // index tile with a ring of two
    // The index tile is staged IW entries per load (HW and HH are multiples
    // of four): 16-byte loads at 16 bits, whose step has the registers to
    // spare and is limited by its vector memory instructions; single entries
    // at FP32, whose registers are all in use.
    constexpr int IW = sizeof(S) == 4 ? 1 : 4;
    constexpr int NQ = HW * HH / IW;             // loads per plane
    constexpr int NE = (NQ + NT - 1) / NT;       // loads per thread
    static_assert(HW * HH % (4 * IW) == 0, "index tiles are staged in whole vectors");
    using IV = typename std::conditional<IW == 1, uint32_t, u32x4>::type;
    constexpr int NR = 2 * RW + 2 * TY;         // ring sites of the tile
    static_assert(NR <= NT, "the ring must fit in the block");

    struct alignas(8) PsiPair { C a, b; };
    __shared__ PsiPair psi[4][RH][RW];
    __shared__ __attribute__((aligned(16))) int kid[6][HH][HW];
    __shared__ double red[NT / 64][6];
    // j_1 + j_2 and both components' second moments of this lane's site of
    // the plane to collide (written by the lane itself one plane earlier)
    __shared__ float mom[15][NT];

    int tx, ty, z0, z1;
    block_item(a, b, tx, ty, z0, z1);

    const int tid = threadIdx.x;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
    const uint32_t hb = a.half_bytes;
    constexpr uint32_t PB = 2 * sizeof(S);      // bytes of a component pair
    constexpr uint32_t DS = kGroup * PB;        // from one direction's run to the next
    const int tly = tid / TX, tlx = tid % TX;

    auto ring_pos = [&](int j, int &hr, int &hc) {
        if (j < RW) { hr = 1; hc = 1 + j; }
        else if (j < 2 * RW) { hr = RH; hc = 1 + j - RW; }
        else if (j < 2 * RW + TY) { hr = 2 + j - 2 * RW; hc = 1; }
        else { hr = 2 + j - 2 * RW - TY; hc = RW; }
    };
    // Job j of a plane whose work list has cnt entries and gives this lane
    // the tile position pos: a site (j < cnt), a ring position, or nothing.
    auto job_at = [&](int j, int cnt, int pos, int &hr, int &hc) -> bool {
        if (j < cnt) { hr = pos / TX + 2; hc = pos % TX + 2; return true; }
        if (j - cnt < NR) { ring_pos(j - cnt, hr, hc); return true; }
        return false;
    };

    // Work-list bounds (uniform; scalar reads) and this lane's entry.
    const cint32 *ws = (const cint32 *)(a.wstart + (size_t)(ty * a.ntx + tx) * (nz + 1));
    struct Bounds { int w0, cnt; };
    auto bounds = [&](int zq) {
        const int zz = wrap(zq, nz);
        const int w0 = ws[zz];
        return Bounds{w0, ws[zz + 1] - w0};
    };
    auto entry = [&](Bounds bd) { return tid < bd.cnt ? (int)a.wpos[bd.w0 + tid] : 0; };

    // This tile column's index tiles (index_tiles_kernel): HW HH entries per
    // plane, planes in order; entry e of a plane is staged by thread e mod NT.
    constexpr uint32_t TB = 4u * (uint32_t)(HW * HH);   // bytes of one plane's index tile
    const __amdgpu_buffer_rsrc_t ridx = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t *>(a.itab + (size_t)(ty * a.ntx + tx) * (size_t)nz * (HW * HH)), 0,
        (int)(TB * (uint32_t)nz), kRsrcWord3);
    auto eok = [&](int j) { return (j + 1) * NT <= NQ || tid + j * NT < NQ; };
    auto fetch_idx = [&](int zq, IV (&v)[NE]) {
        const uint32_t zo = (uint32_t)wrap(zq, nz) * TB;
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            v[j] = IV{};
            if (eok(j)) {
                const uint32_t off = 4u * IW * (uint32_t)(tid + j * NT);
                if constexpr (IW == 1) v[j] = __builtin_amdgcn_raw_buffer_load_b32(ridx, off, zo, 0);
                else v[j] = __builtin_amdgcn_raw_buffer_load_b128(ridx, off, zo, 0);
            }
        }
    };
    auto kslot = [&](int p) { return (p - z0 + 2) % 6; };   // index slot of plane p >= z0 - 2
    auto store_idx = [&](int p, const IV (&v)[NE]) {
        const int q = kslot(p);
#pragma unroll
        for (int j = 0; j < NE; ++j)   // whole vectors, never split into elements (see pair_load)
            if (eok(j)) *reinterpret_cast<IV *>(&kid[q][0][0] + IW * (tid + j * NT)) = v[j];
    };
    auto psi_slot = [&](int p) { return (p - z0 + 1) & 3; };   // density slot of plane p >= z0 - 1

    const __amdgpu_buffer_rsrc_t srcA = half_rsrc(a.src, 0, hb), srcB = half_rsrc(a.src, 1, hb);

    // The 19 pair loads of the site at index-tile position (hr, hc) of plane
    // zw (its populations at byte offset self): f_i = f*_i(x - c_i), or
    // f*_opp(i)(x) when x - c_i is solid; both members of an opposite pair
    // are addressed from the odd member's plane, so the bounce-back is a
    // select of lane offsets.
    auto issue = [&](int zw, int hr, int hc, uint32_t self, H (&raw)[19]) {
        const int qm = kslot(zw - 1), q0 = kslot(zw), qp = kslot(zw + 1);
        const uint32_t self_p = self + DS;
        sfor<19>([&](auto I) {
            constexpr int i = I;
            constexpr int lo = i == 0 ? 0 : ((i & 1) ? i : i - 1);
            const uint32_t soff = dir_off(lo, PB);
            uint32_t off;
            if constexpr (i == 0) {
                off = self;
            } else {
                constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
                const int q = Z == 0 ? q0 : (Z > 0 ? qm : qp);   // plane zw - Z
                const int nb = kid[q][hr - Y][hc - X];
                if constexpr (i == lo) off = nb != kSolidOff ? (uint32_t)nb : self_p;
                else off = nb != kSolidOff ? (uint32_t)nb + DS : self;
            }
            raw[i] = held_load<S>(lo < kSplit ? srcA : srcB, off, soff);
        });
    };
    const C ref0 = a.ref0, ref1 = a.ref1;

    // Densities (and, for a site job with want_mom, the moments) of a
    // completed pull into the LDS plane of zw; ring positions without a
    // fluid site take the wall densities.
    auto consume = [&](int zw, bool is_site, bool is_job, int hr, int hc, int self, const H (&raw)[19],
                       bool want_mom, SiteMoments &sm) {
        C r0 = a.wall0, r1 = a.wall1;
        if (self != kSolidOff) {
            if (is_site && want_mom) {
                Moments<C> m0, m1;
                held_density_momentum<S, 0>(raw, ref0, m0);
                held_density_momentum<S, 1>(raw, ref1, m1);
                r0 = m0.r;
                r1 = m1.r;
                // tau_mix = (rho_1 tau_1 + rho_2 tau_2) / rho below tau_crit:
                // the flux in FP64 (compiled into the HI instances only, so
                // that the others keep their registers)
                if (HI && r0 * a.tau0 + r1 * a.tau1 < a.tau_crit * (r0 + r1)) {
                    held_flux_fp64<S, 0>(raw, m0);
                    held_flux_fp64<S, 1>(raw, m1);
                } else {
                    held_flux<S, 0>(raw, ref0, m0);
                    held_flux<S, 1>(raw, ref1, m1);
                }
                sm.jx = m0.jx + m1.jx;
                sm.jy = m0.jy + m1.jy;
                sm.jz = m0.jz + m1.jz;
                sm.m[0] = m0;
                sm.m[1] = m1;
            } else {
                r0 = held_density<S, 0>(raw, ref0);
                r1 = held_density<S, 1>(raw, ref1);
            }
        }
        if (is_job) psi[psi_slot(zw)][hr - 1][hc - 1] = PsiPair{r0, r1};
    };
    // Jobs of plane zw beyond the first pass (ring positions only: the
    // tile's sites all fit in one pass), one round trip each; and the wall
    // densities at the tile's solid sites.
    auto finish_plane = [&](int zw, int cnt) {
        for (int pass = 1; pass * NT < cnt + NR; ++pass) {
            const int j = tid + pass * NT;
            int hr = 0, hc = 0;
            const bool is_job = job_at(j, cnt, 0, hr, hc);
            const int self = is_job ? kid[kslot(zw)][hr][hc] : kSolidOff;
            H raw[19];
            if (self != kSolidOff) issue(zw, hr, hc, (uint32_t)self, raw);
            __builtin_amdgcn_sched_barrier(0);
            SiteMoments unused;
            consume(zw, false, is_job, hr, hc, self, raw, false, unused);
        }
        if (kid[kslot(zw)][tly + 2][tlx + 2] == kSolidOff)   // solid site of the tile: the wall densities
            psi[psi_slot(zw)][tly + 1][tlx + 1] = PsiPair{a.wall0, a.wall1};
    };

    auto mom_put = [&](const SiteMoments &m) {
        mom[0][tid] = m.jx;
        mom[1][tid] = m.jy;
        mom[2][tid] = m.jz;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            mom[3 + 6 * d][tid] = m.m[d].xx;
            mom[4 + 6 * d][tid] = m.m[d].yy;
            mom[5 + 6 * d][tid] = m.m[d].zz;
            mom[6 + 6 * d][tid] = m.m[d].xy;
            mom[7 + 6 * d][tid] = m.m[d].xz;
            mom[8 + 6 * d][tid] = m.m[d].yz;
        }
    };
    auto mom_get = [&](SiteMoments &m) {
        m.jx = mom[0][tid];
        m.jy = mom[1][tid];
        m.jz = mom[2][tid];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            m.m[d].xx = mom[3 + 6 * d][tid];
            m.m[d].yy = mom[4 + 6 * d][tid];
            m.m[d].zz = mom[5 + 6 * d][tid];
            m.m[d].xy = mom[6 + 6 * d][tid];
            m.m[d].xz = mom[7 + 6 * d][tid];
            m.m[d].yz = mom[8 + 6 * d][tid];
        }
    };
    double acc[6] = {0, 0, 0, 0, 0, 0};
    SiteMoments mc, mn;
    {
        const Moments<C> zm{C(0), C(0), C(0), C(0), C(0), C(0), C(0), C(0), C(0), C(0)};
        mc = SiteMoments{C(0), C(0), C(0), {zm, zm}};
        mn = mc;
    }
    int kc = kSolidOff, pc = 0;   // the site job of the plane to collide: byte offset (kSolidOff: none), tile position
    int kn = kSolidOff, pn = 0;   // ... of the next plane

    // ---- prologue: index tiles of planes z0 - 2 .. z0 + 3; planes z0 - 1,
    // z0 and z0 + 1 pulled, one round trip each.
    {
        IV v[6][NE];
#pragma unroll
        for (int q = 0; q < 6; ++q) fetch_idx(z0 - 2 + q, v[q]);
#pragma unroll
        for (int q = 0; q < 6; ++q) store_idx(z0 - 2 + q, v[q]);
    }
    Bounds b2 = bounds(z0 + 2), b3 = bounds(z0 + 3);
    int pos2 = entry(b2);
    __syncthreads();
    for (int q = 0; q < 3; ++q) {
        const int zw = z0 - 1 + q;
        const Bounds bd = bounds(zw);
        const int pos = entry(bd);
        int hr = 0, hc = 0;
        const bool is_job = job_at(tid, bd.cnt, pos, hr, hc);
        const int self = is_job ? kid[kslot(zw)][hr][hc] : kSolidOff;
        H raw[19];
        if (self != kSolidOff) issue(zw, hr, hc, (uint32_t)self, raw);
        __builtin_amdgcn_sched_barrier(0);
        const bool is_site = tid < bd.cnt;
        SiteMoments unused;
        consume(zw, is_site, is_job, hr, hc, self, raw, q > 0, q == 1 ? mc : (q == 2 ? mn : unused));
        if (q == 1) { kc = is_site ? self : kSolidOff; pc = pos; }
        if (q == 2) { kn = is_site ? self : kSolidOff; pn = pos; }
        finish_plane(zw, bd.cnt);
    }
    mom_put(mc);
    __syncthreads();
    // Nothing of the prologue stays in flight into the loop.
    __builtin_amdgcn_s_waitcnt(0);

    const __amdgpu_buffer_rsrc_t dstA = half_rsrc(a.dst, 0, hb), dstB = half_rsrc(a.dst, 1, hb);
    IV vnext[NE];

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 2 <= z1;   // plane z + 2 is still needed (for the collision of z + 1)

        // D: the pulls of plane z + 2 (the loads go out before this plane's
        // stores)
        H raw[19];
        int self2 = kSolidOff, pos3 = 0;
        Bounds b4{0, 0};
        if (more) {
            fetch_idx(z + 4, vnext);
            pos3 = entry(b3);
            b4 = bounds(z + 4);
            int hr2 = 0, hc2 = 0;
            const bool is_job = job_at(tid, b2.cnt, pos2, hr2, hc2);
            self2 = is_job ? kid[kslot(z + 2)][hr2][hc2] : kSolidOff;
            if (self2 != kSolidOff) issue(z + 2, hr2, hc2, (uint32_t)self2, raw);
        }
        __builtin_amdgcn_sched_barrier(0);

        // E: collide plane z and store
        const int sm_ = psi_slot(z - 1), s0 = psi_slot(z), sp = psi_slot(z + 1);
        const int lx = pc % TX, ly = pc / TX;
        const bool inside = tx * TX + lx < nx && ty * TY + ly < ny;   // not a periodic image
        const bool collide = inside && kc != kSolidOff;
        if (collide) {
            mom_get(mc);
            const PsiPair here = psi[s0][ly + 1][lx + 1];
            const C rho[2] = {here.a, here.b};

            // Eqs. (7), (11): sum_i w_i c_i psi'(x + c_i) from the LDS planes.
            const C nz0 = C(-0.0);
            C n0x = nz0, n0y = nz0, n0z = nz0, n1x = nz0, n1y = nz0, n1z = nz0;
            sfor<19>([&](auto I) {
                constexpr int i = I;
                if constexpr (i > 0) {
                    constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
                    constexpr C wx = C(X * w_of(i)), wy = C(Y * w_of(i)), wz = C(Z * w_of(i));
                    const int sl = Z == 0 ? s0 : (Z > 0 ? sp : sm_);
                    const PsiPair pp = psi[sl][ly + 1 + Y][lx + 1 + X];
                    const C p0 = pp.a, p1 = pp.b;
                    if constexpr (X != 0) { n0x += wx * p0; n1x += wx * p1; }
                    if constexpr (Y != 0) { n0y += wy * p0; n1y += wy * p1; }
                    if constexpr (Z != 0) { n0z += wz * p0; n1z += wz * p1; }
                }
            });
            C Fx[2], Fy[2], Fz[2];
            Fx[0] = rho[0] * (a.G * n1x + a.gx);
            Fy[0] = rho[0] * (a.G * n1y + a.gy);
            Fz[0] = rho[0] * (a.G * n1z + a.gz);
            Fx[1] = rho[1] * (a.G * n0x + a.gx);
            Fy[1] = rho[1] * (a.G * n0y + a.gy);
            Fz[1] = rho[1] * (a.G * n0z + a.gz);
            if (a.wall_kind == 1) {
                // Momentum-balanced walls: the wall part of the force on
                // component a is G rho_a rho^s_b S with S = sum of w_i c_i over
                // the solid neighbours x + c_i; each component gives up its
                // share rho_a / rho of the sum over both components.
                C Sx = C(-0.0), Sy = C(-0.0), Sz = C(-0.0);
                sfor<19>([&](auto I) {
                    constexpr int i = I;
                    if constexpr (i > 0) {
                        constexpr int X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
                        const C sol = kid[kslot(z + Z)][ly + 2 + Y][lx + 2 + X] == kSolidOff ? C(w_of(i)) : C(0);
                        if constexpr (X != 0) Sx += C(X) * sol;
                        if constexpr (Y != 0) Sy += C(Y) * sol;
                        if constexpr (Z != 0) Sz += C(Z) * sol;
                    }
                });
                const C net = a.G * (rho[0] * a.wall1 + rho[1] * a.wall0);
                const C inv_t = recip(rho[0] + rho[1]);
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    const C share = rho[d] * inv_t * net;
                    Fx[d] -= share * Sx;
                    Fy[d] -= share * Sy;
                    Fz[d] -= share * Sz;
                }
            }

            // Eq. (8): u_F = (j_1 + j_2 + F / 2) / rho.
            const C rho_t = rho[0] + rho[1];
            const C inv = recip(rho_t);
            const C ux = (mc.jx + C(0.5) * (Fx[0] + Fx[1])) * inv;
            const C uy = (mc.jy + C(0.5) * (Fy[0] + Fy[1])) * inv;
            const C uz = (mc.jz + C(0.5) * (Fz[0] + Fz[1])) * inv;

            if constexpr (MODE == MODE_CHECK || MODE == MODE_MOMENTS) {
                const bool ok = isfinite(rho[0]) && isfinite(rho[1]) && isfinite(ux) && isfinite(uy) && isfinite(uz);
                acc[0] += (double)rho[0];
                acc[1] += (double)rho[1];
                acc[2] += (double)rho_t * (double)ux;
                acc[3] += (double)rho_t * (double)uy;
                acc[4] += (double)rho_t * (double)uz;
                acc[5] += ok ? 0.0 : 1.0;
            }
            if constexpr (MODE == MODE_MOMENTS) {
                const uint32_t s = (uint32_t)(tx * TX + lx) + (uint32_t)nx * (uint32_t)(ty * TY + ly) + (uint32_t)z * nxy;
                if (a.out_rho0) a.out_rho0[s] = (double)rho[0];
                if (a.out_rho1) a.out_rho1[s] = (double)rho[1];
                if (a.out_u) {
                    a.out_u[s] = (double)ux;
                    a.out_u[(size_t)a.n_sites + s] = (double)uy;
                    a.out_u[2 * (size_t)a.n_sites + s] = (double)uz;
                }
            }
            if constexpr (MODE == MODE_STEP || MODE == MODE_CHECK) {
                const C sref0 = Codec<S>::shifted ? ref0 : C(0), sref1 = Codec<S>::shifted ? ref1 : C(0);
                collide_emit<S>(collide_prepare(a, rho, Fx, Fy, Fz, mc.m, ux, uy, uz, sref0, sref1), dstA, dstB,
                                (uint32_t)kc);
            }
        }
        __builtin_amdgcn_sched_barrier(0);

        // A: the pulls of plane z + 2
        mom_put(mn);
        kc = kn;
        pc = pn;
        if (more) {
            const bool is_site = tid < b2.cnt;
            int hra = 0, hca = 0;
            const bool is_job = job_at(tid, b2.cnt, pos2, hra, hca);
            consume(z + 2, is_site, is_job, hra, hca, self2, raw, true, mn);
            kn = is_site ? self2 : kSolidOff;
            pn = pos2;
            finish_plane(z + 2, b2.cnt);
            store_idx(z + 4, vnext);
            b2 = b3;
            b3 = b4;
            pos2 = pos3;
        }
        __syncthreads();   // B
    }

    if constexpr (MODE == MODE_CHECK || MODE == MODE_MOMENTS) {
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double v = acc[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) red[wv][k] = v;
        }
        __syncthreads();
        if (tid < 6) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NT / 64; ++q) s += red[q][tid];
            a.partials[(size_t)slot * kPartialStride + tid] = s;
        }
    }
}
template <typename S, int TX, int TY, int MODE, bool HI>
__device__ __forceinline__ void step_dispatch(const KArgs<S> &a, int b, int slot) {
    if constexpr (sizeof(S) == 8) step_body<S, TX, TY, MODE>(a, b, slot);
    else step_body_pipe<S, TX, TY, MODE, HI>(a, b, slot);
}

// Waves per SIMD the register allocator must allow: four for the 16-bit
// instances (a few spilled registers cost less than a quarter of the waves,
// and 1024-thread blocks need four), the natural count otherwise.
template <typename S> constexpr int kMinWaves = sizeof(S) <= 4 ? 4 : 1;

// HI: the instance with the FP64 flux at sites below tau_crit (32/16-bit
// storage, advancing modes).
template <typename S, int TX, int TY, int MODE, bool HI = false>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(kMinWaves<S>))) step_kernel(KArgs<S> a) {
    step_dispatch<S, TX, TY, MODE, HI>(a, xcd_remap(blockIdx.x, gridDim.x), blockIdx.x);
}

// Many domains in one launch: work item w = (domain, tile) of a list sorted
// by domain; descs[d] describes domain d with (src, dst) of an even step,
// swapped when flip is set.
template <typename S, int TX, int TY, int MODE, bool HI = false>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(kMinWaves<S>))) batch_kernel(const KArgs<S> *descs, const int2 *work, int flip) {
    const int2 w = work[xcd_remap(blockIdx.x, gridDim.x)];
    KArgs<S> a = descs[w.x];
    if (flip) {
        const S *t = a.src;
        a.src = a.dst;
        a.dst = const_cast<S *>(t);
    }
    step_dispatch<S, TX, TY, MODE, HI>(a, w.y, w.y);
}

__global__ void finalize_kernel(const double *partials, int nblocks, double *out) {
    __shared__ double sh[256];
    const int t = threadIdx.x;
    for (int k = 0; k < kPartialStride; ++k) {
        double s = 0.0;
        for (int j = t; j < nblocks; j += 256) s += partials[(size_t)j * kPartialStride + k];
        sh[t] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (t < w) sh[t] += sh[t + w];
            __syncthreads();
        }
        if (t == 0) out[k] = sh[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Set-up and exchange kernels (one thread per site).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void site_coords(int64_t s, int nx, int ny, int &x, int &y, int &z) {
    x = (int)(s % nx);
    const int64_t r = s / nx;
    y = (int)(r % ny);
    z = (int)(r / ny);
}

__device__ __forceinline__ int64_t site_shift(int x, int y, int z, int dx, int dy, int dz, int nx, int ny, int nz) {
    x += dx; y += dy; z += dz;
    x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
    y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    z = z < 0 ? z + nz : (z >= nz ? z - nz : z);
    return x + (int64_t)nx * (y + (int64_t)ny * z);
}

__global__ void links_kernel(const uint8_t *solid, uint32_t *links, int nx, int ny, int nz) {
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N; s += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        site_coords(s, nx, ny, x, y, z);
        uint32_t L = (solid && solid[s]) ? 1u : 0u;
        if (solid) {
            sfor<19>([&](auto I) {
                constexpr int i = I;
                if constexpr (i > 0) {
                    const int64_t src = site_shift(x, y, z, -cx_of(i), -cy_of(i), -cz_of(i), nx, ny, nz);
                    if (solid[src]) L |= 1u << i;
                }
            });
        }
        links[s] = L;
    }
}

// Equilibrium of Eq. (3) for direction i (double arithmetic).
__device__ __forceinline__ double feq_dir(int i, double rho, double ux, double uy, double uz, int eq_kind) {
    double w = 0, cu = 0;
    sfor<19>([&](auto I) {
        constexpr int j = I;
        if (j == i) {
            w = w_of(j);
            cu = cx_of(j) * ux + cy_of(j) * uy + cz_of(j) * uz;
        }
    });
    const double usq = ux * ux + uy * uy + uz * uz;
    double br = 1.0 + 3.0 * cu + 4.5 * cu * cu * cu - 4.5 * cu * usq;
    if (eq_kind == 1) br += 4.5 * cu * cu - 1.5 * usq;
    return rho * w * br;
}

// Element (in units of S) of component d of direction i of slot k.
__device__ __forceinline__ int64_t pop_elem(int64_t ngroups, int d, int i, int64_t k) {
    const int64_t half_pairs = ngroups * kHalfDirs * kGroup;
    const int64_t pair = (i < kSplit ? 0 : half_pairs) + ((k / kGroup) * kHalfDirs + (i < kSplit ? i : i - kSplit)) * kGroup +
                         k % kGroup;
    return pair * 2 + d;
}

template <typename S>
__device__ __forceinline__ void store_pop(S *dst, int64_t ngroups, int d, int i, int64_t k, double v, double ref) {
    if constexpr (Codec<S>::shifted) v -= w_of(i) * ref;
    dst[pop_elem(ngroups, d, i, k)] = Codec<S>::st((typename Codec<S>::C)v);
}

template <typename S>
__device__ __forceinline__ double load_pop(const S *src, int64_t ngroups, int d, int i, int64_t k, double ref) {
    double v = (double)Codec<S>::ld(src[pop_elem(ngroups, d, i, k)]);
    if constexpr (Codec<S>::shifted) v += w_of(i) * ref;
    return v;
}

// The set-up and exchange kernels address a fluid site s's populations by
// its slot idx[s] (solid sites have none).
// The non-equilibrium part of component a's populations that a velocity
// field's strain implies, for the warm start: f'_i = w_i / (2 T0^2)
// (c_i c_i - T0 I) : Pi^a (the projection of Eq. 10) with the first-order
// Chapman-Enskog flux of the mixture, Pi = -rho T0 tau_mix (grad u + grad u^T)
// (tau_mix of Eqs. 5-6), shared by the components in proportion to their
// densities, Pi^a = (rho_a / rho) Pi.  pi holds rho_a-independent
// Pi / rho at each site, 6 values (xx, yy, zz, xy, xz, yz), component-major.
__device__ __forceinline__ double neq_dir(int i, double rho_a, const double *pi, int64_t N, int64_t t) {
    double out = 0.0;
    sfor<19>([&](auto I) {
        constexpr int j = I;
        if (j == i) {
            constexpr double T0 = 1.0 / 3.0;
            constexpr double X = cx_of(j), Y = cy_of(j), Z = cz_of(j);
            const double c = (X * X - T0) * pi[t] + (Y * Y - T0) * pi[N + t] + (Z * Z - T0) * pi[2 * N + t] +
                             2.0 * (X * Y * pi[3 * N + t] + X * Z * pi[4 * N + t] + Y * Z * pi[5 * N + t]);
            out = rho_a * w_of(j) / (2.0 * T0 * T0) * c;
        }
    });
    return out;
}

// Pi / rho of the warm start at every fluid site (zero on solid sites): the
// derivatives of u by three-point differences along each axis, a solid
// neighbour standing for the wall half a site away with u = 0 (halfway
// bounce-back); Pi / rho = -T0 tau_mix (grad u + grad u^T).
__global__ void strain_kernel(const uint32_t *links, const double *rho0, const double *rho1, const double *u,
                              double tau0, double tau1, int nx, int ny, int nz, double *pi) {
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N; s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t L = links[s];
        double g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // g[d][b] = d u_b / d x_d
        if (!(L & 1u)) {
            int x, y, z;
            site_coords(s, nx, ny, x, y, z);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                // link bit of the minus neighbour (site - e_d: direction +e_d) and of the plus one
                const int bm = 2 * d + 1, bp = 2 * d + 2;
                const int dx = d == 0, dy = d == 1, dz = d == 2;
                const bool wm = (L >> bm) & 1u, wp = (L >> bp) & 1u;
                const int64_t sm = site_shift(x, y, z, -dx, -dy, -dz, nx, ny, nz);
                const int64_t sp = site_shift(x, y, z, dx, dy, dz, nx, ny, nz);
                const double h1 = wm ? 0.5 : 1.0, h2 = wp ? 0.5 : 1.0;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const double v0 = u[b * N + s];
                    const double v1 = wm ? 0.0 : u[b * N + sm], v2 = wp ? 0.0 : u[b * N + sp];
                    g[d][b] = (h1 * h1 * v2 - h2 * h2 * v1 + (h2 * h2 - h1 * h1) * v0) / (h1 * h2 * (h1 + h2));
                }
            }
        }
        const double r0 = rho0[s], r1 = rho1[s], r = r0 + r1;
        const double tau = (L & 1u) || !(r > 0) ? 0.0 : (r0 * tau0 + r1 * tau1) / r;
        const double k = -(1.0 / 3.0) * tau;
        pi[s] = k * 2.0 * g[0][0];
        pi[N + s] = k * 2.0 * g[1][1];
        pi[2 * N + s] = k * 2.0 * g[2][2];
        pi[3 * N + s] = k * (g[0][1] + g[1][0]);
        pi[4 * N + s] = k * (g[0][2] + g[2][0]);
        pi[5 * N + s] = k * (g[1][2] + g[2][1]);
    }
}

// Force per unit density of each component at the fluid sites, F_a / rho_a
// (acc, 6N: component-major, then x, y, z): the Shan-Chen part of Eq. (7)
// with psi = rho, the wall part of Eq. (11) from the wall densities of solid
// neighbours (W2: less the component's density share of the mixture's net
// wall force), and the body acceleration g.  Zero on solid sites.
__global__ void accel_kernel(const uint32_t *links, const double *rho0, const double *rho1, double G, double wall0,
                             double wall1, int wall_kind, double gx, double gy, double gz, int nx, int ny, int nz,
                             double *acc) {
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N; s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t L = links[s];
        double ff[2][3] = {{0, 0, 0}, {0, 0, 0}}, fw[2][3] = {{0, 0, 0}, {0, 0, 0}};
        double a[2][3] = {{0, 0, 0}, {0, 0, 0}};
        if (!(L & 1u)) {
            int x, y, z;
            site_coords(s, nx, ny, x, y, z);
            sfor<19>([&](auto I) {
                constexpr int i = I;
                if constexpr (i > 0) {
                    constexpr double W = w_of(i), X = cx_of(i), Y = cy_of(i), Z = cz_of(i);
                    if ((L >> opp_of(i)) & 1u) {   // x + c_i is solid: component a sees the other's wall density
                        fw[0][0] += W * X * wall1; fw[0][1] += W * Y * wall1; fw[0][2] += W * Z * wall1;
                        fw[1][0] += W * X * wall0; fw[1][1] += W * Y * wall0; fw[1][2] += W * Z * wall0;
                    } else {
                        const int64_t t = site_shift(x, y, z, cx_of(i), cy_of(i), cz_of(i), nx, ny, nz);
                        const double p0 = rho0[t], p1 = rho1[t];
                        ff[0][0] += W * X * p1; ff[0][1] += W * Y * p1; ff[0][2] += W * Z * p1;
                        ff[1][0] += W * X * p0; ff[1][1] += W * Y * p0; ff[1][2] += W * Z * p0;
                    }
                }
            });
            const double r0 = rho0[s], r1 = rho1[s], r = r0 + r1;
            const double g[3] = {gx, gy, gz};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                double w0 = G * fw[0][d], w1 = G * fw[1][d];
                if (wall_kind == 1) {
                    // F_a,wall / rho_a less (F_0,wall + F_1,wall) / rho
                    const double net = (r0 * w0 + r1 * w1) / r;
                    w0 -= net;
                    w1 -= net;
                }
                a[0][d] = G * ff[0][d] + w0 + g[d];
                a[1][d] = G * ff[1][d] + w1 + g[d];
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            acc[d * N + s] = a[0][d];
            acc[(3 + d) * N + s] = a[1][d];
        }
    }
}

// Internal state from fields: f*_j(x) = f_j(x + c_j) if that site is fluid,
// else f_opp(j)(x), with f = f_eq(rho_a, u) (Eq. 3), plus the strain's
// non-equilibrium part when pi is given (warm start).  With acc given, u is
// the force-shifted velocity u_F of Eq. (8) and component a's equilibrium
// takes u_F - (F_a / rho_a) / 2, so that the mixture's population momentum
// sum_i c_i f_i is rho u_F - F / 2 as Eq. (8) requires.
template <typename S>
__global__ void init_fields_kernel(S *dst, const uint32_t *links, const int32_t *idx, const double *rho0,
                                   const double *rho1, const double *u, const double *pi, const double *acc, int nx,
                                   int ny, int nz, int64_t ngroups, int eq_kind, double ref0, double ref1) {
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N; s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t L = links[s];
        if (L & 1u) continue;
        const int64_t k = idx[s];
        int x, y, z;
        site_coords(s, nx, ny, x, y, z);
        sfor<19>([&](auto I) {
            constexpr int j = I;
            // f*_j(x) = f_j(x + c_j) if x + c_j is fluid, else f_opp(j)(x).
            const bool wall = j != 0 && ((L >> opp_of(j)) & 1u);
            const int64_t t = wall ? s : site_shift(x, y, z, cx_of(j), cy_of(j), cz_of(j), nx, ny, nz);
            const int kk = wall ? opp_of(j) : j;
            const double ux = u ? u[t] : 0.0, uy = u ? u[N + t] : 0.0, uz = u ? u[2 * N + t] : 0.0;
            double v[2][3] = {{ux, uy, uz}, {ux, uy, uz}};
            if (acc) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    v[0][d] -= 0.5 * acc[d * N + t];
                    v[1][d] -= 0.5 * acc[(3 + d) * N + t];
                }
            }
            double f0 = feq_dir(kk, rho0[t], v[0][0], v[0][1], v[0][2], eq_kind);
            double f1 = feq_dir(kk, rho1[t], v[1][0], v[1][1], v[1][2], eq_kind);
            if (pi) {
                f0 += neq_dir(kk, rho0[t], pi, N, t);
                f1 += neq_dir(kk, rho1[t], pi, N, t);
            }
            store_pop<S>(dst, ngroups, 0, j, k, f0, ref0);
            store_pop<S>(dst, ngroups, 1, j, k, f1, ref1);
        });
    }
}

// FP64 sums of the distance between two states over all sites (solid sites
// hold 0 in both): [sum (ra - ra_prev)^2, sum ra^2, sum |u - u_prev|^2,
// sum |u|^2, sum ra_prev^2, sum |u_prev|^2] per block into partials
// (kPartialStride per block).
__global__ void residual_kernel(const double *ra, const double *u, const double *ra_prev, const double *u_prev,
                                int64_t N, double *partials) {
    constexpr int K = 6;
    __shared__ double red[4][K];
    double acc[K] = {0, 0, 0, 0, 0, 0};
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N; s += (int64_t)gridDim.x * blockDim.x) {
        const double a = ra[s], ap = ra_prev[s], da = a - ap;
        acc[0] += da * da;
        acc[1] += a * a;
        acc[4] += ap * ap;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = u[d * N + s], vp = u_prev[d * N + s], dv = v - vp;
            acc[2] += dv * dv;
            acc[3] += v * v;
            acc[5] += vp * vp;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double v = acc[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kPartialStride) {
        double v = 0.0;
        if (threadIdx.x < K)
            for (int q = 0; q < 4; ++q) v += red[q][threadIdx.x];
        partials[(size_t)blockIdx.x * kPartialStride + threadIdx.x] = v;
    }
}

template <typename S>
__global__ void set_pops_kernel(S *dst, const uint32_t *links, const int32_t *idx, const double *f, int nx, int ny,
                                int nz, int64_t ngroups, double ref0, double ref1) {
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N; s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t L = links[s];
        if (L & 1u) continue;
        const int64_t k = idx[s];
        int x, y, z;
        site_coords(s, nx, ny, x, y, z);
        sfor<19>([&](auto I) {
            constexpr int j = I;
            const bool wall = j != 0 && ((L >> opp_of(j)) & 1u);
            const int64_t t = wall ? s : site_shift(x, y, z, cx_of(j), cy_of(j), cz_of(j), nx, ny, nz);
            const int kk = wall ? opp_of(j) : j;
#pragma unroll
            for (int d = 0; d < 2; ++d)
                store_pop<S>(dst, ngroups, d, j, k, f[(int64_t)(d * 19 + kk) * N + t], d == 0 ? ref0 : ref1);
        });
    }
}

template <typename S>
__global__ void get_pops_kernel(const S *src, const uint32_t *links, const int32_t *idx, double *f, int nx, int ny,
                                int nz, int64_t ngroups, double ref0, double ref1) {
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N; s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t L = links[s];
        if (L & 1u) {
#pragma unroll
            for (int q = 0; q < 38; ++q) f[(int64_t)q * N + s] = 0.0;
            continue;
        }
        int x, y, z;
        site_coords(s, nx, ny, x, y, z);
        sfor<19>([&](auto I) {
            constexpr int i = I;
            // f_i(x) = f*_i(x - c_i) if x - c_i is fluid, else f*_opp(i)(x).
            const bool wall = i != 0 && ((L >> i) & 1u);
            const int64_t t = wall ? s : site_shift(x, y, z, -cx_of(i), -cy_of(i), -cz_of(i), nx, ny, nz);
            const int kk = wall ? opp_of(i) : i;
            const int64_t k = idx[t];   // t is fluid here
#pragma unroll
            for (int d = 0; d < 2; ++d) f[(int64_t)(d * 19 + i) * N + s] = load_pop<S>(src, ngroups, d, kk, k, d == 0 ? ref0 : ref1);
        });
    }
}

// Index tiles of the step, per tile column col = ty ntx + tx (tiles of
// tx x ty sites) and plane z: the (tx + 4)(ty + 4) sites around the tile (a
// ring of two, periodic) in row-major order, each as the byte offset of its
// population pairs within a buffer half (group_off, pairs of pb bytes) or
// kSolidOff; planes of a column follow one another.
__global__ void index_tiles_kernel(const int32_t *idx, int32_t *out, int nx, int ny, int nz, int tx, int ty, int ntx,
                                   int64_t total, uint32_t pb) {
    const int hw = tx + 4, per = (tx + 4) * (ty + 4);
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(t % per);
        const int64_t r = t / per;
        const int z = (int)(r % nz), col = (int)(r / nz);
        const int x = wrap((col % ntx) * tx - 2 + e % hw, nx), y = wrap((col / ntx) * ty - 2 + e / hw, ny);
        const int32_t v = idx[((int64_t)z * ny + y) * nx + x];
        out[t] = v >= 0 ? (int32_t)group_off((uint32_t)v, pb) : kSolidOff;
    }
}

// Field checks of a restart on the device: counts the fluid sites (bit 0 of
// the link mask clear) and finds the lowest fluid site whose densities are
// not finite, negative, or sum to zero or less, and the lowest whose
// velocity (when given) is not finite.  out[0] += count; out[1], out[2] take
// the minimum (the caller starts them at N).
__global__ void check_fields_kernel(const uint32_t *links, const double *r0, const double *r1, const double *u,
                                    int64_t N, unsigned long long *out) {
    unsigned long long nf = 0, bad_r = (unsigned long long)N, bad_u = (unsigned long long)N;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N; s += (int64_t)gridDim.x * blockDim.x) {
        if (links[s] & 1u) continue;
        ++nf;
        const double a = r0[s], b = r1[s];
        if (!(isfinite(a) && isfinite(b) && a >= 0 && b >= 0 && a + b > 0) && (unsigned long long)s < bad_r)
            bad_r = (unsigned long long)s;
        if (u && !(isfinite(u[s]) && isfinite(u[N + s]) && isfinite(u[2 * N + s])) && (unsigned long long)s < bad_u)
            bad_u = (unsigned long long)s;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nf += __shfl_xor(nf, o, 64);
        const unsigned long long xr = __shfl_xor(bad_r, o, 64), xu = __shfl_xor(bad_u, o, 64);
        bad_r = xr < bad_r ? xr : bad_r;
        bad_u = xu < bad_u ? xu : bad_u;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(out, nf);
        atomicMin(out + 1, bad_r);
        atomicMin(out + 2, bad_u);
    }
}

inline int site_grid(int64_t N) {
    const int64_t b = (N + 255) / 256;
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

template <typename S>
KArgs<S> make_kargs(const StepLaunch &L) {
    using C = typename Codec<S>::C;
    KArgs<S> a;
    a.src = static_cast<const S *>(L.src);
    a.dst = static_cast<S *>(L.dst);
    a.idx = L.idx;
    a.itab = L.itab;
    a.wstart = L.wstart;
    a.wpos = L.wpos;
    a.nx = L.nx; a.ny = L.ny; a.nz = L.nz;
    a.ntx = L.ntx; a.nty = L.nty; a.zchunk = L.zchunk;
    a.btab = L.btab;
    a.half_bytes = (uint32_t)(L.ngroups * kHalfDirs * kGroup * 2 * (int64_t)sizeof(S));
    a.tau0 = (C)L.tau0; a.tau1 = (C)L.tau1; a.G = (C)L.G;
    a.gx = (C)L.gx; a.gy = (C)L.gy; a.gz = (C)L.gz;
    a.wall0 = (C)L.wall0; a.wall1 = (C)L.wall1; a.ref0 = (C)L.ref0; a.ref1 = (C)L.ref1;
    a.tau_crit = (C)L.tau_crit;
    a.eq_kind = L.eq_kind; a.force_kind = L.force_kind; a.wall_kind = L.wall_kind;
    a.partials = L.partials;
    a.out_rho0 = L.out_rho0; a.out_rho1 = L.out_rho1; a.out_u = L.out_u;
    a.n_sites = (int64_t)L.nx * L.ny * L.nz;
    return a;
}

template <typename S, int TX, int TY>
hipError_t launch_typed(Mode mode, const StepLaunch &L, hipStream_t s) {
    const KArgs<S> a = make_kargs<S>(L);
    const dim3 grid((unsigned)(L.btab ? L.nblk : L.ntx * L.nty * L.nzc)), block(TX * TY);
    const bool hi = sizeof(S) < 8 && L.tau_crit > 0;
    switch (mode) {
    case MODE_STEP:
        if (hi) hipLaunchKernelGGL((step_kernel<S, TX, TY, MODE_STEP, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((step_kernel<S, TX, TY, MODE_STEP>), grid, block, 0, s, a);
        break;
    case MODE_CHECK:
        if (hi) hipLaunchKernelGGL((step_kernel<S, TX, TY, MODE_CHECK, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((step_kernel<S, TX, TY, MODE_CHECK>), grid, block, 0, s, a);
        break;
    default: hipLaunchKernelGGL((step_kernel<S, TX, TY, MODE_MOMENTS>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

template <typename S>
hipError_t launch_tiles(Mode mode, const StepLaunch &L, hipStream_t s) {
    if (L.tile_x == 64 && L.tile_y == 4) return launch_typed<S, 64, 4>(mode, L, s);
    if (L.tile_x == 32 && L.tile_y == 8) return launch_typed<S, 32, 8>(mode, L, s);
    if (L.tile_x == 16 && L.tile_y == 16) return launch_typed<S, 16, 16>(mode, L, s);
    if (L.tile_x == 8 && L.tile_y == 32) return launch_typed<S, 8, 32>(mode, L, s);
    if (L.tile_x == 64 && L.tile_y == 8) return launch_typed<S, 64, 8>(mode, L, s);
    if (L.tile_x == 32 && L.tile_y == 16) return launch_typed<S, 32, 16>(mode, L, s);
    if constexpr (sizeof(S) <= 4)
        if (L.tile_x == 64 && L.tile_y == 16) return launch_typed<S, 64, 16>(mode, L, s);
    return hipErrorInvalidValue;
}

template <typename S, int TX, int TY>
int occupancy_typed() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<S, TX, TY, MODE_STEP>, TX * TY, 0) != hipSuccess)
        return 0;
    return n;
}

template <typename S>
int occupancy_tiles(int tx, int ty) {
    if (tx == 64 && ty == 4) return occupancy_typed<S, 64, 4>();
    if (tx == 32 && ty == 8) return occupancy_typed<S, 32, 8>();
    if (tx == 16 && ty == 16) return occupancy_typed<S, 16, 16>();
    if (tx == 8 && ty == 32) return occupancy_typed<S, 8, 32>();
    if (tx == 64 && ty == 8) return occupancy_typed<S, 64, 8>();
    if (tx == 32 && ty == 16) return occupancy_typed<S, 32, 16>();
    if constexpr (sizeof(S) <= 4)
        if (tx == 64 && ty == 16) return occupancy_typed<S, 64, 16>();
    return 0;
}

template <typename S, int TX, int TY>
hipError_t launch_batch_typed(Mode mode, bool hi, const void *descs, const int2 *work, int nwork, int flip,
                              hipStream_t s) {
    const KArgs<S> *d = static_cast<const KArgs<S> *>(descs);
    const dim3 grid((unsigned)nwork), block(TX * TY);
    hi = hi && sizeof(S) < 8;
    switch (mode) {
    case MODE_STEP:
        if (hi) hipLaunchKernelGGL((batch_kernel<S, TX, TY, MODE_STEP, true>), grid, block, 0, s, d, work, flip);
        else hipLaunchKernelGGL((batch_kernel<S, TX, TY, MODE_STEP>), grid, block, 0, s, d, work, flip);
        break;
    case MODE_CHECK:
        if (hi) hipLaunchKernelGGL((batch_kernel<S, TX, TY, MODE_CHECK, true>), grid, block, 0, s, d, work, flip);
        else hipLaunchKernelGGL((batch_kernel<S, TX, TY, MODE_CHECK>), grid, block, 0, s, d, work, flip);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S>
hipError_t launch_batch_tiles(Mode mode, bool hi, int tx, int ty, const void *descs, const int2 *work, int nwork,
                              int flip, hipStream_t s) {
    if (tx == 64 && ty == 4) return launch_batch_typed<S, 64, 4>(mode, hi, descs, work, nwork, flip, s);
    if (tx == 32 && ty == 8) return launch_batch_typed<S, 32, 8>(mode, hi, descs, work, nwork, flip, s);
    if (tx == 16 && ty == 16) return launch_batch_typed<S, 16, 16>(mode, hi, descs, work, nwork, flip, s);
    if (tx == 8 && ty == 32) return launch_batch_typed<S, 8, 32>(mode, hi, descs, work, nwork, flip, s);
    if (tx == 64 && ty == 8) return launch_batch_typed<S, 64, 8>(mode, hi, descs, work, nwork, flip, s);
    if (tx == 32 && ty == 16) return launch_batch_typed<S, 32, 16>(mode, hi, descs, work, nwork, flip, s);
    if constexpr (sizeof(S) <= 4)
        if (tx == 64 && ty == 16) return launch_batch_typed<S, 64, 16>(mode, hi, descs, work, nwork, flip, s);
    return hipErrorInvalidValue;
}

}  // namespace

size_t batch_desc_size(int prec) {
    switch (prec) {
    case LBM_FP64: return sizeof(KArgs<double>);
    case LBM_FP32: return sizeof(KArgs<float>);
    case LBM_FP16S: return sizeof(KArgs<__half>);
    case LBM_BF16S: return sizeof(KArgs<__hip_bfloat16>);
    default: return 0;
    }
}

void fill_batch_desc(int prec, const StepLaunch &L, void *out) {
    switch (prec) {
    case LBM_FP64: *static_cast<KArgs<double> *>(out) = make_kargs<double>(L); break;
    case LBM_FP32: *static_cast<KArgs<float> *>(out) = make_kargs<float>(L); break;
    case LBM_FP16S: *static_cast<KArgs<__half> *>(out) = make_kargs<__half>(L); break;
    case LBM_BF16S: *static_cast<KArgs<__hip_bfloat16> *>(out) = make_kargs<__hip_bfloat16>(L); break;
    default: break;
    }
}

hipError_t launch_batch(int prec, Mode mode, bool hi, int tx, int ty, const void *descs, const int2 *work, int nwork,
                        int flip, hipStream_t s) {
    switch (prec) {
    case LBM_FP64: return launch_batch_tiles<double>(mode, hi, tx, ty, descs, work, nwork, flip, s);
    case LBM_FP32: return launch_batch_tiles<float>(mode, hi, tx, ty, descs, work, nwork, flip, s);
    case LBM_FP16S: return launch_batch_tiles<__half>(mode, hi, tx, ty, descs, work, nwork, flip, s);
    case LBM_BF16S: return launch_batch_tiles<__hip_bfloat16>(mode, hi, tx, ty, descs, work, nwork, flip, s);
    default: return hipErrorInvalidValue;
    }
}

int step_blocks_per_cu(int prec, int tx, int ty) {
    switch (prec) {
    case LBM_FP64: return occupancy_tiles<double>(tx, ty);
    case LBM_FP32: return occupancy_tiles<float>(tx, ty);
    case LBM_FP16S: return occupancy_tiles<__half>(tx, ty);
    case LBM_BF16S: return occupancy_tiles<__hip_bfloat16>(tx, ty);
    default: return 0;
    }
}

bool tile_supported(int tx, int ty) {
    return (tx == 64 && ty == 4) || (tx == 32 && ty == 8) || (tx == 16 && ty == 16) || (tx == 8 && ty == 32) ||
           (tx == 64 && ty == 8) || (tx == 32 && ty == 16) || (tx == 64 && ty == 16);
}

hipError_t launch_step(int prec, Mode mode, const StepLaunch &L, hipStream_t s) {
    switch (prec) {
    case LBM_FP64: return launch_tiles<double>(mode, L, s);
    case LBM_FP32: return launch_tiles<float>(mode, L, s);
    case LBM_FP16S: return launch_tiles<__half>(mode, L, s);
    case LBM_BF16S: return launch_tiles<__hip_bfloat16>(mode, L, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize(const double *partials, int nblocks, double *out, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_index_tiles(const int32_t *idx, int32_t *itab, int nx, int ny, int nz, int tx, int ty, int pair_bytes,
                              hipStream_t s) {
    const int ntx = (nx + tx - 1) / tx, nty = (ny + ty - 1) / ty;
    const int64_t total = (int64_t)ntx * nty * nz * (tx + 4) * (ty + 4);
    hipLaunchKernelGGL(index_tiles_kernel, dim3(site_grid(total)), dim3(256), 0, s, idx, itab, nx, ny, nz, tx, ty, ntx,
                       total, (uint32_t)pair_bytes);
    return hipGetLastError();
}

hipError_t launch_check_fields(const uint32_t *links, const double *rho0, const double *rho1, const double *u,
                               int64_t N, unsigned long long *out, hipStream_t s) {
    hipLaunchKernelGGL(check_fields_kernel, dim3(site_grid(N)), dim3(256), 0, s, links, rho0, rho1, u, N, out);
    return hipGetLastError();
}

hipError_t launch_links(const uint8_t *solid, uint32_t *links, int nx, int ny, int nz, hipStream_t s) {
    hipLaunchKernelGGL(links_kernel, dim3(site_grid((int64_t)nx * ny * nz)), dim3(256), 0, s, solid, links, nx, ny, nz);
    return hipGetLastError();
}

#define LBM_DISPATCH_PREC(prec, S, ...)                         \
    switch (prec) {                                             \
    case LBM_FP64: { using S = double; __VA_ARGS__; break; }    \
    case LBM_FP32: { using S = float; __VA_ARGS__; break; }     \
    case LBM_FP16S: { using S = __half; __VA_ARGS__; break; }   \
    case LBM_BF16S: { using S = __hip_bfloat16; __VA_ARGS__; break; } \
    default: return hipErrorInvalidValue;                       \
    }

hipError_t launch_init_fields(int prec, void *dst, const uint32_t *links, const int32_t *idx, const double *rho0,
                              const double *rho1, const double *u, const double *pi, const double *acc, int nx,
                              int ny, int nz, int64_t ngroups, int eq_kind, const double ref[2], hipStream_t s) {
    const int g = site_grid((int64_t)nx * ny * nz);
    LBM_DISPATCH_PREC(prec, S,
                      hipLaunchKernelGGL(init_fields_kernel<S>, dim3(g), dim3(256), 0, s, static_cast<S *>(dst), links,
                                         idx, rho0, rho1, u, pi, acc, nx, ny, nz, ngroups, eq_kind, ref[0], ref[1]));
    return hipGetLastError();
}

hipError_t launch_accel(const uint32_t *links, const double *rho0, const double *rho1, double G, double wall0,
                        double wall1, int wall_kind, const double g[3], int nx, int ny, int nz, double *acc,
                        hipStream_t s) {
    hipLaunchKernelGGL(accel_kernel, dim3(site_grid((int64_t)nx * ny * nz)), dim3(256), 0, s, links, rho0, rho1, G,
                       wall0, wall1, wall_kind, g[0], g[1], g[2], nx, ny, nz, acc);
    return hipGetLastError();
}

hipError_t launch_strain(const uint32_t *links, const double *rho0, const double *rho1, const double *u, double tau0,
                         double tau1, int nx, int ny, int nz, double *pi, hipStream_t s) {
    hipLaunchKernelGGL(strain_kernel, dim3(site_grid((int64_t)nx * ny * nz)), dim3(256), 0, s, links, rho0, rho1, u,
                       tau0, tau1, nx, ny, nz, pi);
    return hipGetLastError();
}

hipError_t launch_residual(const double *ra, const double *u, const double *ra_prev, const double *u_prev, int64_t N,
                           int nblocks, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, dim3(nblocks), dim3(256), 0, s, ra, u, ra_prev, u_prev, N, partials);
    return hipGetLastError();
}

hipError_t launch_set_pops(int prec, void *dst, const uint32_t *links, const int32_t *idx, const double *f, int nx,
                           int ny, int nz, int64_t ngroups, const double ref[2], hipStream_t s) {
    const int g = site_grid((int64_t)nx * ny * nz);
    LBM_DISPATCH_PREC(prec, S,
                      hipLaunchKernelGGL(set_pops_kernel<S>, dim3(g), dim3(256), 0, s, static_cast<S *>(dst), links,
                                         idx, f, nx, ny, nz, ngroups, ref[0], ref[1]));
    return hipGetLastError();
}

hipError_t launch_get_pops(int prec, const void *src, const uint32_t *links, const int32_t *idx, double *f, int nx,
                           int ny, int nz, int64_t ngroups, const double ref[2], hipStream_t s) {
    const int g = site_grid((int64_t)nx * ny * nz);
    LBM_DISPATCH_PREC(prec, S,
                      hipLaunchKernelGGL(get_pops_kernel<S>, dim3(g), dim3(256), 0, s, static_cast<const S *>(src),
                                         links, idx, f, nx, ny, nz, ngroups, ref[0], ref[1]));
    return hipGetLastError();
}

}  // namespace lbm
