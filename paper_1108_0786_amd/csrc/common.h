// Shared device-side definitions: the D3Q19 velocity set, the storage
// formats of the population deviations, and the device tables of a box.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// D3Q19 (Sec. 2.1): 0 rest; 1..6 axis; 7..18 face diagonals in (d, -d) pairs.
__host__ __device__ constexpr int ex(int a) {
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[a];
}
__host__ __device__ constexpr int ey(int a) {
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[a];
}
__host__ __device__ constexpr int ez(int a) {
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[a];
}
__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
__host__ __device__ constexpr double wgt(int a) {
    return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
// 36 * 2 w_alpha: integer weight of the geometric part of the momentum exchange
__host__ __device__ constexpr int two_w36(int a) { return a == 0 ? 24 : (a <= 6 ? 4 : 2); }

constexpr int kBodyShapeSphere = 0;
constexpr int kBodyShapeCapsule = 1;
constexpr int kBodyShapeSlab = 2;     // tests only: a half-space
constexpr uint8_t kNearBit = 0x80;
constexpr uint8_t kOwnerMask = 0x7f;

// ---------------------------------------------------------------------------
// Storage formats.  Compute type C is double for double storage, float
// otherwise.  The 16-bit formats hold dF * 2^s.
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };

// T in the global address space: pointers read from the box descriptor are
// generic, and casting them lets the compiler use global (not flat) memory
// instructions
template <typename T> using global_t = __attribute__((address_space(1))) T;

// memory access with an optional non-temporal (streaming) hint
template <bool NT, typename P>
__device__ __forceinline__ auto ld(P p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename P, typename T>
__device__ __forceinline__ void st(P p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// R is the raw element type in memory; to_c / from_c convert one element.
// load / store accept generic and global pointers alike.
template <typename S> struct Storage;
template <> struct Storage<double> {
    using C = double;
    using R = double;
    static __device__ __forceinline__ double to_c(double r, float) { return r; }
    static __device__ __forceinline__ double from_c(double v, float) { return v; }
    template <bool NT = false, typename P>
    static __device__ __forceinline__ double load(P p, size_t i, float) { return ld<NT>(p + i); }
    template <bool NT = false, typename P>
    static __device__ __forceinline__ void store(P p, size_t i, double v, float) { st<NT>(p + i, v); }
};
template <> struct Storage<float> {
    using C = float;
    using R = float;
    static __device__ __forceinline__ float to_c(float r, float) { return r; }
    static __device__ __forceinline__ float from_c(float v, float) { return v; }
    template <bool NT = false, typename P>
    static __device__ __forceinline__ float load(P p, size_t i, float) { return ld<NT>(p + i); }
    template <bool NT = false, typename P>
    static __device__ __forceinline__ void store(P p, size_t i, float v, float) { st<NT>(p + i, v); }
};
template <> struct Storage<_Float16> {
    using C = float;
    using R = _Float16;
    static __device__ __forceinline__ float to_c(_Float16 r, float inv_scale) { return (float)r * inv_scale; }
    static __device__ __forceinline__ _Float16 from_c(float v, float scale) { return (_Float16)(v * scale); }
    template <bool NT = false, typename P>
    static __device__ __forceinline__ float load(P p, size_t i, float inv_scale) {
        return to_c(ld<NT>(p + i), inv_scale);
    }
    template <bool NT = false, typename P>
    static __device__ __forceinline__ void store(P p, size_t i, float v, float scale) {
        st<NT>(p + i, from_c(v, scale));
    }
};
__device__ __forceinline__ float bf16_to_float(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}
__device__ __forceinline__ uint16_t float_to_bf16(float f) {
    // round to nearest even, NaN stays NaN: one v_cvt_pk_bf16_f32 on gfx950
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
template <> struct Storage<bf16_t> {
    using C = float;
    using R = uint16_t;
    static __device__ __forceinline__ float to_c(uint16_t r, float inv_scale) { return bf16_to_float(r) * inv_scale; }
    static __device__ __forceinline__ uint16_t from_c(float v, float scale) { return float_to_bf16(v * scale); }
    template <bool NT = false, typename P>
    static __device__ __forceinline__ float load(P p, size_t i, float inv_scale) {
        return to_c(ld<NT>(&p[i].bits), inv_scale);
    }
    template <bool NT = false, typename P>
    static __device__ __forceinline__ void store(P p, size_t i, float v, float scale) {
        st<NT>(&p[i].bits, from_c(v, scale));
    }
};

// Sums over the 64 lanes of a wave in a fixed tree: every lane gets the
// same total, and the order of the additions does not depend on timing.
// The tree: lanes i and i^1, then i^2 (DPP quad permutations), the two
// quads of each half row (row_half_mirror), the two halves of each row of 16
// (row_mirror), and the four row sums as (r0 + r1) + (r2 + r3), read with
// v_readlane.  DPP moves take a few cycles where a shuffle through the LDS
// crossbar takes tens.
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)dpp_move<CTRL>((int)(unsigned)u);
    const unsigned hi = (unsigned)dpp_move<CTRL>((int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int read_lane(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ double read_lane(double v, int lane) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
constexpr int kDppQuadSwap1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadSwap2 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowHalfMirror = 0x141;

template <typename T>
__device__ __forceinline__ T wave_sum_t(T v) {
    v += dpp_move<kDppQuadSwap1>(v);
    v += dpp_move<kDppQuadSwap2>(v);
    v += dpp_move<kDppRowHalfMirror>(v);
    v += dpp_move<kDppRowMirror>(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_t(v); }
__device__ __forceinline__ int wave_sum_int(int v) { return wave_sum_t(v); }

// The owners of the 18 neighbours of a cell (0 fluid, 1 + b body b), five
// bits each, six to a word: three registers, and no array that a run-time
// direction would have to index in private memory.
struct Owners {
    unsigned w[3] = {0u, 0u, 0u};
    __device__ __forceinline__ int get(int a) const {
        const int q = (a - 1) / 6, sh = 5 * ((a - 1) % 6);
        const unsigned word = q == 0 ? w[0] : (q == 1 ? w[1] : w[2]);
        return (int)((word >> sh) & 31u);
    }
    __device__ __forceinline__ void set(int a, int v) { w[(a - 1) / 6] |= (unsigned)v << (5 * ((a - 1) % 6)); }
};

// ---------------------------------------------------------------------------
// Device tables
// ---------------------------------------------------------------------------
struct DevBody {
    double anchor[3], D[3], V[3], O[3], q[4];
    double Xmap[3];            // position at the last remap (bounds the remap box)
    double F[3], T[3];         // hydrodynamic force and torque of the last step
    double radius, half_len, mass;
    double inertia[3];         // principal moments, body frame
    int shape, kinematic;
};

struct DevSpring {
    int i, j;
    double k, gamma, rest_len;
};

struct DevDrive {
    int left, middle, right, gate;
    double amplitude, period, phase_lag;
    long long off_left, off_right;
};

// Momentum-exchange contribution of one boundary link (Eq. hydroF), scratch
// of the sweep: deviation part of e_alpha [2 f~ + 6 w rho e_opp.u_w] and its
// torque about the body position, the integer geometric torque term
// (2 d + 1) x (36 * 2 w_alpha e_alpha), d the integer lever offset, and the
// link's direction alpha.
struct LinkRec {
    double f[3];
    double t[3];
    int s[3];
    int a;
};

// Momentum-exchange sums (Eq. hydroF) of one body over the boundary links of
// one wave of 64 consecutive cells, written by the sweep: the deviation part
// of e_alpha [2 f~ + 6 w rho e_opp.u_w] and its torque about the body
// position, and the exact integer sums of the geometric term 2 w_alpha
// e_alpha: torque (2 d + 1) x (36 * 2 w_alpha e_alpha), d the integer lever
// offset, and force 36 * 2 w_alpha e_alpha.
// One store of a remap in the swapped in-place layout: element `at` of the
// population array gets `v`.
struct RelocRec {
    long long at;
    double v;
};
static_assert(sizeof(LinkRec) == 4 * sizeof(RelocRec), "four relocation records fit one link record");

struct ForceRec {
    double f[3];
    double t[3];
    int s[3];
    int g[3];
    int body;
    int pad;
};

// One tile of the sweep: `first` is the tile's first cell in box `box`,
// (i0, j0, k0) its coordinates.
struct WorkItem {
    int box, first, i0, j0, k0, pad;
};

struct BoxDesc {
    int nx, ny, nz, per;       // per: bit 0 x, 1 y, 2 z periodic
    int N, nb, ns, nd;
    long long stride;          // elements between the arrays of consecutive directions
    double omega;              // 1 / tau
    float omegaf, scale, inv_scale, pad0;
    void *pop0, *pop1;
    uint8_t *flags;
    uint8_t *old_owner;        // N bytes: owner before the last remap
    int *link_cell;
    signed char *link_dir, *link_body;
    LinkRec *link_rec;         // one scratch record per link, written and summed by the sweep; a remap
                               // in the swapped in-place layout lists its moves here (4 per record)
    ForceRec *frec;            // momentum-exchange sums per (wave, body), by body, written by the sweep
    int *grp_pos;              // record of the wave's q-th body at the wave's first link + q
    int *link_base;            // N ints: first link of a boundary cell
    int link_cap;
    int force_avg;             // 1: bodies move with the mean of this and the last step's F, T
    DevBody *bodies;
    DevSpring *springs;
    DevDrive *drives;
    double *traj;
    long long traj_cap;
    void *ctl;                 // control words of the coupling kernel (counter, barrier, remap slices)
    double *flow_sum;          // 3 arrays of N: summed fluid velocity (x, y, z) for the time average, or null
    int *flow_count;           // N: samples in which the cell was fluid
    int flow_every;            // sample the steps n with n % flow_every == 0 (0: none)
    int aa;                    // 1: the populations stream in place in pop0 or pop1 (layout by step parity)
    double force[3];           // tests only: uniform body force on the fluid (Guo's scheme)
    // mutable state, advanced on the device
    long long step;
    int cur;                   // index of the buffer holding the current populations
    int link_count;
    int status;                // 0 ok, else an lbm error code
    int rec_off[17];           // momentum-exchange records of body b: [rec_off[b], rec_off[b + 1])
};

}  // namespace lbm
