// Per-box coupling kernel, run after each sweep:
//   1. momentum-exchange force and torque of every body (Eq. hydroF): the
//      sweep has summed the links of every wave of 64 cells into one record
//      per (wave, body); the box's first workgroup adds the records of each
//      body in a fixed order, and the geometric part 2 w e of the link term,
//      which the records carry as exact integers;
//   2. the same workgroup adds the driving forces (Eqs. FB1-FB3) and the
//      spring-damper forces (Eqs. osci_i/j) and advances every body by one
//      semi-implicit Euler step (Alg. 1);
//   3. the bodies are mapped for the next step (Sec. 2.3): new flags, refill
//      of uncovered cells, near-body marks, the boundary links and the
//      records of the next momentum-exchange sums, skipped when no cell can
//      have changed side since the last mapping.  When all workgroups of the
//      launch can be resident at once, the box's kRedBlocks workgroups wait
//      for the decision and share the mapping (cooperative); otherwise the
//      first workgroup maps alone.
// All sums are in a fixed order, so results do not depend on the launch.
#pragma once
#include "geometry.h"

namespace lbm {

constexpr int kCoupleThreads = 256;
constexpr int kRedBlocks = 32;  // workgroups per box in a coupling launch (they share a remap)
constexpr int kMaxBodies = 16;
constexpr int kMaxSprings = 64;
constexpr int kMaxDrives = 16;
constexpr double kMarginSafety = 1e-9;
constexpr int kSpinLimit = 1 << 20;   // polls of a workgroup barrier before it gives up (about a second)
constexpr int kJoinLimit = 64;        // polls the first workgroup waits for the others to join (tens of us)
constexpr unsigned kJoinGo = 1u << 30, kJoinAbort = 1u << 31;

enum : int { kModeStep = 0, kModeMapOnly = 1 };

// Control words of one box's coupling launch, in device memory, zeroed when
// the box is set up.
struct CoupleCtl {
    unsigned arrived, gen;       // barrier of the box's workgroups: arrivals, generation
    int map_req, cur;            // published by the first workgroup: remap needed, buffer index
    unsigned launches;           // workgroups of this box's coupling launches so far (kRedBlocks each)
    int share[2];                // set by the previous launch, by launch parity: the workgroups stay
                                 // to share a remap
    int lo[3], hi[3];            // ... and the cell box to map
    int counts[kRedBlocks];      // links found in each workgroup's slice of the cell box
    unsigned long long margin[kMaxBodies];  // bits of each body's margin (a non-negative double)
    unsigned owner_changes;      // cells whose owner a mapping has changed, counted since set-up
    int swapped;                 // published by the first workgroup: the remap sees the swapped layout
    unsigned reloc_count;        // stores listed by a remap in the swapped layout
    unsigned join[2];            // by launch parity: workgroups that joined a shared remap, and the
                                 // first workgroup's answer (kJoinGo / kJoinAbort)
};

struct CoupleShared {
    double drv[kMaxDrives][2];  // driving forces of each drive: left, right (x components)
    double spr[kMaxSprings][3]; // force of each spring on its body i (body j feels the opposite)
    int bad[kMaxBodies];
    double red[kCoupleThreads];
    int scan[kCoupleThreads];
    double F[kMaxBodies][3], T[kMaxBodies][3];
    int lo[3], hi[3];          // cell box the remap scans (when map_req)
    int map_req;               // 1: this step ends with a remap
    int ltotal;                // links of the box after the remap
    int parity, hint;          // this launch's parity and share hint
    int sync_ok;               // 0: a barrier of the cooperative remap timed out
    int first;                 // number of the first link of this workgroup's slice
    int share_next;            // the next step may remap: its workgroups should stay
    int rcount;                // cells to refill found in the current round
    int rlist[kCoupleThreads];
    int cur;                   // index of the current population buffer
    int swapped;               // 1: the populations are in the swapped in-place layout (before an odd step)
    // the box's small tables, staged in LDS by the workgroup that finishes the step
    DevBody body[kMaxBodies];
    DevSpring spring[kMaxSprings];
    DevDrive drive[kMaxDrives];
    double margin[kMaxBodies];
    double qmap[kMaxBodies][4];
    double psum[kMaxBodies][6];
    int psumi[kMaxBodies][6];
};

__device__ __forceinline__ double block_min(double v, CoupleShared &sh) {
    const int t = threadIdx.x;
    __syncthreads();
    sh.red[t] = v;
    __syncthreads();
    for (int s = kCoupleThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh.red[t] = fmin(sh.red[t], sh.red[t + s]);
        __syncthreads();
    }
    return sh.red[0];
}

// exclusive prefix sum of v over the block; returns the block total in *tot
__device__ __forceinline__ int block_scan(int v, int *tot, CoupleShared &sh) {
    const int t = threadIdx.x;
    __syncthreads();
    sh.scan[t] = v;
    __syncthreads();
    for (int s = 1; s < kCoupleThreads; s <<= 1) {
        int add = t >= s ? sh.scan[t - s] : 0;
        __syncthreads();
        sh.scan[t] += add;
        __syncthreads();
    }
    *tot = sh.scan[kCoupleThreads - 1];
    return sh.scan[t] - v;
}

template <typename S>
__device__ __forceinline__ double load_dev(const void *p, size_t i, float inv_scale) {
    return (double)Storage<S>::load((const S *)p, i, inv_scale);
}


// ---------------------------------------------------------------------------
// 1. momentum exchange: the sweep's records, body by body
// ---------------------------------------------------------------------------
// The records of body b are [rec_off[b], rec_off[b + 1]).  Wave w of the
// workgroup adds those of bodies w, w + 4, ...: lane l takes records l,
// l + 64, ... of the range in that order (four loads in flight), and the
// lanes are added in a fixed tree (wave_sum).  The sums go to sh.psum /
// sh.psumi; the body table is not needed yet, so this runs while the tables
// are being staged.
// The offsets come from the kernel's snapshot of the descriptor, picked by
// constant indices (an index computed at run time into the snapshot's array
// would move the whole snapshot out of registers).
__device__ __forceinline__ int rec_off_at(const BoxDesc &B, int b) {
    int v = 0;
#pragma unroll
    for (int q = 0; q <= kMaxBodies; ++q) v = b == q ? B.rec_off[q] : v;
    return v;
}

__device__ __forceinline__ void sum_records(const BoxDesc &B, CoupleShared &sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int b = wave; b < B.nb; b += kCoupleThreads / 64) {
        const int h0 = min(rec_off_at(B, b), B.link_cap), h1 = min(rec_off_at(B, b + 1), B.link_cap);
        double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int ia[6] = {0, 0, 0, 0, 0, 0};
        for (int h = h0 + lane; h < h1; h += 4 * 64) {
            ForceRec rec[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (h + 64 * u < h1) rec[u] = B.frec[h + 64 * u];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (h + 64 * u < h1)
#pragma unroll
                    for (int v = 0; v < 3; ++v) {
                        acc[v] += rec[u].f[v];
                        acc[3 + v] += rec[u].t[v];
                        ia[v] += rec[u].s[v];
                        ia[3 + v] += rec[u].g[v];
                    }
        }
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            acc[v] = wave_sum(acc[v]);
            ia[v] = wave_sum_int(ia[v]);
        }
        if (lane == 0)
#pragma unroll
            for (int v = 0; v < 6; ++v) {
                sh.psum[b][v] = acc[v];
                sh.psumi[b][v] = ia[v];
            }
    }
}

// Force and torque of every body: the deviation sums plus the geometric
// part, G = (integer sum) / 36 and its torque S / 72 - f x G, f the
// fractional part of the body position (lever arms are taken from the cell
// R = floor(X)).  Needs the body table in LDS and sum_records done; thread
// b finishes body b (no barrier: rigid_step runs it beside the driving and
// spring forces).
__device__ __forceinline__ void finish_forces(const BoxDesc &B, CoupleShared &sh) {
    const int b = threadIdx.x;
    if (b < B.nb) {
#pragma clang fp contract(off)
        const DevBody &bd = sh.body[b];
        double G[3], fp[3];
        for (int v = 0; v < 3; ++v) {
            G[v] = (double)sh.psumi[b][3 + v] / 36.0;
            const double X = bd.anchor[v] + bd.D[v];
            fp[v] = X - floor(X);
        }
        const double Tg[3] = {(double)sh.psumi[b][0] / 72.0 - (fp[1] * G[2] - fp[2] * G[1]),
                              (double)sh.psumi[b][1] / 72.0 - (fp[2] * G[0] - fp[0] * G[2]),
                              (double)sh.psumi[b][2] / 72.0 - (fp[0] * G[1] - fp[1] * G[0])};
        for (int v = 0; v < 3; ++v) {
            sh.F[b][v] = sh.psum[b][v] + G[v];
            sh.T[b][v] = sh.psum[b][3 + v] + Tg[v];
        }
    }
}

// ---------------------------------------------------------------------------
// 2. rigid bodies
// ---------------------------------------------------------------------------
// B is the kernel's snapshot of the box descriptor (read only); the step
// counter, buffer index and status go to the descriptor itself, Bg.  With
// FLUID the first wave finishes the hydrodynamic force and torque of every
// body (finish_forces) while the other three waves evaluate the driving and
// spring forces; without it (the swimmer in vacuum) sh.F and sh.T are zero.
template <bool FLUID>
__device__ __forceinline__ void rigid_step(const BoxDesc &B, BoxDesc &Bg, CoupleShared &sh) {
    const int nb = B.nb;
    const long long n = B.step;
    const int t = threadIdx.x;
    if (FLUID && t < 64) finish_forces(B, sh);
    // driving, Eqs. FB1-FB3 (delayed right force): the left force of drive d
    // by thread d of the second wave, the right force by thread d of the
    // third, so that the two sines are evaluated side by side
    if (t >= 64 && t - 64 < B.nd) {
        const DevDrive &dv = sh.drive[t - 64];
        const double om = 2.0 * M_PI / dv.period;
        double fl = -dv.amplitude * sin(om * (double)n);
        if (dv.off_left >= 0 && n >= dv.off_left) fl = 0.0;
        sh.drv[t - 64][0] = fl;
    } else if (t >= 128 && t - 128 < B.nd) {
        const DevDrive &dv = sh.drive[t - 128];
        const double om = 2.0 * M_PI / dv.period;
        double fr = dv.amplitude * sin(om * (double)n - dv.phase_lag);
        if (dv.gate && om * (double)n < dv.phase_lag) fr = 0.0;
        if (dv.off_right >= 0 && n >= dv.off_right) fr = 0.0;
        sh.drv[t - 128][1] = fr;
    }
    // springs, Eqs. spring_i, damp_i, osci_i/j: one thread per spring, in the
    // fourth wave
    const int e = t - 192;
    if (e >= 0 && e < B.ns) {
        const DevSpring &sp = sh.spring[e];
        const DevBody &bi = sh.body[sp.i];
        const DevBody &bj = sh.body[sp.j];
        double d[3];
        for (int q = 0; q < 3; ++q) d[q] = (bi.anchor[q] - bj.anchor[q]) + (bi.D[q] - bj.D[q]);
        const double ell = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double coef = -sp.k * (ell - sp.rest_len) / ell;
        for (int q = 0; q < 3; ++q) sh.spr[e][q] = coef * d[q] - sp.gamma * (bi.V[q] - bj.V[q]);
    }
    __syncthreads();
    // one thread per body: total force (Eq. totalFSwimmer) and time integration
    const int b = t;
    if (b < nb) {
        DevBody &bd = sh.body[b];
        // this body's driving and spring forces, summed drive by drive and
        // spring by spring (the order of the plain definition)
        double Fd[3] = {0.0, 0.0, 0.0}, Fs[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < B.nd; ++k) {
            const DevDrive &dv = sh.drive[k];
            const double fl = sh.drv[k][0], fr = sh.drv[k][1];
            if (dv.left == b) Fd[0] = Fd[0] + fl;
            if (dv.right == b) Fd[0] = Fd[0] + fr;
            if (dv.middle == b) Fd[0] = Fd[0] + -(fl + fr);
        }
        for (int k = 0; k < B.ns; ++k) {
            const DevSpring &sp = sh.spring[k];
            if (sp.i == b)
                for (int q = 0; q < 3; ++q) Fs[q] = Fs[q] + sh.spr[k][q];
            if (sp.j == b)
                for (int q = 0; q < 3; ++q) Fs[q] = Fs[q] - sh.spr[k][q];
        }
        // hydrodynamic force and torque that move the body: this step's sums,
        // or their mean with the last step's (bd.F, bd.T still hold those)
        double Fh[3], Th[3];
        for (int q = 0; q < 3; ++q) {
            Fh[q] = B.force_avg ? 0.5 * (sh.F[b][q] + bd.F[q]) : sh.F[b][q];
            Th[q] = B.force_avg ? 0.5 * (sh.T[b][q] + bd.T[q]) : sh.T[b][q];
        }
        for (int q = 0; q < 3; ++q) {
            bd.F[q] = sh.F[b][q];
            bd.T[q] = sh.T[b][q];
        }
        if (bd.kinematic != 1) {
            const double m = bd.mass;
            for (int q = 0; q < 3; ++q) bd.V[q] = bd.V[q] + ((Fh[q] + Fd[q]) + Fs[q]) / m;
        }
        if (bd.kinematic == 0) {
            // Omega += R diag(1/I) R^T T
            const double w = bd.q[0], x = bd.q[1], y = bd.q[2], z = bd.q[3];
            const double R[3][3] = {
                {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
            double bt[3];
            for (int p = 0; p < 3; ++p)
                bt[p] = (R[0][p] * Th[0] + R[1][p] * Th[1] + R[2][p] * Th[2]) / bd.inertia[p];
            for (int p = 0; p < 3; ++p) bd.O[p] = bd.O[p] + (R[p][0] * bt[0] + R[p][1] * bt[1] + R[p][2] * bt[2]);
        }
        for (int q = 0; q < 3; ++q) bd.D[q] = bd.D[q] + bd.V[q];
        {
            const double *O = bd.O;
            const double w = bd.q[0], x = bd.q[1], y = bd.q[2], z = bd.q[3];
            const double pw = -(O[0] * x + O[1] * y + O[2] * z);
            const double px = O[0] * w + (O[1] * z - O[2] * y);
            const double py = O[1] * w + (O[2] * x - O[0] * z);
            const double pz = O[2] * w + (O[0] * y - O[1] * x);
            double qn[4] = {w + 0.5 * pw, x + 0.5 * px, y + 0.5 * py, z + 0.5 * pz};
            const double nrm = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
            for (int q = 0; q < 4; ++q) bd.q[q] = qn[q] / nrm;
        }
        int bad = 0;
        for (int q = 0; q < 3; ++q)
            if (!isfinite(bd.F[q]) || !isfinite(bd.T[q]) || !isfinite(bd.V[q]) || !isfinite(bd.D[q])) bad = 1;
        sh.bad[b] = bad;
        if (B.traj && B.traj_cap > 0) {
            double *rec = B.traj + ((size_t)(n % B.traj_cap) * nb + b) * 16;
            for (int q = 0; q < 3; ++q) {
                rec[q] = bd.D[q];
                rec[3 + q] = bd.V[q];
                rec[6 + q] = bd.O[q];
                rec[9 + q] = bd.F[q];
                rec[12 + q] = bd.T[q];
            }
            rec[15] = (double)n;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int bad = 0;
        for (int q = 0; q < nb; ++q) bad |= sh.bad[q];
        if (bad) Bg.status = -4;
        Bg.step = n + 1;
        if (!B.aa) sh.cur ^= 1;   // in-place streaming keeps its one array
        Bg.cur = sh.cur;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// 3. object mapping
// ---------------------------------------------------------------------------
__device__ __forceinline__ double body_extent(const DevBody &b) {
    if (b.shape == kBodyShapeSlab) return 1e30;   // a half-space: the whole box
    return b.radius + (b.shape == kBodyShapeCapsule ? b.half_len : 0.0);
}

// Largest distance any surface point of body b can have moved since the
// last mapping (translation plus rotation of the farthest point).
__device__ __forceinline__ double moved_bound(const DevBody &b, const double qmap[4]) {
    double dx = 0.0;
    for (int q = 0; q < 3; ++q) {
        const double t = (b.anchor[q] + b.D[q]) - b.Xmap[q];
        dx += t * t;
    }
    double bound = sqrt(dx);
    if (b.shape != kBodyShapeSphere) {
        // rotation angle between q and qmap: 2 atan2(|v|, |w|) of q * conj(qmap)
        const double *p = b.q;
        const double w = p[0] * qmap[0] + p[1] * qmap[1] + p[2] * qmap[2] + p[3] * qmap[3];
        const double vx = -p[0] * qmap[1] + p[1] * qmap[0] - p[2] * qmap[3] + p[3] * qmap[2];
        const double vy = -p[0] * qmap[2] + p[2] * qmap[0] - p[3] * qmap[1] + p[1] * qmap[3];
        const double vz = -p[0] * qmap[3] + p[3] * qmap[0] - p[1] * qmap[2] + p[2] * qmap[1];
        const double ang = 2.0 * atan2(sqrt(vx * vx + vy * vy + vz * vz), fabs(w));
        // a turned half-space moves without bound far from its centre
        if (b.shape == kBodyShapeSlab) bound = ang > 0.0 ? 1e300 : bound;
        else bound += ang * (b.half_len + b.radius + 2.0);
    }
    return bound;
}

// Decide whether the mapping must be redone and, if so, the box of cells to
// scan: the union of every body's old and new bounding box plus two cells.
// Called by the first wave, one lane per body; the lanes combine with wave
// votes and min / max reductions, which do not depend on the order.
__device__ __forceinline__ void decide_map(const BoxDesc &B, BoxDesc &Bg, CoupleShared &sh, bool force) {
    const int nb = B.nb, b = threadIdx.x;
    bool finite = true, need = false, soon = false;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    if (b < nb) {
        const DevBody &bd = sh.body[b];
        // a body whose position is no longer finite cannot be mapped: the box
        // is reported unstable and the flags stay as they are
        for (int q = 0; q < 3; ++q)
            if (!isfinite(bd.anchor[q] + bd.D[q]) || !isfinite(bd.Xmap[q])) finite = false;
        const double moved = moved_bound(bd, sh.qmap[b]);
        need = !(moved < sh.margin[b] - kMarginSafety);
        // may the next step need a remap: two more steps at the present
        // speeds (only decides whether the next step's workgroups stay to
        // share the work; see couple_kernel)
        double ahead = moved + 2.0 * sqrt(bd.V[0] * bd.V[0] + bd.V[1] * bd.V[1] + bd.V[2] * bd.V[2]) + 1e-6;
        const double spin = sqrt(bd.O[0] * bd.O[0] + bd.O[1] * bd.O[1] + bd.O[2] * bd.O[2]);
        if (bd.shape == kBodyShapeCapsule) ahead += 2.0 * spin * (bd.half_len + bd.radius + 2.0);
        if (bd.shape == kBodyShapeSlab && spin > 0.0) ahead = 1e300;
        soon = !(ahead < sh.margin[b] - kMarginSafety);
        const double ext = body_extent(bd);
        for (int q = 0; q < 3; ++q) {
            const double X = bd.anchor[q] + bd.D[q];
            lo[q] = fmin(X, bd.Xmap[q]) - ext;
            hi[q] = fmax(X, bd.Xmap[q]) + ext;
        }
    }
    const bool all_finite = !__any(!finite);
    const bool any_need = force || __any(need);
    const bool any_soon = __any(soon);
    const int nmap = all_finite && any_need ? 1 : 0;
    if (b == 0) {
        if (!all_finite) Bg.status = -4;
        sh.map_req = nmap;
        sh.share_next = nmap || any_soon;
    }
    // the cell box only when a remap is due (the decision is the same in
    // every lane): 36 shuffles of doubles are a large part of a step without one
    if (!nmap) return;
    for (int m = 32; m >= 1; m >>= 1)
        for (int q = 0; q < 3; ++q) {
            lo[q] = fmin(lo[q], __shfl_xor(lo[q], m));
            hi[q] = fmax(hi[q], __shfl_xor(hi[q], m));
        }
    if (b != 0) return;
    const int n[3] = {B.nx, B.ny, B.nz};
    for (int q = 0; q < 3; ++q) {
        // clamp in double before converting, so that no integer overflows
        const double l0 = fmin(fmax(floor(lo[q]) - 2.0, -4.0), (double)n[q] + 4.0);
        const double h0 = fmin(fmax(floor(hi[q]) + 2.0, -4.0), (double)n[q] + 4.0);
        int l = (int)l0, h = (int)h0;
        if (nb == 0) {
            l = 0;
            h = -1;
        }
        if (B.per & (1 << q)) {
            if (l < 0 || h >= n[q] || h - l + 1 >= n[q]) {
                l = 0;
                h = n[q] - 1;
            }
        } else {
            l = max(l, 0);
            h = min(h, n[q] - 1);
        }
        sh.lo[q] = l;
        sh.hi[q] = h;
    }
}

// The object mapping (Sec. 2.3) over the cell box chosen by decide_map.  The
// box is scanned as a linear range of cells t = 0 .. bx*by*bz - 1 (x fastest);
// each pass below covers a slice [t0, t1) of it, the whole range when one
// workgroup maps the box, one contiguous slice per workgroup when all
// kRedBlocks workgroups of the box take part.  Body data come from the
// workgroup's LDS copy (sh.body).
struct MapBox {
    int lo[3], bx, by, ncell;
};

__device__ __forceinline__ MapBox map_box(const CoupleShared &sh) {
    MapBox m;
    for (int q = 0; q < 3; ++q) m.lo[q] = sh.lo[q];
    m.bx = sh.hi[0] - sh.lo[0] + 1;
    m.by = sh.hi[1] - sh.lo[1] + 1;
    const int bz = sh.hi[2] - sh.lo[2] + 1;
    m.ncell = (m.bx > 0 && m.by > 0 && bz > 0) ? m.bx * m.by * bz : 0;
    return m;
}

__device__ __forceinline__ void map_cell(const MapBox &m, int t, int &i, int &j, int &k) {
    i = m.lo[0] + t % m.bx;
    j = m.lo[1] + (t / m.bx) % m.by;
    k = m.lo[2] + t / (m.bx * m.by);
}

// pass 1: new owners; remember the old ones
__device__ __forceinline__ void map_owners(const BoxDesc &B, const CoupleShared &sh, const MapBox &m, int t0, int t1) {
    const int nb = B.nb, nx = B.nx, ny = B.ny, nz = B.nz, per = B.per;
    for (int t = t0 + (int)threadIdx.x; t < t1; t += kCoupleThreads) {
        int i, j, k;
        map_cell(m, t, i, j, k);
        const int c = i + nx * (j + ny * k);
        if (c < 0 || c >= B.N) continue;
        const uint8_t old = B.flags[c] & kOwnerMask;
        int owner = 0;
        for (int b = nb - 1; b >= 0; --b) {
            double r[3];
            int d[3];
            lever_arm(sh.body[b], i, j, k, nx, ny, nz, per, r, d);
            if (inside(sh.body[b], r)) owner = b + 1;
        }
        B.old_owner[c] = old;
        B.flags[c] = (uint8_t)owner;
        if (old != owner) atomicAdd(&((CoupleCtl *)B.ctl)->owner_changes, 1u);
    }
}

// this thread's part of the margin of body b over the slice: the smallest
// distance of a scanned cell centre from the body's surface; until the body
// has moved that far no cell changes side
__device__ __forceinline__ double map_margin(const BoxDesc &B, const DevBody &bd, const MapBox &m, int t0, int t1) {
    double mm = 1e300;
    for (int t = t0 + (int)threadIdx.x; t < t1; t += kCoupleThreads) {
        int i, j, k;
        map_cell(m, t, i, j, k);
        double r[3];
        int d[3];
        lever_arm(bd, i, j, k, B.nx, B.ny, B.nz, B.per, r, d);
        mm = fmin(mm, surface_dist(bd, r));
    }
    return mm;
}

// Equilibrium deviation of direction a at density 1 + drho and velocity u
// (the refill of a cell that left a body), rounding spelled out so that
// every mapping gives the same bits.
__device__ __forceinline__ double refill_value(int a, double drho, double rho, const double u[3]) {
#pragma clang fp contract(off)
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double eu = ex(a) * u[0] + ey(a) * u[1] + ez(a) * u[2];
    return wgt(a) * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
}

// pass 2: refill cells that left a body (equilibrium at the body's velocity,
// density averaged over neighbours that are fluid before and after); needs
// pass 1 done on the neighbours.  The cells to refill are gathered first;
// then one wave refills each, lane a loading the 19 populations of the
// neighbour in direction a, and lane q storing direction q.  The sums run in
// the order one thread would take (directions ascending), so the result
// does not depend on the gathering order.
template <typename S>
__device__ __forceinline__ void map_refill(const BoxDesc &B, CoupleShared &sh, const MapBox &m, int t0, int t1, int cur) {
    if (sh.swapped) return;   // map_swap_gather refilled
    const int nx = B.nx, ny = B.ny, nz = B.nz, per = B.per;
    void *popc = cur ? B.pop1 : B.pop0;
    const size_t stride = (size_t)B.stride;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int base = t0; base < t1; base += kCoupleThreads) {
        __syncthreads();
        if (threadIdx.x == 0) sh.rcount = 0;
        __syncthreads();
        const int t = base + (int)threadIdx.x;
        if (t < t1) {
            int i, j, k;
            map_cell(m, t, i, j, k);
            const int c = i + nx * (j + ny * k);
            if (c >= 0 && c < B.N && B.old_owner[c] != 0 && (B.flags[c] & kOwnerMask) == 0)
                sh.rlist[atomicAdd(&sh.rcount, 1)] = c;
        }
        __syncthreads();
        const int n = sh.rcount;
        for (int e = wave; e < n; e += kCoupleThreads / 64) {
            const int c = sh.rlist[e];
            const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
            double s = 0.0;
            int valid = 0;
            if (lane >= 1 && lane < 19) {
                int ti, tj, tk;
                if (neighbour_rt(lane, i, j, k, nx, ny, nz, per, ti, tj, tk)) {
                    const int nc = ti + nx * (tj + ny * tk);
                    if (B.old_owner[nc] == 0 && (B.flags[nc] & kOwnerMask) == 0) {
                        valid = 1;
                        double v[19];
#pragma unroll
                        for (int q = 0; q < 19; ++q) v[q] = load_dev<S>(popc, (size_t)q * stride + nc, B.inv_scale);
                        s = v[0];
#pragma unroll
                        for (int q = 1; q < 19; ++q) s = s + v[q];
                    }
                }
            }
            double total = 0.0;
            int count = 0;
            for (int a = 1; a < 19; ++a) {
                const double sa = __shfl(s, a, 64);
                if (__shfl(valid, a, 64)) {
                    total = total + sa;
                    ++count;
                }
            }
            const double drho = count ? total / (double)count : 0.0;
            const double rho = 1.0 + drho;
            const DevBody &bd = sh.body[B.old_owner[c] - 1];
            double r[3], u[3];
            int d[3];
            lever_arm(bd, i, j, k, nx, ny, nz, per, r, d);
            wall_velocity(bd, r, u);
            if (lane < 19) {
                const double v = refill_value(lane, drho, rho, u);
                Storage<S>::store((S *)popc, (size_t)lane * stride + c, (typename Storage<S>::C)v, B.scale);
            }
        }
    }
}

// Pass 2 in the swapped layout of in-place streaming (the populations
// before an odd step).  There f_b(x) sits at slot opp(b) of x - e_b when
// that neighbour is fluid, else at slot b of x, so a cell that changes side
// moves its neighbours' populations as well:
//   c uncovered (body -> fluid), x = c + e_b fluid before and after:
//     f_b(x) moves from slot b of x to slot opp(b) of c;
//   c covered (fluid -> body), x likewise:
//     f_b(x), which c pushed at the last step, moves from slot opp(b) of c to
//     slot b of x;
// and the refill of an uncovered cell goes to the slots its new neighbours
// give it.  Some of these stores land where other moves or refills read
// (the slot a move of c empties is where c's own refill of the opposite
// direction goes), so every value is read first and listed (gather, into
// the link-record scratch, which the momentum exchange has consumed by now),
// and the list is stored after a barrier (scatter); no two stores share a
// slot.  The values and the refill arithmetic are those of the own layout,
// so both layouts map bit for bit alike.
__device__ __forceinline__ bool in_map(const MapBox &m, int i, int j, int k) {
    return i >= m.lo[0] && i < m.lo[0] + m.bx && j >= m.lo[1] && j < m.lo[1] + m.by && k >= m.lo[2] &&
           m.bx > 0 && m.by > 0 && k < m.lo[2] + m.ncell / (m.bx * m.by);
}

// fluid before this mapping (old_owner is only written inside the box)
__device__ __forceinline__ bool fluid_before(const BoxDesc &B, const MapBox &m, int c, int i, int j, int k) {
    return in_map(m, i, j, k) ? B.old_owner[c] == 0 : (B.flags[c] & kOwnerMask) == 0;
}

// element of f_b(x) in the swapped layout; before == true: under the flags
// before this mapping, else under the new ones
__device__ __forceinline__ size_t swapped_slot(const BoxDesc &B, const MapBox &m, int b, int c, int i, int j, int k,
                                               bool before) {
    const size_t stride = (size_t)B.stride;
    if (b == 0) return (size_t)c;
    int ti, tj, tk;
    if (neighbour_rt(opp(b), i, j, k, B.nx, B.ny, B.nz, B.per, ti, tj, tk)) {
        const int s = ti + B.nx * (tj + B.ny * tk);
        const bool fl = before ? fluid_before(B, m, s, ti, tj, tk) : (B.flags[s] & kOwnerMask) == 0;
        if (fl) return (size_t)opp(b) * stride + (size_t)s;
    }
    return (size_t)b * stride + (size_t)c;
}

__device__ __forceinline__ void reloc_push(const BoxDesc &B, BoxDesc &Bg, CoupleCtl *ctl, size_t at, double v) {
    const unsigned e = atomicAdd(&ctl->reloc_count, 1u);
    if (e < 4u * (unsigned)B.link_cap) {
        RelocRec r;
        r.at = (long long)at;
        r.v = v;
        ((RelocRec *)B.link_rec)[e] = r;
    } else {
        Bg.status = -6;
    }
}

template <typename S>
__device__ __forceinline__ void map_swap_gather(const BoxDesc &B, BoxDesc &Bg, const CoupleShared &sh, const MapBox &m, int t0,
                                int t1, int cur, CoupleCtl *ctl) {
    const int nx = B.nx, ny = B.ny, nz = B.nz, per = B.per;
    const void *pop = cur ? B.pop1 : B.pop0;
    const size_t stride = (size_t)B.stride;
    for (int t = t0 + (int)threadIdx.x; t < t1; t += kCoupleThreads) {
        int i, j, k;
        map_cell(m, t, i, j, k);
        const int c = i + nx * (j + ny * k);
        if (c < 0 || c >= B.N) continue;
        const bool was = B.old_owner[c] == 0, is = (B.flags[c] & kOwnerMask) == 0;
        if (was == is) continue;
        // loops kept rolled: this runs only at remaps, and the coupling
        // kernel must stay within its registers
#pragma unroll 1
        for (int b = 1; b < 19; ++b) {
            int ti, tj, tk;
            if (!neighbour_rt(b, i, j, k, nx, ny, nz, per, ti, tj, tk)) continue;
            const int x = ti + nx * (tj + ny * tk);
            if (!fluid_before(B, m, x, ti, tj, tk) || (B.flags[x] & kOwnerMask) != 0) continue;
            const size_t from = is ? (size_t)b * stride + x : (size_t)opp(b) * stride + c;
            const size_t to = is ? (size_t)opp(b) * stride + c : (size_t)b * stride + x;
            reloc_push(B, Bg, ctl, to, load_dev<S>(pop, from, B.inv_scale));
        }
        if (!is) continue;
        // refill: density averaged over the neighbours that are fluid before
        // and after (each neighbour's populations summed in direction order,
        // the neighbours added in direction order), as in map_refill
        double total = 0.0;
        int count = 0;
#pragma unroll 1
        for (int a = 1; a < 19; ++a) {
            int ti, tj, tk;
            if (!neighbour_rt(a, i, j, k, nx, ny, nz, per, ti, tj, tk)) continue;
            const int nc = ti + nx * (tj + ny * tk);
            if (!fluid_before(B, m, nc, ti, tj, tk) || (B.flags[nc] & kOwnerMask) != 0) continue;
            double sum = load_dev<S>(pop, (size_t)nc, B.inv_scale);
#pragma unroll 1
            for (int q = 1; q < 19; ++q)
                sum = sum + load_dev<S>(pop, swapped_slot(B, m, q, nc, ti, tj, tk, true), B.inv_scale);
            total = total + sum;
            ++count;
        }
        const double drho = count ? total / (double)count : 0.0;
        const double rho = 1.0 + drho;
        const DevBody &bd = sh.body[B.old_owner[c] - 1];
        double r[3], u[3];
        int d[3];
        lever_arm(bd, i, j, k, nx, ny, nz, per, r, d);
        wall_velocity(bd, r, u);
#pragma unroll 1
        for (int a = 0; a < 19; ++a)
            reloc_push(B, Bg, ctl, swapped_slot(B, m, a, c, i, j, k, false), refill_value(a, drho, rho, u));
    }
}

// Store the listed values: workgroup `part` of `parts` takes one slice.
template <typename S>
__device__ __forceinline__ void map_swap_scatter(const BoxDesc &B, int cur, CoupleCtl *ctl, int part, int parts) {
    void *pop = cur ? B.pop1 : B.pop0;
    const int n = (int)min(__hip_atomic_load(&ctl->reloc_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                           4u * (unsigned)B.link_cap);
    const int chunk = (n + parts - 1) / parts;
    const int e0 = min(part * chunk, n), e1 = min(e0 + chunk, n);
    const RelocRec *list = (const RelocRec *)B.link_rec;
    const size_t lim = (size_t)19 * (size_t)B.stride;
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kCoupleThreads) {
        const RelocRec r = list[e];
        if (r.at >= 0 && (size_t)r.at < lim)
            Storage<S>::store((S *)pop, (size_t)r.at, (typename Storage<S>::C)r.v, B.scale);
    }
}

// pass 3: near-body marks and boundary links of the slice, in cell order,
// numbered from `first`; needs pass 1 done on the neighbours.  With
// write = false only counts.  Returns the number of links in the slice.
__device__ __forceinline__ int map_links(const BoxDesc &B, CoupleShared &sh, const MapBox &m, int t0, int t1, int first,
                         bool write) {
    const int nx = B.nx, ny = B.ny, nz = B.nz, per = B.per;
    int running = first;
    for (int base = t0; base < t1; base += kCoupleThreads) {
        const int t = base + (int)threadIdx.x;
        int c = -1, cnt = 0;
        unsigned mask = 0;
        Owners owners;
        if (t < t1) {
            int i, j, k;
            map_cell(m, t, i, j, k);
            c = i + nx * (j + ny * k);
            if (c < 0 || c >= B.N) c = -1;
            if (c >= 0 && (B.flags[c] & kOwnerMask) == 0) {
                // all 18 neighbour flags are loaded before any is used, so
                // that their latencies overlap (a missing neighbour reads the
                // cell itself and is masked out)
                int nidx[19];
                unsigned ok = 0;
#pragma unroll
                for (int a = 1; a < 19; ++a) {
                    int ti, tj, tk;
                    const bool in = neighbour_rt(a, i, j, k, nx, ny, nz, per, ti, tj, tk);
                    nidx[a] = in ? ti + nx * (tj + ny * tk) : c;
                    ok |= in ? 1u << a : 0u;
                }
                uint8_t nf[19];
#pragma unroll
                for (int a = 1; a < 19; ++a) nf[a] = B.flags[nidx[a]];
#pragma unroll
                for (int a = 1; a < 19; ++a) {
                    const int o = (ok >> a) & 1u ? nf[a] & kOwnerMask : 0;
                    owners.set(a, o);
                    if (o) {
                        mask |= 1u << a;
                        ++cnt;
                    }
                }
            }
        }
        int tot;
        const int off = running + block_scan(cnt, &tot, sh);
        if (write && c >= 0 && (B.flags[c] & kOwnerMask) == 0) {
            B.flags[c] = cnt ? kNearBit : 0;
            if (cnt) {
                B.link_base[c] = off;
                int l = off;
                for (unsigned m = mask; m; m &= m - 1) {
                    const int a = __builtin_ctz(m);
                    if (l < B.link_cap) {
                        B.link_cell[l] = c;
                        B.link_dir[l] = (signed char)a;
                        B.link_body[l] = (signed char)(owners.get(a) - 1);
                    }
                    ++l;
                }
            }
        }
        running += tot;
    }
    return running - first;
}

// The records of the momentum-exchange sums for the new links: one per wave
// of 64 consecutive cells and body that the wave's links reach, grouped by
// body and, within a body, in the order of the waves.  The link list is
// sorted by cell, so the links of a wave are contiguous; the q-th body (in
// ascending order) of the wave that starts at link l0 finds its record at
// grp_pos[l0 + q] (q is smaller than the wave's link count, so these slots
// are the wave's own).  Thread t takes a contiguous range of links and the
// waves that start in it; one block scan per body numbers the records.
// Needs the whole link list written.
__device__ __forceinline__ void map_groups(const BoxDesc &B, BoxDesc &Bg, CoupleShared &sh, int L) {
    const int t = (int)threadIdx.x;
    const int chunk = (L + kCoupleThreads - 1) / kCoupleThreads;
    const int l0 = min(t * chunk, L), l1 = min(l0 + chunk, L);
    // The link lists were written by other workgroups just before, so the
    // loops read eight links at a time, with the loads in flight together.
    // Calls f(l, w) for every link l of [l0, l1), w its wave, and whether it
    // starts its wave.
    auto for_links = [&](auto f) {
        int prev = l0 > 0 ? B.link_cell[l0 - 1] >> 6 : -1;
        for (int q = l0; q < l1; q += 8) {
            int cw[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) cw[u] = q + u < l1 ? B.link_cell[q + u] >> 6 : -1;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (q + u < l1) f(q + u, cw[u], cw[u] != prev);
                prev = cw[u];
            }
        }
    };
    // 1. Every thread ORs the bodies of its links run by run (a run: the links
    // of one wave within the thread's range).  The mask of a run that starts
    // its wave goes to the wave's first link in the scratch words (the link
    // records are free during a mapping); the first run, if it continues a
    // wave from the threads before, is published in the LDS (hw, hm) for the
    // thread that holds the wave's start, with whether it fills the range.
    unsigned *wmask = (unsigned *)B.link_rec;
    int *hw = sh.rlist;                      // wave of the first run, -1 if none
    unsigned *hm = (unsigned *)sh.red;       // its mask; [kCoupleThreads + t]: it fills the range
    int run_start = -1, run_w = -1, first_w = -1;
    unsigned run_m = 0u, first_m = 0u;
    bool first_open = true;                  // still in the first run
    for_links([&](int l, int w, bool starts) {
        if (l > l0 && w != run_w) {          // a run ends
            if (run_start >= 0) wmask[run_start] = run_m;
            else if (first_open) first_m = run_m;
            first_open = false;
            run_m = 0u;
            run_start = -1;
        }
        if (l == l0) first_w = starts ? -1 : w;
        if (starts) run_start = l;
        run_w = w;
        run_m |= 1u << B.link_body[l];
    });
    const bool open_end = l1 > l0 && run_start >= 0;   // the last run starts a wave that may go on
    if (l1 > l0 && run_start < 0 && first_open) first_m = run_m;
    hw[t] = first_w;
    hm[t] = first_m;
    hm[kCoupleThreads + t] = (l1 > l0 && first_open && first_w >= 0) ? 1u : 0u;
    __syncthreads();
    // 2. The last run of a thread may start a wave that the next threads go on
    // with: add their first runs while they belong to it.
    if (open_end) {
        unsigned m = run_m;
        for (int k = t + 1; k < kCoupleThreads && hw[k] == run_w; ++k) {
            m |= hm[k];
            if (!hm[kCoupleThreads + k]) break;
        }
        wmask[run_start] = m;
    }
    __threadfence_block();
    __syncthreads();
    // 3. Number the records body by body, in the order of the waves: one block
    // scan per body; the q-th body of a wave takes the wave's slot l + q.
    unsigned seen = 0;   // bodies with a record here
    for_links([&](int l, int, bool starts) {
        if (starts) seen |= wmask[l];
    });
    int off = 0;   // records of the bodies before b
    for (int b = 0; b < B.nb; ++b) {
        int mine = 0;
        if (seen & (1u << b))
            for_links([&](int l, int, bool starts) {
                if (starts) mine += (wmask[l] >> b) & 1u;
            });
        int total;
        int next = off + block_scan(mine, &total, sh);
        if (seen & (1u << b))
            for_links([&](int l, int, bool starts) {
                if (!starts) return;
                const unsigned m = wmask[l];
                if ((m >> b) & 1u) B.grp_pos[l + __popc(m & ((1u << b) - 1u))] = next++;
            });
        if (threadIdx.x == 0) Bg.rec_off[b] = off;
        off += total;
    }
    if (threadIdx.x == 0)
        for (int b = B.nb; b <= kMaxBodies; ++b) Bg.rec_off[b] = off;
}

// Record the positions and orientations the mapping used (the remap skip
// measures motion from them).
__device__ __forceinline__ void map_record(const BoxDesc &B, const CoupleShared &sh, double *qmaps) {
    const int b = threadIdx.x;
    if (b < B.nb) {
        for (int q = 0; q < 3; ++q) B.bodies[b].Xmap[q] = sh.body[b].anchor[q] + sh.body[b].D[q];
        for (int q = 0; q < 4; ++q) qmaps[4 * b + q] = sh.body[b].q[q];
    }
}

// The whole mapping by one workgroup.
template <typename S>
__device__ __forceinline__ void remap_box(const BoxDesc &B, BoxDesc &Bg, CoupleShared &sh, double *qmaps, double *margins) {
    const MapBox m = map_box(sh);
    CoupleCtl *ctl = (CoupleCtl *)B.ctl;
    if (threadIdx.x == 0) ctl->reloc_count = 0u;
    map_owners(B, sh, m, 0, m.ncell);
    for (int b = 0; b < B.nb; ++b) {
        const double mm = block_min(map_margin(B, sh.body[b], m, 0, m.ncell), sh);
        if (threadIdx.x == 0) margins[b] = mm;
    }
    map_record(B, sh, qmaps);
    __threadfence();
    __syncthreads();
    if (sh.swapped) {
        map_swap_gather<S>(B, Bg, sh, m, 0, m.ncell, sh.cur, ctl);
        __threadfence();
        __syncthreads();
        map_swap_scatter<S>(B, sh.cur, ctl, 0, 1);
    }
    map_refill<S>(B, sh, m, 0, m.ncell, sh.cur);   // nothing to do in the swapped layout
    __threadfence_block();
    __syncthreads();
    const int total = map_links(B, sh, m, 0, m.ncell, 0, true);
    if (threadIdx.x == 0) {
        Bg.link_count = total;
        if (total > B.link_cap) Bg.status = -6;
    }
    __threadfence_block();
    __syncthreads();
    map_groups(B, Bg, sh, min(total, B.link_cap));
}

// Barrier over the kRedBlocks workgroups of one box.  A cooperative launch
// is only made when every workgroup of it can be resident at once; the wait
// is bounded all the same, so that a workgroup never waits for ever: on
// time-out the box is marked failed (status -7) and the kernel drains.
// Waiting workgroups poll with plain device-coherent loads and take one
// acquire fence at the end: an acquire on every poll would invalidate their
// L2 over and over, slowing the workgroup that everyone waits for.
__device__ __forceinline__ bool box_barrier(CoupleCtl *ctl, CoupleShared &sh, BoxDesc &Bg) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this thread's stores visible device-wide
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned g = __hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned a = __hip_atomic_fetch_add(&ctl->arrived, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        if (a == kRedBlocks - 1) {
            __hip_atomic_store(&ctl->arrived, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            int spins = 0;
            while (__hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (++spins > kSpinLimit) {
                    ok = 0;
                    __hip_atomic_store(&Bg.status, -7, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        sh.sync_ok = ok;
    }
    __syncthreads();
    return sh.sync_ok != 0;
}

// Joining a shared remap.  The box's other workgroups join this launch's
// join word; the first workgroup, once it has published its decision, answers
// kJoinGo when all of them have joined (they are then all resident, and the
// remap's barriers can rely on it), or kJoinAbort when it maps alone: when
// there is nothing to map (solo), or when they have not all joined within
// kJoinLimit polls because some are not resident (other work on the device,
// a launch larger than the device holds).  After kJoinAbort every other
// workgroup, joined or not, leaves, and the first one maps by itself, with
// the same results.  A joined workgroup that has waited kSpinLimit polls for
// the answer withdraws, unless the answer came meanwhile.  Workgroups are
// dispatched in order, so the first workgroup of a box is running whenever
// one of the others is.  Returns true if this workgroup takes part in a
// shared remap.
__device__ __forceinline__ bool join_remap(CoupleCtl *ctl, CoupleShared &sh, int parity, bool lead, bool solo) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the decision, visible device-wide
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned *J = &ctl->join[parity];
        int go = 0;
        if (lead) {
            for (int spins = 0;;) {
                const unsigned j = __hip_atomic_load(J, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const bool all = (j & 0xffffu) == (unsigned)(kRedBlocks - 1);
                if (!solo && !all && spins < kJoinLimit) {
                    ++spins;
                    __builtin_amdgcn_s_sleep(4);
                    continue;
                }
                const unsigned answer = !solo && all ? kJoinGo : kJoinAbort;
                unsigned e = j;
                if (__hip_atomic_compare_exchange_strong(J, &e, j | answer, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)) {
                    go = answer == kJoinGo;
                    break;
                }
            }
        } else {
            bool joined = false;
            for (;;) {
                const unsigned j = __hip_atomic_load(J, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (j & kJoinAbort) break;                          // too late: the first maps alone
                unsigned e = j;
                if (__hip_atomic_compare_exchange_strong(J, &e, j + 1u, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)) {
                    joined = true;
                    break;
                }
            }
            for (int spins = 0; joined;) {
                const unsigned j = __hip_atomic_load(J, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (j & kJoinGo) {
                    go = 1;
                    break;
                }
                if (j & kJoinAbort) break;
                if (spins >= kSpinLimit) {
                    unsigned e = j;                                 // withdraw
                    if (__hip_atomic_compare_exchange_strong(J, &e, j - 1u, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT))
                        break;
                    continue;
                }
                ++spins;
                __builtin_amdgcn_s_sleep(4);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        sh.sync_ok = go;
    }
    __syncthreads();
    return sh.sync_ok != 0;
}

// The whole mapping by the kRedBlocks workgroups of a box, r being this
// one's rank: one contiguous slice of the cell range each, with a barrier
// where a pass needs its neighbours' results.  The link count of every
// slice goes through the control block, so that each slice numbers its
// links from the sum of the counts before it: the list comes out in the same
// cell order, and every result bit for bit the same, as with one workgroup.
template <typename S>
__device__ __forceinline__ void remap_coop(const BoxDesc &B, BoxDesc &Bg, CoupleShared &sh, CoupleCtl *ctl, int r, double *qmaps,
                           double *margins) {
    const MapBox m = map_box(sh);
    const int chunk = (m.ncell + kRedBlocks - 1) / kRedBlocks;
    const int t0 = min(r * chunk, m.ncell), t1 = min(t0 + chunk, m.ncell);
    map_owners(B, sh, m, t0, t1);
    for (int b = 0; b < B.nb; ++b) {
        // non-negative doubles order like their bit patterns
        double mm = map_margin(B, sh.body[b], m, t0, t1);
        for (int o = 32; o > 0; o >>= 1) mm = fmin(mm, __shfl_xor(mm, o, 64));
        if ((threadIdx.x & 63) == 0)
            atomicMin(&ctl->margin[b], (unsigned long long)__double_as_longlong(mm));
    }
    if (!box_barrier(ctl, sh, Bg)) return;
    if (r == 0) map_record(B, sh, qmaps);
    if (r == 0 && (int)threadIdx.x < B.nb)
        margins[threadIdx.x] = __longlong_as_double(
            (long long)__hip_atomic_load(&ctl->margin[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (sh.swapped) {
        map_swap_gather<S>(B, Bg, sh, m, t0, t1, sh.cur, ctl);
        if (!box_barrier(ctl, sh, Bg)) return;
        map_swap_scatter<S>(B, sh.cur, ctl, r, kRedBlocks);
    }
    map_refill<S>(B, sh, m, t0, t1, sh.cur);   // nothing to do in the swapped layout
    const int mine = map_links(B, sh, m, t0, t1, 0, false);
    if (threadIdx.x == 0) __hip_atomic_store(&ctl->counts[r], mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!box_barrier(ctl, sh, Bg)) return;
    if (threadIdx.x == 0) {
        int first = 0, total = 0;
        for (int q = 0; q < kRedBlocks; ++q) {
            const int n = __hip_atomic_load(&ctl->counts[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (q < r) first += n;
            total += n;
        }
        sh.first = first;
        sh.ltotal = total;
        if (r == kRedBlocks - 1) {
            Bg.link_count = total;
            if (total > B.link_cap) Bg.status = -6;
        }
    }
    __syncthreads();
    map_links(B, sh, m, t0, t1, sh.first, true);
    // the records of the next momentum-exchange sums need every slice's links
    if (!box_barrier(ctl, sh, Bg)) return;
    if (r == 0) map_groups(B, Bg, sh, min(sh.ltotal, B.link_cap));
}


// Copy n 32-bit words from src to dst with the whole workgroup.
__device__ __forceinline__ void copy_words(void *dst, const void *src, int bytes) {
    const int n = bytes / 4;
    for (int t = threadIdx.x; t < n; t += kCoupleThreads) ((int *)dst)[t] = ((const int *)src)[t];
}

// Stage the box's small tables in LDS.  Each thread first loads its words of
// all five tables into registers (stage_load: the loads of every table are
// in flight together, and other work, the momentum-exchange sums, can be
// issued before they return), then stores them (stage_store).
constexpr int kStageWords = 8;
static_assert(kStageWords * kCoupleThreads >=
                  (int)(sizeof(DevBody) * kMaxBodies + sizeof(DevSpring) * kMaxSprings +
                        sizeof(DevDrive) * kMaxDrives) / 4 + 10 * kMaxBodies,
              "every word of the tables must have a thread");

struct Staged {
    int w[kStageWords];
};

template <bool LOAD>
__device__ __forceinline__ void stage_words(const BoxDesc &B, CoupleShared &sh, const double *qmaps,
                                            const double *margins, Staged &st) {
    const int n0 = (int)sizeof(DevBody) * B.nb / 4, n1 = (int)sizeof(DevSpring) * B.ns / 4;
    const int n2 = (int)sizeof(DevDrive) * B.nd / 4, n3 = 2 * B.nb, n4 = 8 * B.nb;
    const int total = n0 + n1 + n2 + n3 + n4;
#pragma unroll
    for (int k = 0; k < kStageWords; ++k) {
        const int t = (int)threadIdx.x + k * kCoupleThreads;
        if (t >= total) continue;
        int w = t;
        const int *src;
        int *dst;
        if (w < n0) {
            src = (const int *)B.bodies;
            dst = (int *)sh.body;
        } else if ((w -= n0) < n1) {
            src = (const int *)B.springs;
            dst = (int *)sh.spring;
        } else if ((w -= n1) < n2) {
            src = (const int *)B.drives;
            dst = (int *)sh.drive;
        } else if ((w -= n2) < n3) {
            src = (const int *)margins;
            dst = (int *)sh.margin;
        } else {
            w -= n3;
            src = (const int *)qmaps;
            dst = (int *)sh.qmap;
        }
        if constexpr (LOAD) st.w[k] = src[w];
        else dst[w] = st.w[k];
    }
}

__device__ __forceinline__ void stage_load(const BoxDesc &B, CoupleShared &sh, const double *qmaps,
                                           const double *margins, Staged &st) {
    stage_words<true>(B, sh, qmaps, margins, st);
}

__device__ __forceinline__ void stage_store(const BoxDesc &B, CoupleShared &sh, const double *qmaps,
                                            const double *margins, Staged &st) {
    stage_words<false>(B, sh, qmaps, margins, st);
    __syncthreads();
}

__device__ __forceinline__ void stage_out(const BoxDesc &B, CoupleShared &sh) {
    __syncthreads();
    copy_words(B.bodies, sh.body, (int)sizeof(DevBody) * B.nb);
    __threadfence_block();
    __syncthreads();
}

template <typename S>
__global__ __launch_bounds__(kCoupleThreads) void couple_kernel(BoxDesc *boxes, const int *active,
                                                                double *qmaps, double *margins,
                                                                int mode, int force_map, int coop) {
    __shared__ CoupleShared sh;
    // active == null: every box of the context takes part, in order
    const int bi = active ? active[blockIdx.x / kRedBlocks] : (int)(blockIdx.x / kRedBlocks);
    const int r = blockIdx.x % kRedBlocks;
    BoxDesc &Bg = boxes[bi];
    // snapshot of the descriptor, taken before this kernel stores into it, so
    // that no later read has to wait for those stores
    const BoxDesc B = Bg;
    CoupleCtl *ctl = (CoupleCtl *)B.ctl;
    double *qm = qmaps + (size_t)bi * 4 * kMaxBodies;
    double *mg = margins + (size_t)bi * kMaxBodies;
    // the box's other workgroups stay to share a remap only if the previous
    // launch found that one may come (a remap it did not foresee is done by
    // the first workgroup alone).  The hint is kept per launch parity, and
    // the parity is counted by the workgroups themselves, so that every
    // workgroup of a launch reads the same hint however late it starts: the
    // first workgroup writes the next launch's hint while others of this
    // launch may still be about to read theirs.
    // One thread per workgroup counts and reads; the whole workgroup must
    // take the same decision.  The other workgroups need the answer at once
    // (they stay only for a shared remap); the first one only after the step,
    // so there the count is taken by a thread of the last wave and stays in
    // flight while the workgroup stages the tables and sums the records.
    const bool lead = r == 0;
    const int counter = lead ? kCoupleThreads - 64 : 0;
    int h0 = 0, h1 = 0;
    unsigned arrival = 0u;
    if ((int)threadIdx.x == counter) {
        // both hints are read while the count is in flight
        h0 = __hip_atomic_load(&ctl->share[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        h1 = __hip_atomic_load(&ctl->share[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        arrival = __hip_atomic_fetch_add(&ctl->launches, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!lead) {
        if (threadIdx.x == 0) {
            sh.parity = (int)((arrival / kRedBlocks) & 1u);
            sh.hint = sh.parity ? h1 : h0;
        }
        __syncthreads();
        if (!(coop && (mode == kModeMapOnly || force_map || sh.hint != 0))) return;
    }
    if (lead) {
        if (threadIdx.x == 0) {
            sh.cur = B.cur;
            // in-place streaming: the layout the mapping sees is that of the
            // next step, n + 1 after a step
            sh.swapped = B.aa && ((B.step + (mode == kModeStep ? 1 : 0)) & 1) != 0;
        }
        Staged st;
        stage_load(B, sh, qm, mg, st);
        if (mode == kModeStep) sum_records(B, sh);
        stage_store(B, sh, qm, mg, st);
        if (mode == kModeStep) {
            rigid_step<true>(B, Bg, sh);
        }
    }
    if (lead) {
        if ((int)threadIdx.x == counter) {
            sh.parity = (int)((arrival / kRedBlocks) & 1u);
            sh.hint = sh.parity ? h1 : h0;
        }
        if (threadIdx.x < 64) decide_map(B, Bg, sh, force_map || mode == kModeMapOnly);
        stage_out(B, sh);   // begins with a barrier: sh.parity and sh.hint are set
    }
    const int parity = sh.parity;
    const bool share = coop && (mode == kModeMapOnly || force_map || sh.hint != 0);
    if (lead) {
        if (threadIdx.x == 0) {
            __hip_atomic_store(&ctl->share[parity ^ 1], sh.share_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // the next launch's join word (the launch that used it last has ended)
            __hip_atomic_store(&ctl->join[parity ^ 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!share) {
            if (sh.map_req) remap_box<S>(B, Bg, sh, qm, mg);
            return;
        }
        // hand the decision to the box's other workgroups
        if (threadIdx.x == 0) {
            ctl->map_req = sh.map_req;
            ctl->cur = sh.cur;
            ctl->swapped = sh.swapped;
            ctl->reloc_count = 0u;
            for (int q = 0; q < 3; ++q) {
                ctl->lo[q] = sh.lo[q];
                ctl->hi[q] = sh.hi[q];
            }
        }
        if (sh.map_req && (int)threadIdx.x < B.nb)
            ctl->margin[threadIdx.x] = (unsigned long long)__double_as_longlong(1e300);
    }
    // the first workgroup maps alone when nothing is to be mapped, or, with
    // coop == 2 (a test of this path), always
    if (!join_remap(ctl, sh, parity, lead, lead && (!sh.map_req || coop == 2))) {
        if (lead && sh.map_req) remap_box<S>(B, Bg, sh, qm, mg);
        return;
    }
    if (threadIdx.x == 0) {
        sh.map_req = __hip_atomic_load(&ctl->map_req, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sh.cur = __hip_atomic_load(&ctl->cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sh.swapped = __hip_atomic_load(&ctl->swapped, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int q = 0; q < 3; ++q) {
            sh.lo[q] = __hip_atomic_load(&ctl->lo[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh.hi[q] = __hip_atomic_load(&ctl->hi[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    if (!sh.map_req) return;
    if (!lead) copy_words(sh.body, B.bodies, (int)sizeof(DevBody) * B.nb);   // the bodies' new states
    __syncthreads();
    remap_coop<S>(B, Bg, sh, ctl, r, qm, mg);
}

// Integrator-only runs (Sec. 4: the swimmer in vacuum).  One workgroup per
// system advances it nsteps steps with the rigid-body step of couple_kernel
// (driving, springs, integration, trajectory record); with no fluid the
// hydrodynamic force and torque are zero.
__global__ __launch_bounds__(kCoupleThreads) void vacuum_kernel(BoxDesc *systems, long long nsteps) {
    __shared__ CoupleShared sh;
    BoxDesc &Bg = systems[blockIdx.x];
    BoxDesc B = Bg;
    copy_words(sh.body, B.bodies, (int)sizeof(DevBody) * B.nb);
    copy_words(sh.spring, B.springs, (int)sizeof(DevSpring) * B.ns);
    copy_words(sh.drive, B.drives, (int)sizeof(DevDrive) * B.nd);
    for (int t = threadIdx.x; t < kMaxBodies * 3; t += kCoupleThreads) {
        sh.F[t / 3][t % 3] = 0.0;
        sh.T[t / 3][t % 3] = 0.0;
    }
    if (threadIdx.x == 0) sh.cur = B.cur;
    __syncthreads();
    for (long long s = 0; s < nsteps; ++s) {
        rigid_step<false>(B, Bg, sh);
        B.step += 1;
    }
    stage_out(B, sh);
}

}  // namespace lbm
