// Per-box coupling kernel, one workgroup per box, run after each sweep:
//   1. momentum-exchange force and torque of every body (Eq. hydroF), summed
//      in a fixed order (deterministic), with the geometric part 2 w e of the
//      link term accumulated exactly in integers;
//   2. driving forces (Eqs. FB1-FB3), spring-damper forces (Eqs. osci_i/j)
//      and one semi-implicit Euler step of every body (Alg. 1);
//   3. the object mapping of the next step (Sec. 2.3): new flags, refill of
//      uncovered cells, near-body marks and the boundary-link list, skipped
//      when no cell can have changed side since the last mapping.
#pragma once
#include "geometry.h"

namespace lbm {

constexpr int kCoupleThreads = 256;
constexpr int kMaxBodies = 16;
constexpr double kMarginSafety = 1e-9;

enum : int { kModeStep = 0, kModeMapOnly = 1 };

struct CoupleShared {
    double red[kCoupleThreads];
    long long ired[kCoupleThreads];
    int scan[kCoupleThreads];
    double F[kMaxBodies][3], T[kMaxBodies][3];
    int lo[3], hi[3];
    int do_map;
    int cur;                   // index of the current population buffer
};

__device__ __forceinline__ double block_sum(double v, CoupleShared &sh) {
    const int t = threadIdx.x;
    __syncthreads();
    sh.red[t] = v;
    __syncthreads();
    for (int s = kCoupleThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh.red[t] = sh.red[t] + sh.red[t + s];
        __syncthreads();
    }
    return sh.red[0];
}

__device__ __forceinline__ long long block_sum_i(long long v, CoupleShared &sh) {
    const int t = threadIdx.x;
    __syncthreads();
    sh.ired[t] = v;
    __syncthreads();
    for (int s = kCoupleThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh.ired[t] += sh.ired[t + s];
        __syncthreads();
    }
    return sh.ired[0];
}

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
// 1. momentum exchange
// ---------------------------------------------------------------------------
__device__ void momentum_exchange(BoxDesc &B, CoupleShared &sh) {
    const int L = min(B.link_count, B.link_cap);
    for (int b = 0; b < B.nb; ++b) {
        const DevBody &bd = B.bodies[b];
        double acc[6] = {0, 0, 0, 0, 0, 0};
        long long g[3] = {0, 0, 0}, s[3] = {0, 0, 0};
        for (int l = threadIdx.x; l < L; l += kCoupleThreads) {
            if (B.link_body[l] != b) continue;
            const int c = B.link_cell[l];
            const int a = B.link_dir[l];
            int i, j, k, ti, tj, tk;
            decode_cell(c, B.nx, B.ny, i, j, k);
            neighbour_rt(a, i, j, k, B.nx, B.ny, B.nz, B.per, ti, tj, tk);
            double r[3], u[3];
            int d[3];
            lever_arm(bd, ti, tj, tk, B.nx, B.ny, B.nz, B.per, r, d);
            wall_velocity(bd, r, u);
            const int ea[3] = {ex(a), ey(a), ez(a)};
            // e_opp . u = -(e_a . u)
            const double eu = -((double)ea[0] * u[0] + (double)ea[1] * u[1] + (double)ea[2] * u[2]);
            const double2 v = B.link_val[l];
            const double sc = 2.0 * v.x + 6.0 * wgt(a) * v.y * eu;
            const double term[3] = {ea[0] * sc, ea[1] * sc, ea[2] * sc};
            acc[0] += term[0];
            acc[1] += term[1];
            acc[2] += term[2];
            acc[3] += r[1] * term[2] - r[2] * term[1];
            acc[4] += r[2] * term[0] - r[0] * term[2];
            acc[5] += r[0] * term[1] - r[1] * term[0];
            const int cw = two_w36(a);
            const long long ec[3] = {(long long)ea[0] * cw, (long long)ea[1] * cw, (long long)ea[2] * cw};
            const long long dd[3] = {2LL * d[0] + 1, 2LL * d[1] + 1, 2LL * d[2] + 1};
            g[0] += ec[0];
            g[1] += ec[1];
            g[2] += ec[2];
            s[0] += dd[1] * ec[2] - dd[2] * ec[1];
            s[1] += dd[2] * ec[0] - dd[0] * ec[2];
            s[2] += dd[0] * ec[1] - dd[1] * ec[0];
        }
        double tot[6];
        long long gt[3], st[3];
        for (int q = 0; q < 6; ++q) tot[q] = block_sum(acc[q], sh);
        for (int q = 0; q < 3; ++q) gt[q] = block_sum_i(g[q], sh);
        for (int q = 0; q < 3; ++q) st[q] = block_sum_i(s[q], sh);
        if (threadIdx.x == 0) {
#pragma clang fp contract(off)
            double G[3], fp[3];
            for (int q = 0; q < 3; ++q) {
                G[q] = (double)gt[q] / 36.0;
                double X = bd.anchor[q] + bd.D[q];
                fp[q] = X - floor(X);
            }
            const double Tg[3] = {(double)st[0] / 72.0 - (fp[1] * G[2] - fp[2] * G[1]),
                                  (double)st[1] / 72.0 - (fp[2] * G[0] - fp[0] * G[2]),
                                  (double)st[2] / 72.0 - (fp[0] * G[1] - fp[1] * G[0])};
            for (int q = 0; q < 3; ++q) {
                sh.F[b][q] = tot[q] + G[q];
                sh.T[b][q] = tot[3 + q] + Tg[q];
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// 2. rigid bodies (single thread; a handful of bodies)
// ---------------------------------------------------------------------------
__device__ void rigid_step(BoxDesc &B, CoupleShared &sh) {
    const int nb = B.nb;
    const long long n = B.step;
    double Fd[kMaxBodies][3], Fs[kMaxBodies][3];
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < 3; ++q) Fd[b][q] = Fs[b][q] = 0.0;
    // driving, Eqs. FB1-FB3 (delayed right force)
    for (int e = 0; e < B.nd; ++e) {
        const DevDrive &dv = B.drives[e];
        const double om = 2.0 * M_PI / dv.period;
        double fl = -dv.amplitude * sin(om * (double)n);
        double fr = dv.amplitude * sin(om * (double)n - dv.phase_lag);
        if (dv.gate && om * (double)n < dv.phase_lag) fr = 0.0;
        if (dv.off_left >= 0 && n >= dv.off_left) fl = 0.0;
        if (dv.off_right >= 0 && n >= dv.off_right) fr = 0.0;
        const double fm = -(fl + fr);
        Fd[dv.left][0] += fl;
        Fd[dv.right][0] += fr;
        Fd[dv.middle][0] += fm;
    }
    // springs, Eqs. spring_i, damp_i, osci_i/j
    for (int e = 0; e < B.ns; ++e) {
        const DevSpring &sp = B.springs[e];
        const DevBody &bi = B.bodies[sp.i];
        const DevBody &bj = B.bodies[sp.j];
        double d[3];
        for (int q = 0; q < 3; ++q) d[q] = (bi.anchor[q] - bj.anchor[q]) + (bi.D[q] - bj.D[q]);
        const double ell = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double coef = -sp.k * (ell - sp.rest_len) / ell;
        for (int q = 0; q < 3; ++q) {
            const double f = coef * d[q] - sp.gamma * (bi.V[q] - bj.V[q]);
            Fs[sp.i][q] += f;
            Fs[sp.j][q] -= f;
        }
    }
    bool bad = false;
    for (int b = 0; b < nb; ++b) {
        DevBody &bd = B.bodies[b];
        for (int q = 0; q < 3; ++q) {
            bd.F[q] = sh.F[b][q];
            bd.T[q] = sh.T[b][q];
        }
        if (!bd.kinematic) {
            const double m = bd.mass;
            for (int q = 0; q < 3; ++q) bd.V[q] = bd.V[q] + ((sh.F[b][q] + Fd[b][q]) + Fs[b][q]) / m;
            // Omega += R diag(1/I) R^T T
            const double w = bd.q[0], x = bd.q[1], y = bd.q[2], z = bd.q[3];
            const double R[3][3] = {
                {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
            double bt[3];
            for (int p = 0; p < 3; ++p)
                bt[p] = (R[0][p] * sh.T[b][0] + R[1][p] * sh.T[b][1] + R[2][p] * sh.T[b][2]) / bd.inertia[p];
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
        for (int q = 0; q < 3; ++q)
            if (!isfinite(bd.F[q]) || !isfinite(bd.T[q]) || !isfinite(bd.V[q]) || !isfinite(bd.D[q])) bad = true;
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
    if (bad) B.status = -4;
    B.step = n + 1;
}

// ---------------------------------------------------------------------------
// 3. object mapping
// ---------------------------------------------------------------------------
__device__ __forceinline__ double body_extent(const DevBody &b) {
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
    if (b.shape == kBodyShapeCapsule) {
        // rotation angle between q and qmap: 2 atan2(|v|, |w|) of q * conj(qmap)
        const double *p = b.q;
        const double w = p[0] * qmap[0] + p[1] * qmap[1] + p[2] * qmap[2] + p[3] * qmap[3];
        const double vx = -p[0] * qmap[1] + p[1] * qmap[0] - p[2] * qmap[3] + p[3] * qmap[2];
        const double vy = -p[0] * qmap[2] + p[2] * qmap[0] - p[3] * qmap[1] + p[1] * qmap[3];
        const double vz = -p[0] * qmap[3] + p[3] * qmap[0] - p[1] * qmap[2] + p[2] * qmap[1];
        const double ang = 2.0 * atan2(sqrt(vx * vx + vy * vy + vz * vz), fabs(w));
        bound += ang * (b.half_len + b.radius + 2.0);
    }
    return bound;
}

template <typename S>
__device__ void remap(BoxDesc &B, CoupleShared &sh, double *qmaps, double *margins, bool force) {
    const int nb = B.nb;
    if (threadIdx.x == 0) {
        // A body whose position is no longer finite cannot be mapped: report
        // the box as unstable and leave the flags as they are.
        bool finite = true;
        for (int b = 0; b < nb; ++b)
            for (int q = 0; q < 3; ++q) {
                const DevBody &bd = B.bodies[b];
                if (!isfinite(bd.anchor[q] + bd.D[q]) || !isfinite(bd.Xmap[q])) finite = false;
            }
        int need = force ? 1 : 0;
        for (int b = 0; b < nb && !need; ++b)
            if (!(moved_bound(B.bodies[b], qmaps + 4 * b) < margins[b] - kMarginSafety)) need = 1;
        if (!finite) {
            need = 0;
            B.status = -4;
        }
        sh.do_map = need;
        if (need) {
            const int n[3] = {B.nx, B.ny, B.nz};
            for (int q = 0; q < 3; ++q) {
                double lo = 1e300, hi = -1e300;
                for (int b = 0; b < nb; ++b) {
                    const DevBody &bd = B.bodies[b];
                    const double X = bd.anchor[q] + bd.D[q];
                    const double e = body_extent(bd);
                    lo = fmin(lo, fmin(X, bd.Xmap[q]) - e);
                    hi = fmax(hi, fmax(X, bd.Xmap[q]) + e);
                }
                // clamp in double before converting, so that no integer overflows
                lo = fmin(fmax(floor(lo) - 2.0, -4.0), (double)n[q] + 4.0);
                hi = fmin(fmax(floor(hi) + 2.0, -4.0), (double)n[q] + 4.0);
                int l = (int)lo, h = (int)hi;
                if (nb == 0) { l = 0; h = -1; }
                if (B.per & (1 << q)) {
                    if (l < 0 || h >= n[q] || h - l + 1 >= n[q]) { l = 0; h = n[q] - 1; }
                } else {
                    l = max(l, 0);
                    h = min(h, n[q] - 1);
                }
                sh.lo[q] = l;
                sh.hi[q] = h;
            }
        }
    }
    __syncthreads();
    if (!sh.do_map) return;
    const int bx = sh.hi[0] - sh.lo[0] + 1, by = sh.hi[1] - sh.lo[1] + 1, bz = sh.hi[2] - sh.lo[2] + 1;
    const int ncell = (bx > 0 && by > 0 && bz > 0) ? bx * by * bz : 0;
    const int nx = B.nx, ny = B.ny, nz = B.nz, per = B.per;
    // pass 1: new owners; remember the old ones; margin of every body
    double marg[kMaxBodies];
    for (int b = 0; b < nb; ++b) marg[b] = 1e300;
    for (int t = threadIdx.x; t < ncell; t += kCoupleThreads) {
        const int i = sh.lo[0] + t % bx, j = sh.lo[1] + (t / bx) % by, k = sh.lo[2] + t / (bx * by);
        const int c = i + nx * (j + ny * k);
        if (c < 0 || c >= B.N) continue;
        const uint8_t old = B.flags[c] & kOwnerMask;
        int owner = 0;
        for (int b = nb - 1; b >= 0; --b) {
            const DevBody &bd = B.bodies[b];
            double r[3];
            int d[3];
            lever_arm(bd, i, j, k, nx, ny, nz, per, r, d);
            const double d2 = core_dist2(bd, r);
            if (d2 <= bd.radius * bd.radius) owner = b + 1;
            marg[b] = fmin(marg[b], fabs(sqrt(d2) - bd.radius));
        }
        B.old_owner[c] = old;
        B.flags[c] = (uint8_t)owner;
    }
    for (int b = 0; b < nb; ++b) {
        const double m = block_min(marg[b], sh);
        if (threadIdx.x == 0) {
            margins[b] = m;
            for (int q = 0; q < 3; ++q) B.bodies[b].Xmap[q] = B.bodies[b].anchor[q] + B.bodies[b].D[q];
            for (int q = 0; q < 4; ++q) qmaps[4 * b + q] = B.bodies[b].q[q];
        }
    }
    __threadfence_block();
    __syncthreads();
    // pass 2: refill cells that left a body (equilibrium at the body's velocity,
    // density averaged over neighbours that are fluid before and after)
    void *popc = sh.cur ? B.pop1 : B.pop0;
    const size_t N = (size_t)B.N;
    for (int t = threadIdx.x; t < ncell; t += kCoupleThreads) {
        const int i = sh.lo[0] + t % bx, j = sh.lo[1] + (t / bx) % by, k = sh.lo[2] + t / (bx * by);
        const int c = i + nx * (j + ny * k);
        if (c < 0 || c >= B.N) continue;
        const int old = B.old_owner[c];
        if (old == 0 || (B.flags[c] & kOwnerMask) != 0) continue;
        double total = 0.0;
        int count = 0;
        for (int a = 1; a < 19; ++a) {
            int ti, tj, tk;
            if (!neighbour_rt(a, i, j, k, nx, ny, nz, per, ti, tj, tk)) continue;
            const int nc = ti + nx * (tj + ny * tk);
            if (B.old_owner[nc] != 0 || (B.flags[nc] & kOwnerMask) != 0) continue;
            double s = load_dev<S>(popc, nc, B.inv_scale);
            for (int q = 1; q < 19; ++q) s = s + load_dev<S>(popc, (size_t)q * N + nc, B.inv_scale);
            total = total + s;
            ++count;
        }
        const double drho = count ? total / (double)count : 0.0;
        const double rho = 1.0 + drho;
        const DevBody &bd = B.bodies[old - 1];
        double r[3], u[3];
        int d[3];
        lever_arm(bd, i, j, k, nx, ny, nz, per, r, d);
        wall_velocity(bd, r, u);
        const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        for (int a = 0; a < 19; ++a) {
            const double eu = ex(a) * u[0] + ey(a) * u[1] + ez(a) * u[2];
            const double v = wgt(a) * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
            Storage<S>::store((S *)popc, (size_t)a * N + c, (typename Storage<S>::C)v, B.scale);
        }
    }
    __threadfence_block();
    __syncthreads();
    // pass 3: near-body marks and boundary links, in cell order
    int running = 0;
    for (int base = 0; base < ncell; base += kCoupleThreads) {
        const int t = base + (int)threadIdx.x;
        int c = -1, cnt = 0;
        unsigned mask = 0;
        unsigned char owners[19];
        if (t < ncell) {
            const int i = sh.lo[0] + t % bx, j = sh.lo[1] + (t / bx) % by, k = sh.lo[2] + t / (bx * by);
            c = i + nx * (j + ny * k);
            if (c < 0 || c >= B.N) c = -1;
            if (c >= 0 && (B.flags[c] & kOwnerMask) == 0) {
                for (int a = 1; a < 19; ++a) {
                    int ti, tj, tk;
                    owners[a] = 0;
                    if (!neighbour_rt(a, i, j, k, nx, ny, nz, per, ti, tj, tk)) continue;
                    const int o = B.flags[ti + nx * (tj + ny * tk)] & kOwnerMask;
                    if (o) {
                        mask |= 1u << a;
                        owners[a] = (unsigned char)o;
                        ++cnt;
                    }
                }
            }
        }
        int tot;
        const int off = running + block_scan(cnt, &tot, sh);
        if (c >= 0 && (B.flags[c] & kOwnerMask) == 0) {
            B.flags[c] = cnt ? kNearBit : 0;
            if (cnt) {
                B.link_base[c] = off;
                int l = off;
                for (int a = 1; a < 19; ++a) {
                    if (!(mask & (1u << a))) continue;
                    if (l < B.link_cap) {
                        B.link_cell[l] = c;
                        B.link_dir[l] = (signed char)a;
                        B.link_body[l] = (signed char)(owners[a] - 1);
                    }
                    ++l;
                }
            }
        }
        running += tot;
    }
    if (threadIdx.x == 0) {
        B.link_count = running;
        if (running > B.link_cap) B.status = -6;
    }
}

template <typename S>
__global__ __launch_bounds__(kCoupleThreads) void couple_kernel(BoxDesc *boxes, const int *active,
                                                                double *qmaps, double *margins,
                                                                int mode, int force_map) {
    __shared__ CoupleShared sh;
    const int bi = active[blockIdx.x];
    BoxDesc &B = boxes[bi];
    double *qm = qmaps + (size_t)bi * 4 * kMaxBodies;
    double *mg = margins + (size_t)bi * kMaxBodies;
    if (threadIdx.x == 0) sh.cur = B.cur;
    __syncthreads();
    if (mode == kModeStep) {
        momentum_exchange(B, sh);
        if (threadIdx.x == 0) {
            rigid_step(B, sh);
            sh.cur ^= 1;
            B.cur = sh.cur;
        }
        __threadfence_block();
        __syncthreads();
    }
    remap<S>(B, sh, qm, mg, force_map || mode == kModeMapOnly);
}

}  // namespace lbm
