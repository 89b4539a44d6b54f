// C-ABI of the swimmer step library (declared in include/lbmswim.h): context
// management, input validation, device tables, and the launch sequence of
// one coupled step (Alg. 2): sweep (collide, stream, bounce-back) followed by
// the per-box coupling kernel (forces, rigid bodies, next mapping).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbmswim.h"
#include "common.h"
#include "coupling.h"
#include "sweep.h"

using namespace lbm;

namespace {

constexpr int kSweepBlock = 256;

struct HostBox {
    lbm_params p;
    int N = 0;
    std::vector<lbm_body> bodies;
    std::vector<lbm_spring> springs;
    std::vector<lbm_drive> drives;
    int64_t limit = -1;
    int64_t steps = 0;           // host mirror of the device step counter
    DevBody *d_bodies = nullptr;
    DevSpring *d_springs = nullptr;
    DevDrive *d_drives = nullptr;
    int *link_cell = nullptr;
    signed char *link_dir = nullptr, *link_body = nullptr;
    double2 *link_val = nullptr;
    int *link_base = nullptr;
    uint8_t *old_owner = nullptr;
    int link_cap = 0;
    bool mapped = false;
};

}  // namespace

struct lbm_ctx {
    std::vector<HostBox> boxes;
    int storage = LBM_F64;
    hipStream_t stream = nullptr;
    BoxDesc *d_boxes = nullptr;
    double *d_qmaps = nullptr;
    double *d_margins = nullptr;
    int *d_active = nullptr;       // active box indices for the coupling kernel
    WorkItem *d_work = nullptr;    // sweep tiles of the active boxes
    int nwork = 0, nactive = 0;
    std::vector<int> active_host;
    bool work_dirty = true;
    bool force_map = false;
    bool poisoned = false;
    bool timing = false;
    std::vector<hipEvent_t> ev[2];   // start/stop pairs: [0] sweep, [1] coupling
    std::string err;
};

namespace {

int fail(lbm_ctx *c, int code, const std::string &msg) {
    if (c) {
        c->err = msg;
        if (code == LBM_E_HIP) c->poisoned = true;
    }
    return code;
}

#define HIP_TRY(ctx, call)                                                              \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail((ctx), LBM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t storage_bytes(int s) { return s == LBM_F64 ? 8 : (s == LBM_F32 ? 4 : 2); }

int validate_params(lbm_ctx *c, const lbm_params &p) {
    if (p.nx < 3 || p.ny < 3 || p.nz < 3) return fail(c, LBM_E_ARG, "box must be at least 3 cells per axis");
    if ((double)p.nx * p.ny * p.nz > 2.0e9) return fail(c, LBM_E_ARG, "box exceeds 2e9 cells");
    if (!(p.tau > 0.5) || !std::isfinite(p.tau)) return fail(c, LBM_E_ARG, "tau must be finite and > 0.5");
    if (p.storage < LBM_F64 || p.storage > LBM_BF16S) return fail(c, LBM_E_ARG, "unknown storage type");
    if (p.periodic_mask > 7) return fail(c, LBM_E_ARG, "periodic_mask uses bits 0..2 only");
    if (!p.pop[0] || !p.pop[1] || !p.flags) return fail(c, LBM_E_ARG, "pop[0], pop[1] and flags are required");
    if (p.pop[0] == p.pop[1]) return fail(c, LBM_E_ARG, "pop[0] and pop[1] must differ");
    if (p.traj && p.traj_cap <= 0) return fail(c, LBM_E_ARG, "traj_cap must be > 0 with traj");
    if ((p.storage == LBM_F16S || p.storage == LBM_BF16S) && (p.shift_log2 < -30 || p.shift_log2 > 30))
        return fail(c, LBM_E_ARG, "shift_log2 out of range");
    return LBM_OK;
}

BoxDesc make_desc(const HostBox &h, int storage) {
    BoxDesc d;
    memset(&d, 0, sizeof(d));
    d.nx = h.p.nx;
    d.ny = h.p.ny;
    d.nz = h.p.nz;
    d.per = (int)h.p.periodic_mask;
    d.N = h.N;
    d.nb = (int)h.bodies.size();
    d.ns = (int)h.springs.size();
    d.nd = (int)h.drives.size();
    d.omega = 1.0 / h.p.tau;
    d.omegaf = (float)(1.0 / h.p.tau);
    const bool scaled = storage == LBM_F16S || storage == LBM_BF16S;
    d.scale = scaled ? std::ldexp(1.0f, h.p.shift_log2) : 1.0f;
    d.inv_scale = scaled ? std::ldexp(1.0f, -h.p.shift_log2) : 1.0f;
    d.pop0 = h.p.pop[0];
    d.pop1 = h.p.pop[1];
    d.flags = h.p.flags;
    d.old_owner = h.old_owner;
    d.link_cell = h.link_cell;
    d.link_dir = h.link_dir;
    d.link_body = h.link_body;
    d.link_val = h.link_val;
    d.link_base = h.link_base;
    d.link_cap = h.link_cap;
    d.bodies = h.d_bodies;
    d.springs = h.d_springs;
    d.drives = h.d_drives;
    d.traj = h.p.traj;
    d.traj_cap = h.p.traj ? h.p.traj_cap : 0;
    return d;
}

// Upload the static fields of a box descriptor without touching the mutable
// device state (step, cur, link_count, status).
int upload_desc(lbm_ctx *c, int b) {
    BoxDesc d = make_desc(c->boxes[b], c->storage);
    const size_t static_bytes = offsetof(BoxDesc, step);
    HIP_TRY(c, hipMemcpyAsync(c->d_boxes + b, &d, static_bytes, hipMemcpyHostToDevice, c->stream));
    return LBM_OK;
}

int init_common(const lbm_params *params, int nbox, lbm_ctx **out) {
    if (!out) return LBM_E_ARG;
    *out = nullptr;
    if (!params || nbox < 1 || nbox > 65535) return LBM_E_ARG;
    lbm_ctx *c = new lbm_ctx();
    c->storage = params[0].storage;
    c->stream = (hipStream_t)params[0].stream;
    for (int b = 0; b < nbox; ++b) {
        int rc = validate_params(c, params[b]);
        if (rc != LBM_OK) {
            *out = c;
            return rc;
        }
        if (params[b].storage != c->storage) {
            *out = c;
            return fail(c, LBM_E_ARG, "all boxes of a batch must share one storage type");
        }
    }
    c->boxes.resize(nbox);
    for (int b = 0; b < nbox; ++b) {
        HostBox &h = c->boxes[b];
        h.p = params[b];
        h.N = params[b].nx * params[b].ny * params[b].nz;
        if (hipMalloc(&h.link_base, sizeof(int) * h.N) != hipSuccess ||
            hipMalloc(&h.old_owner, h.N) != hipSuccess) {
            *out = c;
            return fail(c, LBM_E_HIP, "out of device memory for per-cell scratch");
        }
        if (hipMemsetAsync(h.p.flags, 0, h.N, c->stream) != hipSuccess ||
            hipMemsetAsync(h.old_owner, 0, h.N, c->stream) != hipSuccess ||
            hipMemsetAsync(h.link_base, 0, sizeof(int) * h.N, c->stream) != hipSuccess) {
            *out = c;
            return fail(c, LBM_E_HIP, "clearing flags failed");
        }
    }
    *out = c;
    HIP_TRY(c, hipMalloc(&c->d_boxes, sizeof(BoxDesc) * nbox));
    HIP_TRY(c, hipMemsetAsync(c->d_boxes, 0, sizeof(BoxDesc) * nbox, c->stream));
    HIP_TRY(c, hipMalloc(&c->d_qmaps, sizeof(double) * 4 * kMaxBodies * nbox));
    HIP_TRY(c, hipMalloc(&c->d_margins, sizeof(double) * kMaxBodies * nbox));
    HIP_TRY(c, hipMemsetAsync(c->d_margins, 0, sizeof(double) * kMaxBodies * nbox, c->stream));
    HIP_TRY(c, hipMalloc(&c->d_active, sizeof(int) * nbox));
    for (int b = 0; b < nbox; ++b) {
        int rc = upload_desc(c, b);
        if (rc != LBM_OK) return rc;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

double body_extent_h(const lbm_body &b) { return b.radius + (b.shape == LBM_CAPSULE ? b.half_len : 0.0); }

int validate_bodies(lbm_ctx *c, const HostBox &h, const lbm_body *bodies, int nb,
                    const lbm_spring *springs, int ns, const lbm_drive *drives, int nd) {
    if (nb < 0 || nb > kMaxBodies) return fail(c, LBM_E_ARG, "between 0 and 16 bodies per box");
    if (ns < 0 || nd < 0 || (nb && !bodies) || (ns && !springs) || (nd && !drives))
        return fail(c, LBM_E_ARG, "null body/spring/drive array");
    const int n[3] = {h.p.nx, h.p.ny, h.p.nz};
    for (int b = 0; b < nb; ++b) {
        const lbm_body &B = bodies[b];
        if (B.shape != LBM_SPHERE && B.shape != LBM_CAPSULE) return fail(c, LBM_E_ARG, "unknown body shape");
        if (!(B.radius > 0) || B.half_len < 0 || (!B.kinematic && !(B.mass > 0)))
            return fail(c, LBM_E_ARG, "body radius and mass must be positive");
        if (!B.kinematic && !(B.inertia[0] > 0 && B.inertia[1] > 0 && B.inertia[2] > 0))
            return fail(c, LBM_E_ARG, "body inertia must be positive");
        const double e = body_extent_h(B);
        for (int q = 0; q < 3; ++q) {
            const double X = B.anchor[q] + B.disp[q];
            if (!std::isfinite(X)) return fail(c, LBM_E_ARG, "body position not finite");
            if (h.p.periodic_mask & (1u << q)) {
                if (2.0 * e + 4.0 >= n[q]) return fail(c, LBM_E_ARG, "body too large for the periodic box");
            } else if (X - e < 1.0 || X + e > n[q] - 1.0) {
                return fail(c, LBM_E_OVERLAP, "body reaches a wall (keep one cell of fluid)");
            }
        }
        const double qn = std::sqrt(B.quat[0] * B.quat[0] + B.quat[1] * B.quat[1] + B.quat[2] * B.quat[2] +
                                    B.quat[3] * B.quat[3]);
        if (std::fabs(qn - 1.0) > 1e-6) return fail(c, LBM_E_ARG, "quaternion must be normalised");
        for (int o = 0; o < b; ++o) {
            const lbm_body &O = bodies[o];
            double d2 = 0;
            for (int q = 0; q < 3; ++q) {
                double d = (B.anchor[q] + B.disp[q]) - (O.anchor[q] + O.disp[q]);
                if (h.p.periodic_mask & (1u << q)) d -= n[q] * std::nearbyint(d / n[q]);
                d2 += d * d;
            }
            // bounding spheres plus one cell of fluid between the bodies
            if (std::sqrt(d2) < body_extent_h(B) + body_extent_h(O) + 1.0)
                return fail(c, LBM_E_OVERLAP, "bodies overlap (or touch)");
        }
    }
    for (int s = 0; s < ns; ++s)
        if (springs[s].i < 0 || springs[s].i >= nb || springs[s].j < 0 || springs[s].j >= nb ||
            springs[s].i == springs[s].j || !(springs[s].rest_len >= 0))
            return fail(c, LBM_E_ARG, "spring indices out of range");
    for (int d = 0; d < nd; ++d) {
        const lbm_drive &D = drives[d];
        if (D.left < 0 || D.left >= nb || D.right < 0 || D.right >= nb || D.middle < 0 || D.middle >= nb ||
            !(D.period > 0))
            return fail(c, LBM_E_ARG, "drive indices out of range or period <= 0");
    }
    return LBM_OK;
}

template <typename F>
int dispatch_storage(int storage, F &&f) {
    switch (storage) {
        case LBM_F64: return f((double *)nullptr);
        case LBM_F32: return f((float *)nullptr);
        case LBM_F16S: return f((_Float16 *)nullptr);
        default: return f((bf16_t *)nullptr);
    }
}

int launch_couple(lbm_ctx *c, const int *active_dev, int nactive, int mode) {
    if (nactive == 0) return LBM_OK;
    return dispatch_storage(c->storage, [&](auto *tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(couple_kernel<S>, dim3(nactive), dim3(kCoupleThreads), 0, c->stream,
                           c->d_boxes, active_dev, c->d_qmaps, c->d_margins, mode, c->force_map ? 1 : 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("couple launch: ") + hipGetErrorString(e));
        return LBM_OK;
    });
}

// Rebuild the sweep tiles and the active-box list for boxes that still run.
int rebuild_work(lbm_ctx *c) {
    std::vector<WorkItem> work;
    c->active_host.clear();
    for (int b = 0; b < (int)c->boxes.size(); ++b) {
        const HostBox &h = c->boxes[b];
        if (h.limit >= 0 && h.steps >= h.limit) continue;
        c->active_host.push_back(b);
        for (int first = 0; first < h.N; first += kSweepBlock) work.push_back({b, first});
    }
    if ((int)work.size() > c->nwork) {
        if (c->d_work) HIP_TRY(c, hipFree(c->d_work));
        HIP_TRY(c, hipMalloc(&c->d_work, sizeof(WorkItem) * std::max<size_t>(work.size(), 1)));
    }
    c->nwork = (int)work.size();
    c->nactive = (int)c->active_host.size();
    if (c->nwork)
        HIP_TRY(c, hipMemcpyAsync(c->d_work, work.data(), sizeof(WorkItem) * work.size(), hipMemcpyHostToDevice,
                                  c->stream));
    if (c->nactive)
        HIP_TRY(c, hipMemcpyAsync(c->d_active, c->active_host.data(), sizeof(int) * c->nactive,
                                  hipMemcpyHostToDevice, c->stream));
    // the host vectors must outlive the asynchronous copies
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->work_dirty = false;
    return LBM_OK;
}

int launch_sweep(lbm_ctx *c) {
    if (c->nwork == 0) return LBM_OK;
    return dispatch_storage(c->storage, [&](auto *tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL((sweep_kernel<S, kSweepBlock>), dim3(c->nwork), dim3(kSweepBlock), 0, c->stream,
                           c->d_boxes, c->d_work);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("sweep launch: ") + hipGetErrorString(e));
        return LBM_OK;
    });
}

template <typename F>
int timed(lbm_ctx *c, int which, F &&launch) {
    if (!c->timing) return launch();
    hipEvent_t a, b;
    HIP_TRY(c, hipEventCreate(&a));
    HIP_TRY(c, hipEventCreate(&b));
    HIP_TRY(c, hipEventRecord(a, c->stream));
    int rc = launch();
    HIP_TRY(c, hipEventRecord(b, c->stream));
    c->ev[which].push_back(a);
    c->ev[which].push_back(b);
    return rc;
}

void drop_events(lbm_ctx *c) {
    for (auto &v : c->ev) {
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
        v.clear();
    }
}

DevBody to_dev(const lbm_body &b) {
    DevBody d;
    memset(&d, 0, sizeof(d));
    for (int q = 0; q < 3; ++q) {
        d.anchor[q] = b.anchor[q];
        d.D[q] = b.disp[q];
        d.V[q] = b.vel[q];
        d.O[q] = b.omega[q];
        d.Xmap[q] = b.anchor[q] + b.disp[q];
        d.inertia[q] = b.inertia[q];
    }
    for (int q = 0; q < 4; ++q) d.q[q] = b.quat[q];
    d.radius = b.radius;
    d.half_len = b.shape == LBM_CAPSULE ? b.half_len : 0.0;
    d.mass = b.mass;
    d.shape = b.shape;
    d.kinematic = b.kinematic;
    return d;
}

lbm_body from_dev(const DevBody &d) {
    lbm_body b;
    memset(&b, 0, sizeof(b));
    for (int q = 0; q < 3; ++q) {
        b.anchor[q] = d.anchor[q];
        b.disp[q] = d.D[q];
        b.vel[q] = d.V[q];
        b.omega[q] = d.O[q];
        b.inertia[q] = d.inertia[q];
    }
    for (int q = 0; q < 4; ++q) b.quat[q] = d.q[q];
    b.radius = d.radius;
    b.half_len = d.half_len;
    b.mass = d.mass;
    b.shape = d.shape;
    b.kinematic = d.kinematic;
    return b;
}

int check_ctx(lbm_ctx *c) {
    if (!c) return LBM_E_ARG;
    if (c->poisoned) return LBM_E_HIP;
    return LBM_OK;
}

int check_box(lbm_ctx *c, int box) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (box < 0 || box >= (int)c->boxes.size()) return fail(c, LBM_E_ARG, "box index out of range");
    return LBM_OK;
}

template <typename S>
__global__ void export_kernel(const BoxDesc *boxes, int bi, double *dst) {
    const BoxDesc &B = boxes[bi];
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t N = (size_t)B.N;
    if (idx >= 19 * N) return;
    const size_t cell = idx % N;
    const S *src = (const S *)(B.cur ? B.pop1 : B.pop0);
    dst[idx] = (B.flags[cell] & kOwnerMask) ? 0.0 : (double)Storage<S>::load(src, idx, B.inv_scale);
}

template <typename S>
__global__ void import_kernel(const BoxDesc *boxes, int bi, const double *srcd) {
    const BoxDesc &B = boxes[bi];
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t N = (size_t)B.N;
    if (idx >= 19 * N) return;
    S *dst = (S *)(B.cur ? B.pop1 : B.pop0);
    Storage<S>::store(dst, idx, (typename Storage<S>::C)srcd[idx], B.scale);
}

}  // namespace

extern "C" {

int lbm_init(const lbm_params *params, lbm_ctx **out) { return init_common(params, 1, out); }

int lbm_init_batch(const lbm_params *params, int32_t nbox, lbm_ctx **out) {
    return init_common(params, nbox, out);
}

int lbm_set_bodies_box(lbm_ctx *c, int32_t box, const lbm_body *bodies, int32_t nb,
                       const lbm_spring *springs, int32_t ns, const lbm_drive *drives, int32_t nd) {
    int rc = check_box(c, box);
    if (rc) return rc;
    HostBox &h = c->boxes[box];
    rc = validate_bodies(c, h, bodies, nb, springs, ns, drives, nd);
    if (rc) return rc;
    // bodies already on the lattice: keep their last mapped positions so that the
    // remap covers both the old and the new cells
    std::vector<DevBody> old(h.bodies.size());
    if (h.mapped && !h.bodies.empty())
        HIP_TRY(c, hipMemcpy(old.data(), h.d_bodies, sizeof(DevBody) * old.size(), hipMemcpyDeviceToHost));
    h.bodies.assign(bodies, bodies + nb);
    h.springs.assign(springs, springs + ns);
    h.drives.assign(drives, drives + nd);
    // link capacity: 18 links per cell of every body's bounding box plus one layer
    long long cap = 0;
    for (const auto &b : h.bodies) {
        const double e = body_extent_h(b) + 2.5;
        const long long side = (long long)std::ceil(2 * e) + 1;
        cap += 18 * side * side * side;
    }
    cap = std::max<long long>(cap, 64);
    if (cap > h.link_cap) {
        if (h.link_cell) {
            HIP_TRY(c, hipFree(h.link_cell));
            HIP_TRY(c, hipFree(h.link_dir));
            HIP_TRY(c, hipFree(h.link_body));
            HIP_TRY(c, hipFree(h.link_val));
        }
        HIP_TRY(c, hipMalloc(&h.link_cell, sizeof(int) * cap));
        HIP_TRY(c, hipMalloc(&h.link_dir, cap));
        HIP_TRY(c, hipMalloc(&h.link_body, cap));
        HIP_TRY(c, hipMalloc(&h.link_val, sizeof(double2) * cap));
        h.link_cap = (int)cap;
    }
    if (!h.d_bodies) {
        HIP_TRY(c, hipMalloc(&h.d_bodies, sizeof(DevBody) * kMaxBodies));
        HIP_TRY(c, hipMalloc(&h.d_springs, sizeof(DevSpring) * 64));
        HIP_TRY(c, hipMalloc(&h.d_drives, sizeof(DevDrive) * 16));
    }
    if (ns > 64 || nd > 16) return fail(c, LBM_E_ARG, "at most 64 springs and 16 drives per box");
    std::vector<DevBody> db(nb);
    for (int b = 0; b < nb; ++b) {
        db[b] = to_dev(bodies[b]);
        if (h.mapped && b < (int)old.size())
            for (int q = 0; q < 3; ++q) db[b].Xmap[q] = old[b].Xmap[q];
    }
    std::vector<DevSpring> ds(ns);
    for (int s = 0; s < ns; ++s) ds[s] = {springs[s].i, springs[s].j, springs[s].k, springs[s].gamma, springs[s].rest_len};
    std::vector<DevDrive> dd(nd);
    for (int d = 0; d < nd; ++d)
        dd[d] = {drives[d].left, drives[d].middle, drives[d].right, drives[d].gate_lagged, drives[d].amplitude,
                 drives[d].period, drives[d].phase_lag, (long long)drives[d].off_left, (long long)drives[d].off_right};
    if (nb) HIP_TRY(c, hipMemcpyAsync(h.d_bodies, db.data(), sizeof(DevBody) * nb, hipMemcpyHostToDevice, c->stream));
    if (ns) HIP_TRY(c, hipMemcpyAsync(h.d_springs, ds.data(), sizeof(DevSpring) * ns, hipMemcpyHostToDevice, c->stream));
    if (nd) HIP_TRY(c, hipMemcpyAsync(h.d_drives, dd.data(), sizeof(DevDrive) * nd, hipMemcpyHostToDevice, c->stream));
    rc = upload_desc(c, box);
    if (rc) return rc;
    int *one = nullptr;
    HIP_TRY(c, hipMalloc(&one, sizeof(int)));
    HIP_TRY(c, hipMemcpyAsync(one, &box, sizeof(int), hipMemcpyHostToDevice, c->stream));
    rc = launch_couple(c, one, 1, kModeMapOnly);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipFree(one));
    h.mapped = true;
    return rc;
}

int lbm_set_bodies(lbm_ctx *c, const lbm_body *bodies, int32_t nb, const lbm_spring *springs, int32_t ns,
                   const lbm_drive *drives, int32_t nd) {
    return lbm_set_bodies_box(c, 0, bodies, nb, springs, ns, drives, nd);
}

int lbm_set_step_limit(lbm_ctx *c, int32_t box, int64_t max_steps) {
    int rc = check_box(c, box);
    if (rc) return rc;
    c->boxes[box].limit = max_steps < 0 ? -1 : max_steps;
    c->work_dirty = true;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int64_t nsteps) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsteps < 0) return fail(c, LBM_E_ARG, "nsteps < 0");
    int64_t done = 0;
    while (done < nsteps) {
        if (c->work_dirty) {
            rc = rebuild_work(c);
            if (rc) return rc;
        }
        if (c->nactive == 0) break;
        // steps until the active set changes
        int64_t run = nsteps - done;
        for (int b : c->active_host) {
            const HostBox &h = c->boxes[b];
            if (h.limit >= 0) run = std::min<int64_t>(run, h.limit - h.steps);
        }
        for (int64_t s = 0; s < run; ++s) {
            rc = timed(c, 0, [&] { return launch_sweep(c); });
            if (rc) return rc;
            rc = timed(c, 1, [&] { return launch_couple(c, c->d_active, c->nactive, kModeStep); });
            if (rc) return rc;
        }
        for (int b : c->active_host) {
            HostBox &h = c->boxes[b];
            h.steps += run;
            if (h.limit >= 0 && h.steps >= h.limit) c->work_dirty = true;
        }
        done += run;
    }
    return LBM_OK;
}

int lbm_body_forces_box(lbm_ctx *c, int32_t box, double *F, double *T, int32_t on_device) {
    int rc = check_box(c, box);
    if (rc) return rc;
    HostBox &h = c->boxes[box];
    const int nb = (int)h.bodies.size();
    if (!F || !T) return fail(c, LBM_E_ARG, "null output");
    if (nb == 0) return LBM_OK;
    if (on_device) {
        for (int b = 0; b < nb; ++b) {
            HIP_TRY(c, hipMemcpyAsync(F + 3 * b, &h.d_bodies[b].F[0], 3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(T + 3 * b, &h.d_bodies[b].T[0], 3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        }
        return LBM_OK;
    }
    std::vector<DevBody> db(nb);
    HIP_TRY(c, hipMemcpyAsync(db.data(), h.d_bodies, sizeof(DevBody) * nb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < 3; ++q) {
            F[3 * b + q] = db[b].F[q];
            T[3 * b + q] = db[b].T[q];
        }
    return LBM_OK;
}

int lbm_body_forces(lbm_ctx *c, double *F, double *T, int32_t on_device) {
    return lbm_body_forces_box(c, 0, F, T, on_device);
}

int lbm_get_bodies_box(lbm_ctx *c, int32_t box, lbm_body *out, int32_t nb) {
    int rc = check_box(c, box);
    if (rc) return rc;
    HostBox &h = c->boxes[box];
    if (nb != (int)h.bodies.size() || (nb && !out)) return fail(c, LBM_E_ARG, "nb does not match the box");
    if (nb == 0) return LBM_OK;
    std::vector<DevBody> db(nb);
    HIP_TRY(c, hipMemcpyAsync(db.data(), h.d_bodies, sizeof(DevBody) * nb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < nb; ++b) out[b] = from_dev(db[b]);
    return LBM_OK;
}

int lbm_get_bodies(lbm_ctx *c, lbm_body *out, int32_t nb) { return lbm_get_bodies_box(c, 0, out, nb); }

int lbm_get_links(lbm_ctx *c, int32_t box, int32_t *cell, int8_t *dir, int8_t *body, int64_t cap, int64_t *n) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!n) return fail(c, LBM_E_ARG, "null count");
    HostBox &h = c->boxes[box];
    BoxDesc d;
    HIP_TRY(c, hipMemcpyAsync(&d, c->d_boxes + box, sizeof(BoxDesc), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *n = d.link_count;
    if (d.link_count > h.link_cap) return fail(c, LBM_E_CAPACITY, "link list overflowed on the device");
    if (d.link_count > cap) return fail(c, LBM_E_CAPACITY, "output capacity too small");
    if (d.link_count == 0) return LBM_OK;
    if (!cell || !dir || !body) return fail(c, LBM_E_ARG, "null output");
    HIP_TRY(c, hipMemcpy(cell, h.link_cell, sizeof(int) * d.link_count, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(dir, h.link_dir, d.link_count, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(body, h.link_body, d.link_count, hipMemcpyDeviceToHost));
    return LBM_OK;
}

int lbm_export_populations(lbm_ctx *c, int32_t box, double *dst) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!dst) return fail(c, LBM_E_ARG, "null destination");
    const size_t total = (size_t)19 * c->boxes[box].N;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    return dispatch_storage(c->storage, [&](auto *tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(export_kernel<S>, dim3(blocks), dim3(256), 0, c->stream, c->d_boxes, (int)box, dst);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("export launch: ") + hipGetErrorString(e));
        return LBM_OK;
    });
}

int lbm_import_populations(lbm_ctx *c, int32_t box, const double *src) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!src) return fail(c, LBM_E_ARG, "null source");
    const size_t total = (size_t)19 * c->boxes[box].N;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    return dispatch_storage(c->storage, [&](auto *tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(import_kernel<S>, dim3(blocks), dim3(256), 0, c->stream, c->d_boxes, (int)box, src);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("import launch: ") + hipGetErrorString(e));
        return LBM_OK;
    });
}

int lbm_step_count(lbm_ctx *c, int32_t box, int64_t *steps) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!steps) return fail(c, LBM_E_ARG, "null output");
    BoxDesc d;
    HIP_TRY(c, hipMemcpyAsync(&d, c->d_boxes + box, sizeof(BoxDesc), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *steps = d.step;
    return LBM_OK;
}

int lbm_status(lbm_ctx *c) {
    int rc = check_ctx(c);
    if (rc) return rc;
    std::vector<BoxDesc> d(c->boxes.size());
    HIP_TRY(c, hipMemcpyAsync(d.data(), c->d_boxes, sizeof(BoxDesc) * d.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t b = 0; b < d.size(); ++b) {
        if (d[b].status == LBM_E_UNSTABLE)
            return fail(c, LBM_E_UNSTABLE, "box " + std::to_string(b) + ": non-finite body force or state");
        if (d[b].status == LBM_E_CAPACITY)
            return fail(c, LBM_E_CAPACITY, "box " + std::to_string(b) + ": link list overflow");
    }
    return LBM_OK;
}

int lbm_set_timing(lbm_ctx *c, int32_t enable) {
    int rc = check_ctx(c);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_events(c);
    c->timing = enable != 0;
    return LBM_OK;
}

int lbm_get_timing(lbm_ctx *c, double out_ms[2], int64_t out_n[2]) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out_ms || !out_n) return fail(c, LBM_E_ARG, "null output");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int w = 0; w < 2; ++w) {
        double tot = 0.0;
        for (size_t i = 0; i + 1 < c->ev[w].size(); i += 2) {
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[w][i], c->ev[w][i + 1]));
            tot += ms;
        }
        out_ms[w] = tot;
        out_n[w] = (int64_t)(c->ev[w].size() / 2);
    }
    return LBM_OK;
}

int lbm_struct_sizes(int64_t out[4]) {
    if (!out) return LBM_E_ARG;
    out[0] = sizeof(lbm_params);
    out[1] = sizeof(lbm_body);
    out[2] = sizeof(lbm_spring);
    out[3] = sizeof(lbm_drive);
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : "null context"; }

void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_events(c);
    for (auto &h : c->boxes) {
        (void)hipFree(h.d_bodies);
        (void)hipFree(h.d_springs);
        (void)hipFree(h.d_drives);
        (void)hipFree(h.link_cell);
        (void)hipFree(h.link_dir);
        (void)hipFree(h.link_body);
        (void)hipFree(h.link_val);
        (void)hipFree(h.link_base);
        (void)hipFree(h.old_owner);
    }
    (void)hipFree(c->d_boxes);
    (void)hipFree(c->d_qmaps);
    (void)hipFree(c->d_margins);
    (void)hipFree(c->d_active);
    (void)hipFree(c->d_work);
    delete c;
}

}  // extern "C"
