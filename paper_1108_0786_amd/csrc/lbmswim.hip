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
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbmswim.h"
#include "common.h"
#include "adjoint.h"
#include "coupling.h"
#include "sweep_aa.h"

using namespace lbm;

namespace {

constexpr int kDefaultBlock = 256;
constexpr int kDefaultGraphSteps = 32;

struct HostBox {
    lbm_params p;
    int N = 0;
    long long stride = 0;
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
    LinkRec *link_rec = nullptr; // momentum-exchange scratch of the sweep, one per link
    ForceRec *frec = nullptr;    // momentum-exchange records, one per (wave, body)
    int *grp_pos = nullptr;      // per link: record of a wave's q-th body at its first link + q
    int *link_base = nullptr;
    uint8_t *old_owner = nullptr;
    CoupleCtl *ctl = nullptr;
    double *flow_sum = nullptr;  // time-averaged flow: 3N sums and N counts (library-owned)
    int *flow_count = nullptr;
    int flow_every = 0;
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
    int coop_remap = 1;            // share the mapping among a box's coupling workgroups (2: join, map alone)
    bool aa = false;               // stream in place (one buffer, layout by step parity)
    bool flow_any = false;         // some box samples the time-averaged flow
    bool force_any = false;        // some box has the test-only body force
    int coop_blocks = 0;           // coupling workgroups that are surely resident at once
    bool poisoned = false;
    bool timing = false;
    int block = kDefaultBlock;
    int xcd_order = 0;
    int nontemporal = 0;
    int graph_steps = kDefaultGraphSteps;
    int ngrid = 0;                 // sweep grid (tiles padded to a multiple of 8)
    hipGraphExec_t graph = nullptr;    // graph_steps steps
    int graph_len = 0;
    hipGraphExec_t tail = nullptr;     // the remainder of the last run shorter than graph_steps
    int tail_len = 0;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    // adjoint scratch
    void *adj_ckpt = nullptr, *adj_seg = nullptr;
    size_t adj_ckpt_bytes = 0, adj_seg_bytes = 0;
    double *adj_lam[2] = {nullptr, nullptr};
    size_t adj_lam_bytes = 0;
    BodyHist *adj_hist = nullptr;
    size_t adj_hist_bytes = 0;
    DevBody *adj_ckpt_bodies = nullptr;
    size_t adj_ckpt_bodies_bytes = 0;
    AdjBody *adj_body = nullptr;
    AdjLinkRec *adj_lrec = nullptr;
    int adj_lrec_cap = 0;
    double *adj_grad = nullptr;
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

// A copy ordered after all work queued on the context's stream, waited for
// before returning (a plain hipMemcpy would run on the null stream, which a
// non-blocking stream does not wait for).
int copy_sync(lbm_ctx *c, void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
    if (bytes == 0) return LBM_OK;
    HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, kind, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int validate_params(lbm_ctx *c, const lbm_params &p) {
    if (p.nx < 3 || p.ny < 3 || p.nz < 3) return fail(c, LBM_E_ARG, "box must be at least 3 cells per axis");
    if ((double)p.nx * p.ny * p.nz > 2.0e9) return fail(c, LBM_E_ARG, "box exceeds 2e9 cells");
    if (!(p.tau > 0.5) || !std::isfinite(p.tau)) return fail(c, LBM_E_ARG, "tau must be finite and > 0.5");
    if (p.storage < LBM_F64 || p.storage > LBM_BF16S) return fail(c, LBM_E_ARG, "unknown storage type");
    if (p.periodic_mask > 7) return fail(c, LBM_E_ARG, "periodic_mask uses bits 0..2 only");
    if (!p.pop[0] || !p.pop[1] || !p.flags) return fail(c, LBM_E_ARG, "pop[0], pop[1] and flags are required");
    if (p.pop[0] == p.pop[1]) return fail(c, LBM_E_ARG, "pop[0] and pop[1] must differ");
    if (p.traj && p.traj_cap <= 0) return fail(c, LBM_E_ARG, "traj_cap must be > 0 with traj");
    if (p.stride != 0 && p.stride < (int64_t)p.nx * p.ny * p.nz)
        return fail(c, LBM_E_ARG, "stride must be 0 or at least nx*ny*nz");
    if ((p.storage == LBM_F16S || p.storage == LBM_BF16S) && (p.shift_log2 < -30 || p.shift_log2 > 30))
        return fail(c, LBM_E_ARG, "shift_log2 out of range");
    if (p.force_average != 0 && p.force_average != 1) return fail(c, LBM_E_ARG, "force_average must be 0 or 1");
    if (p.reserved != 0) return fail(c, LBM_E_ARG, "reserved must be 0");
    for (int q = 0; q < 3; ++q)
        if (!std::isfinite(p.body_force[q])) return fail(c, LBM_E_ARG, "body force not finite");
    return LBM_OK;
}

BoxDesc make_desc(const HostBox &h, int storage, bool aa) {
    BoxDesc d;
    memset(&d, 0, sizeof(d));
    d.nx = h.p.nx;
    d.ny = h.p.ny;
    d.nz = h.p.nz;
    d.per = (int)h.p.periodic_mask;
    d.N = h.N;
    d.stride = h.stride;
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
    d.link_rec = h.link_rec;
    d.frec = h.frec;
    d.grp_pos = h.grp_pos;
    d.link_base = h.link_base;
    d.link_cap = h.link_cap;
    d.force_avg = h.p.force_average;
    d.bodies = h.d_bodies;
    d.springs = h.d_springs;
    d.drives = h.d_drives;
    d.traj = h.p.traj;
    d.traj_cap = h.p.traj ? h.p.traj_cap : 0;
    d.ctl = h.ctl;
    d.flow_sum = h.flow_sum;
    d.flow_count = h.flow_count;
    d.flow_every = h.flow_every;
    d.aa = aa ? 1 : 0;
    for (int q = 0; q < 3; ++q) d.force[q] = h.p.body_force[q];
    return d;
}

// Upload the static fields of a box descriptor without touching the mutable
// device state (step, cur, link_count, status).
int upload_desc(lbm_ctx *c, int b) {
    BoxDesc d = make_desc(c->boxes[b], c->storage, c->aa);
    const size_t static_bytes = offsetof(BoxDesc, step);
    HIP_TRY(c, hipMemcpyAsync(c->d_boxes + b, &d, static_bytes, hipMemcpyHostToDevice, c->stream));
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

int init_common(const lbm_params *params, int nbox, lbm_ctx **out) {
    if (!out) return LBM_E_ARG;
    *out = nullptr;
    if (!params || nbox < 1 || nbox > 65535) return LBM_E_ARG;
    lbm_ctx *c = new lbm_ctx();
    c->storage = params[0].storage;
    for (int b = 0; b < nbox; ++b)
        for (int q = 0; q < 3; ++q) c->force_any = c->force_any || params[b].body_force[q] != 0.0;
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
        h.stride = params[b].stride ? params[b].stride : h.N;
        if (hipMalloc(&h.link_base, sizeof(int) * h.N) != hipSuccess ||
            hipMalloc(&h.old_owner, h.N) != hipSuccess ||
            hipMalloc(&h.ctl, sizeof(CoupleCtl)) != hipSuccess) {
            *out = c;
            return fail(c, LBM_E_HIP, "out of device memory for per-cell scratch");
        }
        if (hipMemsetAsync(h.p.flags, 0, h.N, c->stream) != hipSuccess ||
            hipMemsetAsync(h.old_owner, 0, h.N, c->stream) != hipSuccess ||
            hipMemsetAsync(h.link_base, 0, sizeof(int) * h.N, c->stream) != hipSuccess ||
            hipMemsetAsync(h.ctl, 0, sizeof(CoupleCtl), c->stream) != hipSuccess) {
            *out = c;
            return fail(c, LBM_E_HIP, "clearing flags failed");
        }
    }
    // Non-temporal population loads in the sweep, measured on boxes of 2 to
    // 34 million cells: they pay while the two population buffers of the
    // context hold at most about 768 MiB (FP32 sweep up to 14% faster,
    // FP16S/BF16S 25-29%) and cost 5-12% beyond that; FP64 gains nothing
    // at any size.  Non-temporal stores were slower in every case.
    // The XCD-aware tile order (one contiguous slab of tiles per XCD) pays on
    // states of 2.5 GB and more (5-11% on 5.1-5.2 GB of FP32, 2.5-2.6 GB of
    // FP16S) and costs 2-16% on states of 1 GB and less, so it is on above
    // 2 GiB.
    {
        double state = 0.0;
        for (const HostBox &h : c->boxes) state += 2.0 * 19.0 * (double)h.stride * (double)storage_bytes(c->storage);
        c->nontemporal = c->storage != LBM_F64 && state <= 768.0 * 1024.0 * 1024.0 ? 1 : 0;
        c->xcd_order = state > 2048.0 * 1024.0 * 1024.0 ? 1 : 0;
    }
    // In-place streaming for FP32 storage: on the 256x128x128 swimmer its
    // even steps take 111 us and its odd steps 130 us, against 128 us for
    // every two-buffer step.  The 16-bit formats (bound by their arithmetic)
    // and FP64 are slower in place (73 against 69 us, 258 against 245 us)
    // and keep two buffers.
    c->aa = c->storage == LBM_F32;
    *out = c;
    HIP_TRY(c, hipMalloc(&c->d_boxes, sizeof(BoxDesc) * nbox));
    HIP_TRY(c, hipMemsetAsync(c->d_boxes, 0, sizeof(BoxDesc) * nbox, c->stream));
    HIP_TRY(c, hipMalloc(&c->d_qmaps, sizeof(double) * 4 * kMaxBodies * nbox));
    HIP_TRY(c, hipMalloc(&c->d_margins, sizeof(double) * kMaxBodies * nbox));
    HIP_TRY(c, hipMemsetAsync(c->d_margins, 0, sizeof(double) * kMaxBodies * nbox, c->stream));
    HIP_TRY(c, hipMalloc(&c->d_active, sizeof(int) * nbox));
    {
        // how many coupling workgroups the device holds at once
        int dev = 0, ncu = 0, per_cu = 0;
        HIP_TRY(c, hipGetDevice(&dev));
        HIP_TRY(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        const int rc0 = dispatch_storage(c->storage, [&](auto *tag) -> int {
            using S = std::remove_pointer_t<decltype(tag)>;
            HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, couple_kernel<S>, kCoupleThreads, 0));
            return LBM_OK;
        });
        if (rc0 != LBM_OK) return rc0;
        c->coop_blocks = per_cu * ncu;
    }
    for (int b = 0; b < nbox; ++b) {
        int rc = upload_desc(c, b);
        if (rc != LBM_OK) return rc;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

double body_extent_h(const lbm_body &b) { return b.radius + (b.shape == LBM_CAPSULE ? b.half_len : 0.0); }

// Half axis of a body's core segment in world axes: R(quat) (h, 0, 0), zero
// for a sphere.
void core_half_axis(const lbm_body &b, double a[3]) {
    const double h = b.shape == LBM_CAPSULE ? b.half_len : 0.0;
    const double w = b.quat[0], x = b.quat[1], y = b.quat[2], z = b.quat[3];
    a[0] = h * (1 - 2 * (y * y + z * z));
    a[1] = h * 2 * (x * y + w * z);
    a[2] = h * 2 * (x * z - w * y);
}

// Squared distance between the segments p + s d and q + t e, s, t in [0, 1]:
// minimise over s and t, clamping to the segment ends.
double segment_distance2(const double p[3], const double d[3], const double q[3], const double e[3]) {
    auto dot = [](const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
    auto clamp01 = [](double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); };
    const double r[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    const double aa = dot(d, d), ee = dot(e, e), f = dot(e, r), tiny = 1e-300;
    double s = 0.0, t = 0.0;
    if (aa <= tiny && ee <= tiny) {
        s = t = 0.0;
    } else if (aa <= tiny) {
        t = clamp01(f / ee);
    } else {
        const double c = dot(d, r);
        if (ee <= tiny) {
            s = clamp01(-c / aa);
        } else {
            const double b = dot(d, e), den = aa * ee - b * b;
            s = den > 0.0 ? clamp01((b * f - c * ee) / den) : 0.0;
            t = (b * s + f) / ee;
            if (t < 0.0) {
                t = 0.0;
                s = clamp01(-c / aa);
            } else if (t > 1.0) {
                t = 1.0;
                s = clamp01((b - c) / aa);
            }
        }
    }
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double v = (p[k] + s * d[k]) - (q[k] + t * e[k]);
        d2 += v * v;
    }
    return d2;
}

int validate_bodies(lbm_ctx *c, const HostBox &h, const lbm_body *bodies, int nb,
                    const lbm_spring *springs, int ns, const lbm_drive *drives, int nd) {
    if (nb < 0 || nb > kMaxBodies) return fail(c, LBM_E_ARG, "between 0 and 16 bodies per box");
    if (ns > kMaxSprings || nd > kMaxDrives) return fail(c, LBM_E_ARG, "at most 64 springs and 16 drives per box");
    if (ns < 0 || nd < 0 || (nb && !bodies) || (ns && !springs) || (nd && !drives))
        return fail(c, LBM_E_ARG, "null body/spring/drive array");
    const int n[3] = {h.p.nx, h.p.ny, h.p.nz};
    for (int b = 0; b < nb; ++b) {
        const lbm_body &B = bodies[b];
        if (B.shape != LBM_SPHERE && B.shape != LBM_CAPSULE && B.shape != LBM_SLAB)
            return fail(c, LBM_E_ARG, "unknown body shape");
        if (B.shape == LBM_SLAB) {
            // tests only: a kinematic half-space; it reaches the walls by design
            if (B.kinematic != 1) return fail(c, LBM_E_ARG, "a slab must be kinematic");
            const double qn = std::sqrt(B.quat[0] * B.quat[0] + B.quat[1] * B.quat[1] + B.quat[2] * B.quat[2] +
                                        B.quat[3] * B.quat[3]);
            if (std::fabs(qn - 1.0) > 1e-6) return fail(c, LBM_E_ARG, "quaternion must be normalised");
            for (int q = 0; q < 3; ++q)
                if (!std::isfinite(B.anchor[q] + B.disp[q])) return fail(c, LBM_E_ARG, "body position not finite");
            continue;
        }
        if (B.kinematic < 0 || B.kinematic > 2) return fail(c, LBM_E_ARG, "kinematic must be 0, 1 or 2");
        if (!(B.radius > 0) || B.half_len < 0 || (B.kinematic != 1 && !(B.mass > 0)))
            return fail(c, LBM_E_ARG, "body radius and mass must be positive");
        if (B.kinematic == 0 && !(B.inertia[0] > 0 && B.inertia[1] > 0 && B.inertia[2] > 0))
            return fail(c, LBM_E_ARG, "body inertia must be positive");
        const double e = body_extent_h(B);
        const double qn = std::sqrt(B.quat[0] * B.quat[0] + B.quat[1] * B.quat[1] + B.quat[2] * B.quat[2] +
                                    B.quat[3] * B.quat[3]);
        if (std::fabs(qn - 1.0) > 1e-6) return fail(c, LBM_E_ARG, "quaternion must be normalised");
        double ax[3];
        core_half_axis(B, ax);
        for (int q = 0; q < 3; ++q) {
            const double X = B.anchor[q] + B.disp[q];
            const double eq = B.radius + std::fabs(ax[q]);   // extent along axis q
            if (!std::isfinite(X)) return fail(c, LBM_E_ARG, "body position not finite");
            if (h.p.periodic_mask & (1u << q)) {
                if (2.0 * e + 4.0 >= n[q]) return fail(c, LBM_E_ARG, "body too large for the periodic box");
            } else if (X - eq < 1.0 || X + eq > n[q] - 1.0) {
                return fail(c, LBM_E_OVERLAP, "body reaches a wall (keep one cell of fluid)");
            }
        }
        for (int o = 0; o < b; ++o) {
            const lbm_body &O = bodies[o];
            if (O.shape == LBM_SLAB) continue;   // not checked against a slab (tests only)
            // core segments, the other body moved to its nearest periodic image
            double ao[3], p0[3], d0[3], p1[3], d1[3];
            core_half_axis(O, ao);
            for (int q = 0; q < 3; ++q) {
                double d = (B.anchor[q] + B.disp[q]) - (O.anchor[q] + O.disp[q]);
                if (h.p.periodic_mask & (1u << q)) d -= n[q] * std::nearbyint(d / n[q]);
                p0[q] = d - ax[q];
                d0[q] = 2.0 * ax[q];
                p1[q] = -ao[q];
                d1[q] = 2.0 * ao[q];
            }
            // one cell of fluid between the surfaces
            if (std::sqrt(segment_distance2(p0, d0, p1, d1)) < B.radius + O.radius + 1.0)
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

// Coupling kernel: kRedBlocks workgroups per active box.
int launch_couple(lbm_ctx *c, const int *active_dev, int nactive, int mode) {
    if (nactive == 0) return LBM_OK;
    // every box active (the list is built in box order): no list to read
    if (active_dev == c->d_active && nactive == (int)c->boxes.size()) active_dev = nullptr;
    return dispatch_storage(c->storage, [&](auto *tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        // cooperative only if every workgroup of the launch is resident at once
        const int coop = c->coop_remap && nactive * kRedBlocks <= c->coop_blocks ? c->coop_remap : 0;
        hipLaunchKernelGGL(couple_kernel<S>, dim3(nactive * kRedBlocks), dim3(kCoupleThreads), 0, c->stream,
                           c->d_boxes, active_dev, c->d_qmaps, c->d_margins, mode, c->force_map ? 1 : 0, coop);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("couple launch: ") + hipGetErrorString(e));
        return LBM_OK;
    });
}

void drop_graph(lbm_ctx *c) {
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->tail) (void)hipGraphExecDestroy(c->tail);
    c->graph = nullptr;
    c->graph_len = 0;
    c->tail = nullptr;
    c->tail_len = 0;
}

// Rebuild the sweep tiles and the active-box list for boxes that still run.
int rebuild_work(lbm_ctx *c) {
    std::vector<WorkItem> work;
    c->active_host.clear();
    for (int b = 0; b < (int)c->boxes.size(); ++b) {
        const HostBox &h = c->boxes[b];
        if (h.limit >= 0 && h.steps >= h.limit) continue;
        c->active_host.push_back(b);
    }
    for (int b : c->active_host) {
        const HostBox &h = c->boxes[b];
        const int nx = h.p.nx, ny = h.p.ny;
        for (int first = 0; first < h.N; first += c->block) {
            const int i0 = first % nx, rest = first / nx;
            work.push_back({b, first, i0, rest % ny, rest / ny, 0});
        }
    }
    const int nwork = (int)work.size();
    const int ngrid = (nwork + 7) / 8 * 8;
    if (ngrid > c->ngrid || !c->d_work) {
        if (c->d_work) HIP_TRY(c, hipFree(c->d_work));
        HIP_TRY(c, hipMalloc(&c->d_work, sizeof(WorkItem) * std::max(ngrid, 8)));
    }
    c->nwork = nwork;
    c->ngrid = ngrid;
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
    drop_graph(c);
    return LBM_OK;
}

template <typename S, int BLOCK, bool FLOW>
int launch_sweep_f(lbm_ctx *c) {
    if (c->aa) {
        if (c->nontemporal)
            hipLaunchKernelGGL((sweep_aa_kernel<S, BLOCK, true, FLOW>), dim3(c->ngrid), dim3(BLOCK), 0, c->stream,
                               c->d_boxes, c->d_work, c->nwork, c->xcd_order);
        else
            hipLaunchKernelGGL((sweep_aa_kernel<S, BLOCK, false, FLOW>), dim3(c->ngrid), dim3(BLOCK), 0, c->stream,
                               c->d_boxes, c->d_work, c->nwork, c->xcd_order);
        return LBM_OK;
    }
    if (c->nontemporal)
        hipLaunchKernelGGL((sweep_kernel<S, BLOCK, true, FLOW>), dim3(c->ngrid), dim3(BLOCK), 0, c->stream,
                           c->d_boxes, c->d_work, c->nwork, c->xcd_order);
    else
        hipLaunchKernelGGL((sweep_kernel<S, BLOCK, false, FLOW>), dim3(c->ngrid), dim3(BLOCK), 0, c->stream,
                           c->d_boxes, c->d_work, c->nwork, c->xcd_order);
    return LBM_OK;
}

// The sweep that also samples the time-averaged flow runs only while some
// box samples it; the plain sweep carries no trace of it.
// The sweep with the test-only body force (plain loads, no flow sampling).
template <typename S, int BLOCK>
int launch_sweep_forced(lbm_ctx *c) {
    if (c->aa)
        hipLaunchKernelGGL((sweep_aa_kernel<S, BLOCK, false, false, true>), dim3(c->ngrid), dim3(BLOCK), 0,
                           c->stream, c->d_boxes, c->d_work, c->nwork, c->xcd_order);
    else
        hipLaunchKernelGGL((sweep_kernel<S, BLOCK, false, false, true>), dim3(c->ngrid), dim3(BLOCK), 0, c->stream,
                           c->d_boxes, c->d_work, c->nwork, c->xcd_order);
    return LBM_OK;
}

template <typename S, int BLOCK>
int launch_sweep_t(lbm_ctx *c) {
    if (c->force_any) return launch_sweep_forced<S, BLOCK>(c);
    return c->flow_any ? launch_sweep_f<S, BLOCK, true>(c) : launch_sweep_f<S, BLOCK, false>(c);
}

int launch_sweep(lbm_ctx *c) {
    if (c->nwork == 0) return LBM_OK;
    int rc = dispatch_storage(c->storage, [&](auto *tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        switch (c->block) {
            case 128: return launch_sweep_t<S, 128>(c);
            case 512: return launch_sweep_t<S, 512>(c);
            default: return launch_sweep_t<S, 256>(c);
        }
    });
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("sweep launch: ") + hipGetErrorString(e));
    return LBM_OK;
}

// One coupled step of every active box: sweep, then coupling.
int launch_step(lbm_ctx *c) {
    int rc = launch_sweep(c);
    if (rc) return rc;
    return launch_couple(c, c->d_active, c->nactive, kModeStep);
}

// Capture `len` steps into a graph (*out, replacing what it held).  The
// launches are captured on a private stream (the caller's stream may be the
// legacy default stream, which cannot be captured); the graph is then
// launched on the caller's stream.
int capture_graph(lbm_ctx *c, int len, hipGraphExec_t *out, int *out_len) {
    if (*out) (void)hipGraphExecDestroy(*out);
    *out = nullptr;
    *out_len = 0;
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        c->stream = user;
        return fail(c, LBM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    int rc = LBM_OK;
    for (int s = 0; s < len && rc == LBM_OK; ++s) rc = launch_step(c);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->stream, &g);
    c->stream = user;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    *out_len = len;
    return LBM_OK;
}

// The graphs a run of `run` steps replays: graph_steps steps at a time, and
// the remainder as one graph of its own length (kept until another length is
// needed).  Captures what is missing; launches nothing.
int ensure_graphs(lbm_ctx *c, int64_t run) {
    if (c->timing || c->graph_steps <= 0) return LBM_OK;
    int rc;
    if (run >= c->graph_steps && (!c->graph || c->graph_len != c->graph_steps))
        if ((rc = capture_graph(c, c->graph_steps, &c->graph, &c->graph_len))) return rc;
    const int rem = (int)(run % c->graph_steps);
    if (rem > 0 && (!c->tail || c->tail_len != rem))
        if ((rc = capture_graph(c, rem, &c->tail, &c->tail_len))) return rc;
    return LBM_OK;
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
    const size_t a = idx / N, cell = idx % N;
    const S *src = (const S *)(B.cur ? B.pop1 : B.pop0);
    dst[idx] = (B.flags[cell] & kOwnerMask)
                   ? 0.0
                   : (double)Storage<S>::load(src, current_slot(B, swapped_now(B), (int)a, (int)cell), B.inv_scale);
}

template <typename S>
__global__ void export_cells_kernel(const BoxDesc *boxes, int bi, const int *cells, long long n, double *dst) {
    const BoxDesc &B = boxes[bi];
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int c = cells[m];
    const S *src = (const S *)(B.cur ? B.pop1 : B.pop0);
    const bool ok = c >= 0 && c < B.N;
    for (int a = 0; a < 19; ++a) {
        double v = __longlong_as_double(0x7ff8000000000000LL);
        if (ok)
            v = (B.flags[c] & kOwnerMask)
                    ? 0.0
                    : (double)Storage<S>::load(src, current_slot(B, swapped_now(B), a, c), B.inv_scale);
        dst[(size_t)a * n + m] = v;
    }
}

template <typename S>
__global__ void import_kernel(const BoxDesc *boxes, int bi, const double *srcd) {
    const BoxDesc &B = boxes[bi];
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t N = (size_t)B.N;
    if (idx >= 19 * N) return;
    const size_t a = idx / N, cell = idx % N;
    S *dst = (S *)(B.cur ? B.pop1 : B.pop0);
    // body cells have no slots of their own in the swapped layout
    if (swapped_now(B) && (B.flags[cell] & kOwnerMask)) return;
    Storage<S>::store(dst, current_slot(B, swapped_now(B), (int)a, (int)cell), (typename Storage<S>::C)srcd[idx],
                      B.scale);
}

// Copy the populations of box bi from buffer `from` in one layout to buffer
// `to` in the other (swapped: the swapped in-place layout, else own slots);
// fluid cells only.
template <typename S>
__global__ void relayout_kernel(const BoxDesc *boxes, int bi, int from, int to, int from_swapped, int to_swapped) {
    const BoxDesc &B = boxes[bi];
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t N = (size_t)B.N;
    if (idx >= 19 * N) return;
    const int a = (int)(idx / N), cell = (int)(idx % N);
    if (B.flags[cell] & kOwnerMask) return;
    const S *src = (const S *)(from ? B.pop1 : B.pop0);
    S *dst = (S *)(to ? B.pop1 : B.pop0);
    const auto v = Storage<S>::load(src, current_slot(B, from_swapped != 0, a, cell), B.inv_scale);
    Storage<S>::store(dst, current_slot(B, to_swapped != 0, a, cell), v, B.scale);
}

// Plain streaming copy: each thread moves four 16-byte vectors per round with
// independent loads in flight (a grid that covers the range does one vector
// per thread).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ __launch_bounds__(256) void copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                   size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const u32x4 a = ld<NT>(src + i), b = ld<NT>(src + i + stride), c = ld<NT>(src + i + 2 * stride),
                    d = ld<NT>(src + i + 3 * stride);
        st<NT>(dst + i, a);
        st<NT>(dst + i + stride, b);
        st<NT>(dst + i + 2 * stride, c);
        st<NT>(dst + i + 3 * stride, d);
    }
    for (; i < n; i += stride) st<NT>(dst + i, ld<NT>(src + i));
}

// The sweep's memory access pattern without its arithmetic: 19 streams of n
// elements, stream a at element offset a * stride, one element per thread,
// the 19 loads issued before the 19 stores.
template <typename T, bool NT>
__global__ __launch_bounds__(256) void stream_copy_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                          size_t n, size_t stride) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T v[19];
#pragma unroll
    for (int a = 0; a < 19; ++a)
        v[a] = NT ? __builtin_nontemporal_load(src + (size_t)a * stride + i) : src[(size_t)a * stride + i];
#pragma unroll
    for (int a = 0; a < 19; ++a) dst[(size_t)a * stride + i] = v[a];
}

template <typename T>
void launch_stream_copy(const void *src, void *dst, size_t n, size_t stride, bool nt, hipStream_t stream) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (nt)
        hipLaunchKernelGGL((stream_copy_kernel<T, true>), dim3(blocks), dim3(256), 0, stream, (const T *)src,
                           (T *)dst, n, stride);
    else
        hipLaunchKernelGGL((stream_copy_kernel<T, false>), dim3(blocks), dim3(256), 0, stream, (const T *)src,
                           (T *)dst, n, stride);
}

__global__ void save_hist_kernel(const BoxDesc *boxes, BodyHist *out) {
    const BoxDesc &B = boxes[0];
    const int b = threadIdx.x;
    if (b >= B.nb) return;
    const DevBody &d = B.bodies[b];
    for (int q = 0; q < 3; ++q) {
        out[b].D[q] = d.D[q];
        out[b].V[q] = d.V[q];
        out[b].O[q] = d.O[q];
    }
    for (int q = 0; q < 4; ++q) out[b].q[q] = d.q[q];
}

__global__ void set_layout_kernel(BoxDesc *boxes, int bi, int cur, int aa) {
    boxes[bi].cur = cur;
    boxes[bi].aa = aa;
}

// Switch every box between the two-buffer and the in-place sweep: the
// populations go to the other buffer in the layout of the new mode at the
// box's present step (no copy where both layouts agree).  Graphs captured
// for the old mode are dropped by the caller where needed.
int set_streaming(lbm_ctx *c, bool aa) {
    if (aa == c->aa) return LBM_OK;
    const int nbox = (int)c->boxes.size();
    std::vector<BoxDesc> d(nbox);
    int rc = copy_sync(c, d.data(), c->d_boxes, sizeof(BoxDesc) * nbox, hipMemcpyDeviceToHost);
    if (rc) return rc;
    for (int b = 0; b < nbox; ++b) {
        const bool odd = (d[b].step & 1) != 0;
        const bool from_swapped = c->aa && odd, to_swapped = aa && odd;
        int cur = d[b].cur;
        if (from_swapped != to_swapped) {
            const size_t n = (size_t)19 * c->boxes[b].N;
            const unsigned blocks = (unsigned)((n + 255) / 256);
            rc = dispatch_storage(c->storage, [&](auto *tag) -> int {
                using S = std::remove_pointer_t<decltype(tag)>;
                hipLaunchKernelGGL(relayout_kernel<S>, dim3(blocks), dim3(256), 0, c->stream, c->d_boxes, b, cur,
                                   cur ^ 1, from_swapped ? 1 : 0, to_swapped ? 1 : 0);
                return LBM_OK;
            });
            if (rc) return rc;
            cur ^= 1;
        }
        hipLaunchKernelGGL(set_layout_kernel, dim3(1), dim3(1), 0, c->stream, c->d_boxes, b, cur, aa ? 1 : 0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("relayout: ") + hipGetErrorString(e));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->aa = aa;
    return LBM_OK;
}

__global__ void set_state_kernel(BoxDesc *boxes, long long step, int cur) {
    boxes[0].step = step;
    boxes[0].cur = cur;
}

__global__ void init_adjoint_kernel(AdjBody *adj, const double *w, int nb, double *grad) {
    const int b = threadIdx.x;
    if (b < 3) grad[b] = 0.0;
    if (b >= nb) return;
    AdjBody &a = adj[b];
    for (int q = 0; q < 3; ++q) {
        a.lD[q] = w[3 * b + q];
        a.lV[q] = a.lO[q] = a.lF[q] = a.lT[q] = a.muV[q] = a.lDs[q] = a.lVs[q] = 0.0;
        a.lFn[q] = a.lTn[q] = 0.0;
    }
}

int grow(lbm_ctx *c, void **p, size_t *have, size_t need) {
    if (*have >= need && *p) return LBM_OK;
    if (*p) HIP_TRY(c, hipFree(*p));
    *p = nullptr;
    HIP_TRY(c, hipMalloc(p, need));
    *have = need;
    return LBM_OK;
}

template <typename S>
int adjoint_impl(lbm_ctx *c, int64_t nsteps, int ce, const double *w_host, double *J, double *grad_host) {
    HostBox &h = c->boxes[0];
    const int nb = (int)h.bodies.size();
    const size_t state_bytes = (size_t)19 * h.stride * sizeof(S);
    const int64_t K = (nsteps + ce - 1) / ce;
    int rc;
    // scratch: K checkpoints + the final state; one segment of states
    if ((rc = grow(c, &c->adj_ckpt, &c->adj_ckpt_bytes, state_bytes * (K + 1)))) return rc;
    if ((rc = grow(c, &c->adj_seg, &c->adj_seg_bytes, state_bytes * ce))) return rc;
    for (int q = 0; q < 2; ++q) {
        size_t have = c->adj_lam_bytes;
        if ((rc = grow(c, (void **)&c->adj_lam[q], &have, sizeof(double) * 19 * h.stride))) return rc;
    }
    c->adj_lam_bytes = sizeof(double) * 19 * h.stride;
    if ((rc = grow(c, (void **)&c->adj_hist, &c->adj_hist_bytes, sizeof(BodyHist) * nb * (nsteps + 1)))) return rc;
    if ((rc = grow(c, (void **)&c->adj_ckpt_bodies, &c->adj_ckpt_bodies_bytes, sizeof(DevBody) * kMaxBodies * (K + 1))))
        return rc;
    if (!c->adj_body) HIP_TRY(c, hipMalloc(&c->adj_body, sizeof(AdjBody) * kMaxBodies));
    if (!c->adj_grad) HIP_TRY(c, hipMalloc(&c->adj_grad, sizeof(double) * 4));
    if (c->adj_lrec_cap < h.link_cap) {
        if (c->adj_lrec) HIP_TRY(c, hipFree(c->adj_lrec));
        HIP_TRY(c, hipMalloc(&c->adj_lrec, sizeof(AdjLinkRec) * h.link_cap));
        c->adj_lrec_cap = h.link_cap;
    }
    if (c->work_dirty && (rc = rebuild_work(c))) return rc;
    // current step, buffer and flags at the start
    BoxDesc d0;
    HIP_TRY(c, hipMemcpyAsync(&d0, c->d_boxes, sizeof(BoxDesc), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const long long step0 = d0.step;
    const int cur0 = d0.cur;
    // owner changes made by the mappings so far; any during the forward run
    // (even a cell covered and uncovered again) breaks the fixed-flag reverse pass
    unsigned changes0 = 0, changes1 = 0;
    if ((rc = copy_sync(c, &changes0, &h.ctl->owner_changes, sizeof(unsigned), hipMemcpyDeviceToHost))) return rc;
    auto pop = [&](int cur) { return cur ? h.p.pop[1] : h.p.pop[0]; };
    auto ckpt = [&](int64_t k) { return (char *)c->adj_ckpt + (size_t)k * state_bytes; };
    auto seg = [&](int64_t m) { return (char *)c->adj_seg + (size_t)m * state_bytes; };
    const size_t body_bytes = sizeof(DevBody) * nb;
    // forward pass with checkpoints and the body history
    hipLaunchKernelGGL(save_hist_kernel, dim3(1), dim3(64), 0, c->stream, c->d_boxes, c->adj_hist);
    for (int64_t s = 0; s < nsteps; ++s) {
        const int cur = cur0 ^ (int)(s & 1);
        if (s % ce == 0) {
            HIP_TRY(c, hipMemcpyAsync(ckpt(s / ce), pop(cur), state_bytes, hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(c->adj_ckpt_bodies + (s / ce) * kMaxBodies, h.d_bodies, body_bytes,
                                      hipMemcpyDeviceToDevice, c->stream));
        }
        if ((rc = launch_step(c))) return rc;
        hipLaunchKernelGGL(save_hist_kernel, dim3(1), dim3(64), 0, c->stream, c->d_boxes,
                           c->adj_hist + (size_t)(s + 1) * nb);
    }
    const int cur_end = cur0 ^ (int)(nsteps & 1);
    HIP_TRY(c, hipMemcpyAsync(ckpt(K), pop(cur_end), state_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->adj_ckpt_bodies + K * kMaxBodies, h.d_bodies, body_bytes, hipMemcpyDeviceToDevice,
                              c->stream));
    if ((rc = copy_sync(c, &changes1, &h.ctl->owner_changes, sizeof(unsigned), hipMemcpyDeviceToHost))) return rc;
    if (changes1 != changes0)
        return fail(c, LBM_E_STATE, "the mapping changed during the run; the adjoint holds the flags fixed");
    // objective
    std::vector<BodyHist> fin(nb);
    if ((rc = copy_sync(c, fin.data(), c->adj_hist + (size_t)nsteps * nb, sizeof(BodyHist) * nb,
                        hipMemcpyDeviceToHost)))
        return rc;
    double Jv = 0.0;
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < 3; ++q) Jv += w_host[3 * b + q] * fin[b].D[q];
    *J = Jv;
    // reverse pass
    double *wdev = nullptr;
    HIP_TRY(c, hipMalloc(&wdev, sizeof(double) * 3 * nb));
    if ((rc = copy_sync(c, wdev, w_host, sizeof(double) * 3 * nb, hipMemcpyHostToDevice))) return rc;
    hipLaunchKernelGGL(init_adjoint_kernel, dim3(1), dim3(64), 0, c->stream, c->adj_body, wdev, nb, c->adj_grad);
    HIP_TRY(c, hipMemsetAsync(c->adj_lam[0], 0, c->adj_lam_bytes, c->stream));
    int lcur = 0;  // adj_lam[lcur] holds the adjoint of the populations after the step being reversed
    hipLaunchKernelGGL(adjoint_body_kernel, dim3(1), dim3(kCoupleThreads), 0, c->stream, c->d_boxes, c->adj_body,
                       (const BodyHist *)nullptr, c->adj_hist + (size_t)(nsteps - 1) * nb, c->adj_lrec,
                       (long long)(step0 + nsteps - 1), 0, c->adj_grad);
    const unsigned blocks = (unsigned)((h.N + 255) / 256);
    for (int64_t k = K - 1; k >= 0; --k) {
        const int64_t s0 = k * ce, s1 = std::min<int64_t>(s0 + ce, nsteps);
        const int cur = cur0 ^ (int)(s0 & 1);
        // restore the checkpoint and recompute the segment's states
        HIP_TRY(c, hipMemcpyAsync(pop(cur), ckpt(k), state_bytes, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(h.d_bodies, c->adj_ckpt_bodies + k * kMaxBodies, body_bytes,
                                  hipMemcpyDeviceToDevice, c->stream));
        hipLaunchKernelGGL(set_state_kernel, dim3(1), dim3(1), 0, c->stream, c->d_boxes, step0 + s0, cur);
        for (int64_t m = s0; m < s1; ++m) {
            HIP_TRY(c, hipMemcpyAsync(seg(m - s0), pop(cur0 ^ (int)(m & 1)), state_bytes, hipMemcpyDeviceToDevice,
                                      c->stream));
            if (m + 1 < s1 && (rc = launch_step(c))) return rc;
        }
        for (int64_t n = s1 - 1; n >= s0; --n) {
            AdjArgs args;
            args.state = seg(n - s0);
            args.lam_next = c->adj_lam[lcur];
            args.lam = c->adj_lam[lcur ^ 1];
            args.hist = c->adj_hist + (size_t)n * nb;
            args.adj = c->adj_body;
            args.lrec = c->adj_lrec;
            hipLaunchKernelGGL(adjoint_sweep_kernel<S>, dim3(blocks), dim3(256), 0, c->stream, c->d_boxes, args);
            const long long nprev = (n >= 1) ? (long long)(step0 + n - 1) : -1;
            hipLaunchKernelGGL(adjoint_body_kernel, dim3(1), dim3(kCoupleThreads), 0, c->stream, c->d_boxes,
                               c->adj_body, (const BodyHist *)nullptr,
                               c->adj_hist + (size_t)(n >= 1 ? n - 1 : 0) * nb, c->adj_lrec, nprev, 1, c->adj_grad);
            lcur ^= 1;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("adjoint launch: ") + hipGetErrorString(e));
    HIP_TRY(c, hipMemcpyAsync(grad_host, c->adj_grad, sizeof(double) * 3, hipMemcpyDeviceToHost, c->stream));
    // back to the state after the forward run
    HIP_TRY(c, hipMemcpyAsync(pop(cur_end), ckpt(K), state_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(h.d_bodies, c->adj_ckpt_bodies + K * kMaxBodies, body_bytes, hipMemcpyDeviceToDevice,
                              c->stream));
    hipLaunchKernelGGL(set_state_kernel, dim3(1), dim3(1), 0, c->stream, c->d_boxes, step0 + nsteps, cur_end);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipFree(wdev));
    h.steps += nsteps;
    return LBM_OK;
}

// The input checks of the integrator-only runs (lbm_vacuum_run and its
// allocation-free variant).
int validate_vacuum(const lbm_body *bodies, int32_t nb, const lbm_spring *springs, int32_t ns,
                    const lbm_drive *drives, int32_t nd, int32_t nsys, int64_t nsteps, double *traj,
                    int64_t traj_cap) {
    if (!bodies || nb < 1 || nb > kMaxBodies || ns < 0 || ns > kMaxSprings || nd < 0 || nd > kMaxDrives ||
        (ns && !springs) || (nd && !drives) || nsys < 1 || nsys > 65535 || nsteps < 0 || traj_cap < 0 ||
        (traj && traj_cap == 0))
        return LBM_E_ARG;
    for (int s = 0; s < nsys; ++s) {
        for (int b = 0; b < nb; ++b) {
            const lbm_body &x = bodies[(size_t)s * nb + b];
            if (x.kinematic < 0 || x.kinematic > 2 || !(x.mass > 0) || !(x.inertia[0] > 0) || !(x.inertia[1] > 0) ||
                !(x.inertia[2] > 0))
                return LBM_E_ARG;
        }
        for (int k = 0; k < ns; ++k) {
            const lbm_spring &x = springs[(size_t)s * ns + k];
            if (x.i < 0 || x.i >= nb || x.j < 0 || x.j >= nb || x.i == x.j || !(x.rest_len >= 0)) return LBM_E_ARG;
        }
        for (int d = 0; d < nd; ++d) {
            const lbm_drive &x = drives[(size_t)s * nd + d];
            if (x.left < 0 || x.left >= nb || x.right < 0 || x.right >= nb || x.middle < 0 || x.middle >= nb ||
                !(x.period > 0))
                return LBM_E_ARG;
        }
    }
    return LBM_OK;
}

DevSpring to_dev_spring(const lbm_spring &x) { return {x.i, x.j, x.k, x.gamma, x.rest_len}; }

DevDrive to_dev_drive(const lbm_drive &x) {
    return {x.left, x.middle, x.right, x.gate_lagged, x.amplitude, x.period, x.phase_lag, (long long)x.off_left,
            (long long)x.off_right};
}

// Descriptor of integrator-only system s: its tables in the device arrays
// given, its slice of the caller's trajectory ring.
BoxDesc vacuum_desc(int s, int nb, int ns, int nd, DevBody *bodies, DevSpring *springs, DevDrive *drives, double *traj,
                    int64_t traj_cap) {
    BoxDesc d;
    std::memset(&d, 0, sizeof(d));
    d.nb = nb;
    d.ns = ns;
    d.nd = nd;
    d.bodies = bodies + (size_t)s * nb;
    d.springs = springs + (size_t)s * ns;
    d.drives = drives + (size_t)s * nd;
    d.traj = traj ? traj + (size_t)s * traj_cap * nb * 16 : nullptr;
    d.traj_cap = traj ? traj_cap : 0;
    return d;
}

// Device tables of the allocation-free integrator-only run: one array on
// every GPU the library runs on, held until the process ends.  Host code
// uses the address hipGetSymbolAddress returns on the current device, never
// the array's name.
constexpr size_t kNoAllocScratch = (size_t)1 << 20;
static_assert(kNoAllocScratch == LBM_NOALLOC_SCRATCH_BYTES, "header and library agree on the scratch size");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

std::mutex scratch_mutex;
std::vector<void *> scratch_addr;   // by device ordinal, filled on the first call on that device

// The current device's address of `scratch`, looked up once per device.
int scratch_on_current_device(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return LBM_E_HIP;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if ((int)scratch_addr.size() <= dev) scratch_addr.resize(dev + 1, nullptr);
    if (!scratch_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LBM_E_HIP;
        scratch_addr[dev] = p;
    }
    *out = scratch_addr[dev];
    return LBM_OK;
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// Copy n records of type D converted from the host array src by `conv` to
// the device array dst, through a buffer on the stack (a few records at a
// time, each copy waited for before the buffer is reused).
template <typename D, typename H, typename Conv>
int stage_records(D *dst, const H *src, size_t n, Conv conv, hipStream_t st) {
    constexpr size_t kChunk = 16;
    D buf[kChunk];
    for (size_t q0 = 0; q0 < n; q0 += kChunk) {
        const size_t m = std::min(kChunk, n - q0);
        for (size_t q = 0; q < m; ++q) buf[q] = conv(src[q0 + q]);
        if (hipMemcpyAsync(dst + q0, buf, sizeof(D) * m, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return LBM_E_HIP;
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_adjoint(lbm_ctx *c, int64_t nsteps, int32_t checkpoint_every, const double *dJ_ddisp, double *J,
                double *grad) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->boxes.size() != 1) return fail(c, LBM_E_ARG, "the adjoint runs on a single-box context");
    if (nsteps < 1 || checkpoint_every < 1 || !dJ_ddisp || !J || !grad)
        return fail(c, LBM_E_ARG, "nsteps and checkpoint_every must be >= 1; outputs must be non-null");
    if (c->boxes[0].limit >= 0) return fail(c, LBM_E_ARG, "the adjoint box must not have a step limit");
    if (c->boxes[0].bodies.empty()) return fail(c, LBM_E_STATE, "no bodies set");
    if (c->flow_any) return fail(c, LBM_E_STATE, "stop the flow average before the adjoint (its recomputation would sample)");
    if (c->force_any) return fail(c, LBM_E_STATE, "the adjoint does not cover the test-only body force");
    // the reverse pass keeps and replays its states in the two-buffer layout
    const bool was_aa = c->aa;
    if (was_aa && (rc = set_streaming(c, false))) return rc;
    rc = dispatch_storage(c->storage, [&](auto *tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        return adjoint_impl<S>(c, nsteps, checkpoint_every, dJ_ddisp, J, grad);
    });
    if (was_aa) {
        const int back = set_streaming(c, true);
        if (!rc) rc = back;
    }
    return rc;
}

int lbm_vacuum_run(const lbm_body *bodies, int32_t nb, const lbm_spring *springs, int32_t ns,
                   const lbm_drive *drives, int32_t nd, int32_t nsys, int64_t nsteps, double *traj,
                   int64_t traj_cap, lbm_body *out, void *stream) {
    if (int rc = validate_vacuum(bodies, nb, springs, ns, drives, nd, nsys, nsteps, traj, traj_cap)) return rc;
    std::vector<DevBody> db((size_t)nsys * nb);
    std::vector<DevSpring> ds((size_t)nsys * ns);
    std::vector<DevDrive> dd((size_t)nsys * nd);
    for (size_t q = 0; q < db.size(); ++q) db[q] = to_dev(bodies[q]);
    for (size_t q = 0; q < ds.size(); ++q) ds[q] = to_dev_spring(springs[q]);
    for (size_t q = 0; q < dd.size(); ++q) dd[q] = to_dev_drive(drives[q]);
    DevBody *g_bodies = nullptr;
    DevSpring *g_springs = nullptr;
    DevDrive *g_drives = nullptr;
    BoxDesc *g_desc = nullptr;
    hipStream_t st = (hipStream_t)stream;
    int rc = LBM_OK;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && rc == LBM_OK) rc = LBM_E_HIP;
        return rc == LBM_OK;
    };
    if (ok(hipMalloc(&g_bodies, sizeof(DevBody) * db.size())) &&
        ok(hipMalloc(&g_springs, sizeof(DevSpring) * std::max<size_t>(ds.size(), 1))) &&
        ok(hipMalloc(&g_drives, sizeof(DevDrive) * std::max<size_t>(dd.size(), 1))) &&
        ok(hipMalloc(&g_desc, sizeof(BoxDesc) * nsys))) {
        std::vector<BoxDesc> desc(nsys);
        for (int s = 0; s < nsys; ++s) desc[s] = vacuum_desc(s, nb, ns, nd, g_bodies, g_springs, g_drives, traj, traj_cap);
        if (ok(hipMemcpyAsync(g_bodies, db.data(), sizeof(DevBody) * db.size(), hipMemcpyHostToDevice, st)) &&
            (ds.empty() || ok(hipMemcpyAsync(g_springs, ds.data(), sizeof(DevSpring) * ds.size(),
                                             hipMemcpyHostToDevice, st))) &&
            (dd.empty() || ok(hipMemcpyAsync(g_drives, dd.data(), sizeof(DevDrive) * dd.size(),
                                             hipMemcpyHostToDevice, st))) &&
            ok(hipMemcpyAsync(g_desc, desc.data(), sizeof(BoxDesc) * nsys, hipMemcpyHostToDevice, st))) {
            hipLaunchKernelGGL(vacuum_kernel, dim3(nsys), dim3(kCoupleThreads), 0, st, g_desc, (long long)nsteps);
            if (ok(hipGetLastError()) &&
                ok(hipMemcpyAsync(db.data(), g_bodies, sizeof(DevBody) * db.size(), hipMemcpyDeviceToHost, st)) &&
                ok(hipMemcpyAsync(desc.data(), g_desc, sizeof(BoxDesc) * nsys, hipMemcpyDeviceToHost, st)) &&
                ok(hipStreamSynchronize(st))) {
                for (int s = 0; s < nsys; ++s)
                    if (desc[s].status == LBM_E_UNSTABLE) rc = LBM_E_UNSTABLE;
                if (out)
                    for (size_t q = 0; q < db.size(); ++q) out[q] = from_dev(db[q]);
            }
        }
    }
    if (g_bodies || g_desc) (void)hipStreamSynchronize(st);
    (void)hipFree(g_bodies);
    (void)hipFree(g_springs);
    (void)hipFree(g_drives);
    (void)hipFree(g_desc);
    return rc;
}

int lbm_vacuum_run_noalloc(const lbm_body *bodies, int32_t nb, const lbm_spring *springs, int32_t ns,
                           const lbm_drive *drives, int32_t nd, int32_t nsys, int64_t nsteps, double *traj,
                           int64_t traj_cap, lbm_body *out, void *stream) {
    if (int rc = validate_vacuum(bodies, nb, springs, ns, drives, nd, nsys, nsteps, traj, traj_cap)) return rc;
    const size_t nbod = (size_t)nsys * nb, nspr = (size_t)nsys * ns, ndrv = (size_t)nsys * nd;
    const size_t off_spr = align256(sizeof(DevBody) * nbod);
    const size_t off_drv = off_spr + align256(sizeof(DevSpring) * nspr);
    const size_t off_desc = off_drv + align256(sizeof(DevDrive) * ndrv);
    if (off_desc + sizeof(BoxDesc) * (size_t)nsys > kNoAllocScratch) return LBM_E_ARG;
    void *base = nullptr;
    if (int rc = scratch_on_current_device(&base)) return rc;
    char *p = (char *)base;
    DevBody *g_bodies = (DevBody *)p;
    DevSpring *g_springs = (DevSpring *)(p + off_spr);
    DevDrive *g_drives = (DevDrive *)(p + off_drv);
    BoxDesc *g_desc = (BoxDesc *)(p + off_desc);
    hipStream_t st = (hipStream_t)stream;
    int rc = stage_records(g_bodies, bodies, nbod, [](const lbm_body &x) { return to_dev(x); }, st);
    if (!rc) rc = stage_records(g_springs, springs, nspr, [](const lbm_spring &x) { return to_dev_spring(x); }, st);
    if (!rc) rc = stage_records(g_drives, drives, ndrv, [](const lbm_drive &x) { return to_dev_drive(x); }, st);
    if (!rc) {
        struct Sys { int s; };
        constexpr size_t kChunk = 16;
        Sys idx[kChunk];
        for (size_t s0 = 0; s0 < (size_t)nsys && !rc; s0 += kChunk) {
            const size_t m = std::min(kChunk, (size_t)nsys - s0);
            for (size_t q = 0; q < m; ++q) idx[q].s = (int)(s0 + q);
            rc = stage_records(g_desc + s0, idx, m, [&](const Sys &x) {
                return vacuum_desc(x.s, nb, ns, nd, g_bodies, g_springs, g_drives, traj, traj_cap);
            }, st);
        }
    }
    if (rc) return rc;
    hipLaunchKernelGGL(vacuum_kernel, dim3(nsys), dim3(kCoupleThreads), 0, st, g_desc, (long long)nsteps);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return LBM_E_HIP;
    // results through buffers on the stack
    constexpr size_t kChunk = 16;
    if (out) {
        DevBody buf[kChunk];
        for (size_t q0 = 0; q0 < nbod; q0 += kChunk) {
            const size_t m = std::min(kChunk, nbod - q0);
            if (hipMemcpyAsync(buf, g_bodies + q0, sizeof(DevBody) * m, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return LBM_E_HIP;
            for (size_t q = 0; q < m; ++q) out[q0 + q] = from_dev(buf[q]);
        }
    }
    int status[kChunk];
    for (size_t s0 = 0; s0 < (size_t)nsys; s0 += kChunk) {
        const size_t m = std::min(kChunk, (size_t)nsys - s0);
        for (size_t q = 0; q < m; ++q)
            if (hipMemcpyAsync(&status[q], &g_desc[s0 + q].status, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
                return LBM_E_HIP;
        if (hipStreamSynchronize(st) != hipSuccess) return LBM_E_HIP;
        for (size_t q = 0; q < m; ++q)
            if (status[q] == LBM_E_UNSTABLE) rc = LBM_E_UNSTABLE;
    }
    return rc;
}

int lbm_copy_kernel(const void *src, void *dst, int64_t bytes, int32_t blocks_per_cu, int32_t nontemporal,
                    void *stream) {
    if (!src || !dst || bytes <= 0 || (bytes % 16) != 0 || blocks_per_cu < 0) return LBM_E_ARG;
    const size_t n = (size_t)bytes / 16;
    if ((n + 255) / 256 > 0x7fffffffu) return LBM_E_ARG;
    // blocks_per_cu = 0: one 16-byte vector per thread over the whole range
    const unsigned blocks = blocks_per_cu == 0
                                ? (unsigned)((n + 255) / 256)
                                : (unsigned)std::min<size_t>((n + 1023) / 1024, 256 * (size_t)blocks_per_cu);
    if (nontemporal)
        hipLaunchKernelGGL(copy_kernel<true>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const u32x4 *)src,
                           (u32x4 *)dst, n);
    else
        hipLaunchKernelGGL(copy_kernel<false>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const u32x4 *)src,
                           (u32x4 *)dst, n);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_stream_copy(const void *src, void *dst, int64_t n, int64_t stride, int32_t elem_bytes, int32_t nontemporal,
                    void *stream) {
    if (!src || !dst || n <= 0 || stride < n || (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8))
        return LBM_E_ARG;
    // the grid and the largest element offset must fit their types
    if ((n + 255) / 256 > 0x7fffffffLL || stride > (INT64_MAX / 19) / 8) return LBM_E_ARG;
    const hipStream_t s = (hipStream_t)stream;
    if (elem_bytes == 2) launch_stream_copy<uint16_t>(src, dst, (size_t)n, (size_t)stride, nontemporal != 0, s);
    else if (elem_bytes == 4) launch_stream_copy<uint32_t>(src, dst, (size_t)n, (size_t)stride, nontemporal != 0, s);
    else launch_stream_copy<uint64_t>(src, dst, (size_t)n, (size_t)stride, nontemporal != 0, s);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
}

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
    if (h.mapped && !h.bodies.empty()) {
        rc = copy_sync(c, old.data(), h.d_bodies, sizeof(DevBody) * old.size(), hipMemcpyDeviceToHost);
        if (rc) return rc;
    }
    h.bodies.assign(bodies, bodies + nb);
    h.springs.assign(springs, springs + ns);
    h.drives.assign(drives, drives + nd);
    // link capacity: 18 links per cell of every body's bounding box plus one layer
    long long cap = 0;
    for (const auto &b : h.bodies) {
        if (b.shape == LBM_SLAB) {
            // a plane across the box: at most every face cell of the box twice over
            const long long nx = h.p.nx, ny = h.p.ny, nz = h.p.nz;
            cap += 18 * 2 * (nx * ny + ny * nz + nz * nx);
            continue;
        }
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
            HIP_TRY(c, hipFree(h.link_rec));
            HIP_TRY(c, hipFree(h.frec));
            HIP_TRY(c, hipFree(h.grp_pos));
        }
        HIP_TRY(c, hipMalloc(&h.link_cell, sizeof(int) * cap));
        HIP_TRY(c, hipMalloc(&h.link_dir, cap));
        HIP_TRY(c, hipMalloc(&h.link_body, cap));
        HIP_TRY(c, hipMalloc(&h.link_rec, sizeof(LinkRec) * cap));
        HIP_TRY(c, hipMalloc(&h.frec, sizeof(ForceRec) * cap));
        HIP_TRY(c, hipMalloc(&h.grp_pos, sizeof(int) * cap));
        h.link_cap = (int)cap;
    }
    if (!h.d_bodies) {
        HIP_TRY(c, hipMalloc(&h.d_bodies, sizeof(DevBody) * kMaxBodies));
        HIP_TRY(c, hipMalloc(&h.d_springs, sizeof(DevSpring) * kMaxSprings));
        HIP_TRY(c, hipMalloc(&h.d_drives, sizeof(DevDrive) * kMaxDrives));
    }
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
        int64_t s = 0;
        if (!c->timing && c->graph_steps > 0) {
            if ((rc = ensure_graphs(c, run))) return rc;
            if (run >= c->graph_steps)
                for (; s + c->graph_len <= run; s += c->graph_len) HIP_TRY(c, hipGraphLaunch(c->graph, c->stream));
            if (s < run) {
                HIP_TRY(c, hipGraphLaunch(c->tail, c->stream));
                s += c->tail_len;
            }
        }
        for (; s < run; ++s) {
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

int lbm_prepare(lbm_ctx *c, int64_t nsteps) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsteps < 0) return fail(c, LBM_E_ARG, "nsteps < 0");
    if (c->work_dirty && (rc = rebuild_work(c))) return rc;
    if (c->nactive == 0 || nsteps == 0) return LBM_OK;
    int64_t run = nsteps;
    for (int b : c->active_host) {
        const HostBox &h = c->boxes[b];
        if (h.limit >= 0) run = std::min<int64_t>(run, h.limit - h.steps);
    }
    return ensure_graphs(c, run);
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
    HIP_TRY(c, hipMemcpyAsync(cell, h.link_cell, sizeof(int) * d.link_count, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(dir, h.link_dir, d.link_count, hipMemcpyDeviceToHost, c->stream));
    return copy_sync(c, body, h.link_body, d.link_count, hipMemcpyDeviceToHost);
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

int lbm_export_cells(lbm_ctx *c, int32_t box, const int32_t *cells, int64_t n, double *dst) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!cells || !dst))) return fail(c, LBM_E_ARG, "null cells or destination");
    if (n == 0) return LBM_OK;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    return dispatch_storage(c->storage, [&](auto *tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(export_cells_kernel<S>, dim3(blocks), dim3(256), 0, c->stream, c->d_boxes, (int)box,
                           (const int *)cells, (long long)n, dst);
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

__global__ void flow_mean_kernel(const double *sum, const int *count, long long n, double *mean, int *cnt_out) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int k = count[c];
    for (int q = 0; q < 3; ++q) mean[q * n + c] = k ? sum[q * n + c] / (double)k : 0.0;
    if (cnt_out) cnt_out[c] = k;
}

int lbm_flow_average_begin(lbm_ctx *c, int32_t box, int32_t every) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (every < 0) return fail(c, LBM_E_ARG, "every must be >= 0");
    if (every > 0 && c->force_any) return fail(c, LBM_E_STATE, "no flow average with the test-only body force");
    HostBox &h = c->boxes[box];
    if (every > 0) {
        if (!h.flow_sum) {
            double *sum = nullptr;
            int *cnt = nullptr;
            if (hipMalloc(&sum, sizeof(double) * 3 * (size_t)h.N) != hipSuccess ||
                hipMalloc(&cnt, sizeof(int) * (size_t)h.N) != hipSuccess) {
                (void)hipFree(sum);
                return fail(c, LBM_E_HIP, "out of device memory for the flow average");
            }
            h.flow_sum = sum;
            h.flow_count = cnt;
        }
        HIP_TRY(c, hipMemsetAsync(h.flow_sum, 0, sizeof(double) * 3 * (size_t)h.N, c->stream));
        HIP_TRY(c, hipMemsetAsync(h.flow_count, 0, sizeof(int) * (size_t)h.N, c->stream));
    }
    h.flow_every = every;
    rc = upload_desc(c, box);
    if (rc) return rc;
    c->flow_any = false;
    for (const HostBox &o : c->boxes) c->flow_any = c->flow_any || o.flow_every > 0;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    return LBM_OK;
}

int lbm_flow_average_get(lbm_ctx *c, int32_t box, double *mean, int32_t *count) {
    int rc = check_box(c, box);
    if (rc) return rc;
    const HostBox &h = c->boxes[box];
    if (!mean) return fail(c, LBM_E_ARG, "null output");
    if (!h.flow_sum) return fail(c, LBM_E_STATE, "no flow average was begun on this box");
    const long long n = h.N;
    hipLaunchKernelGGL(flow_mean_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, h.flow_sum,
                       h.flow_count, n, mean, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, LBM_E_HIP, std::string("flow mean launch: ") + hipGetErrorString(e));
    return LBM_OK;
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
        if (d[b].status == LBM_E_SYNC)
            return fail(c, LBM_E_SYNC, "box " + std::to_string(b) + ": coupling workgroups timed out at a barrier");
    }
    return LBM_OK;
}

int lbm_tune(lbm_ctx *c, int32_t key, int64_t value) {
    int rc = check_ctx(c);
    if (rc) return rc;
    switch (key) {
        case LBM_TUNE_BLOCK:
            if (value != 128 && value != 256 && value != 512) return fail(c, LBM_E_ARG, "block must be 128, 256 or 512");
            c->block = (int)value;
            c->work_dirty = true;
            break;
        case LBM_TUNE_XCD_ORDER:
            if (value != 0 && value != 1) return fail(c, LBM_E_ARG, "xcd order is 0 or 1");
            c->xcd_order = (int)value;
            break;
        case LBM_TUNE_GRAPH_STEPS:
            if (value < 0 || value > 4096) return fail(c, LBM_E_ARG, "graph steps in [0, 4096]");
            c->graph_steps = (int)value;
            break;
        case LBM_TUNE_NONTEMPORAL:
            if (value != 0 && value != 1) return fail(c, LBM_E_ARG, "nontemporal is 0 or 1");
            c->nontemporal = (int)value;
            break;
        case LBM_TUNE_FULL_REMAP:
            if (value != 0 && value != 1) return fail(c, LBM_E_ARG, "full remap is 0 or 1");
            c->force_map = value != 0;
            break;
        case LBM_TUNE_COOP_REMAP:
            if (value < 0 || value > 2) return fail(c, LBM_E_ARG, "cooperative remap is 0, 1 or 2");
            c->coop_remap = (int)value;
            break;
        case LBM_TUNE_STREAMING:
            if (value != 0 && value != 1) return fail(c, LBM_E_ARG, "streaming is 0 (two buffers) or 1 (in place)");
            if ((rc = set_streaming(c, value != 0))) return rc;
            break;
        default:
            return fail(c, LBM_E_ARG, "unknown tuning key");
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
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
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    (void)hipFree(c->adj_ckpt);
    (void)hipFree(c->adj_seg);
    (void)hipFree(c->adj_lam[0]);
    (void)hipFree(c->adj_lam[1]);
    (void)hipFree(c->adj_hist);
    (void)hipFree(c->adj_ckpt_bodies);
    (void)hipFree(c->adj_body);
    (void)hipFree(c->adj_lrec);
    (void)hipFree(c->adj_grad);
    for (auto &h : c->boxes) {
        (void)hipFree(h.d_bodies);
        (void)hipFree(h.d_springs);
        (void)hipFree(h.d_drives);
        (void)hipFree(h.link_cell);
        (void)hipFree(h.link_dir);
        (void)hipFree(h.link_body);
        (void)hipFree(h.link_rec);
        (void)hipFree(h.frec);
        (void)hipFree(h.grp_pos);
        (void)hipFree(h.link_base);
        (void)hipFree(h.old_owner);
        (void)hipFree(h.ctl);
        (void)hipFree(h.flow_sum);
        (void)hipFree(h.flow_count);
    }
    (void)hipFree(c->d_boxes);
    (void)hipFree(c->d_qmaps);
    (void)hipFree(c->d_margins);
    (void)hipFree(c->d_active);
    (void)hipFree(c->d_work);
    delete c;
}

}  // extern "C"
