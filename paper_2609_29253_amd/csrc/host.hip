// C-ABI of the patop library: validation, device tables and launches.
//
// set_geometry turns the SI description of the system into device tables in
// units of the fine radial step dr = c / (U fs): the voxel-to-transducer frame
// transform as an affine map of the voxel indices (Sec. 4.1 and Sec. 4.2
// frames), bounding spheres used to bound each brick's bin window
// (Eq. rmin_rmax), the per-bin scale of Eq. ui_area, the polyphase form of the
// convolution and down-sampling (Eq. discrete_conv, Eq. def_downsampling), and
// the midpoint quadrature points of Alg. 2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "geometry.h"
#include "kernels.h"
#include "patop.h"

using namespace patop;
using patop::geom::bounding_sphere;
using patop::geom::cross3;
using patop::geom::dot3;
using patop::geom::grid_box;

// Scratch of pat_forward_noalloc: the FP64 fine-bin coefficients f of one
// forward ([batch][K][Mcount] doubles), in a file-scope device array instead
// of the context's workspace, for callers that cannot allocate.  Every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// uses the array's name as an address: pat_create looks up each device's
// address once (that device current) and the entry point passes that pointer.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

// roctx range over one C-ABI call (host side: it brackets the validation and
// the enqueue of the call's kernels, which a profiler's kernel trace then
// attributes to it; no cost without a profiler attached)
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

constexpr int kMaxDevices = 64;

struct ScratchTable {
    std::mutex mu;
    bool done[kMaxDevices] = {};
    hipError_t err[kMaxDevices] = {};
    void* ptr[kMaxDevices] = {};
};

ScratchTable& scratch_table()
{
    static ScratchTable t;
    return t;
}

// device address of `scratch` on `device`, looked up at its first request with
// that device current (the caller has made it current); the status of the
// lookup is kept with it
hipError_t scratch_lookup(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    ScratchTable& t = scratch_table();
    std::lock_guard<std::mutex> lock(t.mu);
    if (!t.done[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        t.err[device] = e;
        t.ptr[device] = e == hipSuccess ? p : nullptr;
        t.done[device] = true;
    }
    *out = t.ptr[device];
    return t.err[device];
}

}  // namespace

struct pat_ctx {
    int device = 0;
    bool ready = false;
    std::string err;
    // geometry
    int K = 0;
    int64_t N = 0;
    int L = 0, U = 1, mode = 0, precision = 0, max_batch = 1;
    bool truncated = false;
    double work[2] = {-1.0, -1.0};   // area evaluations and pairs per volume (computed on demand)
    size_t ws_bytes = 0;
    LaunchPlan plan{};
    // device allocations
    TrDev* d_tr = nullptr;
    int32_t* d_kperm = nullptr;
    double* d_scale = nullptr;
    double* d_G = nullptr;
    double* d_qpts = nullptr;
    double* d_qdA = nullptr;
    double* d_f = nullptr;
    void* d_W = nullptr;
    double* d_z = nullptr;
    int32_t* d_sup = nullptr;       // support list [N], per-brick counts [nbricks], offsets [nbricks + 1],
                                    // brick order [nbricks]
    double2* d_lut = nullptr;       // E~ / F~ tables [kLutN^2] (lookup-table I_l)
    int32_t* d_items = nullptr;     // (transducer, time tile) forward: work items of both shape groups
};

namespace {

constexpr int32_t kMaxU = 1 << 16;   // up-sampling factors beyond this are rejected

int64_t floordiv64(int64_t a, int64_t b)
{
    int64_t q = a / b;
    return (q * b > a) ? q - 1 : q;
}

const char* kStatusText[] = {"ok",
                             "invalid argument",
                             "transducer frame is not orthonormal",
                             "invalid transducer shape parameters",
                             "grid closer than the radial-function support to a transducer",
                             "invalid system kernel",
                             "geometry not set",
                             "HIP device error",
                             "device out of memory",
                             "unsupported request"};

pat_status fail(pat_ctx* c, pat_status st, const std::string& msg)
{
    if (c) c->err = msg;
    return st;
}

void free_dev(pat_ctx* c)
{
    void** ptrs[] = {(void**)&c->d_tr, (void**)&c->d_kperm, (void**)&c->d_scale, (void**)&c->d_G,
                     (void**)&c->d_qpts, (void**)&c->d_qdA, (void**)&c->d_f, &c->d_W, (void**)&c->d_z,
                     (void**)&c->d_sup, (void**)&c->d_lut, (void**)&c->d_items};
    for (void** p : ptrs) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    c->ready = false;
    c->ws_bytes = 0;
}

struct DevGuard {
    int prev = -1;
    bool ok = false;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DevGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

const char* pat_status_string(int32_t s)
{
    if (s < 0 || s > (int32_t)PAT_E_UNSUPPORTED) return "unknown status";
    return kStatusText[s];
}

const char* pat_last_error(const pat_ctx* c) { return c ? c->err.c_str() : "null context"; }

pat_status pat_create(pat_ctx** out, int32_t device)
{
    if (!out) return PAT_E_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return PAT_E_DEVICE;
    pat_ctx* c = new (std::nothrow) pat_ctx();
    if (!c) return PAT_E_OOM;
    c->device = device;
    {
        // the no-allocation forward's scratch address on this device (kept
        // with its status; pat_forward_noalloc reports a failed lookup)
        DevGuard guard(device);
        void* p = nullptr;
        if (guard.ok) (void)scratch_lookup(device, &p);
    }
    *out = c;
    return PAT_OK;
}

void pat_destroy(pat_ctx* c)
{
    if (!c) return;
    {
        DevGuard g(c->device);
        if (g.ok) (void)hipDeviceSynchronize();
        free_dev(c);
    }
    delete c;
}

pat_status pat_set_geometry(pat_ctx* c, const pat_transducer* tr, int32_t K, const pat_grid* grid,
                            const pat_kernel* kernel, const pat_params* prm)
{
    Range r("pat_set_geometry");
    if (!c) return PAT_E_ARG;
    DevGuard guard(c->device);
    if (!guard.ok) return fail(c, PAT_E_DEVICE, "hipSetDevice failed");
    (void)hipDeviceSynchronize();
    free_dev(c);
    if (!tr || !grid || !kernel || !prm || K < 1) return fail(c, PAT_E_ARG, "null argument or K < 1");
    const pat_params& p = *prm;
    if (!(p.sound_speed > 0.0) || !(p.fs > 0.0) || !(p.t0 >= 0.0) || !std::isfinite(p.t0) || p.L < 1 || p.U < 1 ||
        p.max_batch < 1 || p.reserved != 0)
        return fail(c, PAT_E_ARG, "invalid sampling parameters");
    const int tile_log2 = (p.flags >> 8) & 0xF;
    const bool tiles = (p.flags & PAT_FLAG_TIME_TILES) != 0;
    if ((p.flags & ~(PAT_FLAG_TIME_TILES | 0xF00)) != 0 || (tile_log2 != 0 && (!tiles || tile_log2 < 5 || tile_log2 > 9)))
        return fail(c, PAT_E_ARG, "invalid flags");
    if (tiles && p.area_mode == PAT_AREA_QUADRATURE)
        return fail(c, PAT_E_ARG, "the time-tile forward serves the closed-form area modes");
    if (p.U > kMaxU) return fail(c, PAT_E_UNSUPPORTED, "U above 65536");
    if (p.area_mode != PAT_AREA_CLOSED && p.area_mode != PAT_AREA_QUADRATURE && p.area_mode != PAT_AREA_TRAPEZOID &&
        p.area_mode != PAT_AREA_LUT)
        return fail(c, PAT_E_ARG, "invalid area_mode");
    if (p.area_step < 1 || p.area_step > p.U || (p.area_mode == PAT_AREA_QUADRATURE && p.area_step != 1))
        return fail(c, PAT_E_ARG, "area_step must be in 1..U (1 for the quadrature)");
    if (p.precision != PAT_FP32 && p.precision != PAT_FP64) return fail(c, PAT_E_ARG, "invalid precision");
    if (p.area_mode == PAT_AREA_QUADRATURE &&
        (p.quad_n1 < 1 || p.quad_n2 < 1 || (int64_t)p.quad_n1 * p.quad_n2 > (1 << 16)))
        return fail(c, PAT_E_ARG, "invalid quadrature size");
    if (!kernel->h || kernel->len < 1 || kernel->len > (1 << 24) || !(kernel->kappa > 0.0))
        return fail(c, PAT_E_KERNEL, "empty kernel or kappa <= 0");
    for (int64_t i = 0; i < kernel->len; ++i)
        if (!std::isfinite(kernel->h[i])) return fail(c, PAT_E_KERNEL, "non-finite kernel tap");
    double dlow = 0.0;
    pat_status st = pat_check_geometry(tr, K, grid, kernel->kappa, &dlow);
    if (st != PAT_OK) {
        char buf[160];
        snprintf(buf, sizeof buf, "geometry check failed (%s), distance lower bound %.6g m", pat_status_string(st),
                 dlow);
        return fail(c, st, buf);
    }
    // each extent is >= 1 here; the product is formed only once it is known to fit
    if ((double)grid->n[0] * (double)grid->n[1] * (double)grid->n[2] >= 2147483648.0)
        return fail(c, PAT_E_UNSUPPORTED, "2^31 voxels or more");
    const int64_t N = grid->n[0] * grid->n[1] * grid->n[2];

    const double dr = p.sound_speed / (p.U * p.fs);
    const double r0 = p.t0 * p.U * p.fs;
    const bool surface = p.area_mode != PAT_AREA_QUADRATURE;
    const int step = p.area_step;
    const double da = dr * step;          // device length unit: one area shell
    const double r0a = r0 / step;
    const int64_t nf = kernel->n_first, nl = kernel->n_first + kernel->len - 1;
    const int64_t Mlo = 1 - nl, Mhi = (int64_t)p.U * p.L - nf;
    const int64_t Mcount = Mhi - Mlo + 1;
    if (Mcount < 1 || Mhi > (1 << 30) || Mlo < -(1 << 30)) return fail(c, PAT_E_UNSUPPORTED, "time axis too long");

    // ---- transducer table (da units)
    std::vector<TrDev> T(K);
    std::vector<int32_t> perm;
    int nplan = 0, ncyl = 0;
    double glo[3], ghi[3];
    grid_box(*grid, glo, ghi);
    double dmax_all = 0.0;
    for (int k = 0; k < K; ++k) {
        const pat_transducer& t = tr[k];
        double n3[3];
        cross3(t.e1, t.e2, n3);
        const double* ax[3];
        if (t.shape == PAT_PLANAR) { ax[0] = t.e1; ax[1] = t.e2; ax[2] = n3; ++nplan; }
        else { ax[0] = t.e2; ax[1] = n3; ax[2] = t.e1; ++ncyl; }
        TrDev& d = T[k];
        std::memset(&d, 0, sizeof d);
        double o[3] = {grid->origin[0] - t.c0[0], grid->origin[1] - t.c0[1], grid->origin[2] - t.c0[2]};
        for (int a = 0; a < 3; ++a) {
            d.base[a] = dot3(o, ax[a]) / da;
            for (int q = 0; q < 3; ++q) d.g[a][q] = grid->spacing * ax[a][q] / da;
        }
        double cen[3], rad;
        bounding_sphere(t, cen, rad);
        for (int a = 0; a < 3; ++a) d.cen[a] = cen[a] / da;
        d.rad = rad / da;
        if (t.shape == PAT_PLANAR) { d.p[0] = t.half_w / da; d.p[1] = t.half_h / da; }
        else {
            d.p[0] = t.radius / da; d.p[1] = t.theta_max; d.p[2] = t.half_len / da;
            d.cth = std::cos(t.theta_max); d.sth = std::sin(t.theta_max);
        }
        d.shape = t.shape;
        double far2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double f = std::max(std::fabs(glo[a] - cen[a]), std::fabs(ghi[a] - cen[a]));
            far2 += f * f;
        }
        dmax_all = std::max(dmax_all, std::sqrt(far2) + rad);
    }
    for (int k = 0; k < K; ++k)
        if (T[k].shape == PAT_PLANAR) perm.push_back(k);
    for (int k = 0; k < K; ++k)
        if (T[k].shape == PAT_CYLINDER) perm.push_back(k);
    c->truncated = (int64_t)std::ceil(dmax_all / dr - r0) + nl > (int64_t)p.U * p.L;

    // ---- per-bin scale (Eq. ui_area: U fs / (c tau_{m-1/2}); point method: U fs)
    std::vector<double> scale(Mcount);
    for (int64_t i = 0; i < Mcount; ++i) {
        if (surface) {
            double rm = r0 + (double)(Mlo + i) - 0.5;   // c tau_{m-1/2} / dr
            scale[i] = rm > 0.0 ? p.U * p.fs * dr / rm : 0.0;
        } else {
            scale[i] = p.U * p.fs * dr;
        }
    }
    // ---- polyphase filter G[j] = 1/U sum_{l'=1..U} h[j + l'],  j in [nf - U, nl - 1]
    const int jlo = (int)(nf - p.U), jcnt = (int)(kernel->len + p.U - 1);
    std::vector<double> G(jcnt, 0.0);
    for (int jj = 0; jj < jcnt; ++jj) {
        double acc = 0.0;
        for (int lp = 1; lp <= p.U; ++lp) {
            int64_t n = (int64_t)jlo + jj + lp;
            if (n >= nf && n <= nl) acc += kernel->h[n - nf];
        }
        G[jj] = acc / p.U;
    }
    // ---- quadrature points (midpoint tensor rule, barycentres of equal cells)
    std::vector<double> qp, qdA;
    int Q = 0;
    if (p.area_mode == PAT_AREA_QUADRATURE) {
        Q = p.quad_n1 * p.quad_n2;
        qp.resize((size_t)K * Q * 3);
        qdA.resize(K);
        for (int k = 0; k < K; ++k) {
            const pat_transducer& t = tr[k];
            double n3[3];
            cross3(t.e1, t.e2, n3);
            double* P = qp.data() + (size_t)k * Q * 3;
            if (t.shape == PAT_PLANAR) {
                double du = 2.0 * t.half_w / p.quad_n1, dv = 2.0 * t.half_h / p.quad_n2;
                qdA[k] = du * dv / (dr * dr);
                for (int a = 0; a < p.quad_n1; ++a)
                    for (int b = 0; b < p.quad_n2; ++b) {
                        double u = -t.half_w + (a + 0.5) * du, v = -t.half_h + (b + 0.5) * dv;
                        for (int q = 0; q < 3; ++q)
                            P[3 * (a * p.quad_n2 + b) + q] = (t.c0[q] + u * t.e1[q] + v * t.e2[q]) / dr;
                    }
            } else {
                double dth = 2.0 * t.theta_max / p.quad_n1, dz = 2.0 * t.half_len / p.quad_n2;
                qdA[k] = t.radius * dth * dz / (dr * dr);
                for (int a = 0; a < p.quad_n1; ++a)
                    for (int b = 0; b < p.quad_n2; ++b) {
                        double th = -t.theta_max + (a + 0.5) * dth, z = -t.half_len + (b + 0.5) * dz;
                        double cs = std::cos(th), sn = std::sin(th);
                        for (int q = 0; q < 3; ++q)
                            P[3 * (a * p.quad_n2 + b) + q] =
                                (t.c0[q] + t.radius * cs * t.e2[q] + t.radius * sn * n3[q] + z * t.e1[q]) / dr;
                    }
            }
        }
    }

    // ---- work decomposition
    const int nbx = (int)((grid->n[0] + kBrickX - 1) / kBrickX);
    const int nby = (int)((grid->n[1] + kBrickY - 1) / kBrickY);
    const int nbz = (int)((grid->n[2] + kBrickZ - 1) / kBrickZ);
    const int nbricks = nbx * nby * nbz;
    const int target_wg = 4096;

    // ---- device allocations
    const size_t rs = p.precision == PAT_FP64 ? sizeof(double) : sizeof(float);
    const size_t fbytes = (size_t)p.max_batch * K * Mcount * sizeof(double);
    const size_t wbytes = (size_t)p.max_batch * K * Mcount * rs;
    const size_t zbytes = (size_t)p.max_batch * N * sizeof(double);
    const size_t sbytes = surface ? ((size_t)N + 3 * (size_t)nbricks + 1) * sizeof(int32_t) : 0;
    const size_t lbytes = p.area_mode == PAT_AREA_LUT ? sizeof(double2) * kLutN * kLutN : 0;
    auto dmalloc = [&](void** ptr, size_t bytes) -> bool {
        if (bytes == 0) bytes = 8;
        return hipMalloc(ptr, bytes) == hipSuccess;
    };
    if (!dmalloc((void**)&c->d_tr, sizeof(TrDev) * K) || !dmalloc((void**)&c->d_kperm, sizeof(int32_t) * K) ||
        !dmalloc((void**)&c->d_scale, sizeof(double) * Mcount) || !dmalloc((void**)&c->d_G, sizeof(double) * jcnt) ||
        !dmalloc((void**)&c->d_f, fbytes) || !dmalloc(&c->d_W, wbytes) || !dmalloc((void**)&c->d_z, zbytes) ||
        (surface && !dmalloc((void**)&c->d_sup, sbytes)) || (lbytes && !dmalloc((void**)&c->d_lut, lbytes)) ||
        (Q > 0 && (!dmalloc((void**)&c->d_qpts, sizeof(double) * qp.size()) ||
                   !dmalloc((void**)&c->d_qdA, sizeof(double) * K)))) {
        (void)hipGetLastError();
        free_dev(c);
        return fail(c, PAT_E_OOM, "device allocation failed");
    }
    c->ws_bytes = fbytes + wbytes + zbytes + sbytes + lbytes;
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    up(c->d_tr, T.data(), sizeof(TrDev) * K);
    up(c->d_kperm, perm.data(), sizeof(int32_t) * K);
    up(c->d_scale, scale.data(), sizeof(double) * Mcount);
    up(c->d_G, G.data(), sizeof(double) * jcnt);
    if (surface) {
        // bricks in Morton order of (bx, by, bz): the sparse forward's groups of
        // consecutive support entries then stay spatially compact
        std::vector<std::pair<uint64_t, int32_t>> mk(nbricks);
        for (int b = 0; b < nbricks; ++b) {
            const uint64_t c3[3] = {(uint64_t)(b % nbx), (uint64_t)((b / nbx) % nby), (uint64_t)(b / (nbx * nby))};
            uint64_t key = 0;
            for (int bit = 0; bit < 21; ++bit)
                for (int a = 0; a < 3; ++a) key |= ((c3[a] >> bit) & 1ull) << (3 * bit + a);
            mk[b] = {key, b};
        }
        std::sort(mk.begin(), mk.end());
        std::vector<int32_t> order(nbricks);
        for (int b = 0; b < nbricks; ++b) order[b] = mk[b].second;
        up(c->d_sup + N + 2 * (size_t)nbricks + 1, order.data(), sizeof(int32_t) * nbricks);
    }
    if (Q > 0) {
        up(c->d_qpts, qp.data(), sizeof(double) * qp.size());
        up(c->d_qdA, qdA.data(), sizeof(double) * K);
    }
    if (e == hipSuccess && lbytes) e = launch_lut_build(c->d_lut, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        std::string msg = std::string("upload failed: ") + hipGetErrorString(e);
        free_dev(c);
        return fail(c, PAT_E_DEVICE, msg);
    }

    // ---- launch plan
    LaunchPlan& Lp = c->plan;
    std::memset(&Lp, 0, sizeof Lp);
    KParams& B = Lp.base;
    B.tr = c->d_tr;
    B.K = K;
    for (int a = 0; a < 3; ++a) {
        B.n[a] = grid->n[a];
        B.origin[a] = grid->origin[a] / da;
    }
    B.w = grid->spacing / da;
    B.r0 = r0a;
    B.Mlo = Mlo;
    B.Mcount = Mcount;
    B.step = step;
    B.Jlo = -floordiv64(-Mlo, step);          // ceil(Mlo / step)
    B.Jhi = -floordiv64(-Mhi, step);
    B.nbx = nbx;
    B.nby = nby;
    B.nbz = nbz;
    B.N = N;
    B.qpts = c->d_qpts;
    B.qdA = c->d_qdA;
    B.Q = Q;
    B.lut = c->d_lut;
    Lp.ngroups = 0;
    int off = 0;
    for (int s = 0; s < 2; ++s) {
        int nk = s == 0 ? nplan : ncyl;
        if (nk == 0) continue;
        ShapeGroup& Gp = Lp.groups[Lp.ngroups++];
        Gp.shape = s;
        Gp.kperm = c->d_kperm + off;
        Gp.nk = nk;
        int nchunks = std::max(1, std::min(nk, (target_wg + nbricks - 1) / nbricks));
        Gp.kchunk_fwd = (nk + nchunks - 1) / nchunks;
        Gp.kchunk_adj = Gp.kchunk_fwd;
        off += nk;
    }
    Lp.nbricks = nbricks;
    Lp.ncubes = (int)(((grid->n[0] + 3) / 4) * ((grid->n[1] + 3) / 4) * ((grid->n[2] + 3) / 4));
    Lp.mode = p.area_mode;
    Lp.fp64 = p.precision == PAT_FP64;
    Lp.U = p.U;
    Lp.L = p.L;
    Lp.jlo = jlo;
    Lp.jcnt = jcnt;
    Lp.G = c->d_G;
    Lp.scale = c->d_scale;
    Lp.f = c->d_f;
    Lp.W = c->d_W;
    Lp.z64 = c->d_z;
    if (surface) {
        Lp.sup_list = c->d_sup;
        Lp.sup_cnt = c->d_sup + N;
        Lp.sup_off = c->d_sup + N + nbricks;
        Lp.sup_order = c->d_sup + N + 2 * nbricks + 1;
    }

    // ---- (transducer, time tile) forward: tile width, and each shape group's
    // work items sorted by estimated cost, largest first
    if (tiles) {
        const int64_t J = B.Jhi - B.Jlo + 1;
        int tile = tile_log2 ? 1 << tile_log2 : 512;
        // automatic: the widest tile in 128..512 shells that still gives 8192
        // work items (eight per work-group slot of the device, for the balance
        // of items whose costs differ by orders of magnitude); narrower tiles
        // repeat each pair's setup in more tiles (measured on 128^3 x 256
        // cylinders and 256^3 x 512 planar elements: 128 and 256 are best)
        if (!tile_log2)
            while (tile > 128 && (int64_t)K * ((J + tile - 1) / tile) < 8192) tile >>= 1;
        const int64_t ntiles = (J + tile - 1) / tile;
        if ((int64_t)K * ntiles >= (int64_t)1 << 31) {
            free_dev(c);
            return fail(c, PAT_E_UNSUPPORTED, "too many time tiles");
        }
        const size_t nit = (size_t)K * ntiles;
        double* d_cost = nullptr;
        if (hipMalloc((void**)&c->d_items, sizeof(int32_t) * nit) != hipSuccess ||
            hipMalloc((void**)&d_cost, sizeof(double) * nit) != hipSuccess) {
            (void)hipGetLastError();
            if (d_cost) (void)hipFree(d_cost);
            free_dev(c);
            return fail(c, PAT_E_OOM, "device allocation failed");
        }
        c->ws_bytes += sizeof(int32_t) * nit;
        e = hipMemset(d_cost, 0, sizeof(double) * nit);
        size_t koff = 0;
        for (int g = 0; g < Lp.ngroups && e == hipSuccess; ++g) {
            KParams P = B;
            P.kperm = Lp.groups[g].kperm;
            P.nk = Lp.groups[g].nk;
            e = launch_tile_cost(P, nbricks, tile, (int)ntiles, d_cost + koff * ntiles, nullptr);
            koff += Lp.groups[g].nk;
        }
        std::vector<double> cost(nit);
        if (e == hipSuccess) e = hipMemcpy(cost.data(), d_cost, sizeof(double) * nit, hipMemcpyDeviceToHost);
        (void)hipFree(d_cost);
        std::vector<int32_t> items(nit);
        koff = 0;
        for (int g = 0; g < Lp.ngroups; ++g) {
            const size_t n = (size_t)Lp.groups[g].nk * ntiles;
            int32_t* it = items.data() + koff * ntiles;
            const double* cg = cost.data() + koff * ntiles;
            for (size_t i = 0; i < n; ++i) it[i] = (int32_t)i;
            std::stable_sort(it, it + n, [&](int32_t a, int32_t b) { return cg[a] > cg[b]; });
            Lp.groups[g].items = c->d_items + koff * ntiles;
            Lp.groups[g].nitems = (int)n;
            koff += Lp.groups[g].nk;
        }
        if (e == hipSuccess) e = hipMemcpy(c->d_items, items.data(), sizeof(int32_t) * nit, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            std::string msg = std::string("time-tile set-up failed: ") + hipGetErrorString(e);
            free_dev(c);
            return fail(c, PAT_E_DEVICE, msg);
        }
        Lp.tile = tile;
        Lp.ntiles = (int)ntiles;
    }

    c->K = K;
    c->N = N;
    c->L = p.L;
    c->U = p.U;
    c->mode = p.area_mode;
    c->precision = p.precision;
    c->max_batch = p.max_batch;
    c->work[0] = c->work[1] = -1.0;
    c->ready = true;
    c->err.clear();
    return PAT_OK;
}

enum class Op { forward, forward_sparse, adjoint };

// device buffers must hold whole elements of the context's precision
static bool aligned(const pat_ctx* c, const void* p)
{
    const uintptr_t a = c->precision == PAT_FP64 ? sizeof(double) : sizeof(float);
    return reinterpret_cast<uintptr_t>(p) % a == 0;
}

static pat_status run(pat_ctx* c, const void* in, void* out, int32_t batch, void* stream, Op op)
{
    if (!c) return PAT_E_ARG;
    if (!c->ready) return fail(c, PAT_E_STATE, "set_geometry has not succeeded");
    if (!in || !out || batch < 1 || batch > c->max_batch) return fail(c, PAT_E_ARG, "null buffer or bad batch");
    if (!aligned(c, in) || !aligned(c, out)) return fail(c, PAT_E_ARG, "buffer not aligned to its element size");
    if (op == Op::forward_sparse && c->mode == PAT_AREA_QUADRATURE)
        return fail(c, PAT_E_UNSUPPORTED, "the sparse forward serves the surface methods");
    DevGuard guard(c->device);
    if (!guard.ok) return fail(c, PAT_E_DEVICE, "hipSetDevice failed");
    hipError_t e = op == Op::forward        ? launch_forward(c->plan, in, out, batch, (hipStream_t)stream)
                   : op == Op::forward_sparse ? launch_forward_sparse(c->plan, in, out, batch, (hipStream_t)stream)
                                              : launch_adjoint(c->plan, in, out, batch, (hipStream_t)stream);
    if (e != hipSuccess) return fail(c, PAT_E_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return PAT_OK;
}

pat_status pat_forward(pat_ctx* c, const void* coef, void* signal, int32_t batch, void* stream)
{
    Range r("pat_forward");
    return run(c, coef, signal, batch, stream, Op::forward);
}

pat_status pat_forward_sparse(pat_ctx* c, const void* coef, void* signal, int32_t batch, void* stream)
{
    Range r("pat_forward_sparse");
    return run(c, coef, signal, batch, stream, Op::forward_sparse);
}

pat_status pat_adjoint(pat_ctx* c, const void* signal, void* coef, int32_t batch, void* stream)
{
    Range r("pat_adjoint");
    return run(c, signal, coef, batch, stream, Op::adjoint);
}

pat_status pat_forward_noalloc(pat_ctx* c, const void* coef, void* signal, int32_t batch, void* stream)
{
    Range r("pat_forward_noalloc");
    if (!c) return PAT_E_ARG;
    if (!c->ready) return fail(c, PAT_E_STATE, "set_geometry has not succeeded");
    if (!coef || !signal || batch < 1 || batch > c->max_batch) return fail(c, PAT_E_ARG, "null buffer or bad batch");
    if (!aligned(c, coef) || !aligned(c, signal)) return fail(c, PAT_E_ARG, "buffer not aligned to its element size");
    const double need = (double)batch * c->K * (double)c->plan.base.Mcount * sizeof(double);
    if (need > (double)kScratchBytes) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "forward_noalloc needs %.0f bytes of scratch (batch x K x fine bins x 8), above its static "
                 "%zu bytes; use pat_forward",
                 need, kScratchBytes);
        return fail(c, PAT_E_UNSUPPORTED, buf);
    }
    DevGuard guard(c->device);
    if (!guard.ok) return fail(c, PAT_E_DEVICE, "hipSetDevice failed");
    void* p = nullptr;
    hipError_t e = scratch_lookup(c->device, &p);
    if (e != hipSuccess || !p)
        return fail(c, PAT_E_DEVICE, std::string("scratch address lookup failed: ") + hipGetErrorString(e));
    LaunchPlan plan = c->plan;   // the context's tables; f in the static scratch
    plan.f = static_cast<double*>(p);
    e = launch_forward(plan, coef, signal, batch, (hipStream_t)stream);
    if (e != hipSuccess) return fail(c, PAT_E_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return PAT_OK;
}

pat_status pat_query(const pat_ctx* c, int32_t what, double* out)
{
    if (!out) return PAT_E_ARG;
    if (what == 6) { *out = PATOP_ABI_VERSION; return PAT_OK; }
    if (!c) return PAT_E_ARG;
    if (!c->ready) return PAT_E_STATE;
    switch (what) {
    case 0: *out = c->K; return PAT_OK;
    case 1: *out = (double)c->N; return PAT_OK;
    case 2: *out = (double)c->plan.base.Mcount; return PAT_OK;
    case 3: *out = (double)c->plan.base.Mlo; return PAT_OK;
    case 4: *out = c->truncated ? 1.0 : 0.0; return PAT_OK;
    case 5: *out = (double)c->ws_bytes; return PAT_OK;
    case 9: *out = (double)c->plan.tile; return PAT_OK;
    case 7:
    case 8: {
        pat_ctx* m = const_cast<pat_ctx*>(c);
        if (m->work[0] < 0.0) {
            DevGuard guard(m->device);
            unsigned long long* d = nullptr;
            unsigned long long h[2] = {0, 0};
            hipError_t e = hipMalloc((void**)&d, sizeof h);
            if (e == hipSuccess) e = hipMemcpy(d, h, sizeof h, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = launch_count(m->plan, d, nullptr);
            if (e == hipSuccess) e = hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost);
            if (d) (void)hipFree(d);
            if (e != hipSuccess) return fail(m, PAT_E_DEVICE, std::string("count failed: ") + hipGetErrorString(e));
            m->work[0] = (double)h[0];
            m->work[1] = (double)h[1];
        }
        *out = c->work[what - 7];
        return PAT_OK;
    }
    default: return PAT_E_ARG;
    }
}

}  // extern "C"
