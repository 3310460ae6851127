// api.hip -- host side of the C ABI declared in include/lbm.h: parameter
// derivation (Sec. 2.1-2.3 of Xu, Shi & Xi 2019), argument checks, the
// device-memory layout, the step loop and the synchronising queries.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "lbm_internal.h"

namespace {

int fail(lbm_t *h, int code, const char *fmt, const char *a = "") {
    if (h) {
        char buf[512];
        std::snprintf(buf, sizeof buf, fmt, a);
        h->err = buf;
    }
    return code;
}

int hip_fail(lbm_t *h, hipError_t e, const char *where) {
    if (h) h->err = std::string(where) + ": " + hipGetErrorString(e);
    return LBM_EDEVICE;
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Copy the result block (doubles [0, count) from res + off) to the host.
int read_res(lbm_t *h, hipStream_t s, int off, int count, double *dst) {
    const double *src = reinterpret_cast<const double *>(static_cast<char *>(h->buf) + h->L.off_res) + off;
    hipError_t e = hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? LBM_OK : hip_fail(h, e, "reading results");
}

int require_init(lbm_t *h) {
    if (!h) return LBM_EINVAL;
    if (!h->initialised) return fail(h, LBM_ESTATE, "populations not set (call lbm_set_fields or lbm_set_populations)");
    return LBM_OK;
}

// Take the pending sample of the current state (see lbm_step) into the time
// averages now, with a separate pass over the populations.
int flush_sample(lbm_t *h, hipStream_t s) {
    if (!h->pending_sample) return LBM_OK;
    hipError_t e = lbmk::launch_observe(h, true, s);
    if (e != hipSuccess) return hip_fail(h, e, "observables");
    h->samples += 1;
    h->pending_sample = false;
    return LBM_OK;
}

}  // namespace

extern "C" {

void lbm_default_opts(lbm_opts *o) {
    if (!o) return;
    o->U = 0.1 / std::sqrt(3.0);
    o->T0 = 0.0;
    o->sample_every = 0;
    o->block = 0;
    o->waves_even = 0;
    o->waves_odd = 0;
}

int lbm_derive_params(int N, double Ra, double Pr, int cell, int storage, const lbm_opts *opts,
                      lbm_params *out) {
    if (!out) return LBM_EINVAL;
    lbm_opts o;
    lbm_default_opts(&o);
    if (opts) o = *opts;
    std::memset(out, 0, sizeof *out);
    if (N < 3 || (cell != LBM_SIDE_HEATED && cell != LBM_RAYLEIGH_BENARD) ||
        (storage != LBM_FP64 && storage != LBM_FP32 && storage != LBM_FP16S && storage != LBM_FP16C) || !finite_pos(Ra) ||
        !finite_pos(Pr) || !finite_pos(o.U) || !std::isfinite(o.T0) || o.sample_every < 0)
        return LBM_EINVAL;
    if (N > lbmk::kMaxN) return LBM_ERANGE;
    lbm_params &p = *out;
    p.N = N;
    p.cell = cell;
    p.storage = storage;
    p.Ra = Ra;
    p.Pr = Pr;
    p.U = o.U;
    p.T0 = o.T0;
    p.T_hot = 0.5;
    p.T_cold = -0.5;
    p.H = N;   // node-centred lattice between walls on the planes 0 and N
    p.dT = p.T_hot - p.T_cold;
    // free-fall scaling (Sec. 2.1): Ra = g beta dT H^3/(nu kappa), Pr = nu/kappa,
    // U = sqrt(g beta dT H)
    p.nu = p.U * p.H * std::sqrt(Pr / Ra);
    p.kappa = p.U * p.H / std::sqrt(Ra * Pr);
    p.gbeta = p.U * p.U / (p.H * p.dT);
    // flow rates (Sec. 2.2): nu = (tau_f - 1/2)/3
    p.tau_f = 3.0 * p.nu + 0.5;
    p.s_e = 1.0 / p.tau_f;
    p.s_q = 8.0 * (2.0 * p.tau_f - 1.0) / (8.0 * p.tau_f - 1.0);
    // thermal rates for an isotropic fourth-order error (Sec. 2.3)
    const double r3 = std::sqrt(3.0);
    p.q_k = 3.0 - r3;
    p.q_e = 4.0 * r3 - 6.0;
    p.q_nu = 4.0 * r3 - 6.0;
    p.a_T = 42.0 * r3 * p.kappa - 6.0;
    p.wT0 = (1.0 - p.a_T) / 7.0;
    p.wT1 = (6.0 + p.a_T) / 42.0;
    if (!(p.a_T > -6.0 && p.a_T <= 1.0)) return LBM_ERANGE;
    return LBM_OK;
}

int lbm_state_bytes(int N, int storage, size_t *bytes) {
    if (!bytes || N < 3 || (storage != LBM_FP64 && storage != LBM_FP32 && storage != LBM_FP16S && storage != LBM_FP16C))
        return LBM_EINVAL;
    if (N > lbmk::kMaxN) return LBM_ERANGE;
    *bytes = lbmk::make_layout(N, storage).total;
    return LBM_OK;
}

int lbm_create(int N, double Ra, double Pr, int cell, int storage, const lbm_opts *opts,
               void *dev_buf, size_t buf_bytes, lbm_t **out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    lbm_params p;
    int rc = lbm_derive_params(N, Ra, Pr, cell, storage, opts, &p);
    if (rc != LBM_OK) return rc;
    lbm_opts o;
    lbm_default_opts(&o);
    if (opts) o = *opts;
    int block = o.block ? o.block : 256;
    if (block < 64 || block > 256 || block % 64) return LBM_EINVAL;
    if (o.waves_even < -1 || o.waves_even > 8 || o.waves_odd < -1 || o.waves_odd > 8) return LBM_EINVAL;
    if (dev_buf && (reinterpret_cast<uintptr_t>(dev_buf) % 256)) return LBM_EINVAL;
    lbmk::Layout L = lbmk::make_layout(N, storage);
    if (dev_buf && buf_bytes < L.total) return LBM_ENOMEM;

    lbm_t *h = new (std::nothrow) lbm;
    if (!h) return LBM_ENOMEM;
    h->p = p;
    h->o = o;
    h->L = L;
    h->storage = storage;
    h->block = block;
    {
        int w[2];
        lbmk::default_waves(storage, w);
        h->waves[0] = o.waves_even == 0 ? w[0] : (o.waves_even < 0 ? 0 : o.waves_even);
        h->waves[1] = o.waves_odd == 0 ? w[1] : (o.waves_odd < 0 ? 0 : o.waves_odd);
    }
    h->geo.N = N;
    h->geo.N2 = static_cast<uint32_t>(N) * static_cast<uint32_t>(N);
    h->geo.magic = static_cast<uint32_t>((0x100000000ull + N - 1) / N);
    h->geo.slab = static_cast<uint32_t>(L.slab);
    h->geo.sub = static_cast<uint32_t>(L.sub);
    h->geo.bbits = L.bbits;
    h->geo.bmask = (1u << L.bbits) - 1u;
    if (dev_buf) {
        h->buf = dev_buf;
    } else {
        hipError_t e = hipMalloc(&h->buf, L.total);
        if (e != hipSuccess) {
            delete h;
            return LBM_ENOMEM;
        }
        h->own_buf = true;
    }
    *out = h;
    return LBM_OK;
}

int lbm_destroy(lbm_t *h) {
    if (!h) return LBM_EINVAL;
    for (hipEvent_t ev : h->events) (void)hipEventDestroy(ev);
    if (h->own_buf) (void)hipFree(h->buf);
    delete h;
    return LBM_OK;
}

int lbm_get_params(const lbm_t *h, lbm_params *out) {
    if (!h || !out) return LBM_EINVAL;
    *out = h->p;
    return LBM_OK;
}

int lbm_set_fields(lbm_t *h, const double *uvwT, void *stream) {
    if (!h) return LBM_EINVAL;
    if (!uvwT) return fail(h, LBM_EINVAL, "uvwT is NULL");
    hipStream_t s = as_stream(stream);
    hipError_t e = lbmk::launch_init(h, uvwT, s);
    if (e != hipSuccess) return hip_fail(h, e, "init kernel");
    h->parity = 0;
    h->t = 0;
    h->has_flux = false;
    h->pending_sample = false;
    h->initialised = true;
    if ((e = lbmk::launch_reset_acc(h, s)) != hipSuccess) return hip_fail(h, e, "reset averages");
    h->samples = 0;
    if ((e = lbmk::launch_snapshot(h, s)) != hipSuccess) return hip_fail(h, e, "snapshot");
    return LBM_OK;
}

int lbm_get_fields(lbm_t *h, double *out, void *stream) {
    int rc = require_init(h);
    if (rc) return rc;
    if (!out) return fail(h, LBM_EINVAL, "out is NULL");
    hipError_t e = lbmk::launch_macro(h, out, as_stream(stream));
    return e == hipSuccess ? LBM_OK : hip_fail(h, e, "macro kernel");
}

int lbm_set_populations(lbm_t *h, const double *in, void *stream) {
    if (!h) return LBM_EINVAL;
    if (!in) return fail(h, LBM_EINVAL, "in is NULL");
    hipStream_t s = as_stream(stream);
    hipError_t e = lbmk::launch_set_pop(h, in, s);
    if (e != hipSuccess) return hip_fail(h, e, "set populations");
    h->parity = 0;
    h->has_flux = false;
    h->pending_sample = false;
    h->initialised = true;
    if ((e = lbmk::launch_reset_acc(h, s)) != hipSuccess) return hip_fail(h, e, "reset averages");
    h->samples = 0;
    if ((e = lbmk::launch_snapshot(h, s)) != hipSuccess) return hip_fail(h, e, "snapshot");
    return LBM_OK;
}

int lbm_get_populations(lbm_t *h, double *out, void *stream) {
    int rc = require_init(h);
    if (rc) return rc;
    if (!out) return fail(h, LBM_EINVAL, "out is NULL");
    hipError_t e = lbmk::launch_get_pop(h, out, as_stream(stream));
    return e == hipSuccess ? LBM_OK : hip_fail(h, e, "get populations");
}

int lbm_step(lbm_t *h, int64_t n, void *stream) {
    int rc = require_init(h);
    if (rc) return rc;
    if (h->in_batch) return fail(h, LBM_ESTATE, "cavity of a batch: step it with lbm_batch_step");
    if (n < 0) return fail(h, LBM_EINVAL, "negative step count");
    hipStream_t s = as_stream(stream);
    for (int64_t k = 0; k < n; ++k) {
        hipError_t e;
        if (h->profiling) {
            if (h->events_used + 2 > h->events.size()) {
                for (int m = 0; m < 2; ++m) {
                    hipEvent_t ev;
                    if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(h, e, "event create");
                    h->events.push_back(ev);
                }
            }
            if ((e = hipEventRecord(h->events[h->events_used], s)) != hipSuccess)
                return hip_fail(h, e, "event record");
        }
        // a sample state left by the previous step is observed by the step
        // that leaves it, from the populations it loads anyway
        const bool obs = h->pending_sample;
        if ((e = lbmk::launch_step(h, h->parity, obs, s)) != hipSuccess) return hip_fail(h, e, "step kernel");
        if (h->profiling) {
            if ((e = hipEventRecord(h->events[h->events_used + 1], s)) != hipSuccess)
                return hip_fail(h, e, "event record");
            h->events_used += 2;
        }
        if (obs) {
            if ((e = lbmk::launch_observe_reduce(h, true, s)) != hipSuccess) return hip_fail(h, e, "observables");
            h->samples += 1;
            h->pending_sample = false;
        }
        h->parity ^= 1;
        h->t += 1;
        h->has_flux = true;
        if (h->o.sample_every > 0 && h->t % h->o.sample_every == 0) h->pending_sample = true;
    }
    return LBM_OK;
}

int64_t lbm_time(const lbm_t *h) { return h ? h->t : -1; }

int lbm_observables_raw(lbm_t *h, void *stream, double raw[LBM_NRAW]) {
    int rc = require_init(h);
    if (rc) return rc;
    if (!raw) return fail(h, LBM_EINVAL, "raw is NULL");
    hipStream_t s = as_stream(stream);
    hipError_t e = lbmk::launch_observe(h, false, s);
    if (e != hipSuccess) return hip_fail(h, e, "observables");
    if ((rc = read_res(h, s, lbmk::kResCur, LBM_NRAW, raw)) != LBM_OK) return rc;
    for (int k = 0; k < LBM_NRAW; ++k)
        if (!std::isfinite(raw[k])) return fail(h, LBM_EDIVERGED, "non-finite observable");
    return LBM_OK;
}

int lbm_nondimensional(const lbm_params *p, const double raw[LBM_NRAW], double out[LBM_NOBS]) {
    if (!p || !raw || !out) return LBM_EINVAL;
    const double H = p->H, U = p->U, dT = p->dT, s = std::sqrt(p->Ra * p->Pr);
    const double nf = H / (p->kappa * dT), ng = H / dT;
    out[LBM_NU_HOT] = raw[LBM_RAW_FLUX_HOT] * nf;
    out[LBM_NU_COLD] = -raw[LBM_RAW_FLUX_COLD] * nf;
    out[LBM_NU_HOT_MID] = raw[LBM_RAW_FLUX_HOT_MID] * nf;
    out[LBM_NU_COLD_MID] = -raw[LBM_RAW_FLUX_COLD_MID] * nf;
    out[LBM_NU_HOT_FD] = raw[LBM_RAW_GRAD_HOT] * ng;
    out[LBM_NU_COLD_FD] = -raw[LBM_RAW_GRAD_COLD] * ng;
    out[LBM_NU_HOT_MID_FD] = raw[LBM_RAW_GRAD_HOT_MID] * ng;
    out[LBM_NU_COLD_MID_FD] = -raw[LBM_RAW_GRAD_COLD_MID] * ng;
    out[LBM_RE_RMS] = std::sqrt(raw[LBM_RAW_U2]) * H / p->nu;
    out[LBM_RE_W] = std::sqrt(raw[LBM_RAW_W2]) * H / p->nu;
    const double vt = p->cell == LBM_RAYLEIGH_BENARD ? raw[LBM_RAW_WT] : raw[LBM_RAW_UT];
    out[LBM_NU_VOL] = 1.0 + s * vt / (U * dT);
    out[LBM_EPS_U] = raw[LBM_RAW_EPS_U] * H / (U * U * U);
    out[LBM_EPS_T] = raw[LBM_RAW_EPS_T] * H / (U * dT * dT);
    out[LBM_NU_KIN] = 1.0 + s * out[LBM_EPS_U];
    out[LBM_NU_TH] = s * out[LBM_EPS_T];
    out[LBM_E_KIN] = 0.5 * raw[LBM_RAW_U2] / (U * U);
    out[LBM_RMS_DRHO] = std::sqrt(raw[LBM_RAW_DRHO2]);
    out[LBM_MEAN_T] = raw[LBM_RAW_T];
    out[LBM_RMS_DIV] = std::sqrt(raw[LBM_RAW_DIV2]) * H / U;
    return LBM_OK;
}

int lbm_observables(lbm_t *h, void *stream, double *Nu, double *Re, double *eps_u, double *eps_T) {
    double raw[LBM_NRAW], nd[LBM_NOBS];
    int rc = lbm_observables_raw(h, stream, raw);
    if (rc != LBM_OK) return rc;
    lbm_nondimensional(&h->p, raw, nd);
    if (Nu) *Nu = 0.5 * (nd[LBM_NU_HOT] + nd[LBM_NU_COLD]);
    if (Re) *Re = nd[LBM_RE_RMS];
    if (eps_u) *eps_u = nd[LBM_EPS_U];
    if (eps_T) *eps_T = nd[LBM_EPS_T];
    return LBM_OK;
}

int lbm_averages(lbm_t *h, void *stream, double raw_mean[LBM_NRAW], int64_t *count) {
    int rc = require_init(h);
    if (rc) return rc;
    if (!raw_mean) return fail(h, LBM_EINVAL, "raw_mean is NULL");
    if ((rc = flush_sample(h, as_stream(stream))) != LBM_OK) return rc;
    double acc[LBM_NRAW + 1];
    if ((rc = read_res(h, as_stream(stream), lbmk::kResAcc, LBM_NRAW + 1, acc)) != LBM_OK) return rc;
    const double n = acc[LBM_NRAW];
    if (count) *count = static_cast<int64_t>(n);
    if (n <= 0) return fail(h, LBM_ESTATE, "no samples since the last reset");
    for (int k = 0; k < LBM_NRAW; ++k) {
        raw_mean[k] = acc[k] / n;
        if (!std::isfinite(raw_mean[k])) return fail(h, LBM_EDIVERGED, "non-finite average");
    }
    return LBM_OK;
}

int lbm_reset_averages(lbm_t *h, void *stream) {
    if (!h) return LBM_EINVAL;
    hipError_t e = lbmk::launch_reset_acc(h, as_stream(stream));
    if (e != hipSuccess) return hip_fail(h, e, "reset averages");
    h->samples = 0;
    h->pending_sample = false;
    return LBM_OK;
}

int lbm_residual(lbm_t *h, void *stream, double *max_dT, double *rel_L1_T, double *rel_L2_u) {
    int rc = require_init(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    hipError_t e = lbmk::launch_residual(h, s);
    if (e != hipSuccess) return hip_fail(h, e, "residual");
    double t[5];
    if ((rc = read_res(h, s, lbmk::kResResid, 5, t)) != LBM_OK) return rc;
    for (double v : t)
        if (!std::isfinite(v)) return fail(h, LBM_EDIVERGED, "non-finite residual");
    auto ratio = [](double a, double b) { return a == 0.0 ? 0.0 : (b == 0.0 ? INFINITY : a / b); };
    if (max_dT) *max_dT = t[0];
    if (rel_L1_T) *rel_L1_T = ratio(t[1], t[2]);
    if (rel_L2_u) *rel_L2_u = ratio(t[3], t[4]);
    return LBM_OK;
}

int lbm_run_to_steady(lbm_t *h, int64_t check_every, double tol_max_dT, int64_t max_steps,
                      void *stream, int64_t *steps_taken, double *final_max_dT, double *history,
                      int64_t history_len) {
    int rc = require_init(h);
    if (rc) return rc;
    if (check_every <= 0 || max_steps < 0 || !(tol_max_dT >= 0.0))
        return fail(h, LBM_EINVAL, "bad check interval, step limit or tolerance");
    int64_t done = 0, checks = 0;
    double r = INFINITY;
    while (done < max_steps) {
        const int64_t k = check_every < max_steps - done ? check_every : max_steps - done;
        if ((rc = lbm_step(h, k, stream)) != LBM_OK) return rc;
        done += k;
        if ((rc = lbm_residual(h, stream, &r, nullptr, nullptr)) != LBM_OK) return rc;
        if (history && checks < history_len) history[checks] = r;
        ++checks;
        if (r < tol_max_dT) break;
    }
    if (steps_taken) *steps_taken = done;
    if (final_max_dT) *final_max_dT = r;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Checkpoint file: CkptHeader, the population storage bytes, the result block
// (kResDoubles doubles), then the FNV-1a 64 hash of everything before it.
struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t N, cell, storage, parity, reserved;
    int64_t t, samples;
    double Ra, Pr, U, T0;
    uint64_t pop_bytes, res_doubles;
};
constexpr char kCkptMagic[8] = {'P', '1', '9', '0', '3', 'L', 'B', 'M'};
constexpr size_t kCkptChunk = size_t{64} << 20;

struct Fnv {
    uint64_t h = 0xcbf29ce484222325ull;
    void add(const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
    }
};

struct File {
    FILE *f = nullptr;
    ~File() { if (f) std::fclose(f); }
};

bool same_params(const CkptHeader &c, const lbm_t *h) {
    return c.N == h->p.N && c.cell == h->p.cell && c.storage == h->storage && c.Ra == h->p.Ra &&
           c.Pr == h->p.Pr && c.U == h->p.U && c.T0 == h->p.T0;
}

}  // namespace

extern "C" {

int lbm_save(lbm_t *h, const char *path, void *stream) {
    int rc = require_init(h);
    if (rc) return rc;
    if (!path) return fail(h, LBM_EINVAL, "path is NULL");
    hipStream_t s = as_stream(stream);
    if ((rc = flush_sample(h, s)) != LBM_OK) return rc;
    CkptHeader c{};
    std::memcpy(c.magic, kCkptMagic, 8);
    c.version = 1;
    c.N = h->p.N;
    c.cell = h->p.cell;
    c.storage = h->storage;
    c.parity = h->parity;
    c.t = h->t;
    c.samples = h->samples;
    c.Ra = h->p.Ra;
    c.Pr = h->p.Pr;
    c.U = h->p.U;
    c.T0 = h->p.T0;
    c.pop_bytes = h->L.pop_bytes;
    c.res_doubles = lbmk::kResDoubles;
    File f;
    if (!(f.f = std::fopen(path, "wb"))) return fail(h, LBM_EIO, "cannot open %s for writing", path);
    Fnv sum;
    auto put = [&](const void *p, size_t n) {
        sum.add(p, n);
        return std::fwrite(p, 1, n, f.f) == n;
    };
    if (!put(&c, sizeof c)) return fail(h, LBM_EIO, "short write to %s", path);
    std::vector<char> host(std::min<size_t>(kCkptChunk, h->L.pop_bytes));
    const char *dev = static_cast<const char *>(h->buf) + h->L.off_pop;
    for (size_t o = 0; o < h->L.pop_bytes; o += host.size()) {
        const size_t n = std::min(host.size(), h->L.pop_bytes - o);
        hipError_t e = hipMemcpyAsync(host.data(), dev + o, n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "reading populations");
        if (!put(host.data(), n)) return fail(h, LBM_EIO, "short write to %s", path);
    }
    double res[lbmk::kResDoubles];
    if ((rc = read_res(h, s, 0, lbmk::kResDoubles, res)) != LBM_OK) return rc;
    if (!put(res, sizeof res)) return fail(h, LBM_EIO, "short write to %s", path);
    const uint64_t hash = sum.h;
    if (std::fwrite(&hash, 1, sizeof hash, f.f) != sizeof hash || std::fflush(f.f) != 0)
        return fail(h, LBM_EIO, "short write to %s", path);
    return LBM_OK;
}

int lbm_load(lbm_t *h, const char *path, void *stream) {
    if (!h) return LBM_EINVAL;
    if (!path) return fail(h, LBM_EINVAL, "path is NULL");
    if (h->in_batch) return fail(h, LBM_ESTATE, "cannot load into a cavity of a batch");
    hipStream_t s = as_stream(stream);
    File f;
    if (!(f.f = std::fopen(path, "rb"))) return fail(h, LBM_EIO, "cannot open %s", path);
    CkptHeader c{};
    if (std::fread(&c, 1, sizeof c, f.f) != sizeof c || std::memcmp(c.magic, kCkptMagic, 8) != 0 ||
        c.version != 1)
        return fail(h, LBM_EIO, "%s is not a checkpoint of this library", path);
    if (!same_params(c, h))
        return fail(h, LBM_EINVAL, "checkpoint %s was written for other N, cell, storage or parameters", path);
    if (c.pop_bytes != h->L.pop_bytes || c.res_doubles != lbmk::kResDoubles || c.parity < 0 ||
        c.parity > 1 || c.t < 0 || c.samples < 0)
        return fail(h, LBM_EIO, "checkpoint %s has an inconsistent header", path);
    // first pass: the checksum, before anything reaches the device
    std::vector<char> host(std::min<size_t>(kCkptChunk, c.pop_bytes));
    double res[lbmk::kResDoubles];
    Fnv sum;
    sum.add(&c, sizeof c);
    for (size_t o = 0; o < c.pop_bytes; o += host.size()) {
        const size_t n = std::min<size_t>(host.size(), c.pop_bytes - o);
        if (std::fread(host.data(), 1, n, f.f) != n) return fail(h, LBM_EIO, "%s is truncated", path);
        sum.add(host.data(), n);
    }
    uint64_t hash = 0;
    if (std::fread(res, 1, sizeof res, f.f) != sizeof res ||
        std::fread(&hash, 1, sizeof hash, f.f) != sizeof hash)
        return fail(h, LBM_EIO, "%s is truncated", path);
    sum.add(res, sizeof res);
    if (hash != sum.h) return fail(h, LBM_EIO, "checksum mismatch in %s", path);
    // second pass: copy to the device
    if (std::fseek(f.f, static_cast<long>(sizeof c), SEEK_SET) != 0)
        return fail(h, LBM_EIO, "cannot seek in %s", path);
    char *dev = static_cast<char *>(h->buf) + h->L.off_pop;
    for (size_t o = 0; o < c.pop_bytes; o += host.size()) {
        const size_t n = std::min<size_t>(host.size(), c.pop_bytes - o);
        if (std::fread(host.data(), 1, n, f.f) != n) return fail(h, LBM_EIO, "%s is truncated", path);
        hipError_t e = hipMemcpyAsync(dev + o, host.data(), n, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "writing populations");
    }
    double *dres = reinterpret_cast<double *>(static_cast<char *>(h->buf) + h->L.off_res);
    hipError_t e = hipMemcpyAsync(dres, res, sizeof res, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "writing the result block");
    h->parity = c.parity;
    h->t = c.t;
    h->samples = c.samples;
    h->has_flux = false;
    h->pending_sample = false;
    h->initialised = true;
    if ((e = lbmk::launch_snapshot(h, s)) != hipSuccess) return hip_fail(h, e, "snapshot");
    return LBM_OK;
}

int lbm_centerline_peaks(lbm_t *h, void *stream, double out[5]) {
    int rc = require_init(h);
    if (rc) return rc;
    if (!out) return fail(h, LBM_EINVAL, "out is NULL");
    hipStream_t s = as_stream(stream);
    hipError_t e = lbmk::launch_centerline(h, s);
    if (e != hipSuccess) return hip_fail(h, e, "centreline kernel");
    double pk[4];
    if ((rc = read_res(h, s, lbmk::kResPeak, 4, pk)) != LBM_OK) return rc;
    double raw[LBM_NRAW];
    if ((rc = lbm_observables_raw(h, stream, raw)) != LBM_OK) return rc;
    const double N = h->p.N, U = h->p.U;
    out[0] = pk[0] / U;
    out[1] = (pk[1] + 0.5) / N;
    out[2] = pk[2] / U;
    out[3] = (pk[3] + 0.5) / N;
    out[4] = 0.5 * raw[LBM_RAW_U2] / (U * U);
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(out[k])) return fail(h, LBM_EDIVERGED, "non-finite centreline value");
    return LBM_OK;
}

int lbm_profile(lbm_t *h, int enable) {
    if (!h) return LBM_EINVAL;
    h->profiling = enable != 0;
    return LBM_OK;
}

int lbm_profile_read(lbm_t *h, double *kernel_ms, int64_t *kernels) {
    if (!h || !kernel_ms || !kernels) return LBM_EINVAL;
    double total = 0.0;
    for (size_t k = 0; k + 1 < h->events_used; k += 2) {
        hipError_t e = hipEventSynchronize(h->events[k + 1]);
        if (e != hipSuccess) return hip_fail(h, e, "event synchronize");
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, h->events[k], h->events[k + 1])) != hipSuccess)
            return hip_fail(h, e, "event elapsed");
        total += ms;
    }
    *kernel_ms = total;
    *kernels = static_cast<int64_t>(h->events_used / 2);
    h->events_used = 0;
    return LBM_OK;
}

int lbm_device_copy(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src || bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 ||
        reinterpret_cast<uintptr_t>(src) % 16)
        return LBM_EINVAL;
    if (bytes == 0) return LBM_OK;
    const char *a = static_cast<const char *>(src), *b = static_cast<const char *>(dst);
    if (a < b + bytes && b < a + bytes) return LBM_EINVAL;
    return lbmk::launch_copy(src, dst, bytes, as_stream(stream)) == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

int lbm_nusselt_profile(lbm_t *h, void *stream, double *out) {
    int rc = require_init(h);
    if (rc) return rc;
    if (!out) return fail(h, LBM_EINVAL, "out is NULL");
    hipStream_t s = as_stream(stream);
    hipError_t e = lbmk::launch_profile(h, s);
    if (e != hipSuccess) return hip_fail(h, e, "Nusselt profile");
    const double *src = reinterpret_cast<const double *>(static_cast<char *>(h->buf) + h->L.off_prof) +
                        static_cast<size_t>(lbmk::kProfGroups) * 2 * h->p.N;
    e = hipMemcpyAsync(out, src, h->p.N * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "reading the Nusselt profile");
    for (int k = 0; k < h->p.N; ++k)
        if (!std::isfinite(out[k])) return fail(h, LBM_EDIVERGED, "non-finite Nusselt profile");
    return LBM_OK;
}

int lbm_resample_fields(lbm_t *h, int M, float *out, void *stream) {
    int rc = require_init(h);
    if (rc) return rc;
    if (!out || M < 2 || M > lbmk::kMaxN) return fail(h, LBM_EINVAL, "bad output size or pointer");
    hipError_t e = lbmk::launch_resample(h, M, out, as_stream(stream));
    return e == hipSuccess ? LBM_OK : hip_fail(h, e, "resample");
}

}  // extern "C"

namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune_cache;   // (N, storage, cell) -> block

// Mean duration (ms) of `steps` launches of fn on stream s, timed with events.
template <class F>
int time_steps(F &&fn, int steps, hipStream_t s, double *ms_out, std::string *err) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return LBM_EDEVICE;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return LBM_EDEVICE;
    }
    int rc = fn(2);   // warm-up
    if (rc == LBM_OK && hipEventRecord(a, s) != hipSuccess) rc = LBM_EDEVICE;
    if (rc == LBM_OK) rc = fn(steps);
    if (rc == LBM_OK && hipEventRecord(b, s) != hipSuccess) rc = LBM_EDEVICE;
    float ms = 0.0f;
    if (rc == LBM_OK && (hipEventSynchronize(b) != hipSuccess ||
                         hipEventElapsedTime(&ms, a, b) != hipSuccess)) {
        rc = LBM_EDEVICE;
        *err = "timing events failed";
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms_out = ms / steps;
    return rc;
}

constexpr int kTuneCandidates[] = {64, 128, 192, 256};

}  // namespace

extern "C" {

int lbm_autotune(lbm_t *h, void *stream, int steps_per_candidate, int *best_block, double *best_ms) {
    int rc = require_init(h);
    if (rc) return rc;
    if (steps_per_candidate < 1) return fail(h, LBM_EINVAL, "steps_per_candidate < 1");
    const auto key = std::make_tuple(h->p.N, h->storage, h->p.cell);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            h->block = it->second;
            if (best_block) *best_block = h->block;
            if (best_ms) *best_ms = 0.0;
            return LBM_OK;
        }
    }
    hipStream_t s = as_stream(stream);
    int best = h->block;
    double best_t = INFINITY;
    for (int cand : kTuneCandidates) {
        h->block = cand;
        double ms = 0.0;
        rc = time_steps([&](int n) { return lbm_step(h, n, stream); }, steps_per_candidate, s, &ms, &h->err);
        if (rc != LBM_OK) return rc;
        if (ms < best_t) {
            best_t = ms;
            best = cand;
        }
    }
    h->block = best;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    if (best_block) *best_block = best;
    if (best_ms) *best_ms = best_t;
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

int bfail(lbm_batch_t *b, int code, const std::string &msg) {
    if (b) b->err = msg;
    return code;
}

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

size_t table_bytes(int K) { return up256(static_cast<size_t>(K) * lbmk::kMaxDescBytes); }

// Write the descriptor table (geometry, coefficients, active flags) to the device.
int upload_table(lbm_batch_t *b) {
    std::vector<char> img(table_bytes(b->K));
    size_t nbytes = 0;
    hipError_t e = lbmk::build_batch_table(b, img.data(), &nbytes);
    if (e == hipSuccess)
        e = hipMemcpy(static_cast<char *>(b->buf) + b->off_table, img.data(), nbytes,
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("descriptor table: ") + hipGetErrorString(e));
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_state_bytes(int K, const int *N, int storage, size_t *bytes) {
    if (K < 1 || !N || !bytes) return LBM_EINVAL;
    size_t total = table_bytes(K);
    for (int k = 0; k < K; ++k) {
        size_t s = 0;
        int rc = lbm_state_bytes(N[k], storage, &s);
        if (rc != LBM_OK) return rc;
        total += up256(s);
    }
    *bytes = total;
    return LBM_OK;
}

int lbm_batch_create(int K, const int *N, const double *Ra, const double *Pr, const int *cell,
                     int storage, const lbm_opts *opts, void *dev_buf, size_t buf_bytes,
                     lbm_batch_t **out) {
    if (!out || K < 1 || !N || !Ra || !Pr || !cell) return LBM_EINVAL;
    *out = nullptr;
    size_t need = 0;
    int rc = lbm_batch_state_bytes(K, N, storage, &need);
    if (rc != LBM_OK) return rc;
    if (dev_buf && (reinterpret_cast<uintptr_t>(dev_buf) % 256)) return LBM_EINVAL;
    if (dev_buf && buf_bytes < need) return LBM_ENOMEM;
    lbm_opts o;
    lbm_default_opts(&o);
    if (opts) o = *opts;
    o.sample_every = 0;   // batches do not sample time averages
    lbm_batch_t *b = new (std::nothrow) lbm_batch;
    if (!b) return LBM_ENOMEM;
    b->K = K;
    b->storage = storage;
    b->block = o.block ? o.block : 256;
    if (dev_buf) {
        b->buf = dev_buf;
    } else {
        if (hipMalloc(&b->buf, need) != hipSuccess) {
            delete b;
            return LBM_ENOMEM;
        }
        b->own_buf = true;
    }
    b->off_table = 0;
    size_t off = table_bytes(K);
    for (int k = 0; k < K; ++k) {
        size_t s = 0;
        lbm_state_bytes(N[k], storage, &s);
        lbm_t *h = nullptr;
        rc = lbm_create(N[k], Ra[k], Pr[k], cell[k], storage, &o, static_cast<char *>(b->buf) + off,
                        s, &h);
        if (rc != LBM_OK) {
            lbm_batch_destroy(b);
            return rc;
        }
        h->in_batch = true;
        h->block = b->block;
        b->waves[0] = h->waves[0];
        b->waves[1] = h->waves[1];
        b->cav.push_back(h);
        b->active.push_back(1);
        b->last_res.push_back(INFINITY);
        off += up256(s);
    }
    if ((rc = upload_table(b)) != LBM_OK) {
        lbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch_t *b) {
    if (!b) return LBM_EINVAL;
    for (lbm_t *h : b->cav) lbm_destroy(h);
    if (b->own_buf) (void)hipFree(b->buf);
    delete b;
    return LBM_OK;
}

int lbm_batch_cavity(lbm_batch_t *b, int k, lbm_t **h) {
    if (!b || !h || k < 0 || k >= b->K) return LBM_EINVAL;
    *h = b->cav[k];
    return LBM_OK;
}

int lbm_batch_step(lbm_batch_t *b, int64_t n, void *stream) {
    if (!b) return LBM_EINVAL;
    if (n < 0) return bfail(b, LBM_EINVAL, "negative step count");
    for (int k = 0; k < b->K; ++k) {
        const lbm_t *h = b->cav[k];
        if (!b->active[k]) continue;
        if (!h->initialised) return bfail(b, LBM_ESTATE, "cavity " + std::to_string(k) + " has no populations");
        if (h->parity != b->parity)
            return bfail(b, LBM_ESTATE, "cavity " + std::to_string(k) + " was set after an odd number of batch steps");
    }
    hipStream_t s = as_stream(stream);
    for (int64_t i = 0; i < n; ++i) {
        hipError_t e = lbmk::launch_step_batch(b, b->parity, s);
        if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("batched step: ") + hipGetErrorString(e));
        b->parity ^= 1;
        b->t += 1;
        for (int k = 0; k < b->K; ++k)
            if (b->active[k]) {
                lbm_t *h = b->cav[k];
                h->parity ^= 1;
                h->t += 1;
                h->has_flux = true;
            }
    }
    return LBM_OK;
}

int lbm_batch_run_to_steady(lbm_batch_t *b, int64_t check_every, double tol_max_dT,
                            int64_t max_steps, void *stream, int64_t *steps_k, double *res_k) {
    if (!b) return LBM_EINVAL;
    if (check_every <= 0 || max_steps < 0 || !(tol_max_dT >= 0.0))
        return bfail(b, LBM_EINVAL, "bad check interval, step limit or tolerance");
    int64_t done = 0;
    int rc = LBM_OK;
    auto any_active = [&] {
        for (int a : b->active)
            if (a) return true;
        return false;
    };
    while (done < max_steps && any_active()) {
        const int64_t k = check_every < max_steps - done ? check_every : max_steps - done;
        if ((rc = lbm_batch_step(b, k, stream)) != LBM_OK) return rc;
        done += k;
        bool changed = false;
        for (int c = 0; c < b->K; ++c) {
            if (!b->active[c]) continue;
            double r = 0.0;
            rc = lbm_residual(b->cav[c], stream, &r, nullptr, nullptr);
            if (rc == LBM_EDIVERGED) {   // quarantine: retire it, keep the others going
                r = NAN;
            } else if (rc != LBM_OK) {
                return bfail(b, rc, "cavity " + std::to_string(c) + ": " + b->cav[c]->err);
            }
            b->last_res[c] = r;
            if (!(r >= tol_max_dT)) {    // converged, or diverged (NaN)
                b->active[c] = 0;
                changed = true;
            }
        }
        if (changed && (rc = upload_table(b)) != LBM_OK) return rc;
    }
    for (int c = 0; c < b->K; ++c) {
        if (steps_k) steps_k[c] = b->cav[c]->t;
        if (res_k) res_k[c] = b->last_res[c];
    }
    return LBM_OK;
}

int lbm_batch_autotune(lbm_batch_t *b, void *stream, int steps_per_candidate, int *best_block,
                       double *best_ms) {
    if (!b) return LBM_EINVAL;
    if (steps_per_candidate < 1) return bfail(b, LBM_EINVAL, "steps_per_candidate < 1");
    hipStream_t s = as_stream(stream);
    int best = b->block;
    double best_t = INFINITY;
    for (int cand : kTuneCandidates) {
        b->block = cand;
        int rc = upload_table(b);
        if (rc != LBM_OK) return rc;
        double ms = 0.0;
        rc = time_steps([&](int n) { return lbm_batch_step(b, n, stream); }, steps_per_candidate, s, &ms, &b->err);
        if (rc != LBM_OK) return rc;
        if (ms < best_t) {
            best_t = ms;
            best = cand;
        }
    }
    b->block = best;
    for (lbm_t *h : b->cav) h->block = best;
    int rc = upload_table(b);
    if (rc != LBM_OK) return rc;
    if (best_block) *best_block = best;
    if (best_ms) *best_ms = best_t;
    return LBM_OK;
}

const char *lbm_batch_last_error(const lbm_batch_t *b) { return b ? b->err.c_str() : "NULL batch"; }

const char *lbm_last_error(const lbm_t *h) { return h ? h->err.c_str() : "NULL handle"; }

const char *lbm_strerror(int status) {
    switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ERANGE: return "parameters outside the valid range of the scheme";
    case LBM_ENOMEM: return "buffer too small or allocation failed";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_EDIVERGED: return "non-finite result (diverged)";
    case LBM_ESTATE: return "call not valid in the current state";
    case LBM_EIO: return "checkpoint file missing, short, corrupt or foreign";
    }
    return "unknown status";
}

}  // extern "C"
