// pd_fcbm.hip -- the C entry points of the FCBM-EC peridynamics library for
// gfx950 (plan creation and dispatch by dtype; the per-dtype implementation
// is compiled in pd_inst.hip).
#include "pd_impl.hpp"

namespace pdh {

pd_status check(hipError_t e) {
    if (e == hipSuccess) return PD_OK;
    if (e == hipErrorOutOfMemory) return PD_ENOMEM;
    return PD_EDEVICE;
}

}  // namespace pdh


using namespace pdi;

// ------------------------------------------------ allocation-free solve
// The vectors of pd_static_solve_noalloc live in one file-scope device
// array.  Each GPU that runs the library holds its own copy until the
// process ends; its address on the current device comes from
// hipGetSymbolAddress (in host code `scratch` is only a host-side stand-in),
// looked up once per device and kept.
#include <mutex>

static constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

pd_status scratch_on_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PD_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return PD_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return PD_EDEVICE;
        g_scratch_ptr[dev] = q;
    }
    *out = g_scratch_ptr[dev];
    return PD_OK;
}

}  // namespace

extern "C" {

pd_status pd_plan_create(const pd_grid* grid, const pd_horizon* horizon, const pd_kernel* kernel, const pd_mask* mask,
                         pd_dtype dtype, int flags, void* stream, pd_plan* out) {
    if (!out) return PD_EINVAL;
    return plan_create_impl(grid, horizon, kernel, mask, dtype, flags, S_(stream), out);
}

void pd_plan_destroy(pd_plan plan) { plan_free(plan); }

pd_status pd_plan_query(pd_plan p, pd_plan_info* info) {
    if (!p || !info) return PD_EINVAL;
    info->dim = p->dim;
    info->body_nodes = p->nb;
    info->fft_points = p->nfft;
    info->stencil_size = p->ns;
    info->alpha = p->alpha;
    info->m0 = p->m0;
    info->Wc = p->Wc;
    info->dt_max = p->dt_max;
    info->workspace_bytes = (int64_t)p->bytes + (p->sub32 ? (int64_t)p->sub32->bytes : 0);
    info->lds_per_block = p->max_lds;
    return PD_OK;
}

pd_status pd_force(pd_plan p, const void* u, const void* weight, void* L_out, void* W_out, void* stream) {
    if (!p || !u || !L_out) return PD_EINVAL;
    if (p->kern.weight == PD_WEIGHT_NONE && weight) return PD_EINVAL;
    if (p->kern.weight != PD_WEIGHT_NONE && !weight) return PD_EINVAL;
    if (p->dtype == PD_F32)
        return force_impl<float>(p, (const float*)u, weight, (float*)L_out, (float*)W_out, S_(stream));
    return force_impl<double>(p, (const double*)u, weight, (double*)L_out, (double*)W_out, S_(stream));
}

pd_status pd_force_adjoint(pd_plan p, const void* u, const void* weight, const void* g_bar, void* u_bar,
                           void* weight_bar, void* stream) {
    if (!p || !g_bar) return PD_EINVAL;
    if (weight_bar && !u) return PD_EINVAL;
    if (p->kern.model == PD_BB_NONLINEAR) return PD_EUNSUPPORTED;
    if (p->dtype == PD_F32)
        return adjoint_impl<float>(p, (const float*)u, nullptr, weight, (const float*)g_bar, (float*)u_bar,
                                   (float*)weight_bar, 1.0f, 0, S_(stream));
    return adjoint_impl<double>(p, (const double*)u, nullptr, weight, (const double*)g_bar, (double*)u_bar,
                                (double*)weight_bar, 1.0, 0, S_(stream));
}

pd_status pd_verlet_step(pd_plan p, pd_state* state, const void* b, const void* w, double dt, int nsteps,
                         double* energy_out, void* stream) {
    if (!p || !state) return PD_EINVAL;
    if (p->kern.model == PD_BB_NONLINEAR) return PD_EUNSUPPORTED;
    if (p->dtype == PD_F32)
        return verlet_impl<float>(p, state, (const float*)b, (const float*)w, dt, nsteps, energy_out, S_(stream));
    return verlet_impl<double>(p, state, (const double*)b, (const double*)w, dt, nsteps, energy_out, S_(stream));
}

pd_status pd_verlet_adjoint(pd_plan p, const void* u_n, const void* u_np1, const void* s, void* u_bar, void* v_bar,
                            void* s_bar, void* b_bar, double dt, void* stream) {
    if (!p) return PD_EINVAL;
    if (p->kern.model == PD_BB_NONLINEAR) return PD_EUNSUPPORTED;
    if (p->dtype == PD_F32)
        return verlet_adjoint_impl<float>(p, (const float*)u_n, (const float*)u_np1, (const float*)s, (float*)u_bar,
                                          (float*)v_bar, (float*)s_bar, (float*)b_bar, dt, S_(stream));
    return verlet_adjoint_impl<double>(p, (const double*)u_n, (const double*)u_np1, (const double*)s, (double*)u_bar,
                                       (double*)v_bar, (double*)s_bar, (double*)b_bar, dt, S_(stream));
}

pd_status pd_static_solve(pd_plan p, const void* b, const void* w, void* u_inout, double rtol, int maxit, int options,
                          pd_solve_info* info, void* stream) {
    if (!p) return PD_EINVAL;
    if (p->kern.model == PD_BB_NONLINEAR) return PD_EUNSUPPORTED;
    return static_solve_impl(p, (const double*)b, (const double*)w, (double*)u_inout, rtol, maxit, options, info,
                             S_(stream));
}

pd_status pd_static_solve_noalloc(pd_plan p, const void* b, const void* w, void* u_inout, double rtol, int maxit,
                                  int options, pd_solve_info* info, void* stream) {
    if (!p) return PD_EINVAL;
    if (p->kern.model == PD_BB_NONLINEAR) return PD_EUNSUPPORTED;
    if (p->prof || (p->sub32 && p->sub32->prof)) return PD_EINVAL;   // pass timing creates events
    if (options & ~(PD_SOLVE_MIXED | PD_SOLVE_PRECOND)) return PD_EINVAL;
    if (solve_workspace_bytes(p, options) > kScratchBytes) return PD_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PD_EDEVICE;
    if (dev != p->device) return PD_EINVAL;
    void* ws = nullptr;
    PD_TRY(scratch_on_current_device(&ws));
    return static_solve_impl(p, (const double*)b, (const double*)w, (double*)u_inout, rtol, maxit, options, info,
                             S_(stream), ws, kScratchBytes);
}

pd_status pd_damage_index(pd_plan p, const uint8_t* lambda, void* d_out, void* stream) {
    if (!p) return PD_EINVAL;
    if (p->kern.model == PD_BB_NONLINEAR) return PD_EUNSUPPORTED;
    if (p->dtype == PD_F32) return damage_impl<float>(p, lambda, (float*)d_out, S_(stream));
    return damage_impl<double>(p, lambda, (double*)d_out, S_(stream));
}

const char* pd_status_str(pd_status s) {
    switch (s) {
        case PD_OK: return "ok";
        case PD_EINVAL: return "invalid argument";
        case PD_ENOMEM: return "out of device memory";
        case PD_EDEVICE: return "HIP runtime error";
        case PD_ENOTCONV: return "solver did not converge";
        case PD_ENUMERIC: return "non-finite value";
        case PD_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

pd_status pd_profile_enable(pd_plan p, int enable) {
    if (!p) return PD_EINVAL;
    pd_plan plans[2] = {p, p->sub32};
    for (pd_plan q : plans) {
        if (!q) continue;
        if (enable && !q->prof) q->prof = new std::vector<ProfRec>();
        if (!enable && q->prof) {
            (void)hipDeviceSynchronize();
            for (ProfRec& r : *q->prof) {
                (void)hipEventDestroy(r.a);
                (void)hipEventDestroy(r.b);
            }
            delete q->prof;
            q->prof = nullptr;
        }
    }
    return PD_OK;
}

pd_status pd_profile_read(pd_plan p, pd_pass_time* out, int cap, int* n_out) {
    if (!p || !n_out || (cap > 0 && !out)) return PD_EINVAL;
    std::vector<pd_pass_time> agg;
    pd_plan plans[2] = {p, p->sub32};
    for (pd_plan q : plans) {
        if (!q || !q->prof) continue;
        for (ProfRec& r : *q->prof) {
            float ms = 0.f;
            if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0.f;
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
            size_t k = 0;
            for (; k < agg.size(); ++k)
                if (std::strncmp(agg[k].name, r.name, sizeof(agg[k].name)) == 0) break;
            if (k == agg.size()) {
                pd_pass_time t{};
                std::snprintf(t.name, sizeof(t.name), "%s", r.name);
                agg.push_back(t);
            }
            agg[k].launches += 1;
            agg[k].total_ms += ms;
            agg[k].bytes += r.bytes;
        }
        q->prof->clear();
    }
    *n_out = (int)agg.size();
    for (int i = 0; i < (int)agg.size() && i < cap; ++i) out[i] = agg[i];
    return PD_OK;
}

pd_status pd_test_conv(pd_plan p, const void* x, const int* shift, int parity, void* out, void* stream) {
    if (!p || !x || !out || !shift) return PD_EINVAL;
    if (p->dtype == PD_F32) return test_conv_impl<float>(p, (const float*)x, shift, parity, (float*)out, S_(stream));
    return test_conv_impl<double>(p, (const double*)x, shift, parity, (double*)out, S_(stream));
}

pd_status pd_test_set_lastaxis(pd_plan p, int mode) {
    if (!p || mode < PD_LASTAXIS_AUTO || mode > PD_LASTAXIS_YFFT) return PD_EINVAL;
    p->lastaxis = mode;
    if (p->sub32) p->sub32->lastaxis = mode;
    return PD_OK;
}

pd_status pd_test_set_energy_form(pd_plan p, int form) {
    if (!p || form < PD_ENERGY_DIRECT || form > PD_ENERGY_CONVOLUTION) return PD_EINVAL;
    p->energy_form = form;
    return PD_OK;
}

}  // extern "C"
