// body.hpp -- host-side state of one body, shared by the entry points of api.hip and the request
// server of serve.hip.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/tlsph_dr.h"
#include "internal.hpp"

namespace tlsph {

enum Pass { kDrift = 0, kPassA, kPassB, kPassD, kPassC, kFinish, kNumPass };

struct ProfEvent {
    int pass;
    hipEvent_t a, b;
};

}  // namespace tlsph

struct tlsph_body_s {
    int dim = 0;
    int precision = 32;
    int64_t n = 0;
    hipStream_t stream = nullptr;
    int device = 0;                     // device current at creation: holds the body's memory
    tlsph_allocator alloc{};
    tlsph::DeviceBody db{};
    tlsph::StepParams P{};
    double dp = 0, h = 0, rc = 0, rc2 = 0, rho0 = 0;
    double xmin[3] = {0, 0, 0};
    double extent_min = 0, extent_max = 0;
    std::vector<int32_t> perm;          // internal -> input
    // material / loads / damping
    bool material_set = false;
    double E = 0, nu = 0;
    std::vector<double> bf_free_norm;   // |b| of free particles (for bmax)
    double bmax = 0;
    bool damping_set = false;
    double eta = 0, alpha = 1.0;
    uint64_t seed = 0;
    int scheme = 0;                     // TLSPH_PAIRWISE or TLSPH_PARTICLE
    // host mirror of the step counter
    int64_t step = 0;
    bool dt_valid = false;
    double dt_given = 0.0;
    tlsph::DevState *hst = nullptr;            // pinned mirror of DevState
    bool hst_owned = true;              // false: the mirror belongs to a server
    // profiling
    bool prof = false;
    std::vector<tlsph::ProfEvent> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[tlsph::kNumPass] = {0};
    int64_t prof_n[tlsph::kNumPass] = {0};

    void *dget(size_t bytes) { return alloc.alloc(bytes ? bytes : 256, alloc.ctx); }
    void dput(void *p)
    {
        if (p) alloc.free(p, alloc.ctx);
    }
};

namespace tlsph {

// api.hip helpers used by the server
tlsph_status fail(tlsph_status st, const char *fmt, ...);
// message of a device-detected step failure (TLSPH_E_NONFINITE or TLSPH_E_DIVERGED)
const char *step_error_text(int code);
bool damped_step(uint64_t seed, double alpha, int64_t n);
// tlsph_create_body with an optional caller-owned pinned mirror of the device state
tlsph_status create_body(const tlsph_body_desc *desc, DevState *mirror, tlsph_body *out);
void free_body(tlsph_body b);
tlsph_status pull_state(tlsph_body b);
tlsph_status download_field(tlsph_body b, const void *src, bool real, double *dst_input_order);
// true if step n of the body runs the damping pass
bool body_damped(tlsph_body b, int64_t n);
void update_viscous_limit(tlsph_body b);   // StepParams::dt_visc from the scheme and eta (Eq. 35)
// the body as a row of a batched launch
void fill_inst(tlsph_body b, Inst &I);

}  // namespace tlsph
