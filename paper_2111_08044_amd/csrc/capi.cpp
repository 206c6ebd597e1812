// C ABI of the Floquet brickwork engine (declared in include/floquet.h).
//
// Host responsibilities only: argument validation, FP64 gate construction,
// pass planning (cached per context), launch sequencing on the caller's
// stream, and the final FP64 contractions of the reduced quantities the
// kernels return (bond energies, gradient contractions).
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <array>
#include <map>
#include <string>
#include <vector>

#include "floquet.h"
#include "fl_common.h"
#include "host_math.h"
#include "kernels.h"
#include "noalloc.h"
#include "planner.h"

using cd = std::complex<double>;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int fail_hip(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return FL_EHIP;
}

#define FL_HIP(x)                                      \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return fail_hip(e_, #x); \
    } while (0)

constexpr int kPlanBlock = 16;        // periods per planned block
constexpr int kMaxGatesPerPass = 96;  // cap on gates the planner puts in one pass
constexpr int kReduceGrid = 2048;     // workgroups of the persistent reduction kernels
constexpr int kAdjGrid = 1024;        // workgroups of the persistent reverse pass
constexpr int kAdjLowBits = 4;       // low tile bits of the reverse pass (its kernel takes C at run time)
constexpr int kDense6LowBits = 4;    // low tile bits of the 6-qubit-window forms (their kernel takes C at run time)
constexpr int kWin4Grid = 256;        // workgroups of the 4-qubit-window reverse pass (one per CU)
constexpr int kMinNoallocGrid = 256;  // fewest reduction workgroups fl_expect_energy_noalloc runs
constexpr int kStageSlots = 8;        // pinned host staging slots for uploads
constexpr size_t kStageBytes = 256 << 10;  // bytes per slot: >= 3 x 4096 complex doubles (init tables)

int kmax_of(int dtype) { return dtype == FL_C64 ? FL_KMAX_C64 : FL_KMAX_C128; }

// Geometry of the plain sweep: complex64 on 13-bit tiles with 4 low bits and
// 4-bit register groups, complex128 on 12-bit tiles with 6 low bits and 4-bit
// groups.
fl_geom plain_geom(int L, int dtype) {
    return dtype == FL_C64 ? fl::make_geom(L, FL_KMAX_C64, FL_SWEEP_R_C64, FL_SWEEP_LOWBITS_C64)
                           : fl::make_geom(L, FL_KMAX_C128, 4);
}
size_t amp_bytes(int dtype) { return dtype == FL_C64 ? 8 : 16; }

}  // namespace

struct fl_ctx {
    int L = 0, dtype = 0, variant = 0, dev = 0;
    hipStream_t stream = nullptr;
    fl_geom geom{}, geom_adj{}, geom_rdm{};
    bool have_gates = false, have_h = false;
    double T = 0.0;
    std::vector<cd> h, G;  // FP64, (L-1) x 16
    void* d_gates = nullptr;   // 2 (L-1) gates, 32 reals each, context precision
    void* d_h = nullptr;       // (L-1) bond Hamiltonians, 32 reals each
    double* d_h64 = nullptr;   // the same in FP64 (energy contraction on the device)
    double* d_part = nullptr;  // reduction partials [kReduceGrid][L][16]
    double* d_red = nullptr;   // finalized reductions, 2 x L x 16
    double* h_red = nullptr;   // pinned host copy
    void* d_tabs = nullptr;    // product-state factor tables
    double* d_mpart = nullptr; // gradient partials [kAdjGrid][L-1][16]
    // complex64 reverse pass with window overlaps on the matrix cores:
    // Reverse pass of the 4-qubit-window form (k_adjoint_win4): for the
    // n-period forward plan, its passes and groups in reverse order with the
    // adjoint window fragments, and per reverse group the ops it undoes.
    struct AdjWin4 {
        std::vector<fl_pass> rev;            // reverse passes: the forward's tiles, groups and ops in reverse order (G^dagger)
        std::vector<std::array<int8_t, FL_MAX_OPS>> pos;    // per reverse group: window positions of its ops,
        std::vector<std::array<int16_t, FL_MAX_OPS>> bond;  // and their bonds, in the order the replay meets them
        std::vector<int> nops;
        void* d_mats = nullptr;              // 4 KiB of fragments per reverse group
    };
    std::map<int, AdjWin4> adj_w4;
    double* d_qpart = nullptr; // per-workgroup window overlaps [kWin4Grid][FL_WIN4_MAX_GROUPS][512]
    double* d_qsum = nullptr;  // window overlap of every group of the reverse plans [groups][512]
    size_t qsum_cap = 0;       // doubles allocated at d_qsum
    // Uploads (gates, bond terms, init tables) are copied on the context
    // stream from pinned staging slots; slot k may be refilled once the copy
    // recorded by stage_ev[k] has run.
    unsigned char* h_stage = nullptr;
    hipEvent_t stage_ev[kStageSlots] = {};
    bool stage_used[kStageSlots] = {};
    int stage_next = 0;
    hipEvent_t ev_switch = nullptr;    // orders work across a change of stream
    std::map<std::pair<int, int>, std::vector<fl_pass>> plans;
    std::map<int, std::vector<fl_pass>> adj_plans;
    struct DensePlan {
        std::vector<fl_pass> passes;   // opg[g][0] = window matrix index
        void* d_mats = nullptr;        // 64 KiB of MFMA fragments per window
    };
    std::map<std::pair<int, int>, DensePlan> dense_plans;
    std::vector<std::vector<unsigned char>> dense_host;  // host fragments: sources of in-flight uploads
    std::vector<fl_pass> cover;       // bond cover of the sweep geometry (H0 psi)
    std::vector<fl_pass> cover_rdm;   // bond cover of the reduction geometry
    bool use_grp = false;             // complex64, L >= 14: the reductions run on 13-bit tiles
    fl_geom geom_grp{};               // (L, 13, 5)
    std::vector<fl_pass> cover_grp;   // bond cover of geom_grp in register groups
};

namespace {

uint32_t ntiles(const fl_geom& g) { return 1u << (g.L - g.K); }

const std::vector<fl_pass>& get_plan(fl_ctx* c, int n, bool dagger) {
    auto key = std::make_pair(n, dagger ? 1 : 0);
    auto it = c->plans.find(key);
    if (it != c->plans.end()) return it->second;
    auto& v = c->plans[key];
    v = fl::plan_sweep(c->geom, n, dagger, false, kMaxGatesPerPass);
    return v;
}

const std::vector<fl_pass>& get_adj_plan(fl_ctx* c, int n) {
    auto it = c->adj_plans.find(n);
    if (it != c->adj_plans.end()) return it->second;
    auto& v = c->adj_plans[n];
    v = fl::plan_sweep(c->geom_adj, n, true, true, kMaxGatesPerPass);
    return v;
}

bool is_device_ptr(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

int check_state(const fl_ctx* c, const void* p, const char* name) {
    if (!p) return fail(FL_EINVAL, std::string(name) + " is NULL");
    if (((uintptr_t)p) & 255) return fail(FL_EINVAL, std::string(name) + " is not 256-byte aligned");
    if (!is_device_ptr(p)) return fail(FL_EINVAL, std::string(name) + " is not device memory");
    (void)c;
    return FL_OK;
}

bool finite_all(const double* a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

// Next pinned staging slot, once the upload that last read it has run.
int stage_slot(fl_ctx* c, unsigned char** out, int* slot) {
    const int k = c->stage_next;
    c->stage_next = (k + 1) % kStageSlots;
    if (c->stage_used[k]) FL_HIP(hipEventSynchronize(c->stage_ev[k]));
    *out = c->h_stage + (size_t)k * kStageBytes;
    *slot = k;
    return FL_OK;
}

// One staged upload: up to three (device destination, bytes) copies from
// consecutive regions of one staging slot, then the slot's event.
struct Staged {
    unsigned char* buf = nullptr;
    int slot = 0;
    size_t used = 0;
    void* dst[3] = {};
    size_t off[3] = {}, len[3] = {};
    int n = 0;
};

// Round FP64 complex matrices to `real_bytes` (4: FP32, 8: FP64) reals, 32 per
// 4x4, into the next region of the staged upload.
void stage_mats(Staged& st, void* dst, const std::vector<cd>& m, size_t nmat, int real_bytes) {
    unsigned char* p = st.buf + st.used;
    if (real_bytes == 4) {
        float* t = reinterpret_cast<float*>(p);
        for (size_t i = 0; i < nmat * 16; ++i) {
            t[2 * i] = (float)m[i].real();
            t[2 * i + 1] = (float)m[i].imag();
        }
    } else {
        double* t = reinterpret_cast<double*>(p);
        for (size_t i = 0; i < nmat * 16; ++i) {
            t[2 * i] = m[i].real();
            t[2 * i + 1] = m[i].imag();
        }
    }
    const size_t bytes = nmat * 32 * (size_t)real_bytes;
    st.dst[st.n] = dst;
    st.off[st.n] = st.used;
    st.len[st.n] = bytes;
    ++st.n;
    st.used += (bytes + 255) & ~(size_t)255;
}

// Enqueue the staged copies on the context stream (after every kernel already
// enqueued) and mark the slot busy until they have run.
int stage_commit(fl_ctx* c, const Staged& st) {
    if (st.used > kStageBytes) return fail(FL_EINVAL, "internal: staged upload too large");
    for (int k = 0; k < st.n; ++k)
        FL_HIP(hipMemcpyAsync(st.dst[k], st.buf + st.off[k], st.len[k], hipMemcpyHostToDevice, c->stream));
    FL_HIP(hipEventRecord(c->stage_ev[st.slot], c->stream));
    c->stage_used[st.slot] = true;
    return FL_OK;
}

// Drop the dense window plans (also those of the reverse pass); kernels
// already enqueued may still read them.
int drop_dense_plans(fl_ctx* c) {
    if (c->dense_plans.empty() && c->dense_host.empty() && c->adj_w4.empty()) return FL_OK;
    FL_HIP(hipStreamSynchronize(c->stream));
    for (auto& kv : c->dense_plans)
        if (kv.second.d_mats) (void)hipFree(kv.second.d_mats);
    c->dense_plans.clear();
    for (auto& kv : c->adj_w4)
        if (kv.second.d_mats) (void)hipFree(kv.second.d_mats);
    c->adj_w4.clear();
    c->dense_host.clear();
    return FL_OK;
}

// Gates and G^dagger in the context precision, the bond Hamiltonians in the
// context precision (H0 psi) and in FP64 (the on-device energy contraction).
int install_gates(fl_ctx* c) {
    const int nb = c->L - 1;
    int rc = drop_dense_plans(c);
    if (rc) return rc;
    std::vector<cd> both((size_t)2 * nb * 16);
    for (int b = 0; b < nb; ++b)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                both[(size_t)b * 16 + 4 * i + j] = c->G[(size_t)b * 16 + 4 * i + j];
                both[(size_t)(nb + b) * 16 + 4 * i + j] = std::conj(c->G[(size_t)b * 16 + 4 * j + i]);
            }
    Staged st;
    rc = stage_slot(c, &st.buf, &st.slot);
    if (rc) return rc;
    const int rb = c->dtype == FL_C64 ? 4 : 8;
    stage_mats(st, c->d_gates, both, (size_t)2 * nb, rb);
    if (c->have_h) {
        stage_mats(st, c->d_h, c->h, nb, rb);
        stage_mats(st, c->d_h64, c->h, nb, 8);
    }
    return stage_commit(c, st);
}

void read_c16(const double* src, cd* dst) {
    for (int i = 0; i < 16; ++i) dst[i] = cd(src[2 * i], src[2 * i + 1]);
}

// rho (4x4) from the 16 reals of a bond reduction.
void rho_from16(const double* v, cd* rho) {
    for (int i = 0; i < 4; ++i) rho[5 * i] = v[i];
    int k = 4;
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j) {
            rho[4 * i + j] = cd(v[k], v[k + 1]);
            rho[4 * j + i] = cd(v[k], -v[k + 1]);
            k += 2;
        }
}

// The bond reductions of psi into partials[grid][L][16] (grid <= maxgrid).
int launch_cover_rdm(fl_ctx* c, const void* psi, double* partials, int maxgrid, int* grid_out) {
    if (c->use_grp) {
        const int grid = (int)std::min<uint32_t>(ntiles(c->geom_grp), (uint32_t)maxgrid);
        for (const fl_pass& p : c->cover_grp) {
            hipError_t e = fl::launch_rdm_groups(c->geom_grp, psi, p, partials, grid, c->L, c->stream);
            if (e != hipSuccess) return fail_hip(e, "k_rdm_groups launch");
        }
        *grid_out = grid;
        return FL_OK;
    }
    const int grid = (int)std::min<uint32_t>(ntiles(c->geom_rdm), (uint32_t)maxgrid);
    for (const fl_pass& p : c->cover_rdm) {
        hipError_t e = fl::launch_rdm(c->dtype, c->geom_rdm, psi, p, partials, grid, c->L, c->stream);
        if (e != hipSuccess) return fail_hip(e, "k_rdm launch");
    }
    *grid_out = grid;
    return FL_OK;
}

bool is_dense(const fl_ctx* c) {
    return c->variant == FL_DENSE6_FP32 || c->variant == FL_DENSE6_BF16X3 || c->variant == FL_DENSE4_FP32;
}

// Fuse every register group of a 6-bit-window plan into its 64x64 matrix
// (FP64 product of the embedded gates) and upload the MFMA fragments.
int build_dense_plan(fl_ctx* c, int n, bool dagger, fl_ctx::DensePlan** out) {
    auto key = std::make_pair(n, dagger ? 1 : 0);
    auto it = c->dense_plans.find(key);
    if (it != c->dense_plans.end()) {
        *out = &it->second;
        return FL_OK;
    }
    const int nb = c->L - 1;
    const bool d4 = c->variant == FL_DENSE4_FP32;
    std::vector<fl_pass> plan = fl::plan_sweep(c->geom, n, dagger, false, kMaxGatesPerPass, nullptr,
                                               d4 ? FL_WIN4_MAX_GROUPS : FL_MAX_GROUPS);
    size_t nwin = 0;
    for (const fl_pass& p : plan) nwin += p.ngroups;
    const int mode = c->variant == FL_DENSE6_FP32 ? 0 : 1;
    const size_t fbytes = d4 ? 4096 : (mode == 1 ? 32768 : 65536);   // fragments per window
    std::vector<unsigned char> frags(nwin * fbytes);
    std::vector<cd> U(64 * 64);
    std::vector<cd> Gd((size_t)nb * 16);
    for (int b = 0; b < nb; ++b)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) Gd[(size_t)b * 16 + 4 * i + j] = std::conj(c->G[(size_t)b * 16 + 4 * j + i]);
    size_t w = 0;
    for (fl_pass& p : plan) {
        for (int g = 0; g < p.ngroups; ++g) {
            const cd* gates[FL_MAX_OPS];
            int pos[FL_MAX_OPS];
            for (int k = 0; k < p.nops[g]; ++k) {
                const int gi = p.opg[g][k];
                gates[k] = gi < nb ? &c->G[(size_t)gi * 16] : &Gd[(size_t)(gi - nb) * 16];
                pos[k] = p.opi[g][k];
            }
            if (d4) {
                fl::window_matrix_bits(gates, pos, p.nops[g], 4, U.data());
                fl::window_fragments4(U.data(), reinterpret_cast<float*>(frags.data() + w * fbytes));
            } else {
                fl::window_matrix(gates, pos, p.nops[g], U.data());
                fl::window_fragments(U.data(), mode, frags.data() + w * fbytes);
            }
            p.nops[g] = 1;
            p.opi[g][0] = 0;
            p.opg[g][0] = (int16_t)w;
            ++w;
        }
    }
    fl_ctx::DensePlan dp;
    dp.passes = plan;
    if (nwin) {
        hipError_t e = hipMalloc(&dp.d_mats, frags.size());
        if (e != hipSuccess) return fail(FL_ENOMEM, "window matrices: device allocation failed");
        // stream-ordered; the host copy lives as long as the plan
        c->dense_host.push_back(std::move(frags));
        const auto& src = c->dense_host.back();
        e = hipMemcpyAsync(dp.d_mats, src.data(), src.size(), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            (void)hipFree(dp.d_mats);
            c->dense_host.pop_back();
            return fail_hip(e, "window matrices upload");
        }
    }
    auto& slot = c->dense_plans[key];
    slot = dp;
    *out = &slot;
    return FL_OK;
}

int run_dense(fl_ctx* c, void* psi, int64_t n, bool dagger) {
    const int mode = c->variant == FL_DENSE6_FP32 ? 0 : 1;
    const int64_t q = n / kPlanBlock, r = n % kPlanBlock;
    auto go = [&](int m) -> int {
        fl_ctx::DensePlan* dp = nullptr;
        int rc = build_dense_plan(c, m, dagger, &dp);
        if (rc) return rc;
        for (const fl_pass& p : dp->passes) {
            hipError_t e = c->variant == FL_DENSE4_FP32 ? fl::launch_dense4(c->geom, psi, dp->d_mats, p, c->stream)
                                                         : fl::launch_dense6(mode, c->geom, psi, dp->d_mats, p, c->stream);
            if (e != hipSuccess) return fail_hip(e, "dense window kernel launch");
        }
        return FL_OK;
    };
    for (int64_t i = 0; i < q; ++i) {
        int rc = go(kPlanBlock);
        if (rc) return rc;
    }
    if (r > 0) return go((int)r);
    return FL_OK;
}

int run_periods(fl_ctx* c, void* psi, int64_t n, bool dagger) {
    if (is_dense(c)) return run_dense(c, psi, n, dagger);
    const int64_t q = n / kPlanBlock, r = n % kPlanBlock;
    if (q > 0) {
        const auto& pb = get_plan(c, kPlanBlock, dagger);
        for (int64_t i = 0; i < q; ++i)
            for (const fl_pass& p : pb) {
                hipError_t e = fl::launch_sweep(c->dtype, c->geom, psi, c->d_gates, p, c->stream);
                if (e != hipSuccess) return fail_hip(e, "k_sweep launch");
            }
    }
    if (r > 0) {
        const auto& pr = get_plan(c, (int)r, dagger);
        for (const fl_pass& p : pr) {
            hipError_t e = fl::launch_sweep(c->dtype, c->geom, psi, c->d_gates, p, c->stream);
            if (e != hipSuccess) return fail_hip(e, "k_sweep launch");
        }
    }
    return FL_OK;
}

int run_reverse(fl_ctx* c, void* psi, void* lam, int64_t n) {
    const int grid = (int)std::min<uint32_t>(ntiles(c->geom_adj), kAdjGrid);
    const int64_t q = n / kPlanBlock, r = n % kPlanBlock;
    auto go = [&](const std::vector<fl_pass>& plan) -> int {
        for (const fl_pass& p : plan) {
            hipError_t e = fl::launch_adjoint(c->dtype, c->geom_adj, psi, lam, c->d_gates, p, c->d_mpart, grid,
                                              c->stream);
            if (e != hipSuccess) return fail_hip(e, "k_adjoint launch");
        }
        return FL_OK;
    };
    for (int64_t i = 0; i < q; ++i) {
        int rc = go(get_adj_plan(c, kPlanBlock));
        if (rc) return rc;
    }
    if (r > 0) return go(get_adj_plan(c, (int)r));
    return FL_OK;
}

// The 4-qubit-window form (complex64, full 13-bit tiles) replays its own
// forward windows backwards on the matrix cores (k_adjoint_win4).
bool use_win4_reverse(const fl_ctx* c) {
    return c->dtype == FL_C64 && c->variant == FL_DENSE4_FP32 && c->geom.R == 4 && c->geom.C == FL_DENSE4_LOWBITS &&
           c->geom.C + c->geom.W == FL_KMAX_C64;
}

// The reverse of the n-period forward plan of the 4-qubit-window form: its
// passes and, within each, its groups in reverse order; group k (in that
// order) gets the fragments of U^dagger at k * 4 KiB, the exact transposes of
// the FP32 matrices the forward applied, and the list of ops it undoes.
int get_adj_win4(fl_ctx* c, int n, const fl_ctx::AdjWin4** out) {
    auto it = c->adj_w4.find(n);
    if (it != c->adj_w4.end()) {
        *out = &it->second;
        return FL_OK;
    }
    // the plan build_dense_plan runs for the forward (same planner call)
    const std::vector<fl_pass> fwd =
        fl::plan_sweep(c->geom, n, false, false, kMaxGatesPerPass, nullptr, FL_WIN4_MAX_GROUPS);
    const int nb = c->L - 1;
    fl_ctx::AdjWin4 aw;
    size_t nwin = 0;
    for (const fl_pass& p : fwd) nwin += (size_t)p.ngroups;
    std::vector<unsigned char> frags(std::max<size_t>(nwin, 1) * 4096);
    std::vector<cd> U(256), Ud(256);
    size_t w = 0;
    for (size_t i = fwd.size(); i-- > 0;) {
        const fl_pass& p = fwd[i];
        fl_pass rp = p;
        for (int gr = 0; gr < p.ngroups; ++gr, ++w) {
            const int g = p.ngroups - 1 - gr;
            const cd* gates[FL_MAX_OPS];
            int pos[FL_MAX_OPS];
            std::array<int8_t, FL_MAX_OPS> rpos{};
            std::array<int16_t, FL_MAX_OPS> rbond{};
            for (int k = 0; k < p.nops[g]; ++k) {
                const int gi = p.opg[g][k];
                if (gi < 0 || gi >= nb) return fail(FL_EINVAL, "internal: unexpected gate index in a forward plan");
                gates[k] = &c->G[(size_t)gi * 16];
                pos[k] = p.opi[g][k];
                rpos[p.nops[g] - 1 - k] = (int8_t)p.opi[g][k];
                rbond[p.nops[g] - 1 - k] = (int16_t)gi;
            }
            fl::window_matrix_bits(gates, pos, p.nops[g], 4, U.data());
            for (int r = 0; r < 16; ++r)
                for (int q = 0; q < 16; ++q) Ud[16 * r + q] = std::conj(U[16 * q + r]);
            fl::window_fragments4(Ud.data(), reinterpret_cast<float*>(frags.data() + w * 4096));
            // the reverse pass's group gr: the forward group g, ops reversed
            rp.u0[gr] = p.u0[g];
            rp.nops[gr] = p.nops[g];
            for (int k = 0; k < p.nops[g]; ++k) {
                rp.opi[gr][k] = p.opi[g][p.nops[g] - 1 - k];
                rp.opg[gr][k] = (int16_t)(nb + p.opg[g][p.nops[g] - 1 - k]);   // G^dagger in the gate table
                rp.ops[gr][k] = p.ops[g][p.nops[g] - 1 - k];
            }
            aw.pos.push_back(rpos);
            aw.bond.push_back(rbond);
            aw.nops.push_back(p.nops[g]);
        }
        aw.rev.push_back(rp);
    }
    hipError_t e = hipMalloc(&aw.d_mats, frags.size());
    if (e != hipSuccess) return fail(FL_ENOMEM, "reverse-pass windows: device allocation failed");
    // stream-ordered; the host copy lives as long as the windows
    c->dense_host.push_back(std::move(frags));
    const auto& src = c->dense_host.back();
    e = hipMemcpyAsync(aw.d_mats, src.data(), src.size(), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
        (void)hipFree(aw.d_mats);
        c->dense_host.pop_back();
        return fail_hip(e, "reverse-pass windows upload");
    }
    auto& slot = c->adj_w4[n];
    slot = std::move(aw);
    *out = &slot;
    return FL_OK;
}

// Replay one reverse plan; its group k adds its window overlap to
// d_qsum[(base + k) * 512 ...].
int run_reverse_win4(fl_ctx* c, void* psi, void* lam, const fl_ctx::AdjWin4& aw, size_t base) {
    const int grid = (int)std::min<uint32_t>(ntiles(c->geom), kWin4Grid);
    const unsigned char* mats = static_cast<const unsigned char*>(aw.d_mats);
    size_t k = 0;
    for (const fl_pass& p : aw.rev) {
        hipError_t e = fl::launch_adjoint_win4(c->geom, psi, lam, mats + k * 4096, p, c->d_qpart, grid,
                                               c->d_qsum + (base + k) * 512, c->stream);
        if (e != hipSuccess) return fail_hip(e, "k_adjoint_win4 launch");
        k += (size_t)p.ngroups;
    }
    return FL_OK;
}

// The bond overlap terms (16 reals per bond, summed) of every op undone by a
// reverse plan, from its groups' window overlaps Q (host FP64, the FP64
// adjoint gates).
void overlap_terms_win4(const fl_ctx* c, const fl_ctx::AdjWin4& aw, const double* qsum, std::vector<double>& D) {
    std::vector<cd> Gd((size_t)(c->L - 1) * 16);
    for (int b = 0; b < c->L - 1; ++b)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) Gd[(size_t)b * 16 + 4 * i + j] = std::conj(c->G[(size_t)b * 16 + 4 * j + i]);
    cd Q[256];
    double out[FL_MAX_OPS * 16];
    for (size_t k = 0; k < aw.nops.size(); ++k) {
        const double* q = qsum + k * 512;
        for (int e = 0; e < 256; ++e) Q[e] = cd(q[e], q[256 + e]);
        const cd* gates[FL_MAX_OPS];
        int pos[FL_MAX_OPS];
        for (int o = 0; o < aw.nops[k]; ++o) {
            gates[o] = &Gd[(size_t)aw.bond[k][o] * 16];
            pos[o] = aw.pos[k][o];
        }
        fl::window_overlap_terms(Q, gates, pos, aw.nops[k], out);
        for (int o = 0; o < aw.nops[k]; ++o)
            for (int v = 0; v < 16; ++v) D[(size_t)aw.bond[k][o] * 16 + v] += out[o * 16 + v];
    }
}

int apply_h0(fl_ctx* c, const void* psi, void* out) {
    bool first = true;
    for (const fl_pass& p : c->cover) {
        hipError_t e = fl::launch_apply_h(c->dtype, c->geom, psi, out, c->d_h, p, first ? 1 : 0, c->stream);
        if (e != hipSuccess) return fail_hip(e, "k_apply_h launch");
        first = false;
    }
    return FL_OK;
}

// Stage the three product-state factor tables, copy them to d_tabs and
// launch the init kernel, all in stream order (no host wait).
int upload_tables_and_init(fl_ctx* c, void* psi, const std::vector<cd>& tlo, const std::vector<cd>& tmid,
                           const std::vector<cd>& thi, int a, int b) {
    const size_t n = tlo.size() + tmid.size() + thi.size();
    if (n * 2 * sizeof(double) > kStageBytes || n > (size_t)3 * 4096) return fail(FL_EINVAL, "internal: init tables too large");
    Staged st;
    int rc = stage_slot(c, &st.buf, &st.slot);
    if (rc) return rc;
    double* t = reinterpret_cast<double*>(st.buf);
    size_t k = 0;
    for (const std::vector<cd>* v : {&tlo, &tmid, &thi})
        for (const cd& z : *v) {
            t[k++] = z.real();
            t[k++] = z.imag();
        }
    st.dst[0] = c->d_tabs;
    st.len[0] = k * sizeof(double);
    st.used = st.len[0];
    st.n = 1;
    rc = stage_commit(c, st);
    if (rc) return rc;
    hipError_t e = fl::launch_init(c->dtype, psi, c->L, c->d_tabs, a, b, c->stream);
    if (e != hipSuccess) return fail_hip(e, "k_init launch");
    return FL_OK;
}

}  // namespace

extern "C" {

const char* fl_last_error(void) { return g_err.c_str(); }

int fl_create(fl_ctx** ctx, int L, int dtype, int variant, void* hip_stream) {
    if (!ctx) return fail(FL_EINVAL, "ctx is NULL");
    *ctx = nullptr;
    if (dtype != FL_C64 && dtype != FL_C128) return fail(FL_EINVAL, "dtype must be FL_C64 or FL_C128");
    const int lmax = dtype == FL_C64 ? 34 : 33;
    if (L < 2 || L > lmax) return fail(FL_EINVAL, "L out of range [2, " + std::to_string(lmax) + "]");
    if (variant != FL_PLAIN && variant != FL_DENSE6_FP32 && variant != FL_DENSE6_BF16X3 && variant != FL_DENSE4_FP32)
        return fail(FL_EINVAL, "unknown variant");
    if (variant == FL_DENSE4_FP32 && L < FL_KMAX_C64)
        return fail(FL_EINVAL, "the 4-qubit-window variant needs full 13-bit tiles (L >= 13)");
    if (variant != FL_PLAIN && (dtype != FL_C64 || L < 11))
        return fail(FL_EINVAL, "dense 6-qubit windows need complex64 and L >= 11");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return fail(FL_ENODEV, "no HIP device");
    }
    int dev = 0;
    FL_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    FL_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(FL_ENODEV, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    // the static scratch of fl_expect_energy_noalloc: this device's address
    FL_HIP(fl::scratch_init(dev));
    fl_ctx* c = new fl_ctx();
    c->L = L;
    c->dtype = dtype;
    c->variant = variant;
    c->dev = dev;
    c->stream = (hipStream_t)hip_stream;
    c->geom = (variant == FL_PLAIN)         ? plain_geom(L, dtype)
              : (variant == FL_DENSE4_FP32) ? fl::make_geom(L, FL_KMAX_C64, 4, FL_DENSE4_LOWBITS)
                                            : fl::make_geom(L, FL_KMAX_C64, 6, kDense6LowBits);
    c->geom_adj = fl::make_geom(L, FL_KMAX_ADJ, 4, kAdjLowBits);
    c->geom_rdm = fl::make_geom(L, FL_KMAX_RDM, 2);
    c->cover = fl::plan_cover(c->geom);
    c->cover_rdm = fl::plan_cover(c->geom_rdm);
    c->use_grp = FL_RDM_GROUPS && dtype == FL_C64 && L > FL_KMAX_C64;
    if (c->use_grp) {
        c->geom_grp = fl::make_geom(L, FL_KMAX_C64, FL_RDM_R_C64);
        c->cover_grp = fl::plan_cover_groups(c->geom_grp);
    }
    const int nb = L - 1;
    const size_t rb = dtype == FL_C64 ? 4 : 8;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&c->d_gates, (size_t)2 * nb * 32 * rb);
    if (e == hipSuccess) e = hipMalloc(&c->d_h, (size_t)nb * 32 * rb);
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_h64, (size_t)nb * 32 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_part, (size_t)kReduceGrid * L * 16 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_red, (size_t)2 * L * 16 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_red, (size_t)2 * L * 16 * sizeof(double), 0);
    if (e == hipSuccess) e = hipMalloc(&c->d_tabs, (size_t)3 * 4096 * 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_mpart, (size_t)kAdjGrid * nb * 16 * sizeof(double));
    if (e == hipSuccess && use_win4_reverse(c))
        e = hipMalloc((void**)&c->d_qpart, (size_t)kWin4Grid * FL_WIN4_MAX_GROUPS * 512 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_stage, (size_t)kStageSlots * kStageBytes, 0);
    for (int k = 0; k < kStageSlots && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&c->stage_ev[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_switch, hipEventDisableTiming);
    if (e != hipSuccess) {
        fl_destroy(c);
        (void)hipGetLastError();
        return fail(FL_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    }
    *ctx = c;
    return FL_OK;
}

int fl_destroy(fl_ctx* c) {
    if (!c) return FL_OK;
    // kernels and uploads still in flight read the buffers freed below
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < kStageSlots; ++k)
        if (c->stage_ev[k]) (void)hipEventDestroy(c->stage_ev[k]);
    if (c->ev_switch) (void)hipEventDestroy(c->ev_switch);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    if (c->d_gates) (void)hipFree(c->d_gates);
    if (c->d_h) (void)hipFree(c->d_h);
    if (c->d_h64) (void)hipFree(c->d_h64);
    if (c->d_part) (void)hipFree(c->d_part);
    if (c->d_red) (void)hipFree(c->d_red);
    if (c->h_red) (void)hipHostFree(c->h_red);
    if (c->d_tabs) (void)hipFree(c->d_tabs);
    if (c->d_mpart) (void)hipFree(c->d_mpart);
    for (auto& kv : c->adj_w4)
        if (kv.second.d_mats) (void)hipFree(kv.second.d_mats);
    if (c->d_qpart) (void)hipFree(c->d_qpart);
    if (c->d_qsum) (void)hipFree(c->d_qsum);
    for (auto& kv : c->dense_plans)
        if (kv.second.d_mats) (void)hipFree(kv.second.d_mats);
    delete c;
    return FL_OK;
}

int fl_set_stream(fl_ctx* c, void* hip_stream) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    if (s == c->stream) return FL_OK;
    // The context's own buffers (gate tables, reduction scratch, init
    // tables) are reused across calls: work on the new stream starts after
    // everything already enqueued on the old one.
    FL_HIP(hipEventRecord(c->ev_switch, c->stream));
    FL_HIP(hipStreamWaitEvent(s, c->ev_switch, 0));
    c->stream = s;
    return FL_OK;
}

int fl_set_bonds(fl_ctx* c, const double* h, double T) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if (!h) return fail(FL_EINVAL, "h is NULL");
    if (!(T > 0.0) || !std::isfinite(T)) return fail(FL_EINVAL, "T must be finite and > 0");
    const int nb = c->L - 1;
    if (!finite_all(h, (size_t)nb * 32)) return fail(FL_EINVAL, "h has non-finite entries");
    std::vector<cd> hv((size_t)nb * 16);
    for (int b = 0; b < nb; ++b) read_c16(h + (size_t)b * 32, &hv[(size_t)b * 16]);
    for (int b = 0; b < nb; ++b) {
        const cd* m = &hv[(size_t)b * 16];
        double scale = 0.0, asym = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                scale = std::max(scale, std::abs(m[4 * i + j]));
                asym = std::max(asym, std::abs(m[4 * i + j] - std::conj(m[4 * j + i])));
            }
        if (asym > 1e-12 * std::max(1.0, scale))
            return fail(FL_EINVAL, "h[" + std::to_string(b) + "] is not Hermitian");
    }
    c->h = hv;
    c->G.assign((size_t)nb * 16, cd(0));
    for (int b = 0; b < nb; ++b) fl::gate_exp(&hv[(size_t)b * 16], 0.5 * T, &c->G[(size_t)b * 16]);
    c->T = T;
    c->have_h = true;
    int rc = install_gates(c);
    if (rc) return rc;
    c->have_gates = true;
    return FL_OK;
}

int fl_set_gates(fl_ctx* c, const double* G, const double* h, double T) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if (!G) return fail(FL_EINVAL, "G is NULL");
    const int nb = c->L - 1;
    if (!finite_all(G, (size_t)nb * 32) || (h && !finite_all(h, (size_t)nb * 32)))
        return fail(FL_EINVAL, "non-finite entries");
    std::vector<cd> Gv((size_t)nb * 16);
    for (int b = 0; b < nb; ++b) read_c16(G + (size_t)b * 32, &Gv[(size_t)b * 16]);
    for (int b = 0; b < nb; ++b) {
        const cd* m = &Gv[(size_t)b * 16];
        double dev = 0.0;  // max |G^dagger G - I|
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cd s = 0.0;
                for (int k = 0; k < 4; ++k) s += std::conj(m[4 * k + i]) * m[4 * k + j];
                dev = std::max(dev, std::abs(s - (i == j ? 1.0 : 0.0)));
            }
        if (dev > 1e-10) return fail(FL_EINVAL, "G[" + std::to_string(b) + "] is not unitary");
    }
    if (h) {
        for (int b = 0; b < nb; ++b)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    const cd hij(h[(size_t)b * 32 + 2 * (4 * i + j)], h[(size_t)b * 32 + 2 * (4 * i + j) + 1]);
                    const cd hji(h[(size_t)b * 32 + 2 * (4 * j + i)], h[(size_t)b * 32 + 2 * (4 * j + i) + 1]);
                    if (std::abs(hij - std::conj(hji)) > 1e-12 * std::max(1.0, std::abs(hij)))
                        return fail(FL_EINVAL, "h[" + std::to_string(b) + "] is not Hermitian");
                }
    }
    c->G = Gv;
    c->h.assign((size_t)nb * 16, cd(0));
    if (h)
        for (int b = 0; b < nb; ++b) read_c16(h + (size_t)b * 32, &c->h[(size_t)b * 16]);
    c->have_h = true;
    c->T = T;
    int rc = install_gates(c);
    if (rc) return rc;
    c->have_gates = true;
    return FL_OK;
}

int fl_init_state(fl_ctx* c, void* psi, const double* spinors) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_state(c, psi, "psi");
    if (rc) return rc;
    if (!spinors) return fail(FL_EINVAL, "spinors is NULL");
    const int L = c->L;
    if (!finite_all(spinors, (size_t)L * 4)) return fail(FL_EINVAL, "spinors have non-finite entries");
    std::vector<cd> s((size_t)2 * L);
    for (int i = 0; i < 2 * L; ++i) s[i] = cd(spinors[2 * i], spinors[2 * i + 1]);
    const int a = std::min(L, 12), b = std::min(L - a, 12);
    std::vector<cd> tlo, tmid, thi;
    fl::product_tables(L, s.data(), a, b, tlo, tmid, thi);
    return upload_tables_and_init(c, psi, tlo, tmid, thi, a, b);
}

int fl_init_pairs(fl_ctx* c, void* psi, const double* pairs, const double* tail) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_state(c, psi, "psi");
    if (rc) return rc;
    if (!pairs) return fail(FL_EINVAL, "pairs is NULL");
    const int L = c->L, np = L / 2;
    if ((L & 1) && !tail) return fail(FL_EINVAL, "odd L needs the spinor of the last site (tail)");
    if (!finite_all(pairs, (size_t)np * 8) || ((L & 1) && !finite_all(tail, 4)))
        return fail(FL_EINVAL, "pairs/tail have non-finite entries");
    std::vector<cd> pv((size_t)4 * np), tv(2, cd(1.0));
    for (int i = 0; i < 4 * np; ++i) pv[i] = cd(pairs[2 * i], pairs[2 * i + 1]);
    if (L & 1)
        for (int i = 0; i < 2; ++i) tv[i] = cd(tail[2 * i], tail[2 * i + 1]);
    // table boundaries on pair boundaries: even for even L, odd for odd L
    int a = std::min(L, 12), b = std::min(L - a, 12);
    if (L & 1) {
        a = std::min(L, 11);
        b = std::min(L - a, 12);
    }
    std::vector<cd> tlo, tmid, thi;
    if (!fl::pair_tables(L, pv.data(), tv.data(), a, b, tlo, tmid, thi))
        return fail(FL_EINVAL, "internal: pair table boundary");
    return upload_tables_and_init(c, psi, tlo, tmid, thi, a, b);
}

int fl_apply_period(fl_ctx* c, void* psi, int64_t n, int dagger) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_state(c, psi, "psi");
    if (rc) return rc;
    if (n < 0) return fail(FL_EINVAL, "n_periods < 0");
    if (dagger != 0 && dagger != 1) return fail(FL_EINVAL, "dagger must be 0 or 1");
    if (!c->have_gates) return fail(FL_ESTATE, "no gates: call fl_set_bonds first");
    return run_periods(c, psi, n, dagger == 1);
}

int fl_expect_energy(fl_ctx* c, const void* psi, double out[2], double* rdm) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_state(c, psi, "psi");
    if (rc) return rc;
    if (!out) return fail(FL_EINVAL, "out is NULL");
    if (!c->have_h) return fail(FL_ESTATE, "no bond Hamiltonians: call fl_set_bonds first");
    const int L = c->L;
    int grid = 0;
    rc = launch_cover_rdm(c, psi, c->d_part, kReduceGrid, &grid);
    if (rc) return rc;
    hipError_t e = fl::launch_finalize(c->d_part, grid, L * 16, c->d_red, c->stream);
    if (e != hipSuccess) return fail_hip(e, "k_finalize launch");
    FL_HIP(hipMemcpyAsync(c->h_red, c->d_red, (size_t)L * 16 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    FL_HIP(hipStreamSynchronize(c->stream));
    double E = 0.0;
    for (int b = 0; b < L - 1; ++b) {
        cd rho[16];
        rho_from16(c->h_red + (size_t)b * 16, rho);
        const cd* hb = &c->h[(size_t)b * 16];
        cd tr = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) tr += hb[4 * i + j] * rho[4 * j + i];
        E += tr.real();
        if (rdm)
            for (int k = 0; k < 16; ++k) {
                rdm[(size_t)b * 32 + 2 * k] = rho[k].real();
                rdm[(size_t)b * 32 + 2 * k + 1] = rho[k].imag();
            }
    }
    out[0] = E;
    out[1] = c->h_red[(size_t)(L - 1) * 16];
    return FL_OK;
}

int fl_expect_energy_noalloc(fl_ctx* c, const void* psi, double* out, double* rdm) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_state(c, psi, "psi");
    if (rc) return rc;
    if (!out || ((uintptr_t)out & 7) || !is_device_ptr(out)) return fail(FL_EINVAL, "out must be 8-byte aligned device memory");
    if (rdm && (((uintptr_t)rdm & 7) || !is_device_ptr(rdm)))
        return fail(FL_EINVAL, "rdm must be NULL or 8-byte aligned device memory");
    if (!c->have_h) return fail(FL_ESTATE, "no bond Hamiltonians: call fl_set_bonds first");
    int dev = -1;
    FL_HIP(hipGetDevice(&dev));
    if (dev != c->dev) return fail(FL_EINVAL, "the context's device must be current");
    double* scr = static_cast<double*>(fl::scratch_ptr(dev));
    if (!scr) return fail(FL_ESTATE, "static scratch not set up on this device");
    // scratch: partials [grid][L][16], then the L*16 finalized sums
    const int L = c->L;
    const size_t cap = fl::scratch_bytes() / sizeof(double), row = (size_t)L * 16;
    const size_t fit = cap > row ? (cap - row) / row : 0;
    if (fit < (size_t)kMinNoallocGrid)
        return fail(FL_EINVAL, "L = " + std::to_string(L) + " needs " +
                                   std::to_string((kMinNoallocGrid + 1) * row * sizeof(double)) +
                                   " bytes of static scratch, more than its " + std::to_string(fl::scratch_bytes()));
    const int maxgrid = (int)std::min<size_t>(fit, (size_t)kReduceGrid);
    int grid = 0;
    rc = launch_cover_rdm(c, psi, scr, maxgrid, &grid);
    if (rc) return rc;
    double* fin = scr + (size_t)grid * row;
    hipError_t e = fl::launch_finalize(scr, grid, (int)row, fin, c->stream);
    if (e != hipSuccess) return fail_hip(e, "k_finalize launch");
    e = fl::launch_energy_contract(fin, c->d_h64, L, out, rdm, c->stream);
    if (e != hipSuccess) return fail_hip(e, "k_energy_contract launch");
    return FL_OK;
}

int fl_overlap(fl_ctx* c, const void* phi, int dphi, const void* psi, int dpsi, double out[4]) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    if ((dphi != FL_C64 && dphi != FL_C128) || (dpsi != FL_C64 && dpsi != FL_C128))
        return fail(FL_EINVAL, "dtype must be FL_C64 or FL_C128");
    int rc = check_state(c, phi, "phi");
    if (rc) return rc;
    rc = check_state(c, psi, "psi");
    if (rc) return rc;
    if (!out) return fail(FL_EINVAL, "out is NULL");
    const uint64_t n = 1ull << c->L;
    const uint64_t want = (n + 255) / 256;
    const int grid = (int)std::min<uint64_t>(want, (uint64_t)kReduceGrid);
    hipError_t e = fl::launch_overlap(dphi, phi, dpsi, psi, n, c->d_part, grid, c->stream);
    if (e != hipSuccess) return fail_hip(e, "k_overlap launch");
    e = fl::launch_finalize(c->d_part, grid, 4, c->d_red, c->stream);
    if (e != hipSuccess) return fail_hip(e, "k_finalize launch");
    FL_HIP(hipMemcpyAsync(c->h_red, c->d_red, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    FL_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i < 4; ++i) out[i] = c->h_red[i];
    return FL_OK;
}

int fl_energy_spread(fl_ctx* c, const void* psi, void* ws, double out[3]) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_state(c, psi, "psi");
    if (rc) return rc;
    rc = check_state(c, ws, "ws");
    if (rc) return rc;
    if (ws == psi) return fail(FL_EINVAL, "ws must not alias psi");
    if (!out) return fail(FL_EINVAL, "out is NULL");
    if (!c->have_h) return fail(FL_ESTATE, "no bond Hamiltonians: call fl_set_bonds first");
    rc = apply_h0(c, psi, ws);
    if (rc) return rc;
    double ov[4];
    rc = fl_overlap(c, psi, c->dtype, ws, c->dtype, ov);
    if (rc) return rc;
    out[0] = ov[0];
    out[1] = ov[3];
    out[2] = ov[2];
    return FL_OK;
}

int64_t fl_grad_workspace_bytes(const fl_ctx* c) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    return (int64_t)((1ull << c->L) * amp_bytes(c->dtype));
}

int fl_grad(fl_ctx* c, void* psi_n, void* const* ckpts, int64_t n, int64_t K, const double* gens, int P,
            void* lam, double* grad) {
    if (!c) return fail(FL_EINVAL, "ctx is NULL");
    int rc = check_state(c, psi_n, "psi_n");
    if (rc) return rc;
    rc = check_state(c, lam, "lambda_ws");
    if (rc) return rc;
    if (lam == psi_n) return fail(FL_EINVAL, "lambda_ws must not alias psi_n");
    if (n < 0 || K < 0) return fail(FL_EINVAL, "n_periods and K must be >= 0");
    if (K > 0 && n % K != 0) return fail(FL_EINVAL, "n_periods must be a multiple of K");
    if (P < 0 || (P > 0 && !gens)) return fail(FL_EINVAL, "gens is NULL or P < 0");
    if (!grad) return fail(FL_EINVAL, "grad is NULL");
    if (!c->have_gates || !c->have_h) return fail(FL_ESTATE, "no bonds: call fl_set_bonds first");
    const int L = c->L, nb = L - 1;
    const int64_t nseg = (K > 0) ? n / K : (n > 0 ? 1 : 0);
    const int64_t seglen = (K > 0) ? K : n;
    if (K > 0 && n > 0) {
        if (!ckpts) return fail(FL_EINVAL, "ckpts is NULL");
        for (int64_t s = 0; s < nseg; ++s) {
            rc = check_state(c, ckpts[s], "ckpts[s]");
            if (rc) return rc;
        }
    }
    if (P > 0 && !finite_all(gens, (size_t)nb * P * 32)) return fail(FL_EINVAL, "gens has non-finite entries");
    const size_t bytes = (size_t)(1ull << L) * amp_bytes(c->dtype);
    // 1. bond density matrices of psi_n (explicit terms) -> d_red[0 .. L*16)
    int grid = 0;
    rc = launch_cover_rdm(c, psi_n, c->d_part, kReduceGrid, &grid);
    if (rc) return rc;
    hipError_t e = fl::launch_finalize(c->d_part, grid, L * 16, c->d_red, c->stream);
    if (e != hipSuccess) return fail_hip(e, "k_finalize launch");
    // 2. lambda = H0 psi_n
    rc = apply_h0(c, psi_n, lam);
    if (rc) return rc;
    // 3. reverse replay with checkpoint resets, accumulating D_b
    std::vector<double> Dmx;   // the matrix-core path's bond terms (host FP64)
    if (use_win4_reverse(c)) {
        // A segment's forward was fl_apply_period(K): qb blocks of kPlanBlock
        // periods, then the rr-period remainder; its replay runs the reverse
        // of the remainder plan, then of the block plan qb times.
        const int64_t qb = seglen / kPlanBlock, rr = seglen % kPlanBlock;
        const fl_ctx::AdjWin4* pb = nullptr;
        const fl_ctx::AdjWin4* pr = nullptr;
        if (qb > 0) {
            rc = get_adj_win4(c, kPlanBlock, &pb);
            if (rc) return rc;
        }
        if (rr > 0) {
            rc = get_adj_win4(c, (int)rr, &pr);
            if (rc) return rc;
        }
        const size_t gb = pb ? pb->nops.size() : 0, gr = pr ? pr->nops.size() : 0;
        const size_t need = std::max<size_t>(1, gb + gr) * 512;
        if (need > c->qsum_cap) {
            FL_HIP(hipStreamSynchronize(c->stream));
            if (c->d_qsum) (void)hipFree(c->d_qsum);
            c->d_qsum = nullptr;
            c->qsum_cap = 0;
            e = hipMalloc((void**)&c->d_qsum, need * sizeof(double));
            if (e != hipSuccess) return fail(FL_ENOMEM, "window overlap sums: device allocation failed");
            c->qsum_cap = need;
        }
        e = fl::launch_zero(c->d_qsum, need, c->stream);
        if (e != hipSuccess) return fail_hip(e, "k_zero launch");
        for (int64_t s = nseg - 1; s >= 0; --s) {
            if (pr) {
                rc = run_reverse_win4(c, psi_n, lam, *pr, gb);
                if (rc) return rc;
            }
            for (int64_t i = 0; i < qb; ++i) {
                rc = run_reverse_win4(c, psi_n, lam, *pb, 0);
                if (rc) return rc;
            }
            if (K > 0) FL_HIP(hipMemcpyAsync(psi_n, ckpts[s], bytes, hipMemcpyDeviceToDevice, c->stream));
        }
        std::vector<double> qsum(need);
        FL_HIP(hipMemcpyAsync(c->h_red, c->d_red, (size_t)L * 16 * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
        FL_HIP(hipMemcpyAsync(qsum.data(), c->d_qsum, need * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        FL_HIP(hipStreamSynchronize(c->stream));
        Dmx.assign((size_t)nb * 16, 0.0);
        if (pb) overlap_terms_win4(c, *pb, qsum.data(), Dmx);
        if (pr) overlap_terms_win4(c, *pr, qsum.data() + gb * 512, Dmx);
    } else {
        const int agrid = (int)std::min<uint32_t>(ntiles(c->geom_adj), kAdjGrid);
        e = fl::launch_zero(c->d_mpart, (uint64_t)agrid * nb * 16, c->stream);
        if (e != hipSuccess) return fail_hip(e, "k_zero launch");
        for (int64_t s = nseg - 1; s >= 0; --s) {
            rc = run_reverse(c, psi_n, lam, seglen);
            if (rc) return rc;
            if (K > 0) FL_HIP(hipMemcpyAsync(psi_n, ckpts[s], bytes, hipMemcpyDeviceToDevice, c->stream));
        }
        e = fl::launch_finalize(c->d_mpart, agrid, nb * 16, c->d_red + (size_t)L * 16, c->stream);
        if (e != hipSuccess) return fail_hip(e, "k_finalize launch");
        FL_HIP(hipMemcpyAsync(c->h_red, c->d_red, (size_t)2 * L * 16 * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
        FL_HIP(hipStreamSynchronize(c->stream));
    }
    const double* Dsrc = Dmx.empty() ? c->h_red + (size_t)L * 16 : Dmx.data();
    // 4. contractions on the host (FP64):
    //    dE/dtheta_{b,p} = Re sum_ij A_ij D_ij + tr(gen rho_b),  A = (dG/dtheta) G^dagger
    //    dE/dT          = sum_b Re sum_ij (-(i/2) h_b)_ij D_ij
    const double tau = 0.5 * c->T;
    double gT = 0.0;
    for (int b = 0; b < nb; ++b) {
        cd rho[16], D[16];
        rho_from16(c->h_red + (size_t)b * 16, rho);
        const double* v = Dsrc + (size_t)b * 16;
        for (int i = 0; i < 4; ++i) D[5 * i] = cd(0.0, 2.0 * v[i]);
        int k = 4;
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j) {
                D[4 * i + j] = cd(v[k], v[k + 1]);
                D[4 * j + i] = -std::conj(D[4 * i + j]);
                k += 2;
            }
        const cd* Gb = &c->G[(size_t)b * 16];
        cd Gd[16];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) Gd[4 * i + j] = std::conj(Gb[4 * j + i]);
        for (int p = 0; p < P; ++p) {
            cd gen[16], dG[16], A[16];
            read_c16(gens + ((size_t)b * P + p) * 32, gen);
            fl::gate_exp_derivative(&c->h[(size_t)b * 16], gen, tau, dG);
            fl::mat_mul_n(dG, Gd, A, 4);
            cd s = 0.0, ex = 0.0;
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    s += A[4 * i + j] * D[4 * i + j];
                    ex += gen[4 * i + j] * rho[4 * j + i];
                }
            grad[(size_t)b * P + p] = s.real() + ex.real();
        }
        cd sT = 0.0;
        for (int i = 0; i < 16; ++i) sT += cd(0.0, -0.5) * c->h[(size_t)b * 16 + i] * D[i];
        gT += sT.real();
    }
    grad[(size_t)nb * P] = gT;
    return FL_OK;
}

// ---------------------------------------------------------------- host helpers

int fl_xyz_bonds(int L, const double* J, const double* fields, double* h_out) {
    if (L < 2 || L > 64) return fail(FL_EINVAL, "L out of range");
    if (!J || !fields || !h_out) return fail(FL_EINVAL, "NULL argument");
    for (int b = 0; b < L - 1; ++b) {
        cd h[16];
        fl::xyz_bond(J + 3 * b, fields + 3 * b, fields + 3 * (b + 1), h);
        for (int k = 0; k < 16; ++k) {
            h_out[(size_t)b * 32 + 2 * k] = h[k].real();
            h_out[(size_t)b * 32 + 2 * k + 1] = h[k].imag();
        }
    }
    return FL_OK;
}

int fl_host_gates(int nb, const double* h, double T, double* G_out) {
    if (nb < 1 || !h || !G_out) return fail(FL_EINVAL, "bad argument");
    for (int b = 0; b < nb; ++b) {
        cd hm[16], G[16];
        read_c16(h + (size_t)b * 32, hm);
        fl::gate_exp(hm, 0.5 * T, G);
        for (int k = 0; k < 16; ++k) {
            G_out[(size_t)b * 32 + 2 * k] = G[k].real();
            G_out[(size_t)b * 32 + 2 * k + 1] = G[k].imag();
        }
    }
    return FL_OK;
}

int fl_host_ground_states(int n, const double* h, double* g_out, double* e_out) {
    if (n < 1 || !h || !g_out) return fail(FL_EINVAL, "bad argument");
    if (!finite_all(h, (size_t)n * 32)) return fail(FL_EINVAL, "h has non-finite entries");
    for (int k = 0; k < n; ++k) {
        cd hm[16], g[4];
        double e0 = 0.0;
        read_c16(h + (size_t)k * 32, hm);
        fl::ground_state4(hm, g, &e0);
        for (int i = 0; i < 4; ++i) {
            g_out[(size_t)k * 8 + 2 * i] = g[i].real();
            g_out[(size_t)k * 8 + 2 * i + 1] = g[i].imag();
        }
        if (e_out) e_out[k] = e0;
    }
    return FL_OK;
}

int fl_host_gate_derivative(const double* h, const double* gen, double T, double* dG_out) {
    if (!h || !gen || !dG_out) return fail(FL_EINVAL, "NULL argument");
    cd hm[16], gm[16], dG[16];
    read_c16(h, hm);
    read_c16(gen, gm);
    fl::gate_exp_derivative(hm, gm, 0.5 * T, dG);
    for (int k = 0; k < 16; ++k) {
        dG_out[2 * k] = dG[k].real();
        dG_out[2 * k + 1] = dG[k].imag();
    }
    return FL_OK;
}

int fl_xyz_generators(int L, double* gens_out) {
    if (L < 2 || L > 64 || !gens_out) return fail(FL_EINVAL, "bad argument");
    const double zero[3] = {0, 0, 0};
    for (int b = 0; b < L - 1; ++b)
        for (int a = 0; a < 3; ++a) {
            double J[3] = {0, 0, 0};
            J[a] = 1.0;
            cd h[16];
            fl::xyz_bond(J, zero, zero, h);
            for (int k = 0; k < 16; ++k) {
                gens_out[((size_t)b * 3 + a) * 32 + 2 * k] = h[k].real();
                gens_out[((size_t)b * 3 + a) * 32 + 2 * k + 1] = h[k].imag();
            }
        }
    return FL_OK;
}

int fl_tile_map(int L, int dtype, int h, uint64_t* out) {
    if (dtype != FL_C64 && dtype != FL_C128) return fail(FL_EINVAL, "bad dtype");
    if (L < 2 || L > 24 || !out) return fail(FL_EINVAL, "bad argument");
    const fl_geom g = plain_geom(L, dtype);
    if (g.W > 0 && (h < g.C || h + g.W > L)) return fail(FL_EINVAL, "window out of range");
    if (g.W == 0) h = g.C;
    const uint64_t nt = 1ull << (L - g.K);
    for (uint64_t t = 0; t < nt; ++t) {
        const uint64_t base = fl_tile_base(t, g.C, g.W, h);
        for (uint32_t j = 0; j < (1u << g.K); ++j) out[(t << g.K) + j] = base + fl_tile_offset(j, g.C, h);
    }
    return FL_OK;
}

int fl_host_window_matrix(const double* G, const int* pos, int nops, int mode, double* U_out, void* frag_out) {
    if (!G || !pos || nops < 0 || nops > 64 || !U_out) return fail(FL_EINVAL, "bad argument");
    if (mode < -1 || mode > 2) return fail(FL_EINVAL, "mode must be -1, 0, 1 or 2");
    const int nbits = mode == 2 ? 4 : 6, n = 1 << nbits;
    std::vector<cd> g((size_t)nops * 16);
    std::vector<const cd*> gp(nops);
    for (int k = 0; k < nops; ++k) {
        if (pos[k] < 0 || pos[k] > nbits - 2) return fail(FL_EINVAL, "gate position out of the window");
        read_c16(G + (size_t)k * 32, &g[(size_t)k * 16]);
        gp[k] = &g[(size_t)k * 16];
    }
    std::vector<cd> U((size_t)n * n);
    fl::window_matrix_bits(gp.data(), pos, nops, nbits, U.data());
    for (int i = 0; i < n * n; ++i) {
        U_out[2 * i] = U[i].real();
        U_out[2 * i + 1] = U[i].imag();
    }
    if (frag_out) {
        if (mode == 2) fl::window_fragments4(U.data(), static_cast<float*>(frag_out));
        else if (mode == 0 || mode == 1) fl::window_fragments(U.data(), mode, frag_out);
        else return fail(FL_EINVAL, "fragments need mode 0, 1 or 2");
    }
    return FL_OK;
}

int fl_host_window_overlaps(const double* Q, const double* G, const int* pos, int nops, double* out) {
    if (!Q || !G || !pos || nops < 0 || nops > 64 || !out) return fail(FL_EINVAL, "bad argument");
    for (int k = 0; k < nops; ++k)
        if (pos[k] < 0 || pos[k] > 2) return fail(FL_EINVAL, "gate position outside a 4-bit window");
    std::vector<cd> q(256), g((size_t)nops * 16);
    for (int e = 0; e < 256; ++e) q[e] = cd(Q[2 * e], Q[2 * e + 1]);
    std::vector<const cd*> gp(nops);
    for (int k = 0; k < nops; ++k) {
        read_c16(G + (size_t)k * 32, &g[(size_t)k * 16]);
        gp[k] = &g[(size_t)k * 16];
    }
    fl::window_overlap_terms(q.data(), gp.data(), pos, nops, out);
    return FL_OK;
}

int fl_plan_query(int L, int dtype, int kind, int64_t n, int dagger, int32_t* buf, int64_t cap, int64_t* needed) {
    if (dtype != FL_C64 && dtype != FL_C128) return fail(FL_EINVAL, "bad dtype");
    if (L < 2 || L > (dtype == FL_C64 ? 34 : 33)) return fail(FL_EINVAL, "L out of range");
    if (n < 0 || n > 100000) return fail(FL_EINVAL, "n out of range for a query");
    if (!needed) return fail(FL_EINVAL, "needed is NULL");
    std::vector<fl_pass> plan;
    fl_geom g;
    if (kind == 0) {
        g = plain_geom(L, dtype);
        const int64_t q = n / kPlanBlock, r = n % kPlanBlock;
        std::vector<fl_pass> pb, pr;
        if (q > 0) pb = fl::plan_sweep(g, kPlanBlock, dagger != 0, false, kMaxGatesPerPass);
        if (r > 0) pr = fl::plan_sweep(g, (int)r, dagger != 0, false, kMaxGatesPerPass);
        for (int64_t i = 0; i < q; ++i) plan.insert(plan.end(), pb.begin(), pb.end());
        plan.insert(plan.end(), pr.begin(), pr.end());
    } else if (kind == 1) {
        g = fl::make_geom(L, FL_KMAX_ADJ, 4, kAdjLowBits);
        const int64_t q = n / kPlanBlock, r = n % kPlanBlock;
        std::vector<fl_pass> pb, pr;
        if (q > 0) pb = fl::plan_sweep(g, kPlanBlock, true, true, kMaxGatesPerPass);
        if (r > 0) pr = fl::plan_sweep(g, (int)r, true, true, kMaxGatesPerPass);
        for (int64_t i = 0; i < q; ++i) plan.insert(plan.end(), pb.begin(), pb.end());
        plan.insert(plan.end(), pr.begin(), pr.end());
    } else if (kind == 2) {
        g = fl::make_geom(L, FL_KMAX_RDM, 2);
        plan = fl::plan_cover(g);
    } else if (kind == 4 || kind == 5) {
        if (dtype != FL_C64 || L < (kind == 4 ? 11 : FL_KMAX_C64))
            return fail(FL_EINVAL, "dense plans need complex64 and L >= 11 (6-qubit) or 13 (4-qubit windows)");
        g = kind == 4 ? fl::make_geom(L, FL_KMAX_C64, 6, kDense6LowBits)
                      : fl::make_geom(L, FL_KMAX_C64, 4, FL_DENSE4_LOWBITS);
        const int64_t q = n / kPlanBlock, r = n % kPlanBlock;
        std::vector<fl_pass> pb, pr;
        const int mg = kind == 5 ? FL_WIN4_MAX_GROUPS : FL_MAX_GROUPS;
        if (q > 0) pb = fl::plan_sweep(g, kPlanBlock, dagger != 0, false, kMaxGatesPerPass, nullptr, mg);
        if (r > 0) pr = fl::plan_sweep(g, (int)r, dagger != 0, false, kMaxGatesPerPass, nullptr, mg);
        for (int64_t i = 0; i < q; ++i) plan.insert(plan.end(), pb.begin(), pb.end());
        plan.insert(plan.end(), pr.begin(), pr.end());
    } else if (kind == 3) {
        g = plain_geom(L, dtype);
        plan = fl::plan_cover(g);
    } else if (kind == 6) {
        if (dtype != FL_C64 || L <= FL_KMAX_C64) return fail(FL_EINVAL, "the grouped cover needs complex64 and L >= 14");
        g = fl::make_geom(L, FL_KMAX_C64, FL_RDM_R_C64);
        plan = fl::plan_cover_groups(g);
    } else {
        return fail(FL_EINVAL, "kind must be 0..6");
    }
    std::vector<int> words;
    fl::serialize_plan(g, plan, words);
    *needed = (int64_t)words.size();
    if (buf) {
        const int64_t m = std::min<int64_t>(cap, (int64_t)words.size());
        for (int64_t i = 0; i < m; ++i) buf[i] = words[i];
    }
    return FL_OK;
}

}  // extern "C"
