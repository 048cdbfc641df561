// Host-side internals shared by the library's translation units: call
// context, error reporting, launch wrapper with optional event timing, the
// workspace layout, and the per-shape pipeline entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "../../include/nep.h"
#include "nep_device.hpp"

namespace nep {

constexpr int kMaxTypes = 16;

nep_status fail(nep_status code, const char* fmt, ...);
void clear_error();

// Event timing of launches (nep_profile_enable).
bool profiling_on();
void profile_begin(const char* name, hipStream_t st, void** token);
void profile_end(void* token, hipStream_t st);

#define NEP_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t _e = (call);                                                            \
        if (_e != hipSuccess)                                                              \
            return ::nep::fail(NEP_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(_e)); \
    } while (0)

#define NEP_LAUNCH(name, kernel, grid, block, shmem, stream, ...)                                       \
    do {                                                                                                \
        void* _tok = nullptr;                                                                           \
        if (::nep::profiling_on()) ::nep::profile_begin(name, stream, &_tok);                           \
        hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                            \
        hipError_t _e = hipGetLastError();                                                              \
        if (_tok) ::nep::profile_end(_tok, stream);                                                     \
        if (_e != hipSuccess)                                                                           \
            return ::nep::fail(NEP_ERR_HIP, "launch of %s failed: %s", name, hipGetErrorString(_e));    \
    } while (0)

enum class Mode { Descriptors, Forward, LossGrad, Backward };

// A resolved launch plan (nep_plan with the defaults filled in).
struct Plan {
    int team_desc, team_force, team_tangent, team_cg;
    int cg_blocks, outer_chunk;
    int network;  // 1 = matrix-core tiles, 2 = lane per atom, 3 = inside the sweeps
    int cg_rows;  // 0 = pair-per-lane coefficient sweep; 1..3 = moment rows per lane
};

// Team size (lanes per atom) of the pair sweeps and the grid defaults.
constexpr int kTeam = 8;
constexpr int kMaxAngRows = 2048;
constexpr int kOuterChunk = 64;
constexpr int kNetwork = 1;

// Defaults for zero fields; NEP_ERR_INVALID_ARG for values out of range.
nep_status resolve_plan(const nep_plan* p, Plan* out);

// Everything one call needs, already validated.
struct Ctx {
    Dims dm;
    Plan plan;
    bool f64;
    hipStream_t stream;
    Mode mode;
    int Ns;
    long Na;
    long pairs;
    // batch / neighbours
    const int64_t* atom_offset;
    const int* types;
    const int64_t* row;
    const int* seg;
    const void* pair_data;
    const int* reverse;
    const int* atom_struct;
    const int* species_order;
    const int64_t* species_offset;
    // parameters
    const void* theta;
    const void* qscale;
    // targets (LossGrad) or seeds (Backward)
    const double* Et;
    const void* Ft;
    const double* Wt;
    const uint8_t* has_v;
    double lam_e, lam_f, lam_v;
    const double* dE;
    const void* dF;
    const double* dW;
    // outputs
    double* loss;
    void* grad;
    // fused Adam/AMSGrad step after the gradient (nep_train_step)
    int adam;
    AdamArgs adam_args;
    void* theta_out;
    void* m;
    void* v;
    void* vmax;
    double* E_out;
    void* F_out;
    double* W_out;
    void* desc_out;
    // workspace
    unsigned char* ws;
    size_t ws_bytes;
};

// Workspace carve-up (byte offsets), identical for every shape of given sizes.
struct Layout {
    size_t q, A, S0, S1, Eat, e, t, F, Fown, Wat, ubar, dq, dA, abar, alpha, beta, gam, h;
    size_t Es, Ws, ebar, Ubar, lossp, outer_part, ang_part, stage, nbr_totals;
    size_t total;
    int outer_rows, ang_rows, outer_chunk;
};

Layout make_layout(const Dims& dm, const Plan& plan, bool f64, int Ns, long Na, long pairs);

// Calls f(std::integral_constant<int, S>) for the team size s in {4, 8, 16}.
template <typename T, class F>
T with_team_size(int s, F&& f) {
    switch (s) {
        case 4: return f(std::integral_constant<int, 4>{});
        case 16: return f(std::integral_constant<int, 16>{});
        default: return f(std::integral_constant<int, 8>{});
    }
}
// Calls f(std::integral_constant<int, R>) for rows r in {1, 2, 3} of the
// row-owned coefficient sweep.
template <typename T, class F>
T with_cg_rows(int r, F&& f) {
    switch (r) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 3: return f(std::integral_constant<int, 3>{});
        default: return f(std::integral_constant<int, 2>{});
    }
}
template <class F>
nep_status with_team(int s, F&& f) {
    return with_team_size<nep_status>(s, static_cast<F&&>(f));
}
// the coefficient-gradient sweep also runs with 32-lane teams (its per-team
// LDS block makes wide teams the way to fit more waves per CU for large moment
// blocks with many angular neighbours)
template <typename T, class F>
T with_cg_team_size(int s, F&& f) {
    if (s == 32) return f(std::integral_constant<int, 32>{});
    return with_team_size<T>(s, static_cast<F&&>(f));
}

// Blocks of `threads` threads with `shm` bytes of dynamic LDS that the current
// device holds at once for kernel `fn` (occupancy per CU times CUs, cached per
// kernel, device and launch shape); -1 if the runtime query fails.
int resident_blocks(const void* fn, int threads, size_t shm);
// cg_rows_geom with the T-independent part computed once per shape (host).
CgRowsGeom cg_rows_geom_host(int T, int NA, int KA, int LM, int rbytes, int rows);

// Per-shape pipeline (forward / loss+grad / backward / descriptors).
using ShapeFn = nep_status (*)(const Ctx&);
struct ShapeEntry {
    int KR, KA, NR, NA, L, H4, H5;
    ShapeFn f32, f64;
};
const ShapeEntry* find_shape(const Dims& dm);
const ShapeEntry* shape_table(int* count);

nep_status build_neighbors(const Ctx& c, const nep_batch* b, nep_neighbors* nb, void* ws, size_t ws_bytes);
nep_status gather_batch(const Ctx& c, const nep_batch* src, const nep_neighbors* sn, const nep_targets* st,
                        const int* ids, int n, long Na, int64_t* dst_off, void* dst_pos, int* dst_types,
                        double* dst_cells, nep_neighbors* dn, double* dst_E, void* dst_F, double* dst_W,
                        uint8_t* dst_hv, void* ws, size_t ws_bytes);

// ZBL pair term (nep_zbl.hip): adds scale * (E, F, W) of the term; arguments
// already validated. ws holds zbl_workspace_bytes(Na).
size_t zbl_workspace_bytes(long Na);
nep_status zbl_add(const Dims& dm, bool f64, const nep_zbl* z, const nep_batch* b, const nep_neighbors* nb,
                   double scale, double* energy, void* force, double* virial, void* ws, hipStream_t st);

}  // namespace nep
