// The launch sequence of one call for one descriptor shape and precision.
//
//   descriptors : descriptor
//   forward     : descriptor -> network_forward -> force -> structure
//   loss+grad   : forward, structure(loss, seeds) -> tangent -> network_backward
//                 -> angular_coeff_grad -> outer_grad -> final_reduce
//   backward    : descriptor -> network_forward -> seeds -> tangent -> ... -> final_reduce
#pragma once

#include "nep_internal.hpp"
#include "nep_kernels.hpp"
#include "nep_reduce.hpp"

namespace nep {

template <typename R, class Sh>
nep_status run_shape(const Ctx& c) {
    const Layout L = make_layout(c.dm, c.plan, c.f64, c.Ns, c.Na, c.pairs);
    if (c.ws_bytes < L.total) return fail(NEP_ERR_WORKSPACE, "workspace holds %zu bytes, %zu needed", c.ws_bytes, L.total);
    auto Wr = [&](size_t off) { return reinterpret_cast<R*>(c.ws + off); };
    auto Wd = [&](size_t off) { return reinterpret_cast<double*>(c.ws + off); };
    const Dims dm = c.dm;
    const hipStream_t st = c.stream;
    const int Na = int(c.Na);
    const R* theta = static_cast<const R*>(c.theta);
    const R* qscale = static_cast<const R*>(c.qscale);
    const Rec<R>* pairs = static_cast<const Rec<R>*>(c.pair_data);
    auto team_grid = [&](int S) { return (Na + kBlock / S - 1) / (kBlock / S); };
    nep_status rs = NEP_OK;

    // LDS of the angular-coefficient gradient block (dynamic; <= one CU's 160 KB).
    // A block that does not fit with the plan's team size (many species in
    // FP64: T^2 accumulator blocks) runs with 32-lane teams, the smallest block;
    // the grid and the partial rows are the plan's either way.
    int team_cg = c.plan.team_cg;
    auto cg_bytes = [&](int S) {
        return with_cg_team_size<size_t>(S, [&](auto S_) { return CoeffGradSmem<R, Sh, decltype(S_)::value>::bytes(dm.T); });
    };
    if (cg_bytes(team_cg) > 160 * 1024) team_cg = 32;
    const size_t cg_shm = cg_bytes(team_cg);
    // the row-owned form: LDS of one wavefront, wavefronts per block
    const CgRowsGeom cg_rows_gm =
        cg_rows_geom_host(dm.T, Sh::NA, Sh::KA, Sh::LM, int(sizeof(R)), c.plan.cg_rows > 0 ? c.plan.cg_rows : 1);
    const int cg_rows_nw = cg_rows_waves(cg_rows_gm.wave_bytes);
    if (c.mode == Mode::LossGrad || c.mode == Mode::Backward) {
        if (c.plan.cg_rows > 0 && cg_rows_gm.wave_bytes > 160 * 1024)
            return fail(NEP_ERR_UNSUPPORTED, "row-owned angular coefficient sweep needs %zu bytes of LDS per wavefront",
                        cg_rows_gm.wave_bytes);
        if (c.plan.cg_rows == 0 && cg_shm > 160 * 1024)
            return fail(NEP_ERR_UNSUPPORTED, "angular coefficient block of %d-lane teams needs %zu bytes of LDS",
                        team_cg, cg_shm);
        if (OuterTiles<R>::lds_bytes(dm) > 160 * 1024 || dm.H > kBlock ||
            OuterTiles<R>::tiles(dm) > OuterTiles<R>::WAVES * OuterTiles<R>::MAXTW)
            return fail(NEP_ERR_UNSUPPORTED, "network of %d hidden units too large for the outer-product tiles", dm.H);
    }

    R* q = (c.mode == Mode::Descriptors || c.desc_out) && c.desc_out ? static_cast<R*>(c.desc_out) : Wr(L.q);
    // network 3: each atom's network runs in its team at the end of the
    // descriptor (forward) and tangent (Hessian-vector product) sweeps, and
    // when forces are wanted the descriptor sweep also runs the force pass
    const bool fused = c.plan.network == 3 && c.mode != Mode::Descriptors;
    const bool fused_force = fused && (c.mode == Mode::Forward || c.mode == Mode::LossGrad);
    Rec<R>* hslots = reinterpret_cast<Rec<R>*>(Wr(L.h));
    if (Na > 0 && (rs = with_team(c.plan.team_desc, [&](auto S_) -> nep_status {
            constexpr int S = decltype(S_)::value;
            if (fused_force)
                NEP_LAUNCH("descriptor", (k_descriptor<R, Sh, S, 2>), dim3(team_grid(S) + dm.T), dim3(kBlock), 0, st,
                           dm, theta, c.species_order, c.species_offset, Na, c.row, c.seg, pairs, q, Wr(L.A), Wr(L.S0), qscale, Wr(L.Eat), Wr(L.e),
                           Wr(L.t), c.reverse, hslots, Wr(L.Fown), Wr(L.Wat));
            else if (fused)
                NEP_LAUNCH("descriptor", (k_descriptor<R, Sh, S, 1>), dim3(team_grid(S) + dm.T), dim3(kBlock), 0, st,
                           dm, theta, c.species_order, c.species_offset, Na, c.row, c.seg, pairs, q, Wr(L.A), Wr(L.S0), qscale, Wr(L.Eat), Wr(L.e),
                           Wr(L.t), nullptr, nullptr, nullptr, nullptr);
            else
                NEP_LAUNCH("descriptor", (k_descriptor<R, Sh, S, 0>), dim3(team_grid(S) + dm.T), dim3(kBlock), 0, st,
                           dm, theta, c.species_order, c.species_offset, Na, c.row, c.seg, pairs, q, Wr(L.A), Wr(L.S0), nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, nullptr, nullptr);
            return NEP_OK;
        })))
        return rs;
    if (c.mode == Mode::Descriptors) return NEP_OK;

    const bool lane_net = c.plan.network == 2;
    const int net_grid = lane_net ? int((c.Na + 63) / 64) + dm.T : int((c.Na + Mfma<R>::M - 1) / Mfma<R>::M) + dm.T;
    if (Na > 0 && lane_net)
        NEP_LAUNCH("network_forward", (k_network_forward_lane<R, Sh>), dim3(net_grid), dim3(64), 0, st, dm, theta,
                   qscale, c.species_order, c.species_offset, q, Wr(L.Eat), Wr(L.e), Wr(L.t));
    if (Na > 0 && !lane_net && !fused)
        NEP_LAUNCH("network_forward", (k_network_forward<R, Sh>), dim3(net_grid), dim3(64), 0, st, dm, theta, qscale,
                   c.species_order, c.species_offset, q, Wr(L.Eat), Wr(L.e), Wr(L.t));

    double* Es = c.E_out ? c.E_out : Wd(L.Es);
    double* Ws = c.W_out ? c.W_out : Wd(L.Ws);
    R* F = c.F_out ? static_cast<R*>(c.F_out) : Wr(L.F);
    const bool loss = c.mode == Mode::LossGrad;

    if (c.mode == Mode::Forward || loss) {
        if (Na > 0 && (rs = with_team(c.plan.team_force, [&](auto S_) -> nep_status {
                constexpr int S = decltype(S_)::value;
                if (fused_force) {
                } else if constexpr (sizeof(R) == 8) {
                    NEP_LAUNCH("force", (k_force_lockstep<R, Sh, S>), dim3(team_grid(S) + dm.T), dim3(kBlock), 0,
                               st, dm, theta, c.species_order, c.species_offset, Na, c.row, c.seg, pairs, c.reverse,
                               Wr(L.A), Wr(L.e), hslots, Wr(L.Fown), Wr(L.Wat));
                } else {
                    // the segment-crossing force sweep: c^A, eps_k and the segment
                    // tables in dynamic LDS
                    const size_t shm = force_lds(dm.T, Sh::NA, Sh::KA, Sh::KR, kBlock / S, int(sizeof(R))).bytes;
                    const size_t stat = size_t(kBlock / S) * Sh::NA * Sh::LM * sizeof(R);
                    if (shm + stat > 64 * 1024)
                        NEP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_force<R, Sh, S>),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(shm)));
                    NEP_LAUNCH("force", (k_force<R, Sh, S>), dim3(team_grid(S) + dm.T), dim3(kBlock), shm, st, dm,
                               theta, c.species_order, c.species_offset, Na, c.row, c.seg, pairs, c.reverse, Wr(L.A),
                               Wr(L.e), hslots, Wr(L.Fown), Wr(L.Wat));
                }
                NEP_LAUNCH("force_gather", (k_force_gather<R, S>), dim3(team_grid(S)), dim3(kBlock), 0, st, Na,
                           c.row, reinterpret_cast<const Rec<R>*>(Wr(L.h)), Wr(L.Fown), F);
                return NEP_OK;
            })))
            return rs;
        if (c.Ns > 0)
            NEP_LAUNCH("structure", (k_structure<R>), dim3(c.Ns), dim3(kRedBlock), 0, st, c.Ns, c.Na, c.atom_offset,
                       Wr(L.Eat), Wr(L.Wat), F, loss ? 1 : 0, c.Et, static_cast<const R*>(c.Ft), c.Wt, c.has_v,
                       c.lam_e, c.lam_f, c.lam_v, Es, Ws, Wd(L.ebar), Wd(L.Ubar), Wr(L.ubar), Wd(L.lossp));
        if (!loss) return NEP_OK;
    } else {
        const long n = 9L * c.Ns > 3L * c.Na ? 9L * c.Ns : 3L * c.Na;
        if (n > 0)
            NEP_LAUNCH("seeds", (k_seeds<R>), dim3(int((n + kRedBlock - 1) / kRedBlock)), dim3(kRedBlock), 0, st,
                       c.Ns, c.Na, c.dE, static_cast<const R*>(c.dF), c.dW, Wd(L.ebar), Wd(L.Ubar), Wr(L.ubar));
    }

    int ang_rows_used = L.ang_rows;  // partial rows the coefficient sweep writes
    if (Na > 0) {
        if ((rs = with_team(c.plan.team_tangent, [&](auto S_) -> nep_status {
                constexpr int S = decltype(S_)::value;
                if (fused)
                    NEP_LAUNCH("tangent", (k_tangent<R, Sh, S, true>), dim3(team_grid(S) + dm.T), dim3(kBlock), 0, st,
                               dm, theta, c.species_order, c.species_offset, c.atom_struct, Na, c.row, c.seg, pairs, Wr(L.ubar), Wd(L.Ubar),
                               Wr(L.A), Wr(L.dq), Wr(L.dA), Wr(L.S1), qscale, Wd(L.ebar), Wr(L.e), Wr(L.t),
                               Wr(L.abar), Wr(L.alpha), Wr(L.beta), Wr(L.gam));
                else
                    NEP_LAUNCH("tangent", (k_tangent<R, Sh, S, false>), dim3(team_grid(S) + dm.T), dim3(kBlock), 0, st,
                               dm, theta, c.species_order, c.species_offset, c.atom_struct, Na, c.row, c.seg, pairs, Wr(L.ubar), Wd(L.Ubar),
                               Wr(L.A), Wr(L.dq), Wr(L.dA), Wr(L.S1), nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr);
                return NEP_OK;
            })))
            return rs;
        if (fused) {
        } else if (lane_net)
            NEP_LAUNCH("network_backward", (k_network_backward_lane<R, Sh>), dim3(net_grid), dim3(64), 0, st, dm,
                       theta, qscale, c.species_order, c.species_offset, c.atom_struct, Wd(L.ebar), Wr(L.dq),
                       Wr(L.e), Wr(L.t), Wr(L.abar), Wr(L.alpha), Wr(L.beta), Wr(L.gam));
        else
            NEP_LAUNCH("network_backward", (k_network_backward<R, Sh>), dim3(net_grid), dim3(64), 0, st, dm, theta,
                       qscale, c.species_order, c.species_offset, c.atom_struct, Wd(L.ebar), Wr(L.dq), Wr(L.e),
                       Wr(L.t), Wr(L.abar), Wr(L.alpha), Wr(L.beta), Wr(L.gam));
        if (c.plan.cg_rows > 0) {
            if constexpr (sizeof(R) != 4)
                return fail(NEP_ERR_UNSUPPORTED, "the row-owned coefficient sweep is built for FP32 only");
            else if ((rs = with_cg_rows<nep_status>(c.plan.cg_rows, [&](auto R_) -> nep_status {
                    constexpr int ROWS = decltype(R_)::value;
                    const size_t shm = size_t(cg_rows_nw) * cg_rows_gm.wave_bytes;
                    const void* kfn = reinterpret_cast<const void*>(&k_angular_coeff_grad_rows<R, Sh, ROWS>);
                    if (shm > 64 * 1024)
                        NEP_HIP(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, int(shm)));
                    // each wavefront walks a fixed range of tiles, so the grid is
                    // the number of blocks the GPU holds at once (no second round),
                    // at most the plan's partial rows
                    const int resident = resident_blocks(kfn, 64 * cg_rows_nw, shm);
                    if (resident < 0) return fail(NEP_ERR_HIP, "occupancy query of the coefficient sweep failed");
                    const int grid = std::max(1, std::min(L.ang_rows / cg_rows_nw, resident));
                    ang_rows_used = grid * cg_rows_nw;
                    // atoms ordered by angular pair count within groups of tiles
                    // when a wavefront walks enough tiles to amortise the ordering
                    const long tiles_ub = (long(Na) + cg_rows_gm.teams - 1) / cg_rows_gm.teams + dm.T;
                    const long per_wave = (tiles_ub + ang_rows_used - 1) / ang_rows_used;
                    const int group_tiles = per_wave >= 4 ? kCgSortTiles : 0;
                    NEP_LAUNCH("angular_coeff_grad", (k_angular_coeff_grad_rows<R, Sh, ROWS>),
                               dim3(grid), dim3(64 * cg_rows_nw), shm, st, dm, c.species_order,
                               c.species_offset, c.atom_struct, Na, c.row, c.seg, pairs, Wr(L.ubar), Wd(L.Ubar),
                               Wr(L.A), Wr(L.dA), Wr(L.e), Wr(L.abar), group_tiles, Wd(L.ang_part));
                    return NEP_OK;
                })))
                return rs;
        } else if ((rs = with_cg_team_size<nep_status>(team_cg, [&](auto S_) -> nep_status {
                constexpr int S = decltype(S_)::value;
                if (cg_shm > 64 * 1024)
                    NEP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_angular_coeff_grad<R, Sh, S>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, int(cg_shm)));
                NEP_LAUNCH("angular_coeff_grad", (k_angular_coeff_grad<R, Sh, S>), dim3(L.ang_rows), dim3(kBlock),
                           cg_shm, st, dm, c.types, c.atom_struct, Na, c.row, c.seg, pairs, Wr(L.ubar), Wd(L.Ubar),
                           Wr(L.A), Wr(L.dA), Wr(L.e), Wr(L.abar), Wd(L.ang_part));
                return NEP_OK;
            })))
            return rs;
        // FP32 sub-chunks of 32 atoms (half the barrier rounds of 16) unless a
        // 32-atom block's LDS (> 32 KB) would cut the blocks per CU of a grid
        // with work for several of them (>= 1024 blocks); FP64 takes 16
        const size_t lds32 = OuterTiles<R, 32>::lds_bytes(dm);
        const bool sc32 = sizeof(R) == 4 && lds32 <= 64 * 1024 && (lds32 <= 32 * 1024 || L.outer_rows < 1024);
        const size_t og_shm = sc32 ? OuterTiles<R, 32>::lds_bytes(dm) : OuterTiles<R, 16>::lds_bytes(dm);
        auto outer_sc = [&](auto TW_, auto SC_) -> nep_status {
            constexpr int TW = decltype(TW_)::value, SC = decltype(SC_)::value;
            if (og_shm > 64 * 1024)
                NEP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_outer_grad<R, Sh, TW, SC>),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, int(og_shm)));
            NEP_LAUNCH("outer_grad", (k_outer_grad<R, Sh, TW, SC>), dim3(L.outer_rows), dim3(kBlock), og_shm, st, dm,
                       qscale, c.species_order, c.species_offset, L.outer_chunk, q, Wr(L.dq), Wr(L.abar), Wr(L.e),
                       Wr(L.alpha), Wr(L.beta), Wr(L.gam), Wr(L.S0), Wr(L.S1), fused ? 1 : 0, Wd(L.outer_part));
            return NEP_OK;
        };
        auto outer = [&](auto TW_) -> nep_status {
            if constexpr (sizeof(R) == 4)
                if (sc32) return outer_sc(TW_, std::integral_constant<int, 32>{});
            return outer_sc(TW_, std::integral_constant<int, 16>{});
        };
        switch (OuterTiles<R>::tiles_per_wave(dm)) {
            case 1: rs = outer(std::integral_constant<int, 1>{}); break;
            case 2: rs = outer(std::integral_constant<int, 2>{}); break;
            case 4: rs = outer(std::integral_constant<int, 4>{}); break;
            default: rs = outer(std::integral_constant<int, 6>{}); break;
        }
        if (rs) return rs;
    }
    if (Na > 0 && dm.offB1 > 0)
        NEP_LAUNCH("reduce_stage", k_reduce_stage<kRedBlock / 64>, dim3(int((dm.offB1 + 63) / 64), kStageGroups), dim3(kRedBlock), 0,
                   st, dm, Sh::NR * Sh::KR, Wd(L.outer_part), L.outer_rows, Wd(L.ang_part), ang_rows_used, Wd(L.stage),
                   c.species_offset, L.outer_chunk);
    NEP_LAUNCH("final_reduce", (k_final_reduce<R>), dim3(int((dm.offB1 + kRedBlock) / kRedBlock)), dim3(kRedBlock), 0,
               st, dm, c.Ns, c.atom_offset, Wd(L.stage), Na > 0 ? kStageGroups : 0, Wd(L.ebar), Wd(L.lossp), c.lam_e,
               c.lam_f, c.lam_v, static_cast<R*>(c.grad), loss ? c.loss : nullptr, c.adam, c.adam_args,
               static_cast<R*>(c.theta_out), static_cast<R*>(c.m), static_cast<R*>(c.v), static_cast<R*>(c.vmax));
    return NEP_OK;
}

}  // namespace nep

// Instantiates both precisions of one shape and registers them.
#define NEP_SHAPE_TU(KR, KA, NR, NA, L, H4, H5)                                                       \
    namespace nep {                                                                                   \
    nep_status shape_f32_##KR##_##KA##_##NR##_##NA##_##L##_##H4##_##H5(const Ctx& c) {                \
        return run_shape<float, Shape<KR, KA, NR, NA, L, H4, H5>>(c);                                 \
    }                                                                                                 \
    nep_status shape_f64_##KR##_##KA##_##NR##_##NA##_##L##_##H4##_##H5(const Ctx& c) {                \
        return run_shape<double, Shape<KR, KA, NR, NA, L, H4, H5>>(c);                                \
    }                                                                                                 \
    }
