/*
 * libnep — neuroevolution-potential (NEP) training hot path on AMD Instinct
 * MI355X (gfx950): batched descriptors, energies, forces and virials over many
 * periodic structures, the weighted energy/force/virial loss, its analytic
 * gradient with respect to every parameter, and the Adam/AMSGrad update.
 *
 * The operations follow the TorchNEP paper (arXiv 2606.19557):
 *   site energies Eq. (1); descriptor scaling Eq. (2); per-species network
 *   Eq. (3); loss Eqs. (4)-(7); gradient g_t = dL/dtheta and Adam/AMSGrad
 *   Eqs. (8)-(13); radial descriptor Eqs. (15)-(16); Chebyshev basis with
 *   cosine cutoff Eqs. (17)-(18); angular moments Eq. (19); three-body
 *   invariant Eq. (20); 4-body and 5-body contractions of the moments
 *   (Methods, "NEP descriptors").
 *
 * Conventions (all entry points):
 *   - Every array argument is a DEVICE pointer owned by the caller unless the
 *     comment says "host". The library keeps no pointer after a call returns
 *     and allocates no device memory: temporaries live in the caller's
 *     workspace `ws` of `ws_bytes` bytes (size from nep_workspace_size).
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL
 *     is the default stream), except nep_build_neighbors, which synchronises
 *     the stream once to learn the pair count.
 *   - Return value: NEP_OK (0) or a negative nep_status. Arguments are
 *     validated on the host before anything is launched; on error nothing is
 *     written and nep_last_error() (thread-local) describes the problem.
 *   - dtype selects the bulk floating-point type of positions, pair vectors,
 *     forces, parameters, gradients, descriptors and scaler: NEP_F32 or
 *     NEP_F64. Energies, virials, loss values and loss seeds are always double.
 *   - Layouts are row-major and densely packed.
 *
 * Parameter vector theta (length from nep_param_count), in this order:
 *   c_R[a][b][n][k]  (T*T*(n_max_r+1)*(basis_r+1))  radial coefficients, Eq. (16),
 *                    a = species of the centre atom, b = species of the neighbour;
 *   c_A[a][b][n][k]  (T*T*(n_max_a+1)*(basis_a+1))  angular coefficients, Eq. (19);
 *   for each species t: W0[t][mu][nu] (H*D), b0[t][mu] (H), w1[t][mu] (H), Eq. (3);
 *   b1               (1) shared output bias, Eq. (3).
 * Descriptor vector q (length D): radial n = 0..n_max_r; then for l = 1..l_max
 * and n = 0..n_max_a the three-body q_nl = sum_m A_nlm^2 (real orthonormal
 * harmonics); then, if l_max_4b = 2, q4_n (n = 0..n_max_a), the (2 2 2)
 * Wigner-3j contraction of the complex l = 2 moments; then, if l_max_5b = 1,
 * q5_n = (sum_m A_n1m^2)^2.
 */
#ifndef NEP_H
#define NEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nep_status;

enum {
    NEP_OK = 0,
    NEP_ERR_INVALID_ARG = -1, /* null pointer, negative size, inconsistent sizes */
    NEP_ERR_UNSUPPORTED = -2, /* model shape without a compiled kernel, rc_a > rc_r, ... */
    NEP_ERR_CAPACITY = -3,    /* neighbour buffer too small; required counts reported */
    NEP_ERR_WORKSPACE = -4,   /* workspace smaller than nep_workspace_size */
    NEP_ERR_HIP = -5          /* a HIP runtime call failed; message in nep_last_error */
};

enum { NEP_F32 = 0, NEP_F64 = 1 };

/* Launch plan: the tile shapes of the pair sweeps and of the gradient
 * reductions. Any zero field takes its default. Results differ between plans
 * only by floating-point summation order. nep_autotune picks one by timing
 * the candidates on the caller's batch. */
typedef struct {
    int32_t team_descriptor;   /* lanes per atom in the descriptor sweep: 4, 8 or 16 (default 8) */
    int32_t team_force;        /* lanes per atom in the force sweep and force gather (default 8) */
    int32_t team_tangent;      /* lanes per atom in the tangent sweep (default 8) */
    int32_t team_coeff_grad;   /* lanes per atom in the angular coefficient-gradient sweep: 4, 8, 16 or 32 (default 8);
                                  a team size whose LDS block (T^2 accumulator blocks) exceeds a CU's 160 KB runs
                                  with 32-lane teams */
    int32_t coeff_grad_blocks; /* grid cap of that sweep = its FP64 partial rows, 1..65536 (default 2048) */
    int32_t outer_chunk;       /* atoms per work item of the network/radial outer products, 8..4096 (default 64) */
    int32_t network;           /* per-species network passes: 1 = matrix-core tiles of 32 atoms (16 in FP64),
                                  2 = one lane per atom in 64-atom wavefronts, weights as wave-uniform
                                  (scalar) operands; 3 = inside the descriptor and tangent sweeps, each
                                  atom's team splitting the hidden units (no network launches), the
                                  descriptor sweep then also running the force pass; default 1 */
    int32_t coeff_grad_rows;   /* angular coefficient-gradient sweep: 0 = teams of team_coeff_grad lanes, one pair
                                  per lane (default); 1, 2 or 3 = moment rows per lane: ceil(N_A / rows) lanes per
                                  atom, each running every pair of its atom for its rows (team_coeff_grad unused) */
} nep_plan;

/* Model hyper-parameters (the model keys of the paper's input file, Table I). */
typedef struct {
    int32_t num_types;  /* T >= 1 species */
    int32_t n_max_r;    /* radial channels n = 0..n_max_r */
    int32_t n_max_a;    /* angular channels n = 0..n_max_a */
    int32_t basis_r;    /* Chebyshev functions k = 0..basis_r (radial) */
    int32_t basis_a;    /* Chebyshev functions k = 0..basis_a (angular) */
    int32_t l_max;      /* three-body harmonics l = 1..l_max */
    int32_t l_max_4b;   /* 0 (off) or 2 (4-body term on) */
    int32_t l_max_5b;   /* 0 (off) or 1 (5-body term on) */
    int32_t hidden;     /* neurons H of the hidden layer */
    int32_t dtype;      /* NEP_F32 or NEP_F64 */
    double rc_r;        /* radial cutoff (Angstrom) */
    double rc_a;        /* angular cutoff, 0 < rc_a <= rc_r */
    const nep_plan* plan; /* host, launch plan or NULL for the defaults; read during each call only.
                             The workspace size depends on it. */
} nep_model;

/* A packed batch of fully periodic structures. Structure s owns atoms
 * atom_offset[s] .. atom_offset[s+1]-1. A structure may be empty (nep_gather_batch
 * makes one for an out-of-range id): its E_s and W_s are 0 and it takes no part
 * in the loss (N_s and N_v of Eqs. 4-7 count only structures with atoms). */
typedef struct {
    int32_t num_structures;     /* Ns >= 0 */
    int64_t num_atoms;          /* Na = atom_offset[Ns] */
    const int64_t* atom_offset; /* [Ns+1], atom_offset[0] = 0, non-decreasing */
    const void* positions;      /* [Na][3] dtype, Cartesian Angstrom, any image */
    const int32_t* types;       /* [Na] species in [0, T) */
    const double* cells;        /* [Ns][3][3] rows = cell vectors a, b, c */
} nep_batch;

/* Neighbour lists (caller-allocated, filled by nep_build_neighbors).
 * Row i holds every (j, image) with |r_ij| < rc_r, r_ij = r_j + n.H - r_i.
 * The row is grouped by neighbour species b = 0..T-1; inside each group the
 * pairs with |r_ij| < rc_a come first. */
typedef struct {
    int64_t capacity;         /* pairs `pairs` can hold */
    int64_t* row_offset;      /* [Na+1] first pair of each row */
    int32_t* seg_count;       /* [Na][T][2]: {pairs, angular pairs} per neighbour species */
    void* pairs;              /* [capacity][4] dtype: r_ij x, y, z and the neighbour index j
                                 stored bit-for-bit in the 4th slot (int32 in float, int64 in double) */
    int32_t* reverse;         /* [capacity] index of the reverse pair (j, i, -n) of each pair, -1 if absent */
    int32_t* atom_struct;     /* [Na] structure index of each atom */
    int32_t* species_order;   /* [Na] atoms sorted by species (stable) */
    int64_t* species_offset;  /* [T+1] start of each species in species_order */
    int64_t num_pairs;        /* host, written by nep_build_neighbors (also on NEP_ERR_CAPACITY);
                                 at most 2^31 - 1 pairs per batch */
    int64_t num_angular_pairs;/* host, written by nep_build_neighbors */
    int32_t* species_runs;    /* [Ns][T][2] or NULL: when set, nep_build_neighbors writes for each
                                 structure s and species t the run {start, end} of s's species-t
                                 atoms inside species_order ({0, 0} when s has none), and
                                 nep_gather_batch on these lists gathers the minibatch's species
                                 order from them instead of sorting it */
} nep_neighbors;

/* Reference data and loss weights, Eqs. (4)-(7). */
typedef struct {
    const double* energy;       /* [Ns] target energies */
    const void* force;          /* [Na][3] dtype target forces */
    const double* virial;       /* [Ns][9] target virials */
    const uint8_t* has_virial;  /* [Ns] 1 = structure has a virial label, or NULL = all labelled */
    double lambda_e, lambda_f, lambda_v;
} nep_targets;

typedef struct {
    double lr, beta1, beta2, eps; /* paper defaults 0.9, 0.999, 1e-8 */
    int32_t amsgrad;              /* 1 = keep the running maximum, 0 = plain Adam */
    int32_t amsgrad_mode;         /* 0 = maximum of the bias-corrected second moment (Eq. 12);
                                     1 = maximum of the raw second moment, then bias correction
                                     (the torch.optim.Adam form) */
} nep_adam_cfg;

/* Number of parameters P and descriptor length D (host outputs). Pure host call. */
nep_status nep_param_count(const nep_model* model, int64_t* num_params, int64_t* num_descriptors);

/* Workspace bytes (host output) for any call on a batch of Ns structures, Na
 * atoms and num_pairs neighbour pairs (use nep_neighbors.num_pairs). Pure host. */
nep_status nep_workspace_size(const nep_model* model, int32_t num_structures, int64_t num_atoms,
                              int64_t num_pairs, size_t* bytes);

/* Builds the neighbour lists of a batch (once per dataset; the paper keeps
 * them on the GPU, Results, "Training efficiency"). Cutoffs from the model.
 * Cell lists: each cell is binned into slabs at least r_c^R wide along every
 * lattice direction (at most one bin per atom); every atom scans the bins
 * within reach, periodic images included, with distances tested in FP64.
 * Positions need not be wrapped into the cell. Rows are deterministic.
 * On NEP_ERR_CAPACITY nbr->num_pairs holds the required pair count; grow
 * nbr->pairs and call again. ws must hold nep_workspace_size(..., 0) bytes
 * (the bins live there during the call). */
nep_status nep_build_neighbors(const nep_model* model, const nep_batch* batch, nep_neighbors* nbr, void* ws,
                               size_t ws_bytes, void* stream);

/* Data loader of a training epoch (mini-batch training, Methods): copies the
 * structures ids[0..num_ids) of a packed dataset `src`, with their neighbour
 * lists (built once for the dataset) and targets, into a packed minibatch, in
 * the order given. Atoms, neighbour indices j and reverse-pair indices are
 * renumbered; the minibatch's species order is gathered from src_nbr->species_runs
 * when the dataset's lists carry them, else sorted again; energies, virials
 * and has_virial (1 when the dataset has no mask) follow their structures.
 * ids is a device array; an id outside [0, src Ns) selects an empty structure.
 * The caller allocates the minibatch arrays: atom_offset [num_ids+1], cells
 * [num_ids][3][3], positions/force [num_atoms][3], types [num_atoms], and nbr
 * (row_offset [num_atoms+1], seg_count, atom_struct, species_order, species_offset,
 * pairs/reverse of nbr->capacity), where num_atoms and the pair count are the
 * sums of the selected structures' counts (kept by the caller on the host);
 * nbr->num_pairs and num_angular_pairs are left to the caller. Sizes that do
 * not match give wrong lists but no access outside the given arrays.
 * src_targets may be NULL (then energy, force, virial are not written); any of
 * energy, force, virial, has_virial may be NULL. ws: 8 (num_ids + 1) bytes, plus
 * 4 T (num_ids + 1) when src_nbr->species_runs is set. nbr->species_runs is not
 * written. */
nep_status nep_gather_batch(const nep_model* model, const nep_batch* src, const nep_neighbors* src_nbr,
                            const nep_targets* src_targets, const int32_t* ids, int32_t num_ids, int64_t num_atoms,
                            int64_t* atom_offset, void* positions, int32_t* types, double* cells, nep_neighbors* nbr,
                            double* energy, void* force, double* virial, uint8_t* has_virial, void* ws,
                            size_t ws_bytes, void* stream);

/* Energies E_s = sum_i E_i (Eq. 1), forces F_k = -dE/dr_k and virials
 * W_s = -sum_{i in s, j} r_ij (x) dE_i/dr_ij (9 components, row-major).
 *   theta   [P] dtype; q_scale [D] dtype (Eq. 2 factors 1/(q_max - q_min));
 *   energy  [Ns] double (required); force [Na][3] dtype or NULL;
 *   virial  [Ns][9] double or NULL; descriptor [Na][D] dtype or NULL (unscaled q). */
nep_status nep_forward(const nep_model* model, const void* theta, const void* q_scale, const nep_batch* batch,
                       const nep_neighbors* nbr, double* energy, void* force, double* virial, void* descriptor,
                       void* ws, size_t ws_bytes, void* stream);

/* ZBL short-range repulsion (the screened-Coulomb correction the paper lists
 * among NEP's supported terms; Methods). The form is the universal potential
 * of Ziegler, Biersack and Littmark:
 *   phi(r) = k_e Z_a Z_b / r * sum_k c_k exp(-d_k r / a_ab),
 *   a_ab = 0.8854 a_0 / (Z_a^0.23 + Z_b^0.23),
 *   (c, d) = (0.18175, 3.19980), (0.50986, 0.94229), (0.28022, 0.40290), (0.02817, 0.20162),
 * k_e = 14.399645 eV A, a_0 = 0.529177210903 A, times the switch f(r) = 1 below
 * r_inner, (1 + cos(pi (r - r_inner) / (r_outer - r_inner))) / 2 up to r_outer,
 * 0 beyond. Atom i takes E_i = 1/2 sum_j phi(r_ij); forces and virials follow
 * the conventions of nep_forward. The term has no trainable parameter. */
typedef struct {
    const int32_t* atomic_number; /* host [T] nuclear charge of each species, 1..118; read during the call */
    double r_inner, r_outer;      /* switch range (Angstrom), 0 <= r_inner < r_outer <= model rc_r */
} nep_zbl;

/* Adds scale * (E, F, W) of the ZBL term to energy [Ns] (double), force
 * [Na][3] (dtype) and virial [Ns][9] (double); any of the three may be NULL.
 * scale = +1 after nep_forward gives NEP + ZBL predictions; scale = -1 on a
 * dataset's targets once makes nep_loss_and_grad train NEP + ZBL (the loss and
 * its gradient are unchanged by moving a parameter-free term to the targets).
 * Pairs come from the radial lists of nep_build_neighbors; a pair at distance
 * 0 contributes nothing. Deterministic (fixed summation order). ws: at least
 * 80 * num_atoms bytes (per-atom partial sums). */
nep_status nep_zbl_add(const nep_model* model, const nep_zbl* zbl, const nep_batch* batch, const nep_neighbors* nbr,
                       double scale, double* energy, void* force, double* virial, void* ws, size_t ws_bytes,
                       void* stream);

/* The weighted loss L = lambda_e Delta_E + lambda_f Delta_F + lambda_v Delta_V
 * (Eqs. 4-7; N_s, N_a, N_a^s over the batch's non-empty structures; Delta_V over
 * the labelled ones)
 * and its gradient dL/dtheta (the g_t of Adam, Eq. 8), computed analytically.
 *   loss [4] double device: {L, Delta_E, Delta_F, Delta_V};
 *   grad [P] dtype, overwritten;
 *   energy [Ns] double, force [Na][3] dtype, virial [Ns][9] double: optional
 *   prediction outputs (NULL = not returned). */
nep_status nep_loss_and_grad(const nep_model* model, const void* theta, const void* q_scale,
                             const nep_batch* batch, const nep_neighbors* nbr, const nep_targets* targets,
                             double* loss, void* grad, double* energy, void* force, double* virial, void* ws,
                             size_t ws_bytes, void* stream);

/* Vector-Jacobian product of (E, F, W) with respect to theta:
 *   grad = sum_s dE[s] dE_s/dtheta + sum_i dF[i] . dF_i/dtheta + sum_s dW[s] : dW_s/dtheta.
 *   dE [Ns] double, dF [Na][3] dtype, dW [Ns][9] double (any may be NULL = zero);
 *   grad [P] dtype, overwritten. */
nep_status nep_backward(const nep_model* model, const void* theta, const void* q_scale, const nep_batch* batch,
                        const nep_neighbors* nbr, const double* dE, const void* dF, const double* dW, void* grad,
                        void* ws, size_t ws_bytes, void* stream);

/* Autotuner of the launch plan (the tiling choice of the packed batch). Times
 * nep_loss_and_grad on this batch under candidate plans, `repeats` timed runs
 * each after one warm-up, with HIP events around every kernel launch:
 *   phase 1: team sizes 4, 8, 16 in all four pair sweeps (and 32 in the
 *            coefficient-gradient sweep); each sweep kernel keeps its fastest;
 *   phase 2: (coeff_grad_blocks, outer_chunk) pairs, chosen by the summed time
 *            of the two kernels and the reductions that read their rows;
 *   phase 3: the three network implementations, by the summed time of the
 *            network kernels and the sweeps that host the fused variant.
 * Candidates whose workspace exceeds ws_bytes or whose LDS exceeds a CU are
 * skipped. Writes the chosen plan to *plan_out (host); model->plan is ignored.
 * The arguments are those of nep_loss_and_grad (loss and grad are overwritten).
 * Synchronises the stream; clears event records of nep_profile_enable. */
nep_status nep_autotune(const nep_model* model, const void* theta, const void* q_scale, const nep_batch* batch,
                        const nep_neighbors* nbr, const nep_targets* targets, double* loss, void* grad, void* ws,
                        size_t ws_bytes, int32_t repeats, nep_plan* plan_out, void* stream);

/* One Adam/AMSGrad step t (1-based) of Eqs. (8)-(13), in place on theta, m, v,
 * vmax (all [P] of dtype; vmax unused when cfg->amsgrad = 0, may be NULL). */
nep_status nep_adam_step(int64_t num_params, int32_t dtype, void* theta, const void* grad, void* m, void* v,
                         void* vmax, int64_t t, const nep_adam_cfg* cfg, void* stream);

/* One training step: nep_loss_and_grad followed by nep_adam_step on the same
 * stream, with the Adam/AMSGrad update (Eqs. 8-13, step t, 1-based) taken in
 * the kernel that finishes the gradient, one launch fewer than the two calls.
 * theta [P] is read by the whole pass and updated in place at its end; m, v,
 * vmax [P] as in nep_adam_step; loss [4] and grad [P] as in nep_loss_and_grad
 * (grad holds the gradient at the old theta). Results are bitwise those of the
 * two calls. Errors as in either call; nothing is launched on an error. */
nep_status nep_train_step(const nep_model* model, void* theta, const void* q_scale, const nep_batch* batch,
                          const nep_neighbors* nbr, const nep_targets* targets, void* m, void* v, void* vmax,
                          int64_t t, const nep_adam_cfg* cfg, double* loss, void* grad, void* ws, size_t ws_bytes,
                          void* stream);

/* nep_train_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the workspace taken from a static device
 * array of 128 MiB inside the library instead of a caller argument. Each GPU
 * the library runs on holds its own copy of that array from the first call on
 * it until the process ends; the call runs on the current device (stream must
 * belong to it) and calls no hipMalloc, hipFree or other allocating routine.
 * All calls on one GPU share the array and it keeps the last call's contents
 * (nothing in it needs to start at zero): calls that overlap on one GPU (two
 * streams, two host threads) race and give undefined results.
 * Returns NEP_ERR_WORKSPACE, before touching the device, when the batch needs
 * more than 128 MiB of workspace (nep_workspace_size); other arguments and
 * errors as in nep_train_step. */
nep_status nep_train_step_noalloc(const nep_model* model, void* theta, const void* q_scale, const nep_batch* batch,
                                  const nep_neighbors* nbr, const nep_targets* targets, void* m, void* v, void* vmax,
                                  int64_t t, const nep_adam_cfg* cfg, double* loss, void* grad, void* stream);

/* Eq. (2) factors from descriptors: q_scale[nu] = 1/(max_i q[i][nu] - min_i q[i][nu]),
 * or 1 where that range is below 1e-10. descriptor [Na][D], q_scale [D], dtype. */
nep_status nep_descriptor_scale(int64_t num_atoms, int64_t num_descriptors, int32_t dtype, const void* descriptor,
                                void* q_scale, void* stream);

/* Thread-local description of the last error (empty string if none). */
const char* nep_last_error(void);

/* Per-kernel timing with HIP events (for measurement only; adds a small cost).
 * nep_profile_enable(1) starts recording every launch of every later call on
 * its stream; nep_profile_read synchronises, then copies up to `cap` entries
 * (host arrays) of kernel name, launch count and total milliseconds, and
 * returns the number of distinct kernels in *count. enable(0) stops and clears. */
nep_status nep_profile_enable(int32_t on);
nep_status nep_profile_read(int32_t cap, char (*names)[64], int64_t* launches, double* total_ms, int32_t* count);
/* Restrict that recording to launches of one kernel (its name as nep_profile_read
 * reports it; host string, copied), so a timed loop carries two events per
 * launch of that kernel only; NULL or "" records every kernel again. */
nep_status nep_profile_only(const char* kernel_name);

#ifdef __cplusplus
}
#endif

#endif /* NEP_H */
