// Internal plan of the Chebyshev recurrence (shared by the moment, batched and
// tuning entry points).
#pragma once

#include <vector>

#include "common.hpp"

namespace tbk {

constexpr int kReduceChunk = 2048;                 // partials per first-level reduction block
constexpr size_t kPartialBudget = 256ull << 20;    // bytes of block partials kept between reductions

struct KpmPlan {
    tbk_kpm_config cfg{};
    int Rp = 1, L = 1, VPT = 1, log2_slice = 0, n_chunks = 1, reduce_every = 1;
    int Rv = 1;                 // block partials per step (2 Rp with the doubling identities)
    int Mr = 1;                 // reduced rows: M, or M / 2 + 1 with the doubling identities
    int64_t n_tiles = 0, G = 0;
    int64_t G_real = 0;         // blocks that own tiles (G rounded up for the XCD block order)
    bool tile_is_slice = false;
    int uniform_width = 0;      // > 0 when every slice stores this many entries per row
    size_t elem = 0, vec_bytes = 0;
    size_t off_state = 0, off_r = 0, off_a = 0, off_b = 0, off_part = 0, off_l1 = 0, off_raw = 0, off_flag = 0,
           total = 0;
    bool block = false;         // block Hamiltonian (kpm_block.hip)
    int norb = 1;               // orbitals per atom of a block Hamiltonian (4 or 9)
    bool geom = false;          // blocks formed in the step from bond displacements
    double geom_params[12] = {};   // integrals at r0, r0, beta (h->sk_geom)
    bool seeded = false;        // start vectors generated on the device from `seed`
    uint64_t seed = 0;
    int32_t n_start = 0;        // 0: fresh run; >= 2: continue from the state kept in the workspace
};

// Leading bytes of the recurrence workspace: the record of the last completed
// run, which a later call with n_start > 0 continues.  The vectors r, T_a, T_b
// follow at offsets that depend only on (rows, R, precision), not on M.
struct KpmState {
    uint64_t magic;             // kStateMagic once a run has completed
    int64_t n_rows, n_entries;
    int32_t R, precision, fmt, next_n;   // next_n = M of that run: the next moment to compute
    double a, b;
};
constexpr uint64_t kStateMagic = 0x54424b504d535431ull;
constexpr size_t kStateMu0 = 512;      // byte offset of mu_0 per vector (<= 64 doubles)
constexpr size_t kStateBytes = 1024;

// Timing of the recurrence step launches (kpm_step_timer): while on, a run
// records a HIP event before and after each stretch of consecutive step
// launches (between two moment reductions) on its stream, and adds the elapsed
// times once the stream has been synchronised.  One per host thread.
struct StepTimer {
    bool on = false;
    double ms = 0.0;              // accumulated step time
    int64_t launches = 0;         // step launches timed
    std::vector<hipEvent_t> ev;   // event pool; pairs (start, end)
    size_t used = 0;              // events recorded by the current run
    hipError_t mark(hipStream_t s);
    hipError_t collect();         // after the stream is synchronised
};
StepTimer &step_timer();

// Per-launch scalars of a step (pointers go as separate restrict parameters).
template <class VT> struct StepScalars {
    int64_t n_rows;
    int64_t n_tiles;
    int32_t log2_slice;
    int32_t Rp;              // padded vector count = L * VPT
    int32_t tiles_per_block;
    int32_t xcd_remap;
    VT c1;                   // 2/a (1/a on the first step)
    VT shift;                // b
    VT hop;                  // the one off-diagonal value when `uniform`
    int32_t uniform;         // 1: values are not read, every real entry is `hop`
    int32_t compact;         // 1: columns from the 16-bit offsets (col where they escape)
};

// Pointers of one step launch.
template <class VT> struct StepPtrs {
    const int64_t *ptr;
    const int32_t *col;
    const int16_t *col16;
    const VT *val;
    const VT *onsite;
    const VT *tcur;
    const VT *tprev;
    VT *tnext;
    const VT *r;
    double *partial;
};

// One recurrence step on a block Hamiltonian (pl.norb = 4 or 9 orbitals per
// atom, norb x norb blocks; kpm_block.hip): the same contract as the one-orbital step kernel,
// rows = orbital rows, sa.n_rows = orbital rows, slices over atoms.
template <class VT>
tbk_status launch_step_block(const KpmPlan &pl, bool first, bool diag, hipStream_t s, const StepPtrs<VT> &p,
                             const StepScalars<VT> &a);

int pad_vectors(int R);
tbk_kpm_config default_config(const tbk_ham *h, int32_t R, int32_t precision);
tbk_status make_plan(const tbk_ham *h, int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                     KpmPlan &pl);
tbk_status check_moment_args(const tbk_ham *h, const KpmPlan &pl, const double *a, const double *b,
                             const void *r, void *work, int64_t work_bytes, double *mu);
// r: start vectors in the caller's order (or NULL with pl.seeded).  With start
// and left (row order, [rows][Rp], device) the pair form runs instead:
// T_0 = start, mu_n = Re <left|T_n(Ht) start>, no spectrum guard.
tbk_status run_plan(const tbk_ham *h, const KpmPlan &pl, double a, double b, const void *r, int32_t R,
                    int32_t M, int32_t precision, char *w, double *mu, hipStream_t s,
                    const void *start = nullptr, const void *left = nullptr);

// One run of the recurrence for vector type VT (double: c128, float: c64), L
// threads per row and VPT vectors per thread; instantiated in kpm_inst_*.hip.
template <class VT, int L, int VPT>
tbk_status run_moments_inst(const tbk_ham *h, const KpmPlan &pl, double a, double b, const VT *r, int32_t R,
                            int32_t M, char *work, double *mu, hipStream_t s, const VT *start, const VT *left);

}  // namespace tbk
