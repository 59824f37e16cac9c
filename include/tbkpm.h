/*
 * tbkpm.h -- C ABI of the MI355X (gfx950) kernel-polynomial DOS library.
 *
 * The library computes, on one GPU, the density-of-states step of linear-scaling
 * quantum transport (paper Sec. 2.4): a sparse orthogonal tight-binding
 * Hamiltonian (Eq. (1)) assembled from a neighbour list, the Chebyshev
 * recurrence T_{n+1} = 2 Ht T_n - T_{n-1} with Ht = (H - b)/a, the moments
 * mu_n = <r|T_n|r> over random-phase vectors r, and the Jackson-damped DOS of
 * Eq. (4).  The KPM details follow the published kernel polynomial method
 * (Weisse, Wellein, Alvermann & Fehske, Rev. Mod. Phys. 78, 275 (2006)).
 *
 * Conventions shared by every entry point:
 *  - Every call returns a tbk_status; TBK_OK is 0.  On an error nothing is
 *    written to the outputs unless stated, and tbk_last_error() describes it.
 *    No call aborts, exits or throws across the ABI.
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary CPU memory owned by the caller.  The library keeps
 *    no pointer after a call returns.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue work
 *    on it and return without waiting, except where a host output is written:
 *    those synchronise `stream` before returning.
 *  - Builders may allocate temporary device memory (stream-ordered) and free it
 *    before returning; kpm_moments allocates nothing and uses `work`.
 *  - Complex vectors are interleaved (re, im) pairs: c128 = 2 x double,
 *    c64 = 2 x float.  A block of R vectors is stored row-major [rows][R]:
 *    element (row i, vector v) at index i*R + v.
 */
#ifndef TBKPM_H
#define TBKPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TBK_OK = 0,
    TBK_ERR_INVALID_ARG = 1,      /* an argument is outside its documented range   */
    TBK_ERR_BUFFER_TOO_SMALL = 2, /* a caller buffer is smaller than required       */
    TBK_ERR_NOT_FINITE = 3,       /* NaN/Inf in coordinates or parameters           */
    TBK_ERR_SPECTRUM = 4,         /* |mu_n| > mu_0: (a, b) does not bound spec(H)   */
    TBK_ERR_UNSUPPORTED = 5,      /* valid but unsupported (e.g. degree > 256)      */
    TBK_ERR_DEVICE = 6            /* a HIP call failed; text in tbk_last_error()    */
} tbk_status;

/* Text of the last error on the calling thread; valid until its next call. */
const char *tbk_last_error(void);

/* ABI revision of this header (incremented on any incompatible change). */
#define TBK_ABI_VERSION 14
int32_t tbk_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Hamiltonian storage                                                       */
/* ------------------------------------------------------------------------ */

/* Storage formats of the off-diagonal part of H (the onsite diagonal is a
 * separate vector).  SELL = sliced ELLPACK: rows are grouped in slices of
 * `slice` consecutive rows; slice s stores w_s entries per row (w_s = largest
 * degree in the slice) column-major: entry k of row i lives at
 *   ptr[s] + k * slice + (i - s * slice).
 * Padding entries hold col = own row and value 0. */
typedef enum {
    TBK_CSR_F64 = 0,   /* CSR, double values: entries of row i at [ptr[i], ptr[i+1]) */
    TBK_SELL_F64 = 1,  /* SELL, double values                                          */
    TBK_SELL_F32 = 2,  /* SELL, float values (for the complex-float recurrence)         */
    TBK_BSELL4_F64 = 3, /* block SELL over atoms, n_orb = 4 or 9 orbitals per atom, double
                           n_orb x n_orb blocks (tb_build_hamiltonian_sk only): ptr
                           [n_slices+1] over atom slices of `slice` atoms; col [n_entries]
                           neighbour atom row of each block (own row on padding); val
                           [n_orb^2 n_entries], block q row-major at n_orb^2 q (zero on
                           padding); n_rows = n_orb atoms                              */
    TBK_BSELL4_F32 = 4, /* the same with float blocks (complex-float recurrence)        */
    TBK_BGEOM_F64 = 5,  /* block SELL over atoms that stores each bond's displacement
                           instead of its block (tb_build_hamiltonian_sk, one species,
                           no networks): ptr, col as TBK_BSELL4_*; val [3 n_entries],
                           (dx, dy, dz) from the row atom to col[q] (minimum image; zero
                           on padding); the recurrence forms every block from it and the
                           integrals in h->sk_geom (28 B per bond read instead of
                           n_orb^2 values: the matrix-free form for models whose
                           blocks do not fit in memory)                              */
    TBK_BGEOM_F32 = 6   /* the same with float displacements (complex-float
                           recurrence, blocks formed in float); val [4 n_entries]:
                           slot q holds (dx, dy, dz, c) with c the bits of col[q] as
                           a float, one 16-byte record, the only bond data the
                           recurrence reads                                          */
} tbk_format;

/* Distance-scaled hopping model of Eq. (1):
 *   t_ij = t_pair[s_i * n_species + s_j] * exp(-beta (r_ij / r0 - 1)),  r_ij < r_cut
 *   H_ii = onsite[s_i]
 * onsite and t_pair are host arrays ([n_species], [n_species^2], symmetric). */
typedef struct {
    double r_cut;          /* hopping cutoff (A), strict r < r_cut            */
    double r0;             /* reference bond length (A)                       */
    double beta;           /* decay exponent                                  */
    int32_t n_species;     /* S >= 1                                          */
    int32_t reorder;       /* 1: rows in spatial cell order (perm filled);
                              0: rows in the caller's atom order              */
    const double *onsite;  /* host [S] (eV)                                   */
    const double *t_pair;  /* host [S*S] (eV)                                 */
} tbk_tb_params;

/* A Hamiltonian in device memory.  tbk_hamiltonian_size fills the size fields;
 * the caller allocates the device arrays with those sizes and sets the
 * pointers; tb_build_hamiltonian fills the arrays. */
typedef struct {
    int32_t fmt;           /* tbk_format                                        */
    int32_t slice;         /* SELL slice height (rows), a power of two in
                              [1, 1024]; ignored for CSR                        */
    int64_t n_rows;        /* rows = atoms (one orbital per atom)               */
    int64_t n_ptr;         /* entries of ptr: n_rows+1 (CSR), n_slices+1 (SELL) */
    int64_t n_entries;     /* stored entries incl. SELL padding                 */
    int64_t n_bonds;       /* unordered neighbour pairs                         */
    int32_t max_degree;    /* largest row degree                                */
    int32_t has_onsite;    /* 1 if some onsite energy is non-zero               */
    int32_t n_seg;         /* independent systems stacked along the rows (>= 1) */
    int64_t *ptr;          /* device int64 [n_ptr]                              */
    int32_t *col;          /* device int32 [n_entries] (row indices of H)       */
    void *val;             /* device double|float [n_entries]                   */
    void *onsite;          /* device double|float [n_rows] (same type as val)   */
    int32_t *perm;         /* device int32 [n_rows]: row -> caller atom index   */
    int64_t *seg_rows;     /* device int64 [n_seg+1]: rows of system s are
                              [seg_rows[s], seg_rows[s+1]); may be NULL when
                              n_seg == 1                                       */
    int32_t uniform_hop;   /* out (build): 1 when every stored off-diagonal
                              value equals hop_value (e.g. a pristine lattice
                              in SELL_F32); 0 otherwise and for learned H      */
    double hop_value;      /* out (build): that value, as stored (eV)         */
    int16_t *col16;        /* optional device int16 [n_entries] (NULL = none):
                              column minus row of each stored entry, or -32768
                              where that does not fit in 16 bits (col holds
                              every column); filled by tb_build_hamiltonian
                              when non-NULL, read by the recurrence with
                              compact_columns = 1                              */
    int32_t n_orb;         /* out (build): orbitals per atom, 1 for the one-
                              orbital builders, 4 or 9 for tb_build_hamiltonian_sk;
                              perm[row] / n_orb is the caller's atom           */
    double sk_geom[12];    /* out (build, TBK_BGEOM_*): the ten integrals of
                              tbk_sk_params at r0, then r0 and beta            */
} tbk_ham;

/*
 * Size query (neighbour search + degree count on the GPU, Eq. (1)'s N(i)).
 *   pos     device double [n][3] (A); periodic axes may hold any value, they
 *           are wrapped; open axes are binned over the coordinates' range.
 *   species device int32 [n], each in [0, n_species).
 *   box     host double[3]: periodic lengths (ignored on open axes).
 *   periodic host int32[3]: 1 = periodic axis.
 *   h       in: fmt, slice; out: n_rows, n_ptr, n_entries, n_bonds, max_degree,
 *           has_onsite, n_seg = 1.
 * Errors: INVALID_ARG (n < 1, n >= 2^31, periodic length < 2 r_cut, species
 * out of range, bad fmt/slice, r_cut/r0/beta not positive), NOT_FINITE (a
 * coordinate is NaN/Inf), UNSUPPORTED (degree > 256), DEVICE.
 * Synchronises `stream`.
 */
tbk_status tbk_hamiltonian_size(const double *pos, const int32_t *species, int64_t n,
                                const double box[3], const int32_t periodic[3],
                                const tbk_tb_params *p, tbk_ham *h, void *stream);

/*
 * Builds H (Eq. (1)) into the buffers of `h` (sized by tbk_hamiltonian_size
 * for the same inputs): columns of each row ascending, both triangles computed
 * from the same FP64 distance (H is exactly symmetric), onsite[i] = onsite of
 * the row's species, perm[i] = caller atom of row i.  Writes the row
 * Gershgorin bounds [E_lo, E_hi] (eV, FP64) to spec_bounds (host).
 * Errors: as tbk_hamiltonian_size, plus BUFFER_TOO_SMALL when the sizes in `h`
 * are smaller than what these inputs need, INVALID_ARG for a NULL array.
 * Synchronises `stream`.
 */
tbk_status tb_build_hamiltonian(const double *pos, const int32_t *species, int64_t n,
                                const double box[3], const int32_t periodic[3],
                                const tbk_tb_params *p, tbk_ham *h,
                                double spec_bounds[2], void *stream);

/*
 * Several independent structures at once ("segments", e.g. finite-temperature
 * snapshots of different sizes), stacked along the atom index: structure s
 * holds atoms [seg_atoms[s], seg_atoms[s+1]) of pos/species (seg_atoms: host
 * int64 [n_seg+1], seg_atoms[0] = 0, strictly increasing), its periodic box is
 * boxes[3 s .. 3 s + 2] (host), and periodic[3] applies to all.  Neighbours are
 * searched only inside a structure; the rows of structure s are the row range
 * [seg_atoms[s], seg_atoms[s+1]) of the stacked H, whose table tb_build_*
 * copies to h->seg_rows (device int64 [n_seg+1], caller-allocated).
 * spec_bounds: host double [n_seg][2], Gershgorin [E_lo, E_hi] per structure.
 * Errors as the single-structure calls, plus INVALID_ARG for a bad table.
 */
tbk_status tbk_hamiltonian_size_batched(const double *pos, const int32_t *species, int32_t n_seg,
                                        const int64_t *seg_atoms, const double *boxes,
                                        const int32_t periodic[3], const tbk_tb_params *p,
                                        tbk_ham *h, void *stream);
tbk_status tb_build_hamiltonian_batched(const double *pos, const int32_t *species, int32_t n_seg,
                                        const int64_t *seg_atoms, const double *boxes,
                                        const int32_t periodic[3], const tbk_tb_params *p,
                                        tbk_ham *h, double *spec_bounds, void *stream);

/* ------------------------------------------------------------------------ */
/* Chebyshev moments                                                         */
/* ------------------------------------------------------------------------ */

typedef enum {
    TBK_PREC_F64 = 0,  /* c128 vectors, double H (CSR_F64 or SELL_F64)              */
    TBK_PREC_C32 = 1   /* c64 vectors, float H (SELL_F32); moments summed in double  */
} tbk_precision;

/* Launch shape of the recurrence kernel.  Every shape computes bitwise the
 * same vectors T_n; the moments differ only in the order in which per-block
 * double partial sums are added (a few ulp); the shape sets the speed.  A tile is 256/L rows with
 * L = R_pad / vectors_per_thread threads per row (R_pad = R rounded up to a
 * power of two). */
typedef struct {
    int32_t vectors_per_thread; /* 1, or 2 (C32 only, R >= 2): vectors per thread  */
    int32_t tiles_per_block;    /* >= 1: consecutive tiles one workgroup handles    */
    int32_t nontemporal;        /* 1: streamed arrays use non-temporal loads/stores */
    int32_t xcd_remap;          /* block order over the 8 XCDs (workgroup b runs on
                                   XCD b % 8): 0 = dispatch order; 1 = each XCD
                                   sweeps a contiguous eighth of the rows; 2, 3 =
                                   each XCD takes runs of 16 (2) or 64 (3)
                                   consecutive blocks, the XCDs' runs side by side
                                   (one front over the chip, neighbour rows in the
                                   XCD's own L2)                                  */
    int32_t rows_per_thread;    /* 1, 2 or 4: rows (from consecutive tiles) a
                                   thread advances together; 4 takes effect with
                                   one vector per thread row on width-3 slices and
                                   runs as 2 elsewhere.  Block Hamiltonians with one
                                   vector (atom form, displacement form): staging of
                                   each tile's rows through LDS, 1 = when the launch
                                   has >= 2048 tiles, 2 = always, 4 = never        */
    int32_t persistent;         /* kpm_moments_batched only: 1 = all steps in one
                                   cooperative launch (a team of workgroups per
                                   structure, barrier per step); 0 = one launch
                                   per step                                        */
    int32_t doubling;           /* kpm_moments only: 1 = two moments per step from
                                   mu_2k = 2<T_k|T_k> - mu_0 and
                                   mu_2k-1 = 2 Re<T_k|T_k-1> - mu_1 (exact for
                                   Hermitian H; M/2 steps and no read of r)        */
    int32_t uniform_values;     /* kpm_moments only: 1 = do not read the stored
                                   off-diagonal values, use h->hop_value (needs
                                   h->uniform_hop = 1; same results bit for bit,
                                   4 or 8 B less per stored entry)                */
    int32_t compact_columns;    /* kpm_moments only: 1 = read the 16-bit column
                                   offsets h->col16 (needs them) and col only
                                   where an offset does not fit: 2 B less per
                                   stored entry, same results bit for bit         */
    int32_t atom_rows;          /* block Hamiltonians (TBK_BSELL4_*) only: 1 = a
                                   thread owns every orbital row of one atom, so a
                                   neighbour's orbital rows of T_n are gathered
                                   once per atom; 0 = a thread per orbital row.
                                   Ignored for the other formats                 */
} tbk_kpm_config;

/* The launch shape kpm_moments uses for (h, R, precision) when none is given
 * (written to *cfg).  Errors: INVALID_ARG (NULL pointer, R outside [1, 64],
 * precision/format mismatch). */
tbk_status kpm_default_config(const tbk_ham *h, int32_t R, int32_t precision, tbk_kpm_config *cfg);

/* Bytes of device workspace kpm_moments needs for (h, R, M, precision) with the
 * default launch shape (kpm_workspace_size) or a given one (cfg may be NULL). */
tbk_status kpm_workspace_size(const tbk_ham *h, int32_t R, int32_t M, int32_t precision,
                              int64_t *bytes);
tbk_status kpm_workspace_size_config(const tbk_ham *h, int32_t R, int32_t M, int32_t precision,
                                     const tbk_kpm_config *cfg, int64_t *bytes);

/*
 * Scale of the Chebyshev expansion (Sec. 2.4: the expansion needs the spectrum
 * mapped into [-1, 1]) from spectral bounds, for n systems:
 *   a[s] = margin (E_hi - E_lo) / 2,  b[s] = (E_hi + E_lo) / 2,
 * with [E_lo, E_hi] = spec_bounds[2 s], spec_bounds[2 s + 1] (host double,
 * eV; e.g. the Gershgorin bounds the builders return) and margin >= 1 (1.01
 * keeps the scaled spectrum inside [-1, 1] with room for rounding).  a, b:
 * host double [n], caller-allocated.  Host arithmetic only.
 * Errors: INVALID_ARG (n < 1, NULL, margin < 1 or not finite, E_hi <= E_lo),
 * NOT_FINITE (a bound is NaN/Inf); nothing is written on an error.
 */
tbk_status kpm_scale(int32_t n, const double *spec_bounds, double margin, double *a, double *b);

/*
 * Chebyshev moments of Ht = (H - b)/a over R random vectors (Sec. 2.4 and the
 * trace of Eq. (4) by random phases):
 *   T_0 = r, T_1 = Ht r, T_{n+1} = 2 Ht T_n - T_{n-1},
 *   mu[s][v][n] = Re <r_v|T_n>_s  (n = 0..M-1; the overlap is restricted to the
 *   rows of system s).
 * Every step is one pass over H on the GPU with the overlap accumulated in
 * double inside the same kernel; per-block partial sums are reduced in a fixed
 * order, so results are bitwise reproducible for a given launch shape.
 *   a, b   host double [n_seg]: scale a > 0 and shift of each system.
 *   r      device c128|c64 [n_rows][R] in the CALLER's atom order (not read
 *          when n_start > 0; may then be NULL).
 *   n_start 0: a fresh run, moments 0 .. M-1.  n_start >= 2: continue the run
 *          whose state `work` holds (checkpoint/resume of the recurrence):
 *          the last completed call on this `work` was a fresh or continued run
 *          of the same Hamiltonian (same sizes and values), R, precision, a and
 *          b that ended at moment n_start - 1 (its M was n_start); work keeps
 *          T_{n_start-1}, T_{n_start-2}, the start vectors and mu_0, and this
 *          call writes only mu[.][.][n_start .. M-1], bit for bit what one run
 *          with this M would write (any launch shape: the vectors do not
 *          depend on it).  Direct form only (cfg->doubling = 0).
 *   work   device, >= kpm_workspace_size bytes, 256-byte aligned.  Its
 *          leading bytes hold the run's state (a record of the run, the start
 *          vectors, T_{n-1} and T_{n-2}) at offsets that do not depend on M,
 *          so one buffer sized for the largest M serves every call of a run
 *          split over calls.
 *   mu     device double [n_seg][R][M].
 * Errors: INVALID_ARG (R < 1 or R > 64, M < 2, a <= 0, precision/format
 * mismatch; n_start not 0 and not in [2, M), doubling with n_start > 0, or
 * work holding no state that ends at n_start - 1 for these arguments),
 * BUFFER_TOO_SMALL (work_bytes), SPECTRUM (some |mu_n| > mu_0 (1 + 1e-6):
 * (a, b) does not bound the spectrum; mu is still written), DEVICE.
 * Synchronises `stream` (to read the spectrum check and, with n_start > 0,
 * the state record).
 */
tbk_status kpm_moments(const tbk_ham *h, const double *a, const double *b, const void *r,
                       int32_t R, int32_t M, int32_t precision, int32_t n_start, void *work,
                       int64_t work_bytes, double *mu, void *stream);

/* kpm_moments with an explicit launch shape (cfg may be NULL = default); the
 * workspace must be sized by kpm_workspace_size_config for the same cfg.
 * Extra errors: INVALID_ARG for a shape outside the ranges of tbk_kpm_config. */
tbk_status kpm_moments_config(const tbk_ham *h, const double *a, const double *b, const void *r,
                              int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                              int32_t n_start, void *work, int64_t work_bytes, double *mu,
                              void *stream);

/*
 * kpm_moments_config without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a static device array of
 * the library, 64 MiB on each GPU it runs on, held until the process ends; this
 * call makes no allocation (no hipMalloc, hipFree or allocating library
 * routine).  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents: n_start > 0 continues the run the last call on this
 * GPU left there (as kpm_moments_config continues the run its `work` holds),
 * and calls that overlap on one GPU (several host threads or streams) race.
 * Arguments, results (bit for bit those of kpm_moments_config with the same
 * cfg) and errors as kpm_moments_config, plus BUFFER_TOO_SMALL when
 * kpm_workspace_size_config for these arguments exceeds 64 MiB (e.g. up to
 * about 2.7 M rows for one complex-float vector).  The step timer does not
 * time this call.  Synchronises `stream`.
 */
tbk_status kpm_moments_noalloc(const tbk_ham *h, const double *a, const double *b, const void *r,
                               int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                               int32_t n_start, double *mu, void *stream);

/*
 * kpm_moments_config with the random-phase start vectors (Sec. 2.4) generated
 * on the device instead of read from an [n_rows][R] array:
 *   r[i][v] = exp(i phi), phi = 2 pi (x >> 11) 2^-53, x = output number
 *   i R + v of SplitMix64 started at state `seed` (Steele, Lea & Flood 2014),
 * with i the caller's atom index (so the phases do not depend on the row order
 * the builder chose).  Same workspace, n_start and errors as
 * kpm_moments_config (a continued run reads the phases kept in `work`, so
 * `seed` is then unused).
 */
tbk_status kpm_moments_seeded(const tbk_ham *h, const double *a, const double *b, uint64_t seed,
                              int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                              int32_t n_start, void *work, int64_t work_bytes, double *mu,
                              void *stream);

/* The phases kpm_moments_seeded uses, written out: r device c128 (precision
 * 0) or c64 (precision 1) [n][R], caller-allocated.  Asynchronous on `stream`.
 * Errors: INVALID_ARG (n < 0, R outside [1, 64], bad precision, r NULL). */
tbk_status tbk_random_phase(uint64_t seed, int64_t n, int32_t R, int32_t precision, void *r,
                            void *stream);

/*
 * Moments of every structure of a stacked Hamiltonian (tb_build_hamiltonian_
 * batched) in one recurrence launch per step: structure s is scaled by its own
 * a[s] > 0, b[s] (host double [n_seg]) and mu is device double
 * [n_seg][R][M], mu[s][v][n] = Re <r_v|T_n>_s over the rows of s.  r is
 * [n_rows][R] in the caller's stacked atom order.  The workspace size depends
 * on the structures' sizes and is queried with kpm_workspace_size_batched
 * (which reads h->seg_rows and synchronises `stream`).  Launch shapes as in
 * kpm_moments_config (xcd_remap and rows_per_thread are not used here); with
 * cfg->persistent = 1 all M - 1 steps run in one cooperative launch (DEVICE if a
 * team barrier times out; UNSUPPORTED with more structures than co-resident
 * workgroups).
 * Errors as kpm_moments; SPECTRUM if any structure's moments leave [-mu_0, mu_0].
 */
tbk_status kpm_workspace_size_batched(const tbk_ham *h, int32_t R, int32_t M, int32_t precision,
                                      const tbk_kpm_config *cfg, int64_t *bytes, void *stream);
tbk_status kpm_moments_batched(const tbk_ham *h, const double *a, const double *b, const void *r,
                               int32_t R, int32_t M, int32_t precision, const tbk_kpm_config *cfg,
                               void *work, int64_t work_bytes, double *mu, void *stream);

/*
 * Timing of the recurrence step kernels alone (a measurement aid for the
 * bandwidth of Sec. 2.4's sparse products): while enabled on the calling
 * thread, kpm_moments* and kpm_moments_batched (one launch per step) record
 * HIP events on their stream before and after every stretch of consecutive
 * step launches (the moment reductions between stretches are outside them)
 * and add the elapsed times when the call synchronises.
 * kpm_step_timer(1) enables and clears, kpm_step_timer(0) disables;
 * kpm_step_timer_read returns the milliseconds and the number of step
 * launches timed since the last read or enable, then clears them.  The pair
 * form used by lsqt_vac_moments and the persistent launch are not timed.
 * Errors: INVALID_ARG (enable not 0/1, NULL).
 */
tbk_status kpm_step_timer(int32_t enable);
tbk_status kpm_step_timer_read(double *ms, int64_t *launches);

/*
 * Bandwidth probes (measurement aid: the HBM ceilings a bandwidth-bound step
 * such as the recurrence of Sec. 2.4 is rated beside):
 *   mode 1: copy `bytes` from src to dst (device, 16-byte aligned, no overlap);
 *   mode 0: read `bytes` of src; dst (device, >= 4 tbk_bandwidth_probe_words()
 *           bytes) receives one XOR fold per workgroup so that every load is used.
 * bytes: a positive multiple of 16.  Asynchronous on `stream`; the caller times
 * it (e.g. HIP events).  Loads and stores are non-temporal 16-byte accesses,
 * four in flight per thread, 8 workgroups of 256 threads per compute unit.
 * Errors: INVALID_ARG (mode, size, alignment, NULL), DEVICE.
 * tbk_bandwidth_probe_words: the word count of mode 0's output on the current
 * device (-1 on a HIP error).
 */
tbk_status tbk_bandwidth_probe(const void *src, void *dst, int64_t bytes, int32_t mode, void *stream);
int64_t tbk_bandwidth_probe_words(void);

/* ------------------------------------------------------------------------ */
/* Autotuning                                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t slice;              /* chosen SELL slice height                      */
    tbk_kpm_config config;      /* chosen launch shape                           */
    double ms_per_step;         /* measured time of one recurrence step (ms);
                                   -1 when tuning is switched off               */
    int32_t candidates;         /* (slice, shape) pairs timed                    */
    int32_t from_cache;         /* 1 when the answer came from the cache         */
} tbk_tune_result;

/*
 * Picks the SELL slice height and the recurrence launch shape for one
 * structure (same inputs as tb_build_hamiltonian) and vector count R (the
 * sparse matrix-vector products of the Chebyshev expansion are the cost of
 * the LSQT step, Sec. 2.4; only their speed depends on the choice): builds
 * H for each candidate slice, times `steps` recurrence steps of every
 * candidate shape on the GPU (HIP events on `stream`), returns the fastest.
 * Only speed depends on the choice.  Results are cached per device and
 * problem class (size bucket, R, precision, format, degree, onsite) in
 * memory, and in the file named by the environment variable
 * TBKPM_AUTOTUNE_CACHE when set; TBKPM_AUTOTUNE=0 returns the defaults
 * untimed.  Allocates (and frees) temporary device memory.
 * Errors: as tb_build_hamiltonian; INVALID_ARG for R outside [1, 64], steps
 * outside [1, 1000], a CSR format or a precision/format mismatch.
 * Synchronises `stream`.
 */
tbk_status tbk_autotune(const double *pos, const int32_t *species, int64_t n,
                        const double box[3], const int32_t periodic[3],
                        const tbk_tb_params *p, int32_t fmt, int32_t R, int32_t precision,
                        int32_t steps, tbk_tune_result *out, void *stream);

/* tbk_autotune for one form of the recurrence: `form` gives the fields
 * doubling and uniform_values (the other fields are ignored; NULL = the
 * direct form); the returned config carries them.  The cache key includes the
 * form.  Extra error: INVALID_ARG when uniform_values = 1 and the structure's
 * hoppings are not all equal at some candidate slice height. */
tbk_status tbk_autotune_form(const double *pos, const int32_t *species, int64_t n,
                             const double box[3], const int32_t periodic[3],
                             const tbk_tb_params *p, int32_t fmt, int32_t R, int32_t precision,
                             int32_t steps, const tbk_kpm_config *form, tbk_tune_result *out,
                             void *stream);

/* ------------------------------------------------------------------------ */
/* Learned hoppings (radial descriptor + per-bond MLP)                       */
/* ------------------------------------------------------------------------ */

/*
 * Model of the learned hoppings.  Per unordered bond {i, j} (r_ij below the
 * hopping cutoff) the MLP input is x = [f_0..f_7(r_ij) || v_i + v_j] (16
 * values), standardised as (x - shift) / scale, where v_i = sum_j f(r_ij) over
 * the descriptor cutoff (node feature of Eq. (2) with identity c_nk) and
 * f_k(r) = [T_k(2 (r/r_cut - 1)^2 - 1) + 1] / 2 * f_c(r),
 * f_c(r) = [1 + cos(pi r / r_cut)] / 2 (Eq. (2) radial functions; the cosine
 * form of the smooth cutoff is this library's choice).  The MLP is
 * 16 -> 32 -> tanh -> 32 -> tanh -> 1 with parameters (FP32, 1633, device)
 *   W1 [32][16], b1 [32], W2 [32][32], b2 [32], W3 [32], b3 [1]
 * and every product uses bfloat16 operands (round to nearest even) with FP32
 * accumulation.  The hopping is t_ij = t_plain(r_ij) (1 + y_ij).
 */
typedef struct {
    double r_cut;          /* descriptor cutoff (A)                       */
    int32_t n_radial;      /* radial functions per atom; must be 8        */
    const double *shift;   /* host [16] feature shifts                    */
    const double *scale;   /* host [16] feature scales (non-zero)         */
    const float *params;   /* device [1633] MLP parameters                */
    int32_t n_species;     /* with c_nk: species count                    */
    const double *c_nk;    /* host [n_species][n_species][8][8] descriptor
                              coefficients per species pair (symmetric in
                              the pair), or NULL for the identity: the bond
                              descriptor C_n(r) = sum_k c_nk f_k(r) replaces
                              f in the node and the bond features (Eq. (2));
                              taken by tb_build_hamiltonian_sk_learned only */
} tbk_mlp_model;

#define TBK_MLP_PARAMS 1633

/* Node features v [n][n_radial] (device double) of stacked structures (same
 * structure arguments as tb_build_hamiltonian_batched), cutoff r_cut. */
tbk_status tbk_descriptor(const double *pos, int32_t n_seg, const int64_t *seg_atoms,
                          const double *boxes, const int32_t periodic[3], double r_cut,
                          int32_t n_radial, double *v, void *stream);

/* Unordered bonds i < j (atom indices) within r_cut, ordered by (i, j): the
 * edges {i, j} of Eq. (1)/(2) whose hoppings the learned model predicts (half
 * of the edges: H_ji follows from H_ij by the symmetry stated with Eq. (2)).
 * Same structure arguments as tbk_descriptor (minimum image, strict r < r_cut).
 * bi, bj int32 and br double (device, capacity cap).  *n_bonds receives the
 * count; BUFFER_TOO_SMALL (nothing written) if it exceeds cap.
 * Synchronises `stream`. */
tbk_status tbk_bonds(const double *pos, int32_t n_seg, const int64_t *seg_atoms,
                     const double *boxes, const int32_t periodic[3], double r_cut, int64_t cap,
                     int32_t *bi, int32_t *bj, double *br, int64_t *n_bonds, void *stream);

/* tbk_descriptor with descriptor coefficients per species pair (Eq. (2)):
 * v_i = sum_j C(r_ij), C_n(r) = sum_k c_nk[s_i][s_j][n][k] f_k(r).
 * species device int32 [n] in [0, n_species); c_nk host double
 * [n_species][n_species][n_radial][n_radial], symmetric in the species pair.
 * Errors: as tbk_descriptor; INVALID_ARG (species, asymmetric c_nk),
 * NOT_FINITE.  Synchronises `stream`. */
tbk_status tbk_descriptor_species(const double *pos, const int32_t *species, int32_t n_seg,
                                  const int64_t *seg_atoms, const double *boxes,
                                  const int32_t periodic[3], double r_cut, int32_t n_radial,
                                  int32_t n_species, const double *c_nk, double *v, void *stream);

/* Standardised MLP inputs X [nb][16] as bfloat16 bits (device uint16), one
 * rounding from double: the edge features of Eq. (2) (the bond's radial
 * functions f_k(r_ij)) followed by the sum of the node features v_i + v_j.
 * bi, bj, br from tbk_bonds, v from tbk_descriptor; shift, scale: host [16].
 * Asynchronous on `stream`.  Errors: UNSUPPORTED (n_radial != 8), INVALID_ARG
 * (NULL, a zero or non-finite scale or shift). */
tbk_status tbk_bond_features(int64_t nb, const int32_t *bi, const int32_t *bj, const double *br,
                             const double *v, int32_t n_radial, double r_cut, const double *shift,
                             const double *scale, uint16_t *X, void *stream);

/* tbk_bond_features with the bond descriptor C(r_ij) of the bond's species
 * pair in place of f(r_ij) (same c_nk as tbk_descriptor_species).
 * Synchronises `stream`. */
tbk_status tbk_bond_features_species(int64_t nb, const int32_t *bi, const int32_t *bj,
                                     const double *br, const int32_t *species, const double *v,
                                     int32_t n_radial, double r_cut, int32_t n_species,
                                     const double *c_nk, const double *shift, const double *scale,
                                     uint16_t *X, void *stream);

/* Onsite-network inputs of Eq. (2) (the node feature v_i of each atom):
 * X[i] = bfloat16 bits of [(v_i - shift) / scale || 0 x 8] (16 values, the
 * bond network's input width), one rounding from double.  v device double
 * [n][n_radial] (tbk_descriptor); shift, scale host [8]; X device uint16
 * [n][16].  Errors: UNSUPPORTED (n_radial != 8), INVALID_ARG. */
tbk_status tbk_node_features(int64_t n, const double *v, int32_t n_radial, const double *shift,
                             const double *scale, uint16_t *X, void *stream);

/* Mean and standard deviation (host double [16] each) of the unstandardised
 * bond features over nb bonds (FP64, fixed summation order); used as the
 * fixed feature shift and scale of a model (the input normalisation of the
 * networks of Eq. (2); Sec. 2.1 normalises during training).  Synchronises
 * `stream`.  Errors: UNSUPPORTED (n_radial != 8), INVALID_ARG (nb < 1, NULL). */
tbk_status tbk_feature_moments(int64_t nb, const int32_t *bi, const int32_t *bj, const double *br,
                               const double *v, int32_t n_radial, double r_cut, double *mean,
                               double *stddev, void *stream);

/* Synthetic training target of the learned-hopping workload (the paper
 * trains the networks of Eq. (2) against reference data; here the reference
 * is a coordination-corrected form of the Eq. (1) hopping): the residual
 * y*_b = kappa (z_i + z_j - 2 z0) of t = t_plain (1 + y*), with
 * z_i = v[i][0] (device float [nb] output).  Asynchronous on `stream`. */
tbk_status tbk_coordination_target(int64_t nb, const int32_t *bi, const int32_t *bj,
                                   const double *v, int32_t n_radial, double kappa, double z0,
                                   float *y, void *stream);

/* Forward pass of the hopping network of Eq. (2) (the model of tbk_mlp_model):
 * y [nb] (device float) of inputs X (bf16 bits [nb][16], tbk_bond_features);
 * params device float [1633].  Asynchronous on `stream`.  Errors:
 * INVALID_ARG (nb < 0, NULL). */
tbk_status tbk_mlp_forward(int64_t nb, const uint16_t *X, const float *params, float *y,
                           void *stream);

/* Training of the hopping network of Eq. (2) by gradient descent (Sec. 2.1;
 * the loss here is a weighted squared error of the hopping residual, since the
 * band-structure loss of Eq. (3) needs DFT data):
 * loss L = (1/nb) sum_b w_b (y_b - y*_b)^2 (w = NULL: all ones) and dL/dparams
 * by the analytic backward pass, every product with bfloat16 operands as in
 * the forward pass: grad device float [1633], loss device double [1] (may be
 * NULL).  Uses `work` (device, >= tbk_mlp_workspace_size(nb) bytes).
 * Deterministic (fixed-order FP64 reduction of per-wavefront partials).
 * Errors: INVALID_ARG (nb < 1, NULL), BUFFER_TOO_SMALL (work). */
tbk_status tbk_mlp_workspace_size(int64_t nb, int64_t *bytes);
tbk_status tbk_mlp_loss_grad(int64_t nb, const uint16_t *X, const float *target,
                             const float *weight, const float *params, float *grad,
                             double *loss, void *work, int64_t work_bytes, void *stream);

/* One step of the AdamW optimizer the paper trains with (Sec. 2.1; Loshchilov
 * & Hutter, decoupled weight decay) on n FP32 parameters p (device) with
 * gradient g and FP32 moment estimates m, v (device, updated in place);
 * t = 1-based step count after this update:
 *   m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 *   p -= lr [(m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) + wd p].
 * Asynchronous on `stream`.  Errors: INVALID_ARG (n < 0, t < 1, NULL, lr or
 * wd < 0, beta outside [0, 1), eps <= 0). */
tbk_status tbk_adamw_step(int64_t n, float *p, const float *g, float *m, float *v, int64_t t,
                          double lr, double beta1, double beta2, double eps, double wd,
                          void *stream);

/* Training loop on the GPU (Sec. 2.1: AdamW over epochs of the training set;
 * network of Eq. (2)): `epochs` passes over the nb bonds in minibatches of
 * `batch`, one tbk_mlp_loss_grad and one tbk_adamw_step per minibatch; *step
 * counts the updates.  shuffle_seed = 0 takes the bonds in their stored order;
 * otherwise epoch e takes the nb / 16 chunks of 16 consecutive bonds in the
 * order c -> (mul_e c + add_e) mod (nb / 16), with mul_e coprime to nb / 16 in
 * the middle half of its range and add_e drawn from SplitMix64(shuffle_seed)
 * (deterministic; the last nb % 16 bonds stay last).  Minibatches then mix
 * chunks of every structure instead of one structure's bonds at a time, while
 * each 16-bond tile still reads contiguous features.
 * params, m, v device float [1633],
 * updated in place.  loss_history (host [epochs]) receives each epoch's mean
 * loss.  work >= tbk_mlp_workspace_size(min(batch, nb)) + 7168 bytes.
 * Each minibatch's AdamW update is applied inside its gradient reduction (the
 * arithmetic of tbk_adamw_step).  Synchronises `stream` once per epoch.
 * Errors: as tbk_mlp_loss_grad; INVALID_ARG (epochs < 1, batch < 1, *step < 0,
 * AdamW hyper-parameters as tbk_adamw_step). */
tbk_status tbk_mlp_train(int64_t nb, const uint16_t *X, const float *target, const float *weight,
                         float *params, float *m, float *v, int64_t *step, int32_t epochs,
                         int64_t batch, uint64_t shuffle_seed, double lr, double beta1, double beta2,
                         double eps, double wd, double *loss_history, void *work,
                         int64_t work_bytes, void *stream);

/*
 * Learned assembly (inference fused into assembly): as
 * tb_build_hamiltonian_batched (SELL formats), but each bond's hopping is
 * t_plain(r) (1 + y) with y the MLP output of the bond, evaluated once per
 * unordered bond and written to both H_ij and H_ji.  bond_y (device float,
 * capacity bond_cap, may be NULL) receives y per bond in tbk_bonds order;
 * *n_bonds (may be NULL) the bond count.  spec_bounds as in the batched build,
 * from the learned values.
 */
tbk_status tb_build_hamiltonian_learned(const double *pos, const int32_t *species, int32_t n_seg,
                                        const int64_t *seg_atoms, const double *boxes,
                                        const int32_t periodic[3], const tbk_tb_params *p,
                                        const tbk_mlp_model *model, tbk_ham *h,
                                        double *spec_bounds, float *bond_y, int64_t bond_cap,
                                        int64_t *n_bonds, void *stream);

/* ------------------------------------------------------------------------ */
/* DOS reconstruction                                                        */
/* ------------------------------------------------------------------------ */

/*
 * Jackson-damped DOS of Eq. (4) from moments averaged over vectors:
 *   rho(E) = [g_0 mu_0 + 2 sum_{n=1}^{M-1} g_n mu_n T_n(x)] / (a pi sqrt(1-x^2)),
 *   x = (E - b)/a, rho = 0 for |x| >= 1,
 *   g_n = [(M-n+1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))] / (M+1)
 *   (kernel = 0), or g_n = 1 (kernel = 1, no damping).
 * rho integrates to mu_0 (states per eV of the whole system); the spin and
 * volume factor 2/Omega of Eq. (4) is the caller's.
 *   mu device double [M]; E device double [nE]; rho device double [nE].
 * Errors: INVALID_ARG (M < 1, a <= 0, nE < 0, kernel not 0/1), DEVICE.
 */
tbk_status kpm_dos(const double *mu, int32_t M, double a, double b, int32_t kernel,
                   const double *E, int32_t nE, double *rho, void *stream);

/*
 * Average of the moments over the R random vectors (the stochastic trace of
 * Eq. (4), Sec. 2.4: each vector gives an unbiased estimate, their mean the
 * estimate kpm_dos reconstructs from):
 *   mean[s][n] = (1/R) sum_{v=0}^{R-1} mu[s][v][n], summed in v order.
 *   mu device double [n_seg][R][M] (kpm_moments, kpm_moments_batched);
 *   mean device double [n_seg][M], caller-allocated (may not alias mu).
 * Asynchronous on `stream`.  Errors: INVALID_ARG (n_seg, R or M < 1, NULL).
 */
tbk_status kpm_mean_moments(const double *mu, int32_t n_seg, int32_t R, int32_t M, double *mean,
                            void *stream);

/* kpm_dos for n_struct structures in one launch (stacked snapshots):
 *   mu  device double [n_struct][M] (each already averaged over vectors),
 *   a, b host double [n_struct] (scale > 0 and shift of each structure),
 *   E   device double [n_struct][nE] (each structure's own grid),
 *   rho device double [n_struct][nE].
 * Errors: as kpm_dos, INVALID_ARG for n_struct outside [1, 65535].  Copies a
 * and b to the device and synchronises `stream` before returning. */
tbk_status kpm_dos_batched(const double *mu, int32_t M, int32_t n_struct, const double *a,
                           const double *b, int32_t kernel, const double *E, int32_t nE,
                           double *rho, void *stream);

/* ------------------------------------------------------------------------ */
/* Multi-orbital Slater-Koster Hamiltonian (s, p or s, p, d per atom)        */
/* ------------------------------------------------------------------------ */

/* Two-centre parameters of one species (Sec. 3: Slater-Koster blocks formed
 * from bond directions; Slater & Koster, Phys. Rev. 94, 1498 (1954), Table I,
 * s, p and d rows).  Every integral is scaled by f(r) = exp(-beta (r/r0 - 1))
 * for r < r_cut. */
typedef struct {
    double r_cut, r0, beta;     /* cutoff and reference length (Angstrom), decay */
    double e_s, e_p;            /* onsite energies (eV)                            */
    double v_ss_sigma, v_sp_sigma, v_pp_sigma, v_pp_pi;   /* at r0 (eV)          */
    int32_t reorder;            /* 1 = atom rows in cell-list order (as
                                   tbk_tb_params.reorder)                          */
    int32_t orbitals;           /* 4 = s, px, py, pz; 9 = those and dxy, dyz, dzx,
                                   dx2-y2, d3z2-r2                                 */
    double e_d;                 /* d onsite energy (eV), orbitals = 9             */
    double v_sd_sigma, v_pd_sigma, v_pd_pi;                /* at r0 (eV),          */
    double v_dd_sigma, v_dd_pi, v_dd_delta;                /* orbitals = 9         */
    /* Several species (pair_v != NULL; the single-species integrals and onsite
     * energies above are then unused):
     *   n_species  in [1, 16]; species[i] (device, the builder's argument) in
     *              [0, n_species);
     *   pair_v     host double [n_species][n_species][10]: the ten integrals
     *              (order as above) of the ordered species pair (A, B); a mixed
     *              integral (sp, sd, pd) has the lower angular momentum on A, and
     *              the equal-l integrals (ss, pp, dd) must not depend on the order;
     *   species_e  host double [n_species][3]: e_s, e_p, e_d of each species.
     * A bond i -> j takes the blocks with l_a <= l_b from (s_i, s_j) and the
     * others from (s_j, s_i), by <b_i|H|a_j> = (-1)^(l_a + l_b) of the reversed
     * bond's entry. */
    int32_t n_species;
    const double *pair_v;
    const double *species_e;
} tbk_sk_params;

/*
 * Orbital Hamiltonian with N = sk->orbitals orbitals on every atom: row N r + a
 * (a = s, x, y, z, then the five d for N = 9) for atom row r; for a bond with
 * direction cosines c (from i to j, minimum image) and f = f(r):
 *   <s|s> = f V_ss_sigma, <s_i|p_j,b> = f c_b V_sp_sigma, <p_i,a|s_j> = -f c_a V_sp_sigma,
 *   <p_i,a|p_j,b> = f [c_a c_b V_pp_sigma + (delta_ab - c_a c_b) V_pp_pi],
 * and with N = 9 the s-d, p-d and d-d entries of the same table (blocks with
 * the lower angular momentum on the row side as tabulated, the others by
 * <b_i|a_j> = (-1)^(l_a + l_b) <a_i|b_j>); onsite diag(e_s, e_p x3, e_d x5).
 * Stored as a SELL/CSR matrix of N n rows (entry N q + b of an orbital row:
 * q-th neighbour in cell-list order, its orbital b; columns not sorted), so
 * kpm_moments, kpm_dos and the VAC calls take it as is, or in the block
 * format (h->fmt = TBK_BSELL4_*).  perm[N r + a] = N atom + a (the caller's
 * orbital order); n_orb = N; spec_bounds: host double[2], row Gershgorin bounds.
 *   species device int32 [n] (all 0: one species); other arguments as for
 *   tbk_hamiltonian_size / tb_build_hamiltonian.
 * Errors: as tb_build_hamiltonian; NOT_FINITE for a non-finite parameter;
 * INVALID_ARG for orbitals other than 4 and 9.  Both calls synchronise `stream`.
 */
tbk_status tbk_hamiltonian_size_sk(const double *pos, const int32_t *species, int64_t n,
                                   const double box[3], const int32_t periodic[3],
                                   const tbk_sk_params *sk, tbk_ham *h, void *stream);
tbk_status tb_build_hamiltonian_sk(const double *pos, const int32_t *species, int64_t n,
                                   const double box[3], const int32_t periodic[3],
                                   const tbk_sk_params *sk, tbk_ham *h, double spec_bounds[2],
                                   void *stream);

/* Onsite network of Eq. (2): the onsite energy of shell l (s, p, d) on an atom
 * of species a is e_{a,l} + y_{a,l}, y_{a,l} the output of network (a, l) on
 * the atom's node features (tbk_node_features of its descriptor v_i at cutoff
 * r_cut; the shape and bfloat16 products of tbk_mlp_model).
 *   params device float [n_species][n_shells][TBK_MLP_PARAMS], n_shells = 2
 *   for orbitals = 4, 3 for 9; n_species as in tbk_sk_params (1 without
 *   pair_v). */
typedef struct {
    double r_cut;          /* descriptor cutoff (A)              */
    const double *shift;   /* host [8] node-feature shifts       */
    const double *scale;   /* host [8] node-feature scales       */
    const float *params;   /* device, see above                  */
    int32_t n_species;     /* with c_nk, as in tbk_mlp_model     */
    const double *c_nk;    /* host, as in tbk_mlp_model, or NULL */
} tbk_onsite_model;

/*
 * Learned Slater-Koster Hamiltonian (Eq. (2): the two-centre integrals of a
 * bond are network outputs of its edge features, the angular factors P_lambda
 * of the table unchanged): as tb_build_hamiltonian_sk, but bond {i, j} uses the
 * integrals v_l (1 + y_l(ij)), l = 0 .. K-1 (K = 4 for orbitals = 4, 10 for 9,
 * in the order of tbk_sk_params), where y_l is the output of network l on the
 * bond's standardised features [f_0..7(r_ij) || v_i + v_j] (the inputs, the
 * network shape and the bfloat16 products of tbk_mlp_model).  One network per
 * integral: model->params is device float [K][TBK_MLP_PARAMS].  With onsite
 * (may be NULL) the onsite energies are those of tbk_onsite_model; model may
 * be NULL when onsite is given (fixed two-centre integrals).  bond_y (device float, capacity
 * bond_cap >= K n_bonds, may be NULL) receives y [K][n_bonds] in tbk_bonds
 * order (bonds i < j of the hopping cutoff sk->r_cut); *n_bonds (may be NULL)
 * the bond count.  spec_bounds from the learned values.
 * Errors: as tb_build_hamiltonian_sk; INVALID_ARG (incomplete model,
 * n_radial != 8), BUFFER_TOO_SMALL (bond_y).  Synchronises `stream`.
 */
tbk_status tb_build_hamiltonian_sk_learned(const double *pos, const int32_t *species, int64_t n,
                                           const double box[3], const int32_t periodic[3],
                                           const tbk_sk_params *sk, const tbk_mlp_model *model,
                                           const tbk_onsite_model *onsite, tbk_ham *h,
                                           double spec_bounds[2], float *bond_y, int64_t bond_cap,
                                           int64_t *n_bonds, void *stream);

/* ------------------------------------------------------------------------ */
/* Velocity autocorrelation conductivity, Eq. (3)                            */
/* ------------------------------------------------------------------------ */

/*
 * Velocity operator along `axis` (0, 1, 2 = x, y, z), V = (i / hbar)[H, X],
 * in the layout of a built Hamiltonian h (single structure):
 *   vx[q] = H_q (x_col - x_row) / hbar  for every stored entry q (0 on padding),
 * the displacement between the two atoms (perm[row] / h->n_orb) taken with the minimum-image
 * convention (the bond of the hopping), hbar = 0.6582119569 eV fs, so that
 * (V psi)_i = i sum_q vx[q] psi_col(q) in Angstrom / fs.
 * For a block Hamiltonian (TBK_BSELL4_*) every value of block q is scaled by
 * the displacement between the row atom and col[q] (the orbitals sit on their
 * atom): vx has the layout of h->val, n_orb^2 values per block.
 *   pos  device double [atoms][3] (the positions h was built from, caller's
 *        atom order); box, periodic: host, as for tb_build_hamiltonian.
 *   vx   device, same type as h->val, as many elements as h->val holds
 *        (h->n_entries, or n_orb^2 h->n_entries for blocks).
 * Asynchronous on `stream`.  Errors: INVALID_ARG (NULL, axis, box, format),
 * UNSUPPORTED (stacked structures).
 */
tbk_status tb_build_velocity(const double *pos, const double box[3], const int32_t periodic[3],
                             int32_t axis, const tbk_ham *h, void *vx, void *stream);

/* Terms of the Chebyshev-Bessel series of exp(-i H dt / hbar) used when
 * lsqt_vac_moments gets n_cheb <= 0: the first k past z = a dt / hbar with
 * |J_k(z)| < 1e-15, plus one.  -1 on a bad argument. */
int32_t lsqt_chebyshev_terms(double a, double dt);

/* Bytes of device workspace lsqt_vac_moments needs for the same (R, M,
 * precision, time_batch, cfg): the workspace of the recurrence of R * B vectors
 * (B = the time batch, below), six [n_rows][R_pad] vectors and, when B > 1, the
 * batch's start and left vectors and moments. */
tbk_status lsqt_workspace_size(const tbk_ham *h, int32_t R, int32_t M, int32_t precision,
                               int32_t time_batch, const tbk_kpm_config *cfg, int64_t *bytes);

/*
 * Correlation moments of Eq. (3) with the random-phase trace of Sec. 2.4:
 *   phi_R(0) = r_v, phi_L(0) = V r_v; for j = 0 .. n_t - 1 (t_j = j dt fs)
 *     nu[j][v][m] = Re <phi_L(t_j)| T_m(Ht) V |phi_R(t_j)>,  m = 0 .. M-1,
 *     then phi_R, phi_L <- exp(-i H dt / hbar) (.) by the Chebyshev-Bessel
 *     series exp(-i b dt/hbar) sum_k (2 - delta_k0) (-i)^k J_k(a dt/hbar) T_k(Ht)
 *     with n_cheb terms (<= 0: lsqt_chebyshev_terms).
 * Summed over a complete basis, nu[j][.][m] is the T_m moment of
 * Tr[delta(E - H) Re(V V(t_j))]; lsqt_sigma turns nu into sigma(E, t).
 *   r    device c128|c64 [n_rows][R] start vectors, caller's atom order;
 *   vx   from tb_build_velocity (scalar or block layout, as h);
 *   time_batch  B: the recurrences of B consecutive time steps run together as
 *        one recurrence of R * B vectors (each step's moments are independent of
 *        the others', so only the order of the FP64 sums' tiling changes; the
 *        matrix is read once per B steps); 0 = max(1, 16 / R), 1 = one step at a
 *        time; R * B <= 64;
 *   cfg  launch shape of that recurrence of R * B vectors (NULL = default;
 *        doubling must be 0);
 *   nu   device double [n_t][R][M].
 * Synchronises `stream`.  Errors: as kpm_moments_config; INVALID_ARG (dt <= 0,
 * n_t outside [1, 10^6], doubling, time_batch < 0, R * B > 64); UNSUPPORTED
 * (several structures, the displacement form, blocks of other than 4 or 9
 * orbitals); SPECTRUM when a moment is not finite.
 */
tbk_status lsqt_vac_moments(const tbk_ham *h, const void *vx, double a, double b, const void *r,
                            int32_t R, int32_t M, int32_t n_t, double dt, int32_t n_cheb,
                            int32_t precision, int32_t time_batch, const tbk_kpm_config *cfg,
                            void *work, int64_t work_bytes, double *nu, void *stream);

/*
 * Running conductivity of Eq. (3) without the prefactor 2 e^2 / Omega:
 *   C_j(E) = [g_0 nu_0 + 2 sum g_m nu_m T_m(x)] / (a pi sqrt(1 - x^2)) of
 *            nu[j] (the kpm_dos reconstruction, same kernels),
 *   sigma[j][e] = trapezoidal integral of C over t_0 .. t_j (sigma[0] = 0).
 *   nu device double [n_t][M] (averaged over vectors); E device [nE];
 *   sigma device double [n_t][nE], in (Angstrom/fs)^2 fs / eV.
 * Errors: as kpm_dos; INVALID_ARG (n_t outside [1, 65535], dt <= 0).
 */
tbk_status lsqt_sigma(const double *nu, int32_t M, int32_t n_t, double dt, double a, double b,
                      int32_t kernel, const double *E, int32_t nE, double *sigma, void *stream);

/* ------------------------------------------------------------------------ */
/* Transport post-processing: integrated DOS, frames, mobility               */
/* ------------------------------------------------------------------------ */

/*
 * Integrated DOS (states below E) of the kernel-damped expansion of kpm_dos,
 * in closed form: with x = (E - b)/a = cos(theta),
 *   N(E) = g_0 mu_0 (1 - theta/pi) - (2/pi) sum_{n=1}^{M-1} g_n mu_n sin(n theta) / n,
 * N = 0 for x <= -1 and g_0 mu_0 for x >= 1 (the integral of each T_n against
 * the Chebyshev weight; no energy grid, so no states are lost at the band
 * edges).  States of the whole system without the spin factor, as kpm_dos;
 * N(E) - N(E_neutral) counts the carriers behind the concentration axis of the
 * mobility curve (Sec. 3).
 *   mu device double [M]; E device double [nE]; N device double [nE].
 * Asynchronous on `stream`.  Errors: as kpm_dos.
 */
tbk_status kpm_integrated_dos(const double *mu, int32_t M, double a, double b, int32_t kernel,
                              const double *E, int32_t nE, double *N, void *stream);

/*
 * Frame average and mobility (Sec. 2.4: LSQT results of several MD frames are
 * averaged; Sec. 3: mobility against carrier concentration):
 *   sigma    device double [n_frames][n_t][nE]: lsqt_sigma of each frame on
 *            one common energy grid,
 *   N        device double [n_frames][nE]: kpm_integrated_dos of each frame on
 *            the same grid,
 *   n_ref    states below the charge-neutrality point (e.g. half the orbitals
 *            of a half-filled band),
 * out (device double [nE] each):
 *   sigma_sc[e] = max over j of the frame mean of sigma[.][j][e] (the plateau
 *                 of the running conductivity: the semiclassical value),
 *   carriers[e] = frame mean of N[.][e] - n_ref,
 *   mobility[e] = 0.1 sigma_sc[e] / |carriers[e]| in cm^2 / (V s), NaN where
 *                 carriers[e] = 0.
 * The factor 0.1: with sigma = (2 e^2 / A) sigma_sc and n = 2 carriers / A
 * (spin 2, area A), mu = sigma / (e n) = e sigma_sc / carriers, and
 * e Angstrom^2 / (eV fs) = 0.1 cm^2 / (V s); area and spin cancel.
 * Asynchronous on `stream`.  Errors: INVALID_ARG (counts, NULL), NOT_FINITE (n_ref).
 */
tbk_status lsqt_mobility(const double *sigma, int32_t n_frames, int32_t n_t, int32_t nE, const double *N,
                         double n_ref, double *sigma_sc, double *carriers, double *mobility, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TBKPM_H */
