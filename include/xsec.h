/*
 * xsec.h -- C ABI of the MI355X line-by-line cross-section library (libxsec.so).
 *
 * The library computes molecular absorption cross sections sigma(nu) from a line
 * list, following the ExoCross paper (Yurchenko, Al-Refaie & Tennyson,
 * arXiv:1801.09803):
 *   - line intensity I (cm/molecule), Sec. "Intensities and partition function", Eq. 1,
 *     with the partition function Q(T) summed over the states, Eq. 2;
 *   - Doppler / Gaussian / Lorentzian / Voigt line profiles, Sec. "Line profiles",
 *     Eq. 15-19, sampled on the grid (the "sampling method");
 *   - sigma(nu_k) = sum over lines of I f(nu_k - nu_fi), Sec. "Cross sections", Eq. 6-8;
 *   - an equidistant grid of N points including both ends, Eq. 9;
 *   - line wings truncated at a cut-off (25 cm^-1 by default), Sec. "Off-set";
 *   - the Vectorized Voigt approximation and its area-normalised form, Sec.
 *     "Vectorized Voigt approximation" and "Binned Vectorized Voigt with the line area
 *     preserved";
 *   - emission cross sections from the emissivity (Eq. for the emissivity), radiative
 *     lifetimes, the cooling function, and the moments of the partition function with
 *     the specific heat;
 *   - two-temperature (vibrational / rotational) non-LTE populations.
 *
 * Conventions
 *   Units: wavenumbers and energies in cm^-1, T in K, P in the unit of P0 (bar by
 *   default), gamma_ref in cm^-1 per P0, mass in Da, A in s^-1, sigma in
 *   cm^2/molecule (the paper's table of units).
 *   Transitions follow the ExoMol two-file format: upper and lower state indices
 *   into the states arrays (index_base 0, or 1 for ExoMol running numbers).
 *   nu = E[upper] - E[lower] must be > 0.
 *
 * Memory and streams
 *   Arrays documented as "device" are device pointers owned by the caller; the
 *   library never frees them and does not keep them past the call (it copies what
 *   it needs into plan-owned workspace).  "host" arrays are read during the call.
 *   `stream` is a hipStream_t passed as void* (NULL = the default stream).  Every
 *   call enqueues its work on that stream and returns without waiting, except where
 *   a call is documented as synchronous.
 *
 * Errors
 *   Every call returns an xs_status; no exception crosses the ABI.  On failure
 *   xs_last_error() returns a thread-local message describing the first problem.
 *   A failed call leaves the plan usable (its previous line set stays valid unless
 *   the failing call was xs_set_lines, which then leaves no line set).
 *
 * Thread safety: one plan must not be used from two host threads at once.
 */
#ifndef XSEC_H
#define XSEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XS_ABI_VERSION 6

typedef struct xs_plan xs_plan;
typedef struct xs_graph xs_graph;
typedef struct xs_stream xs_stream;

typedef enum {
    XS_OK = 0,
    XS_ERR_ARG = 1,          /* invalid argument (sizes, ranges, null pointers)          */
    XS_ERR_INDEX = 2,        /* a transition's state index is outside the states array  */
    XS_ERR_NU_NONPOS = 3,    /* a transition has E[upper] - E[lower] <= 0               */
    XS_ERR_HIP = 4,          /* the HIP runtime reported an error                        */
    XS_ERR_OOM = 5,          /* device allocation failed                                 */
    XS_ERR_STATE = 6,        /* call out of order (e.g. no states or lines set)          */
    XS_ERR_UNSUPPORTED = 7,  /* option combination not implemented                       */
    XS_ERR_INJECTED = 8      /* a fault injected for testing (environment variable
                                XS_FAULT_INJECT, see xs_stream_chunk) stopped the call
                                before any copy or device work                           */
} xs_status;

typedef enum {
    XS_DOPPLER = 0,      /* Gaussian with the Doppler HWHM of Eq. 16                      */
    XS_GAUSS_FIXED = 1,  /* Gaussian with a constant HWHM alpha_fixed (Eq. 15)            */
    XS_LORENTZ = 2,      /* Lorentzian with HWHM gamma_L of Eq. 18 (Eq. 17)               */
    XS_VOIGT = 3,        /* Voigt: Doppler (x) Lorentz (Eq. 19, normalised convolution)   */
    XS_GH_SAMPLED = 4,   /* Voigt as a Gauss-Hermite sum of shifted Lorentzians (Eq. 30),
                            sampled at the grid points                                   */
    XS_GH_BINNED = 5,    /* bin-averaged Gauss-Hermite Voigt, area-conserving (Eq. 31)   */
    XS_VVOIGT = 6,       /* Vectorized Voigt (Sec. "Vectorized Voigt approximation"): the
                            Voigt profile within vv_radius of the centre; beyond it the
                            Voigt profile of a line at 1 cm^-1 (Doppler width of Eq. 16 at
                            nu = 1, the line's own Lorentz width), at the same offset from
                            the centre, times beta (1, or with vv_beta the ratio of the two
                            profiles at vv_radius, which makes the profile continuous).
                            The radius region is the grid points with
                            ceil((nu - R - nu_a)/dnu) <= k <= floor((nu + R - nu_a)/dnu).
                            Calls return XS_ERR_ARG when sqrt(ln2) R / alpha_ref < 2e4 at a
                            requested T (alpha_ref the reference's Doppler HWHM), where the
                            reference wing would lose its closed form.                   */
    XS_VVOIGT_NORM = 7,  /* XS_VVOIGT with each line's intensity divided by dnu times the
                            sum of its profile values over its whole cut-off window (the
                            window on the grid extended past its ends), so that a line whose
                            window lies on the grid adds exactly I to dnu sum_k sigma_k
                            (Sec. "Binned Vectorized Voigt with the line area preserved"); a
                            line whose profile sums to zero adds nothing                  */
    XS_DOPPLER_BINNED = 8,  /* bin-averaged Doppler Gaussian (Sec. "Binned Gaussian profile
                            with analytical integrals"): sigma_k = I/(2 dnu) [erf(x+) -
                            erf(x-)], x+- = sqrt(ln2)(nu_k +- dnu/2 - nu)/alpha_D, evaluated
                            in double (erfc differences in the tails); same windows as the
                            sampled profiles                                                */
    XS_LORENTZ_BINNED = 9,  /* bin-averaged Lorentzian (Sec. "Binned Lorentzian profile with
                            analytical integrals", Eq. 27-28 with the minus sign between nu_k
                            and nu restored): sigma_k = I/(pi dnu) [atan(y+) - atan(y-)],
                            y+- = (nu_k +- dnu/2 - nu)/gamma_L; gamma_L = 0 gives the step
                            limit (I/dnu in the line's bin)                                  */
    XS_SUPERLINES = 10      /* super-line histogram (Sec. "Super-lines", the Bin option):
                            sigma_k = (sum of I over the lines with floor((nu - nu_a)/dnu +
                            0.5) = k) / dnu, half-open bins; the super-line intensity of
                            grid point k is dnu sigma_k.  No profile, no cut-off            */
} xs_profile;

typedef enum {
    XS_FP64 = 0,         /* profiles and sums in double precision                         */
    XS_FP32 = 1          /* profiles in single precision with double-precision line
                            setup (intensity exponents, Q(T), centre-to-grid offsets) and
                            compensated single-precision accumulation; sigma is float    */
} xs_precision;

typedef enum {
    XS_BROAD_CONST = 0,      /* gamma_const, n_const for every line                        */
    XS_BROAD_PER_LINE = 1,   /* gamma_ref[i], n_exp[i] given per transition                */
    XS_BROAD_A0_JLOWER = 2   /* ExoMol "a0" scheme: table indexed by the lower state's J   */
} xs_broadening;

typedef struct {
    double nu_a, nu_b;     /* grid bounds, both included (Eq. 9), nu_b > nu_a              */
    int64_t n_points;      /* grid points N >= 2; dnu = (nu_b - nu_a)/(N - 1)              */
    double cutoff;         /* wing cut-off (cm^-1) > 0; window |nu_k - nu| <= cutoff       */
    double mass_da;        /* molecular mass (Da) > 0, for Eq. 16                          */
    double T0, P0;         /* reference temperature / pressure of gamma_ref (Eq. 18)      */
    int32_t profile;       /* xs_profile                                                   */
    int32_t precision;     /* xs_precision                                                 */
    int32_t broadening;    /* xs_broadening                                                */
    int32_t index_base;    /* 0, or 1 for ExoMol running numbers                           */
    double alpha_fixed;    /* HWHM for XS_GAUSS_FIXED                                      */
    double gamma_const;    /* gamma_ref for XS_BROAD_CONST                                 */
    double n_const;        /* temperature exponent for XS_BROAD_CONST                      */
    int32_t slices_per_wave; /* tile shape: 64-point slices per wavefront (1, 2, 4, or 8
                                for XS_FP32 with 1 or 2 wavefronts per workgroup);
                                0 = library default (2)                                  */
    int32_t waves_per_block; /* tile shape: wavefronts per workgroup for XS_FP32 (1, 2, 4
                                or 8); 0 = library default (2); XS_FP64 always uses 4    */
    int32_t a_is_log;        /* 1: the A array given to xs_set_lines holds ln A (s^-1)    */
    int32_t n_split;         /* workgroups sharing one tile: workgroup q sums the LDS batches
                                q, q + n_split, ... of the tile's sorted lines (every share
                                gets the same mix of centre and wing lines) and a fixed-order
                                compensated pass adds the shares: 1..64, or 0 = chosen from
                                the plan's grid and line counts                          */
    int32_t tp_block;        /* (T, P) points per forward launch (workgroups of one tile for
                                consecutive (T, P) run back to back): 1..256, or 0 = chosen
                                per call (8, fewer when the FP32 Voigt core rows of
                                16 B per line and (T, P) would exceed 16 GiB)            */
    int32_t vv_beta;         /* XS_VVOIGT(_NORM): 1 = continuity factor beta, 0 = beta = 1
                                (the paper's usual choice)                               */
    double vv_radius;        /* XS_VVOIGT(_NORM): radius R (cm^-1) of the Voigt region, > 0;
                                0 = 4 cm^-1 (the paper's value)                          */
    int32_t gh_nodes;        /* XS_GH_SAMPLED / XS_GH_BINNED: nodes of the Gauss-Hermite rule
                                of Eq. 30-31, 1..64; 0 = 30 (the paper's usual N_GH)     */
} xs_opts;

/* Fill *opts with defaults: cutoff 25, T0 296 K, P0 1 bar, Voigt, FP32, per-line
 * broadening, index_base 0.  Grid and mass must still be set.  */
xs_status xs_opts_default(xs_opts* opts);

/* Create a plan for a grid and profile.  *out receives the plan (owned by the
 * caller until xs_plan_destroy).  Validates the options (XS_ERR_ARG). */
xs_status xs_plan_create(const xs_opts* opts, xs_plan** out);

/* Free the plan and all of its device workspace.  NULL is accepted. */
xs_status xs_plan_destroy(xs_plan* plan);

/* States (Eq. 2; the .states file's energy, total degeneracy and J columns).
 * E: device double[n_states] (cm^-1); g: device int32[n_states] (g_tot > 0);
 * J: device int32[n_states] or NULL (needed only for XS_BROAD_A0_JLOWER).
 * The arrays are copied into the plan on `stream`.  Replaces any previous states
 * and invalidates the line set. */
xs_status xs_set_states(xs_plan* plan, int64_t n_states, const double* E, const int32_t* g,
                        const int32_t* J, void* stream);

/* a0 broadening table (Sec. "Broadening parameters"): host float arrays indexed by
 * the lower state's J = 0..n_j-1; lower states with J >= n_j use the last row. */
xs_status xs_set_broadening_table(xs_plan* plan, int32_t n_j, const float* gamma_ref,
                                  const float* n_exp);

/* Transitions (the .trans file: upper index, lower index, Einstein A).
 * upper, lower: device int32[n_lines]; A: device float[n_lines] (s^-1);
 * gamma_ref, n_exp: device float[n_lines] for XS_BROAD_PER_LINE, else NULL.
 * Computes per-line wavenumbers nu = E[upper] - E[lower] and line constants,
 * drops lines whose cut-off window misses the grid, and sorts the rest by centre
 * into the plan's workspace (original indices are kept for gradients).
 * SYNCHRONOUS: waits for `stream` to check indices and wavenumbers; returns
 * XS_ERR_INDEX or XS_ERR_NU_NONPOS for invalid transitions (no line set then). */
xs_status xs_set_lines(xs_plan* plan, int64_t n_lines, const int32_t* upper, const int32_t* lower,
                       const float* A, const float* gamma_ref, const float* n_exp, void* stream);

/* Number of lines kept by the last xs_set_lines (window overlaps the grid). */
xs_status xs_lines_kept(const xs_plan* plan, int64_t* n_kept);

/* Intensity thresholds (Sec. "Intensity thresholds"). */
typedef enum {
    XS_THRESHOLD_NONE = 0,     /* every line                                                  */
    XS_THRESHOLD_CONSTANT = 1, /* keep lines with I >= i_crit (cm/molecule)                    */
    XS_THRESHOLD_HITRAN = 2    /* HITRAN's dynamic cut-off: keep lines with I >= i_crit (nu/
                                  nu_crit) tanh(c2 nu/(2T)) for nu <= nu_crit, I >= i_crit above;
                                  the paper's defaults are nu_crit = 2000 cm^-1, i_crit = 1e-29 */
} xs_threshold;

/* Set the plan's intensity threshold for the following cross sections (and graphs
 * created afterwards; existing graphs refuse to launch).  I is Eq. 1 at each call's T
 * (in double); dropped lines contribute nothing, and the tile kernels sweep only the kept
 * lines of each (T, P) (a per-(T, P) compaction in sorted order).  mode: xs_threshold;
 * i_crit >= 0; nu_crit > 0 for XS_THRESHOLD_HITRAN.  Host-only, no device work.
 * xs_cross_section_adjoint returns XS_ERR_UNSUPPORTED while a threshold is set. */
xs_status xs_set_intensity_threshold(xs_plan* plan, int32_t mode, double i_crit, double nu_crit);

/* Intensity kind of the cross sections (Sec. "Intensities and partition function"). */
typedef enum {
    XS_ABSORPTION = 0,   /* Eq. 1: I = g_up A/(8 pi c nu^2) exp(-c2 E_low/T)(1 - exp(-c2 nu/T))/Q;
                            sigma in cm^2/molecule                                          */
    XS_EMISSION = 1      /* the emissivity of the transition's upper state,
                            eps = h c g_up A nu exp(-c2 E_up/T)/(4 pi Q) (erg/s/sr/molecule;
                            the printed formula's unit needs the factor h c); sigma in
                            erg/s/sr/molecule per cm^-1                                     */
} xs_intensity_kind;

/* Set the intensity kind of the following cross sections (default XS_ABSORPTION), with
 * the same profiles, grid and cut-off.  Graphs captured before a change refuse to launch
 * (XS_ERR_STATE); an open line-list stream fails its next chunk, and a checkpoint resumes
 * only under the kind it was written with.  An intensity threshold compares the quantity
 * summed (the emissivity for XS_EMISSION).  xs_cross_section_adjoint returns
 * XS_ERR_UNSUPPORTED for XS_EMISSION.  Host-only, no device work. */
xs_status xs_set_intensity_kind(xs_plan* plan, int32_t kind);

/* Partition function Q(T) of Eq. 2 and its derivative dQ/dT, summed on the device
 * in double precision, for n_T temperatures.  T: host double[n_T] (> 0);
 * Q, dQdT: device double[n_T] or NULL. */
xs_status xs_partition_function(xs_plan* plan, int32_t n_T, const double* T, double* Q,
                                double* dQdT, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): xs_partition_function without any
 * allocation.  The temperatures travel to the device as a kernel argument and the partial
 * sums live in a fixed scratch array of the library (XS_NOALLOC_MAX_T temperatures plus
 * 2 x 256 partial sums per temperature, ~1 MiB of doubles per GPU, held until the process
 * ends).  Results are bitwise those of xs_partition_function.  T: host double[n_T] (> 0),
 * 1 <= n_T <= XS_NOALLOC_MAX_T (XS_ERR_ARG otherwise, before any device work); Q, dQdT:
 * device double[n_T] or NULL.  The plan's states must be on the current device.  Every
 * call on one GPU uses that GPU's one scratch array: calls that overlap in time on one
 * GPU (other streams, other host threads) race and must be ordered by the caller. */
#define XS_NOALLOC_MAX_T 256
xs_status xs_partition_function_noalloc(xs_plan* plan, int32_t n_T, const double* T, double* Q,
                                        double* dQdT, void* stream);

/* Non-LTE populations (Sec. "Treating non-local thermodynamic equilibrium"): each state's
 * energy splits as E = E_vib + E_rot, with E_vib the energy of the lowest state of its
 * vibrational (vibronic) manifold (the lowest-J state, which on a rotational ladder is the
 * manifold's lowest energy), and its population per degeneracy is
 *   F = exp(-c2 E_vib/T_vib) exp(-c2 E_rot/T_rot).
 * labels: device int32[n_states], the manifold of each state in [0, n_labels); E_vib is the
 * lowest energy among the states of a manifold (state energies must be >= 0).  NULL
 * returns to LTE.  Invalidates the line set: xs_set_lines must follow (it then carries the
 * vibrational energies of each line's states).  SYNCHRONOUS (checks the labels):
 * XS_ERR_INDEX for a label out of range, XS_ERR_ARG for a negative energy. */
xs_status xs_set_vibrational_labels(xs_plan* plan, int32_t n_labels, const int32_t* labels, void* stream);

/* Cross sections with non-LTE populations for n_tp (T_rot, T_vib, P) points: as
 * xs_cross_section (T_rot in the Doppler width, the broadening and the rotational
 * populations), with the absorption intensity
 *   I = g_up A/(8 pi c nu^2) (F_low - F_up) / Q(T_vib, T_rot),   Q = sum g F,
 * (Eq. 1's population difference; negative for an inverted transition) or, for
 * XS_EMISSION, the emissivity h c g_up A nu F_up/(4 pi Q).  T_rot, T_vib, P: host
 * double[n_tp].  Needs a line set made after xs_set_vibrational_labels (XS_ERR_STATE).
 * xs_cross_section on such a line set takes T_vib = T_rot (the LTE values); graphs and
 * streams do the same.  xs_cross_section_adjoint returns XS_ERR_UNSUPPORTED. */
xs_status xs_cross_section_nlte(xs_plan* plan, int32_t n_tp, const double* T_rot, const double* T_vib,
                                const double* P, void* sigma, void* stream);

/* Non-LTE partition function Q(T_vib, T_rot) = sum g F over the plan's states, in double
 * precision (a fixed-order device sum).  T_rot, T_vib: host double[n_T]; Q: device
 * double[n_T].  Needs xs_set_vibrational_labels (XS_ERR_STATE). */
xs_status xs_partition_function_nlte(xs_plan* plan, int32_t n_T, const double* T_rot, const double* T_vib,
                                     double* Q, void* stream);

/* Moments of the partition function and the specific heat (Sec. "Partition function",
 * the equation for C_p), summed on the device in double precision in a fixed order over
 * the plan's states, for n_T temperatures, with x = c2 E/T:
 *   Q = sum g e^-x,  Q' = T dQ/dT = sum g x e^-x,  Q'' = sum g x^2 e^-x,
 *   C_p = R [Q''/Q - (Q'/Q)^2] + 5R/2  (J/K/mol; the internal states' heat capacity plus
 *   the ideal gas's 5R/2; the printed formula lacks the square, and its T^2 d^2Q/dT^2 is
 *   Q'' - 2Q').
 * T: host double[n_T] (> 0); Q, Q1, Q2, Cp: device double[n_T] or NULL. */
xs_status xs_partition_moments(xs_plan* plan, int32_t n_T, const double* T, double* Q, double* Q1,
                               double* Q2, double* Cp, void* stream);

/* Radiative lifetimes (Sec. "Radiative lifetime"): tau_i = 1 / sum of A over the given
 * transitions whose upper state is i (s), +inf for a state that no transition leaves.
 * upper: device int32[n_lines] (the plan's index_base); A: device float[n_lines] (ln A with
 * a_is_log); tau: device double[n_states of the plan].  The transitions are independent of
 * the plan's line set (every transition counts, whether or not its window meets the grid).
 * The sums are FP64 atomic additions: their order, and so the last bits, may vary between
 * runs.  SYNCHRONOUS (waits for `stream` to check the indices): XS_ERR_INDEX for an upper
 * index out of range. */
xs_status xs_lifetimes(xs_plan* plan, int64_t n_lines, const int32_t* upper, const float* A, double* tau,
                       void* stream);

/* Cooling function (Sec. "Cooling function"): the total power emitted per molecule and
 * steradian, the sum of the emissivities of the given transitions,
 *   W(T) = h c / (4 pi Q(T)) sum g_up A nu exp(-c2 E_up/T)  (erg/s/sr/molecule),
 * for n_T temperatures.  Computed as one pass over the transitions that sums A nu per
 * upper state (FP64 atomic additions, order not fixed) and, per temperature, a fixed-order
 * pass over the states.  upper, lower: device int32[n_lines]; A: device float[n_lines];
 * T: host double[n_T] (> 0); W: device double[n_T].  SYNCHRONOUS (waits to check the
 * transitions): XS_ERR_INDEX, XS_ERR_NU_NONPOS as for xs_set_lines. */
xs_status xs_cooling_function(xs_plan* plan, int64_t n_lines, const int32_t* upper, const int32_t* lower,
                              const float* A, int32_t n_T, const double* T, double* W, void* stream);

/* Cross sections for n_tp (T, P) pairs (Eq. 6-8 with the sampling method).
 * T, P: host double[n_tp] (T > 0, P >= 0; P = 0 gives the pure Doppler limit).
 * sigma: device array [n_tp][n_points], nu fastest; float for XS_FP32, double for
 * XS_FP64.  The result overwrites sigma.  The (T, P) points are processed in blocks
 * of tp_block, each block in one forward launch that makes one pass over the sorted
 * lines per tile.  XS_FP32 with XS_VOIGT sizes the buffer of its double-precision core
 * values from a bound kept with the line set: a call waits on `stream` once (to read the
 * bound back) when the line set is new or its highest temperature exceeds the highest one
 * the bound covers; otherwise, and for every other profile and precision, it does not wait.
 * The result of a (T, P) point does not depend on the other points of the call. */
xs_status xs_cross_section(xs_plan* plan, int32_t n_tp, const double* T, const double* P,
                           void* sigma, void* stream);

/* Graph capture of xs_cross_section (the batching extension: a whole (T, P) grid from
 * one recorded launch sequence, replayed without host work or waits).
 * xs_graph_create records the sequence for n_tp (T, P) points (host arrays, as for
 * xs_cross_section) writing into the device array sigma [n_tp][n_points] (kept by
 * the graph: it must stay allocated while the graph is used).  The graph owns its
 * own workspace (xs_graph_workspace_bytes), sized from a bound that holds for every
 * temperature up to the captured one, so the recording involves waits and allocation
 * but a replay involves neither.  SYNCHRONOUS.  *out receives the graph.
 * xs_graph_launch replays it on `stream`; it returns XS_ERR_STATE once the plan's
 * states, lines or tile configuration have changed since the capture.
 * xs_graph_set_tp replaces the (T, P) values used by later replays (enqueued on
 * `stream`, ordered with replays on the same stream); each new T must be > 0 and
 * <= the T captured at its position (XS_ERR_ARG otherwise), P >= 0.
 * xs_graph_destroy waits for the device and frees the graph (NULL accepted); destroy
 * graphs before their plan. */
xs_status xs_graph_create(xs_plan* plan, int32_t n_tp, const double* T, const double* P,
                          void* sigma, xs_graph** out);
xs_status xs_graph_set_tp(xs_graph* graph, const double* T, const double* P, void* stream);
xs_status xs_graph_launch(xs_graph* graph, void* stream);
xs_status xs_graph_destroy(xs_graph* graph);
size_t xs_graph_workspace_bytes(const xs_graph* graph);

/* Tile configuration of the forward launches: wavefronts per workgroup (4, or 1, 2, 8
 * for XS_FP32), 64-point slices per wavefront (1, 2, 4; 8 for XS_FP32 with 1 or 2
 * wavefronts per workgroup), n_split and tp_block as in
 * xs_opts; 0 selects the default.  SYNCHRONOUS (waits for the device, then rebuilds
 * the tile dispatch order).  Invalidates captured graphs.
 * xs_get_tile_config writes {waves, slices, n_split, tp_block, n_split and tp_block
 * used by the last xs_cross_section}. */
xs_status xs_set_tile_config(xs_plan* plan, int32_t waves, int32_t slices, int32_t n_split,
                             int32_t tp_block);
xs_status xs_get_tile_config(const xs_plan* plan, int32_t out[6]);

/* Autotuner of the tile configuration (the batching extension).  Times the forward
 * launches (and the split combine) over the first min(n_tp, 16) (T, P) points (at
 * most one default block) in a coordinate search: eleven (waves, slices) shapes at
 * their default n_split, then n_split in 1, 2, 4, .. 64 for the best shape, then smaller
 * tp_block values; a candidate is timed twice when one run is under 20 ms.  It stops
 * once budget_ms of wall time is spent (the first candidate always runs) and keeps the
 * fastest per (T, P).  out (host int32[4] or NULL) receives {waves, slices,
 * n_split, tp_block}.  SYNCHRONOUS; uses plan workspace; invalidates captured graphs. */
xs_status xs_autotune(xs_plan* plan, int32_t n_tp, const double* T, const double* P,
                      double budget_ms, void* stream, int32_t out[4]);

/* Line-list streaming (chunked reading of a line list too large for one call, as the
 * paper's program reads its transition files in chunks; here the chunks come from
 * host memory and the sums stay on the device).
 * xs_stream_begin starts accumulating the cross sections of n_tp (T, P) points
 * (host arrays, as for xs_cross_section) over the chunks passed to xs_stream_chunk;
 * sigma (device [n_tp][n_points], float for XS_FP32, double for XS_FP64) receives
 * the result at xs_stream_end.  The stream owns device accumulators (a sum and a
 * compensation per value), a chunk result and two chunk buffers, and an internal copy
 * stream of default priority; its work runs on `stream`.  *out receives the stream.
 * xs_stream_chunk takes the next chunk: n transitions as host arrays (upper, lower,
 * A as for xs_set_lines; gamma_ref and n_exp for XS_BROAD_PER_LINE, else NULL).  Use
 * pinned host memory: the chunk is copied asynchronously on the copy stream while the
 * previous chunk is prepared and computed on `stream`, and the host arrays must stay
 * unchanged until the next xs_stream_chunk (or xs_stream_end) call has returned.
 * Each chunk replaces the plan's line set (as xs_set_lines: synchronous, and invalid
 * transitions return XS_ERR_INDEX / XS_ERR_NU_NONPOS, reported one call later).
 * xs_stream_end computes the last chunk, writes sigma = sum + compensation, waits for
 * it (SYNCHRONOUS) and frees the stream (also after an error); lines_kept (host, or
 * NULL) receives the number of transitions whose window overlapped the grid.
 * xs_stream_checkpoint computes any pending chunk and writes the accumulators, the
 * (T, P) points and the chunk counts to the file `path` (SYNCHRONOUS; written to
 * path.tmp, then renamed).  xs_stream_resume creates a stream from such a file for a
 * plan with the same grid (range and points), cut-off, profile and its options, mass,
 * broadening scheme and constants (and a0 table length), index base, A convention,
 * precision and intensity kind; any difference returns XS_ERR_ARG naming it.  States,
 * the broadening table's values and lines are not in the file: set the states before
 * resuming; chunks then continue the sums.
 * xs_stream_stats writes {chunks passed, transitions passed, transitions kept}.
 * Fault injection (for tests of checkpoint and resume): with the environment variable
 * XS_FAULT_INJECT=chunk:k set when xs_stream_chunk is called, the call that would pass the
 * chunk of index k (0-based, counting every chunk of the accumulation, also those before
 * a resume) returns XS_ERR_INJECTED after validating its arguments and before any copy
 * or device work; the stream keeps its state and stays usable. */
xs_status xs_stream_begin(xs_plan* plan, int32_t n_tp, const double* T, const double* P,
                          void* sigma, void* stream, xs_stream** out);
xs_status xs_stream_chunk(xs_stream* st, int64_t n, const int32_t* upper, const int32_t* lower,
                          const float* A, const float* gamma_ref, const float* n_exp);
/* A chunk already in device memory (a line list kept resident in HBM, such as a list of
 * 4e9 transitions at 12 B each): upper, lower, A (and gamma_ref, n_exp for
 * XS_BROAD_PER_LINE) are device arrays of n transitions.  Nothing is copied: a pending
 * host chunk is computed first, then this chunk is prepared (as xs_set_lines: synchronous,
 * XS_ERR_INDEX / XS_ERR_NU_NONPOS at once) and its cross sections are added into the
 * accumulators on the stream's compute stream.  The arrays are read only during the call.
 * Counts as one chunk (fault injection included). */
xs_status xs_stream_chunk_device(xs_stream* st, int64_t n, const int32_t* upper, const int32_t* lower,
                                 const float* A, const float* gamma_ref, const float* n_exp);
xs_status xs_stream_end(xs_stream* st, int64_t* lines_kept);
xs_status xs_stream_checkpoint(xs_stream* st, const char* path);
xs_status xs_stream_resume(xs_plan* plan, const char* path, void* sigma, void* stream,
                           xs_stream** out);
xs_status xs_stream_stats(const xs_stream* st, int64_t out[3]);

/* Adjoint of xs_cross_section for one (T, P) with the Voigt profile (not in the paper:
 * the derivative of Eq. 1, 2, 16, 18 and of the Voigt profile).  Given dL/dsigma on the
 * grid it returns dL/dT, dL/dP and, per transition in the caller's order of the last
 * xs_set_lines, dL/d(ln A), dL/d(gamma_ref) and dL/dn (lines whose window misses the grid
 * get 0).  Profiles are recomputed; nothing is kept from the forward call.
 * dL_dsigma: device float[n_points] (XS_FP32) or double[n_points] (XS_FP64);
 * dL_dT, dL_dP: device double[1] or NULL; dL_dlogA, dL_dgamma_ref, dL_dn: device
 * double arrays of n_lines values (n_lines of the last xs_set_lines), for both precisions
 * (per-line gradients of a loss on cross sections of ~1e-20 cm^2 lie far below the float
 * range), or NULL (gamma_ref / n outputs need XS_BROAD_PER_LINE).
 * Returns XS_ERR_UNSUPPORTED for other profiles. */
xs_status xs_cross_section_adjoint(xs_plan* plan, double T, double P, const void* dL_dsigma,
                                   double* dL_dT, double* dL_dP, void* dL_dlogA,
                                   void* dL_dgamma_ref, void* dL_dn, void* stream);

/* Kernel timing (tracing).  While enabled, every launch of the forward tile kernel,
 * of the split combine, of the double-precision Voigt core pre-pass and of the line
 * preparation (prep, sort, gather) is bracketed by hipEvents recorded on the call's
 * stream (graph replays are not recorded).
 * xs_set_timing(plan, 1) clears the accumulated times and enables recording;
 * xs_set_timing(plan, 0) stops it.  xs_kernel_times waits for the recorded events
 * (synchronous) and returns the accumulated milliseconds and launch counts. */
typedef struct {
    double forward_ms;          /* tile kernels (one launch per block of (T, P)), and the
                                   adjoint kernel                                          */
    double core_ms;             /* FP32 per-(line, T, P) pre-passes: Voigt core values
                                   (count + evaluation) and line records                   */
    double prep_ms;             /* xs_set_lines device work                                */
    int64_t forward_launches;
    int64_t core_launches;
    int64_t prep_launches;
    double combine_ms;          /* sums of split tiles (n_split > 1)                       */
    int64_t combine_launches;
    int64_t forward_tp;         /* (T, P) results computed by the forward launches         */
    double far_ms;              /* FP32 Voigt: node-sampled far wing and window ends (far,
                                   finish and ends kernels, one set per forward launch of
                                   the segmented sweep)                                     */
    int64_t far_launches;
} xs_timings;

xs_status xs_set_timing(xs_plan* plan, int enable);
xs_status xs_kernel_times(xs_plan* plan, xs_timings* out);

/* Measurement aid, no part of the cross-section method: n_threads threads (a positive
   multiple of 256) each run iters (>= 1) iterations of 16 independent FP32 FMA chains, one
   v_fma_f32 per chain and iteration, and write one float each to out[n_threads] (device
   memory), asynchronously on stream.  A counter run over it calibrates the VALU-issue
   counters (SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, GRBM_GUI_ACTIVE) against a kernel that keeps
   the vector ALUs busy, as a device copy of known size calibrates the HBM byte counters.
   XS_ERR_ARG for a NULL out or out-of-range sizes, XS_ERR_HIP if the launch fails. */
xs_status xs_valu_probe(float* out, int64_t n_threads, int32_t iters, void* stream);

/* Bytes of device memory the plan currently holds. */
size_t xs_workspace_bytes(const xs_plan* plan);

/* Thread-local description of the last error ("" if none). */
const char* xs_last_error(void);

/* XS_ABI_VERSION of the built library. */
int xs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XSEC_H */
