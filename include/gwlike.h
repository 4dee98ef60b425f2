/*
 * gwlike.h -- C ABI of the batched frequency-domain compact-binary log-likelihood library
 * for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for a batch of B parameter points theta, the Gaussian-noise
 * log-likelihood ratio of the paper's Eq. 2 (section 2, "Bayesian Inference"):
 *
 *     logL(theta) = sum_det [ <d|h(theta)> - 1/2 <h(theta)|h(theta)> ],
 *     <a|b>       = 4 df Re sum_k conj(a_k) b_k / S_k,
 *
 * which is Eq. 2's exponent -(2/T)|d - h|^2 / S summed over independent bins (T = 1/df),
 * minus the same with h = 0 (the theta-independent 1/(2 pi S) prefactor cancels). The paper
 * names this evaluation the dominant cost of inference (section 2.2) and the bottleneck that
 * its parallel nested sampling spreads over processes (section 3, "Parallel prior sampling");
 * here the batch axis B plays the role of those processes.
 *
 * Signal model (the paper names none that is available; these conventions are the library's):
 * TaylorF2 inspiral, 3.5PN non-spinning phase with aligned-spin 1.5PN (beta) and 2PN (sigma)
 * terms, Newtonian amplitude A = sqrt(5/24) pi^(-2/3) (G Mc/c^3)^(5/6) c / D_L,
 *     h_+ = A f^(-7/6) (1 + cos^2 i)/2 e^{-i Psi(f)},  h_x = -i A f^(-7/6) cos(i) e^{-i Psi(f)},
 *     Psi(f) = 2 pi f t_c - phi_c - pi/4 + 3/(128 eta v^5) sum_k phi_k v^k,  v = (pi G M f / c^3)^(1/3),
 * projected on L-shaped detectors on a spherical Earth (radius 6.371e6 m):
 *     h_det = (F_+ h_+ + F_x h_x) e^{-2 pi i f dt_det},  dt_det = -(r_det . k) / c.
 * Fourier convention x~(f) = int x(t) e^{-2 pi i f t} dt.
 *
 * Parameter layout theta[B][11], row-major float64, columns:
 *   0 chirp mass Mc (Msun, detector frame)   1 q = m2/m1 in (0, 1]   2 chi1   3 chi2 (aligned)
 *   4 luminosity distance (Mpc)              5 right ascension (rad) 6 declination (rad)
 *   7 inclination (rad)                      8 polarisation psi (rad) 9 coalescence phase (rad)
 *   10 geocentre coalescence time t_c (s)
 * A row with a non-finite value, q outside (0, 1], Mc <= 0, D_L <= 0 or |chi| >= 1 yields
 * logL = NaN (and a NaN gradient row); the call still returns GWL_OK. So does a row whose phase
 * could exceed 2^39 cycles somewhere on the event's grid (bounded at set-up by
 * sum_m |a_m| max|g_m(f)| + max_det |t_c + dt_det| f_max over the post-Newtonian terms a_m g_m(f)
 * of the phase in cycles; e.g. |t_c| f_max >= 2^39): beyond that a float64 phase no longer
 * resolves a cycle finely enough, and the float64 kernels' table index would not be exact.
 *
 * Conventions for every call:
 *   - Device pointers are HIP device (HBM) addresses on the current device; host pointers are
 *     ordinary process memory. The caller owns every buffer it passes; the library owns the
 *     opaque handles and the device tables inside them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). Calls that take a
 *     stream are asynchronous and stream-ordered: outputs are valid once the stream has
 *     reached the call. Event handles are immutable after creation and may be used
 *     concurrently from several streams. A multi-event plan owns one workspace: launches of
 *     the same plan must not overlap (issue them on one stream, or wait between them).
 *   - Argument errors are detected on the host before any launch and return GWL_E_INVALID or
 *     GWL_E_SHAPE with a message in gwl_last_error(); a failing HIP call returns
 *     GWL_E_DEVICE. No C++ exception crosses this interface. Nothing is written on error.
 */
#ifndef GWLIKE_H
#define GWLIKE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GWL_OK = 0,
  GWL_E_INVALID = -1,     /* bad argument value (null pointer, non-positive size, bad PSD, ...) */
  GWL_E_SHAPE = -2,       /* sizes inconsistent with each other or beyond the supported range    */
  GWL_E_DEVICE = -3,      /* a HIP runtime call failed (message names it)                      */
  GWL_E_NOMEM = -4,       /* device allocation failed                                          */
  GWL_E_UNSUPPORTED = -5, /* valid request the library does not implement                      */
  GWL_E_INTERNAL = -6
} gwl_status;

typedef enum { GWL_FP64 = 0, GWL_MIXED = 1 } gwl_precision;

/* Largest detector count per event. */
#define GWL_MAX_DET 4
/* Number of parameters per point. */
#define GWL_NPARAM 11

/* An L-shaped detector: vertex latitude and longitude, azimuths of the x and y arms measured
 * clockwise from local North (all radians). Arms are horizontal. */
typedef struct {
  double lat, lon, xarm_az, yarm_az;
} gwl_detector;

/* gwl_event_create flags */
#define GWL_F_ISCO_CUTOFF 1u

typedef struct gwl_event_s* gwl_event;
typedef struct gwl_plan_s* gwl_plan;

/* Thread-local text of the last error on this thread ("" if none). */
const char* gwl_last_error(void);

/* Library version string. */
const char* gwl_version(void);

/*
 * Create an event: one data segment seen by `ndet` detectors on a common frequency grid.
 *   data   device, float64 [ndet][M][2]  (complex d~_k, interleaved re, im; strain/Hz)
 *   psd    device, float64 [ndet][M]     (one-sided noise PSD S_k > 0, 1/Hz)
 *   fgrid  device, float64 [M]           (bin frequencies f_k > 0, Hz)
 *   dets   host,   gwl_detector [ndet]
 *   df     frequency spacing = 1/T (s^-1); the 4 df of the inner product uses it
 *   gmst   Greenwich sidereal angle (rad) of the segment, held fixed across the segment
 *   flags  0, or GWL_F_ISCO_CUTOFF: the model is zero above the gravitational-wave frequency of
 *          the innermost stable circular orbit of the point's total mass M,
 *          f_isco = c^3 / (6^(3/2) pi G M) (twice the orbital frequency at r = 6 G M / c^2): both
 *          inner products keep only the bins with f_k <= f_isco. The grid must then increase
 *          (GWL_E_INVALID otherwise). Not available with relative binning, the calibration model
 *          or multi-event plans (GWL_E_UNSUPPORTED). The cut moves with the masses in whole bins,
 *          so gwl_logl_grad returns the derivative with the point's bins held fixed.
 * The call prepares the per-bin tables of the factored likelihood on the device (event
 * preparation, section 2 Eq. 2 rearranged: u_k = 4 df f_k^(-7/6) conj(d_k)/S_k and
 * K_det = 4 df sum_k f_k^(-7/3)/S_k) and synchronises `stream` before returning, so the
 * caller may free data, psd and fgrid afterwards. Returns GWL_E_INVALID if any PSD value is
 * not finite and positive, any f_k is not finite and positive, or any data value is not finite.
 */
gwl_status gwl_event_create(const double* data, const double* psd, const gwl_detector* dets, int ndet,
                            const double* fgrid, int64_t M, double df, double gmst, unsigned flags,
                            void* stream, gwl_event* out);

/*
 * Relative binning (paper section 5: summary data against a fiducial waveform). Same inputs as
 * gwl_event_create plus the fiducial point theta_fid (host, float64 [11]) and the edge spacing
 * eps (radians). The edges are the grid bins where floor(dpsi(f)/eps) changes, plus both ends,
 * with dpsi(f) = 2 pi sum_g sign(g) (f/f_g)^g over g = -5/3, -2/3, 1, 5/3, 7/3 (f_g = f_hi for
 * g > 0, f_lo for g < 0). Per detector and edge the event keeps the summary data
 * V_e = sum_k u_k p0_k hat_e(f_k) (u_k as above, p0_k the fiducial's phasor, hat_e the
 * piecewise-linear function that is 1 at edge e and 0 at its neighbours). Calls on this event
 * then evaluate <d|h> as Re sum_e V_e rho(f_e) with rho the phasor of the phase difference from
 * the fiducial (linear interpolation of h/h0 between edges), on the edges only, and <h|h>
 * exactly. Accurate for points whose phase differs from the fiducial's by much less than eps
 * across any two edges. GWL_E_INVALID if theta_fid is outside the model's domain.
 */
gwl_status gwl_event_create_rb(const double* data, const double* psd, const gwl_detector* dets, int ndet,
                               const double* fgrid, int64_t M, double df, double gmst, const double* theta_fid,
                               double eps, unsigned flags, void* stream, gwl_event* out);

/*
 * Detector calibration model (paper section 2: amplitude and phase corrections at frequency
 * nodes, typically ten per detector). Same inputs as gwl_event_create plus nnode (4..16). The
 * model becomes h_cal,det(f) = h_det(f) (1 + dA_det(f)) exp(i dphi_det(f)), dA and dphi cubic
 * Catmull-Rom splines in ln f through nnode node values at frequencies spaced uniformly in ln f
 * from the first to the last grid bin (a linearly extrapolated ghost node beyond each end).
 * On such an event gwl_logl_batch and gwl_logl_grad take theta [B][11 + 2 nnode ndet]: the 11
 * signal parameters, then per detector its nnode amplitude values followed by its nnode phase
 * values (radians); grad has the same shape. <h|h> stays exact (per-event spline moments).
 * With relative binning: gwl_event_create_rb_cal.
 */
gwl_status gwl_event_create_cal(const double* data, const double* psd, const gwl_detector* dets, int ndet,
                                const double* fgrid, int64_t M, double df, double gmst, int nnode, unsigned flags,
                                void* stream, gwl_event* out);

/*
 * Relative binning and the calibration model together: the event of gwl_event_create_rb (same
 * edges and summary data against theta_fid) whose model carries the calibration factor of
 * gwl_event_create_cal (nnode nodes per detector, spanning the grid from its first to its last
 * bin). The factor is smooth in f, so its product with h / h0 is interpolated between edges like
 * h / h0 itself: <d|h_cal> = Re sum_e V_e rho(f_e) (1 + dA(f_e)) exp(i dphi(f_e)), on the edges
 * only; <h_cal|h_cal> stays exact, its spline moments taken over every grid bin. theta and grad
 * have 11 + 2 nnode ndet columns, as on a calibrated event. Both precisions run the float64 edge
 * loop.
 */
gwl_status gwl_event_create_rb_cal(const double* data, const double* psd, const gwl_detector* dets, int ndet,
                                   const double* fgrid, int64_t M, double df, double gmst, const double* theta_fid,
                                   double eps, int nnode, unsigned flags, void* stream, gwl_event* out);

/* Relative-binning sizes: number of edges (0 for an ordinary event) and of grid bins. */
gwl_status gwl_event_rb_info(gwl_event ev, int64_t* nedge, int64_t* nbins);

/* Release an event and its device tables. Null is accepted. The caller must ensure no work
 * using the event is still pending on any stream. */
gwl_status gwl_event_destroy(gwl_event ev);

/* Query sizes of an event (any pointer may be null). */
gwl_status gwl_event_info(gwl_event ev, int* ndet, int64_t* M, double* df);

/*
 * logL for a batch (paper Eq. 2, as the ratio above).
 *   theta  device, float64 [B][11];  logl device, float64 [B].
 *   prec   GWL_FP64: every step in float64.
 *          GWL_MIXED: float64 for the post-Newtonian phase, the time-shift term and its
 *          reduction modulo one cycle, and for every per-point scalar and reduction; float32
 *          for the per-bin phasor, complex multiply-accumulate over short blocks of bins.
 * B = 0 is a no-op. The call allocates nothing once the event's workspace on `stream` is large
 * enough: the event keeps one workspace per stream, grown (outside graph capture only) by the
 * first call that needs more. On a stream that is capturing a graph a call that would need to
 * grow it returns GWL_E_INVALID: reserve it first with gwl_event_reserve (or one ordinary call of
 * the same size on that stream).
 * GWL_MIXED on a relative-binning event runs the float64 edge loop: its few hundred edge terms are
 * each a sum over hundreds of bins, and float32 roundings on them would not stay within the
 * accuracy the mixed path keeps elsewhere (1e-3 absolute on logL).
 */
gwl_status gwl_logl_batch(gwl_event ev, const double* theta, int64_t B, gwl_precision prec, double* logl,
                          void* stream);

/*
 * gwl_logl_batch over a batch whose length the device decides: only the first *live points of
 * theta[B][11] are evaluated and written to logl (the rest of logl is left as it was), with
 * live a device int64 read by the kernels when they run (values above B count as B, below 1 as
 * none). The launch is sized for B, so the call can be captured once and replayed for batches
 * of any length up to B, e.g. the shrinkage draws of the slice-sampling chains still moving
 * (gwl_slice_draws sets *live). Point groups past *live leave the evaluation kernel at once; the
 * launch splits each point group's bins over enough workgroups that a quarter of the point groups
 * still fill the chip. Not for calibrated events (GWL_E_UNSUPPORTED).
 */
gwl_status gwl_logl_batch_live(gwl_event ev, const double* theta, int64_t B, const int64_t* live, gwl_precision prec,
                               double* logl, void* stream);

/*
 * Grow the event's workspace on `stream` to what a gwl_logl_batch (with_grad = 0) or
 * gwl_logl_grad (with_grad = 1) call with these arguments needs, so that such calls allocate
 * nothing, also under graph capture. Must not be called while `stream` is capturing (it may
 * allocate, and then returns GWL_E_INVALID there). Growing synchronises `stream` before the old
 * buffer is freed. The workspace lives until the event is destroyed.
 */
gwl_status gwl_event_reserve(gwl_event ev, int64_t B, gwl_precision prec, int with_grad, void* stream);

/*
 * gwl_logl_batch without any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc). Same arguments and results as
 * gwl_logl_batch, to rounding (the launch shape may differ). Its workspace (per-point set-up rows,
 * partial sums and completion counters) lives in fixed device arrays, GWL_NOALLOC_SCRATCH_BYTES
 * plus 64 KiB, that every GPU the library runs on holds until the process ends; the call
 * allocates nothing, also not on its first use. It takes the tuned launch shape when that shape's
 * workspace fits, else one with fewer workgroups per point group, else the set-up inside the
 * evaluation kernel, which needs no workspace. All calls on one GPU share the arrays, so calls
 * that overlap on one GPU (other streams, other threads) race and must not be issued;
 * consecutive calls on one stream are fine. The first call on each device looks up the arrays'
 * device addresses (hipGetSymbolAddress): make it outside graph capture. GWL_E_SHAPE for B
 * outside [0, 2^30]; GWL_E_UNSUPPORTED for a calibrated event.
 */
#define GWL_NOALLOC_SCRATCH_BYTES (64ull << 20)
gwl_status gwl_logl_batch_noalloc(gwl_event ev, const double* theta, int64_t B, gwl_precision prec, double* logl,
                                  void* stream);

/*
 * logL and its gradient with respect to all 11 parameters (adjoint of the same evaluation,
 * fused with the forward pass; feeds gradient-based proposals of the sampler in section 3).
 *   grad   device, float64 [B][11] (same column order as theta).
 */
gwl_status gwl_logl_grad(gwl_event ev, const double* theta, int64_t B, gwl_precision prec, double* logl,
                         double* grad, void* stream);

/*
 * Detector-frame strain h_det(f_k) for a batch of points (the signal model above), used to
 * build injections and to check the model on its own.
 *   theta  device float64 [B][11]; fgrid device float64 [M]; dets host [ndet]
 *   out    device float64 [B][ndet][M][2] (complex, interleaved)
 */
gwl_status gwl_waveform(const double* theta, int64_t B, const gwl_detector* dets, int ndet, const double* fgrid,
                        int64_t M, double gmst, double* out, void* stream);

/*
 * Several events of uneven size in one persistent launch (the batch axis of the paper's
 * parallel prior sampling, section 3, extended across events).
 * gwl_multi_plan_create builds the work list (event, point group, bin range), sizes the
 * workspace for the given per-event batch sizes B_e, picks tile shapes, and captures the whole
 * evaluation (queue reset, per-point set-up, persistent kernel, per-event finalisation) in a
 * HIP graph bound to the events. The events must outlive the plan. Calibrated events (of
 * gwl_event_create_cal or gwl_event_create_rb_cal) are not in the persistent queue: each launch
 * runs their own set-up, bin-loop and epilogue kernels after the graph (on side streams of the
 * plan's own, joined back into the launch's stream; workspaces allocated here), with theta and
 * grad of 11 + 2 nnode ndet columns; the ISCO cut-off is not supported in plans.
 *   evs       host [E] event handles;  B_e host int64 [E] (each >= 0)
 *   with_grad 0: logL only; 1: logL and gradient
 */
gwl_status gwl_multi_plan_create(const gwl_event* evs, int E, const int64_t* B_e, gwl_precision prec,
                                 int with_grad, gwl_plan* out);

/*
 * gwl_multi_plan_create with the queue order chosen by the caller: order 0 takes the tuned one (as
 * gwl_multi_plan_create), 1 queues events by ascending work (small events finish first: lower
 * per-event latency), 2 by descending work (large items first, small ones fill the tail of the
 * launch). The chunk length is the tuned one either way. Results do not depend on the order (every item writes its
 * own partial sums, added in a fixed order). GWL_E_INVALID for another order.
 */
gwl_status gwl_multi_plan_create_order(const gwl_event* evs, int E, const int64_t* B_e, gwl_precision prec,
                                       int with_grad, int order, gwl_plan* out);

/*
 * Run a plan. theta[e], logl[e], grad[e] are device pointers ([B_e][P_e], [B_e], [B_e][P_e], P_e = 11
 * or 11 + 2 nnode ndet on a calibrated event);
 * grad may be null when the plan has no gradient. The pointer tables are host arrays of E
 * entries. If event_latency_us is non-null it receives, per event, the time from the start of
 * the launch to the completion of that event's results (device clock), and the call then
 * synchronises `stream`. Calibrated events run on side streams of the plan's own, forked from
 * `stream` after the persistent launch and joined back into it before the call returns: work
 * queued on `stream` afterwards sees every result.
 */
gwl_status gwl_multi_launch(gwl_plan pl, const double* const* theta, double* const* logl, double* const* grad,
                            double* event_latency_us, void* stream);

gwl_status gwl_plan_destroy(gwl_plan pl);

/* Shape of a plan: the bin-chunk length shared by all events, whether events are queued by
 * descending work (1) or ascending work (0), and the number of work items. Any pointer may be
 * null. */
gwl_status gwl_plan_info(gwl_plan pl, int* chunk, int* descending, int64_t* items);

/*
 * Time candidate shapes of a multi-event plan for this workload (events, B_e, precision,
 * with_grad) and record the fastest in the JSON cache `cache_path` (null = in memory only):
 * chunk lengths 1024..16384 bins and both queue orders, each timed over three graph launches on
 * synthetic valid parameter points. gwl_multi_plan_create then uses the recorded shape for the
 * same workload (same event order, B_e and bin counts). Allocates a plan per candidate and
 * synchronises the device. GWL_E_SHAPE if no candidate fits.
 */
gwl_status gwl_multi_autotune(const char* cache_path, const gwl_event* evs, int E, const int64_t* B_e,
                              gwl_precision prec, int with_grad);

/*
 * Time candidate tile shapes for (event, B, precision, with_grad) on the device and record the
 * fastest in the JSON cache file `cache_path` (created or updated; null = in-memory only).
 * Candidates vary the wavefronts per workgroup, the workgroups per group of 64 points, whether
 * the per-point set-up runs in the evaluation kernel and, for the value with several workgroups
 * per point group, whether the last workgroup to finish or a second kernel adds their sums (the
 * same bits either way). Later calls with a matching shape use the cached choice. Synchronises
 * the device.
 */
gwl_status gwl_autotune(const char* cache_path, gwl_event ev, int64_t B, gwl_precision prec, int with_grad);

/* The bin-loop shape a gwl_logl_batch / gwl_logl_grad call with these arguments would use: the
 * number of bin chunks and the chunk length in bins (from the autotuner's cache, else the
 * heuristic). Either output pointer may be null. */
gwl_status gwl_launch_shape(gwl_event ev, int64_t B, gwl_precision prec, int with_grad, int* nchunk,
                            int* chunk_bins);

/* The evaluation kernel's layout for such a call: wavefronts per workgroup (each takes one chunk
 * of bins for the workgroup's 64 points; the chunks are added in LDS), workgroups per group of 64
 * points (nchunk = waves x groups), and whether the per-point set-up runs inside that kernel (1)
 * or in a set-up kernel before it (0). (Which kernel adds the workgroups' sums is not reported:
 * it does not change the result.) Any output pointer may be null. */
gwl_status gwl_launch_layout(gwl_event ev, int64_t B, gwl_precision prec, int with_grad, int* waves, int* groups,
                             int* setup);

/* Load tile choices from a JSON cache written by gwl_autotune (missing file = GWL_E_INVALID). */
gwl_status gwl_autotune_load(const char* cache_path);

/*
 * Kernel timing for measurement. While enabled, every launch of the evaluation kernel (the bin
 * loop with its reduction and, for the value, the epilogue) made by gwl_logl_batch and
 * gwl_logl_grad is bracketed by two HIP events recorded on the caller's stream (the stream the
 * kernel runs on). gwl_profile_read waits for those events and returns the number
 * of bracketed launches and their summed duration in milliseconds since the previous read,
 * then forgets them. Either pointer may be null. Disabling keeps unread records.
 */
gwl_status gwl_profile_enable(int on);
gwl_status gwl_profile_read(int64_t* launches, double* total_ms);

/*
 * Slice-sampling support for a sampler above the likelihood (the walks that propose the
 * candidates of the paper's section 3 algorithm; procedure: Neal 2003, "Slice sampling",
 * sections 4.1 and 4.2). One slice move of n chains in d dimensions is: place an interval
 * [x - u0 dirn, x + (1 - u0) dirn] on each chain's line, step its ends out by whole lengths while
 * they lie inside the region (at most jl = floor(m u1) steps to the left and jr = m - 1 - jl to
 * the right), then draw t uniformly from [lo, hi], shrinking the interval to the draw after
 * every draw outside, until a draw lands inside. These calls do the bookkeeping; the caller
 * evaluates ln L at the points they write and passes the values back. The region is {p in the
 * unit cube, ln L(p) >= lmin}; a NaN ln L counts as outside.
 *
 * All arrays are float64 device memory, row-major, owned by the caller; `lmin` points to one
 * device double; `done` is one byte per chain (0 or 1). Every product and sum is rounded on its
 * own, in the order written above (no fused multiply-add), so the results equal those of the
 * same steps taken one array operation at a time. Calls are stream-ordered on `stream`;
 * GWL_E_SHAPE for n < 1, d < 1, m < 1 or G < 1, for more than 2^30 points (m n or G n) or more
 * than 2^31 coordinates (m n d or G n d); GWL_E_INVALID for a null pointer.
 *
 * gwl_slice_ends: lo = -u0, hi = 1 - u0, jl, jr as above, and the m - 1 ends each chain's stepping
 *   out may examine (its left ends lo - s for s < jl and right ends hi + s for s < jr): slot s of
 *   chain i, pts[(s n + i) d ..] = x_i + t dirn_i with t = lo_i - s for s < jl_i and
 *   t = hi_i + (s - jl_i) above; pts holds (m - 1) n rows (none for m = 1, when pts may be null).
 * gwl_slice_ends_select: with logl[(m - 1) n] the values at those slots: lo -= the number of left
 *   ends inside before the first outside (jl if none), hi += the same on the right (jr if none).
 *   Nothing to do for m = 1.
 * The shrinkage draws of a move come in groups of G, each group for the chains still moving,
 * listed in list[0 .. *nact) (int32 chain indices, device; *nact a device int64, taken as at
 * most n; entries outside [0, n) are skipped):
 * gwl_slice_list_init: list = 0, 1, .., n - 1 and *nact = n (the first group of a move).
 * gwl_slice_move_begin: the start of a move in one launch: xn = x, done = 0 and the list of all
 *   chains (as gwl_slice_list_init). gwl_slice_move_end: moved |= done (bytes) and x = xn.
 * gwl_slice_draws: for list entry j (chain i = list[j]), G draws, each from the interval as it
 *   would be if the earlier draws had fallen outside: t_k = a + u_k (b - a) from (a, b) =
 *   (lo, hi), then a = t_k if t_k < 0 else b = t_k, with u_k = u[k n + i]; writes t[j G + k],
 *   the points pts[(j G + k) d ..] = x_i + t_k dirn_i (the live points are the first *nact G
 *   rows of pts[G n][d]), a[i] and b[i]. Sets *live = *nact G (for gwl_logl_batch_live), adds
 *   it to *calls if calls is not null, and sets *nact_next = 0. nact_next must not be nact.
 * gwl_slice_select: with logl[*nact G] the values at those points, for every listed chain not
 *   yet done: the first draw inside the region (if any) gives xn = x + t dirn and done = 1;
 *   otherwise the chain takes (lo, hi) = (a, b) and is appended to list_next (*nact_next counts
 *   them; the order of the appended chains depends on scheduling). list_next and nact_next must
 *   differ from list and nact. The cube test recomputes x + t dirn with the same rounding as the
 *   points gwl_slice_draws wrote, so those points are not read again.
 */
gwl_status gwl_slice_ends(int64_t n, int d, int m, const double* x, const double* dirn, const double* u0,
                          const double* u1, double* pts, double* lo, double* hi, double* jl, double* jr, void* stream);
gwl_status gwl_slice_ends_select(int64_t n, int d, int m, const double* pts, const double* logl, const double* lmin,
                                 double* lo, double* hi, const double* jl, const double* jr, void* stream);
gwl_status gwl_slice_list_init(int64_t n, int* list, int64_t* nact, void* stream);
gwl_status gwl_slice_move_begin(int64_t n, int d, const double* x, double* xn, unsigned char* done, int* list,
                                int64_t* nact, void* stream);
gwl_status gwl_slice_move_end(int64_t n, int d, const unsigned char* done, unsigned char* moved, const double* xn,
                              double* x, void* stream);
gwl_status gwl_slice_draws(int64_t n, int d, int G, const int* list, const int64_t* nact, const double* x,
                           const double* dirn, const double* lo, const double* hi, const double* u, double* t,
                           double* pts, double* a, double* b, int64_t* live, int64_t* nact_next, int64_t* calls,
                           void* stream);
gwl_status gwl_slice_select(int64_t n, int d, int G, const int* list, const int64_t* nact, const double* x,
                            const double* dirn, const double* t, const double* logl, const double* lmin,
                            const double* a, const double* b, double* xn, unsigned char* done, double* lo, double* hi,
                            int* list_next, int64_t* nact_next, void* stream);

/*
 * Prior transform for a sampler above the likelihood (the prior-sampling step of the paper's
 * section 2: nested sampling draws points uniformly in the unit cube and maps them to parameters
 * through the prior's inverse CDF). Columns are independent; column j maps u to
 *   theta = g_j(c0_j + c1_j clamp(u, 0, 1))   (the argument in one fused multiply-add)
 * with g_j the identity (a uniform prior on [c0, c0 + c1]), the cube root (density ~ x^2 on
 * [a, b]: c0 = a^3, c1 = b^3 - a^3), asin (density ~ cos x, e.g. declination on [-pi/2, pi/2]:
 * c0 = -1, c1 = 2) or acos (density ~ sin x, e.g. inclination on [0, pi]: c0 = -1, c1 = 2, which
 * maps u = 0 to pi). asin and acos arguments are clamped to [-1, 1]. Points outside the cube
 * are clamped into it first, so a sampler may pass candidates it will judge itself.
 *
 * u and theta: n x d float64 row-major device arrays owned by the caller (they must not
 * overlap); map, c0, c1: host arrays of d entries, copied at the call. Stream-ordered on
 * `stream`. GWL_E_SHAPE for n < 1 or d outside [1, GWL_PRIOR_MAX_DIM]; GWL_E_INVALID for a null
 * pointer or an unknown map code.
 */
#define GWL_PRIOR_MAX_DIM 64
typedef enum { GWL_MAP_LINEAR = 0, GWL_MAP_CBRT = 1, GWL_MAP_ASIN = 2, GWL_MAP_ACOS = 3 } gwl_prior_map;
gwl_status gwl_prior_transform(int64_t n, int d, const int* map, const double* c0, const double* c1, const double* u,
                               double* theta, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GWLIKE_H */
