/*
 * wf.h -- C ABI of the widefield radio-interferometric measurement operator on one
 * MI355X (gfx950).
 *
 * The operator is the hybrid w-stacking / w-projection model of Dabbech & Wiaux,
 * "A distributed resource-adaptive implementation of the widefield radio-
 * interferometric measurement model for scalable image formation":
 *
 *   y = Phi x + n                        (Sect. 2, eq. 3)
 *   Phi = [Phi_1 .. Phi_P]^T,  Phi_p = G_p F Z_p              (Sect. 3.2, eq. 6)
 *   Phi^dag Phi = sum_p Z_p^dag F^dag G_p^dag G_p F Z_p        (Sect. 3.3, eq. 7-8)
 *
 * Z_p is the w-layer of bin p times the grid correction, F the 2x-oversampled 2-D DFT,
 * G_p the sparse de-gridding matrix whose rows are Kaiser-Bessel taps convolved with a
 * per-visibility residual-w Fourier kernel (Sect. 3.1).  The number of w-bins P and the
 * strategy are chosen at build time from the memory model (eq. 9) and the cost model
 * (eq. 10) by the decision tree of Sect. 3.4 / Fig. 2, under one GPU's memory.
 *
 * Conventions
 *  - Every call returns wf_status; 0 (WF_OK) is success.  No C++ exception crosses the
 *    ABI.  On failure wf_last_error() returns a thread-local message.
 *  - Image pixel (i, j) of an nx x ny image is at direction cosines
 *    l = (i - nx/2) cell, m = (j - ny/2) cell; images are row-major [ny][nx] (rows = m).
 *    nx, ny must be even powers of two in [8, 8192] (the grid is 2nx x 2ny).
 *  - Visibilities are ordered [chan][row] in the caller's row order; complex values are
 *    interleaved FP32 (re, im).  Images for several channels are [nchan][ny][nx].
 *  - Apply calls are asynchronous on the HIP stream passed in (NULL = default stream);
 *    all their pointer arguments are DEVICE memory owned by the caller.  The operator
 *    owns its sparse matrices and work grids; a handle belongs to the device that was
 *    current at build time.  Calls on one handle must not overlap (they share the work
 *    grids); distinct handles are independent.
 */
#ifndef WF_H
#define WF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wf_op wf_op;
typedef struct wf_mlp wf_mlp;

typedef enum {
  WF_OK = 0,
  WF_EINVAL = 1,   /* bad argument: shape, non-finite uvw, field too wide (2L^2 >= 1) */
  WF_ENOMEM = 2,   /* device or host allocation failed                               */
  WF_EBUDGET = 3,  /* no strategy of the decision tree fits the memory budget        */
  WF_EHIP = 4,     /* a HIP runtime call failed                                      */
  WF_ENOTSUP = 5   /* valid request the library does not implement                  */
} wf_status;

typedef enum { WF_STORE_F32 = 0, WF_STORE_F16 = 1, WF_STORE_BF16 = 2 } wf_store;

/* Strategy of Sect. 3.4 / Fig. 2: (a) precomputed G, (b) precomputed holographic H,
 * (c) G computed on the fly.  WF_AUTO runs the decision tree: (a) when G fits the
 * budget, else (b) when H fits (its exact size is known after the symbolic pass), else
 * (c); WF_EBUDGET when not even (c)'s row data fits.  A holographic operator stores
 * H_p = G_p^dag G_p as dense stencils per active 32 x 32 grid tile (side 2 Tmax - 1,
 * Tmax the largest patch side reaching the tile) and applies Phi^dag Phi only:
 * wf_forward / wf_adjoint / wf_get_row return WF_ENOTSUP for it.  Needs tile 32.
 * An on-the-fly operator keeps no values of G.  It writes G chunk by chunk (runs of
 * whole row groups of one bin, at most 2.5% of the budget share each) into a transient
 * buffer of each branch at every apply, in one of two forms (option otf_form):
 *  - factorised: the build stores each row's thresholded residual kernel (n' x n'
 *    values, times its weight, in the store format; about n'^2 / T^2 ~ 0.4 of G's
 *    values) and its 2J Kaiser-Bessel taps (evaluated in FP64, kept in FP32); an apply
 *    only convolves the kernel with the taps (FP32);
 *  - rebuilt: only coordinates, weight and patch word are kept per row (about 48 bytes);
 *    an apply repeats the FP64 value pass of the build of (a), so that its results equal
 *    those of (a) up to the order of FP32 atomic additions.
 * wf_get_row returns WF_ENOTSUP for it. */
typedef enum { WF_AUTO = 0, WF_PRECOMP_G = 1, WF_PRECOMP_H = 2, WF_ONTHEFLY = 3 } wf_strategy;

typedef struct {
  int32_t nx, ny;   /* image side in pixels                                    */
  double cell_rad;  /* pixel size as a direction-cosine step; field L = n cell */
} wf_image_shape;

typedef struct {
  int32_t J;               /* Kaiser-Bessel support (odd), default 7                  */
  double beta;             /* Kaiser-Bessel shape, default 2.34 J                     */
  int32_t oversample;      /* grid oversampling o (Sect. 3.2), must be 2              */
  double alpha;            /* w-kernel sampling margin over the chirp band, default 2 */
  int32_t smax;            /* largest residual-kernel side (odd, <= 31), default 31   */
  double eps_w;            /* kernel energy dropped by the hard threshold, 1e-6       */
  int32_t nbins;           /* 0: planner chooses P (eq. 10); > 0 forces P (<= 255)    */
  wf_strategy strategy;    /* WF_AUTO: decision tree                                  */
  wf_store store;          /* value precision of the stored G                         */
  double plan_fraction;    /* planning / clustering subset fraction, default 0.01     */
  double budget_fraction;  /* share of memory_budget for the sparse matrix, 0.65      */
  uint64_t seed;           /* SplitMix64 state for the subset draw                    */
  int32_t tile;            /* grid tile side of the fused G^dag G kernel (0 = auto:
                              32); a power of two with tile + J + smax - 2 <= 101, so
                              that an item's FP64 accumulator fits one LDS (160 KiB)   */
  int32_t max_rows_per_item; /* rows per work item, <= 1024 (0 = auto: 1024)           */
  int32_t branches;        /* concurrent branches of an apply, <= 16 (0 = auto: one per
                              channel up to 4; a single channel runs on one branch)   */
  const wf_mlp* surrogate; /* NULL: exact residual kernels.  Otherwise the rows of
                              residual-kernel side 9..15 (smaller kernels cost less to
                              build exactly than an inference) whose kernel the network
                              predicts with log10 error at most log10(surrogate_tol) use
                              the prediction (square fields).  Under strategy (c)
                              the factorised form stores the predicted kernels; the
                              rebuilt form re-infers them at every apply from a copy
                              of the network's parameters taken at build.  Either way
                              the network must outlive the build call only.  Not
                              with strategy (b).                                      */
  double surrogate_tol;    /* predicted relative L2 error bound, default 1e-3          */
  const float* weights;    /* NULL: unit weights.  Otherwise host FP32 [total rows] in
                              the [chan][row] order of the visibilities: row k of the
                              operator is scaled by weights[k], Phi_W = diag(w) Phi, so
                              Phi_W^dag Phi_W = Phi^dag diag(w^2) Phi (data weighting,
                              Sect. 2).  Finite; scaled G values must fit the storage
                              format (WF_EINVAL when FP16 would overflow).  Read during
                              the build only.                                         */
  const uint8_t* flags;    /* NULL: no flags.  Otherwise host [total rows], same order;
                              non-zero discards the measurement (Sect. 3.5 input files)
                              before planning: its row is never built, wf_forward
                              writes 0 there and wf_adjoint ignores it.  Read during the
                              build only.                                             */
  int32_t otf_form;        /* form of strategy (c): 0 auto (factorised when its stored
                              kernels fit the budget share, else rebuilt), 1 rebuilt at
                              every apply, 2 factorised (WF_EBUDGET when its kernels do
                              not fit)                                                */
} wf_options;

/* Fill *opt with the defaults listed above. */
void wf_default_options(wf_options* opt);

/* Build the operator (workflow stages 1-3 of Sect. 3.5 / Fig. 3: plan, partition,
 * precompute).
 *  uvw_m      host [nrows][3] FP64 baseline coordinates in metres (copied).
 *  chan_rows  NULL: every channel uses all nrows rows of uvw_m.  Otherwise host
 *             [nchan] row counts; channel c uses its own consecutive block of
 *             chan_rows[c] rows of uvw_m (sum must equal nrows).  Each channel is an
 *             independent operator with its own w-bins (wideband model, Sect. 2).
 *  freqs_hz   host [nchan] channel frequencies; uvw in wavelengths = uvw_m f / c.
 *  shape      image geometry, shared by all channels.
 *  memory_budget_bytes  device memory the planner may assume (e.g. 288e9).
 *  opt        NULL for defaults.
 *  hip_stream stream for the build's device work (NULL = default stream); the call
 *             returns after the build has completed.
 *  out        receives the handle.
 * Errors: WF_EINVAL (shapes, non-finite uvw, 2L^2 >= 1), WF_EBUDGET (nothing fits),
 * WF_ENOTSUP (holographic or on-the-fly strategy requested/required), WF_ENOMEM, WF_EHIP. */
wf_status wf_build_operator(const double* uvw_m, int64_t nrows, const int64_t* chan_rows,
                            const double* freqs_hz, int32_t nchan, wf_image_shape shape,
                            uint64_t memory_budget_bytes, const wf_options* opt,
                            void* hip_stream, wf_op** out);

/* Briggs robust weights for wf_options.weights.  The paper names density-aware data
 * weighting (Sect. 2) without a formula; this is the published definition (D. S.
 * Briggs, PhD thesis, 1995), per channel:
 *   W_c  = sum of the natural weights w_k of the samples whose (u, v) -- or whose
 *          conjugate (-u, -v), the image being real -- falls in Fourier cell c of the
 *          image (du = 1 / (nx cell_rad), dv = 1 / (ny cell_rad); index
 *          floor(u / du + 1/2) modulo nx, likewise v);
 *   f^2  = (5 10^-robust)^2 sum_k w_k / sum_k w_k W_c(k);
 *   w'_k = w_k / (1 + W_c(k) f^2)   (robust -> +inf: natural; -> -inf: uniform).
 * out receives the operator weights sqrt(w'_k): the imaging weight multiplies each
 * sample once in Phi^dag diag(w') y = Phi_W^dag Phi_W-style sums.
 *  uvw_m, nrows, chan_rows, freqs_hz, nchan, shape: as for wf_build_operator.
 *  natural  host FP32 [total rows] natural weights (NULL = ones; finite, >= 0).
 *  flags    host [total rows] (NULL = none): flagged samples get 0 and are left out.
 *  out      host FP32 [total rows].
 * Device work (density gridding with FP64 atomics, reductions) on hip_stream;
 * synchronous.  Errors: WF_EINVAL, WF_ENOMEM, WF_EHIP. */
wf_status wf_briggs_weights(const double* uvw_m, int64_t nrows, const int64_t* chan_rows,
                            const double* freqs_hz, int32_t nchan, wf_image_shape shape,
                            double robust, const float* natural, const uint8_t* flags,
                            float* out, void* hip_stream);

/* Allocation-free variant of wf_briggs_weights, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  One channel, every array already on the device:
 *  d_uvw_m    device FP64 [nrows][3] metres; freq_hz the channel's frequency.
 *  d_natural  device FP32 [nrows] natural weights (NULL = ones);
 *  d_flags    device [nrows] (NULL = none): flagged samples get 0 and are left out.
 *  d_out      device FP32 [nrows] operator weights sqrt(w'_k), as wf_briggs_weights.
 * The density grid and the two sums live in a static device array of the library
 * (WF_BRIGGS_NOALLOC_MAX_CELLS + 2 doubles, 32 MiB, one per device, held until the
 * process ends); nx * ny beyond WF_BRIGGS_NOALLOC_MAX_CELLS is WF_EINVAL.  Nothing is
 * allocated; the array is cleared by a kernel at every call.  Asynchronous on
 * hip_stream: f^2 is formed on the device, nothing is read back.  Calls that overlap
 * on one device share the array and race: order them on one stream.  Device data is
 * not validated (non-finite coordinates give unspecified weights, never an access out
 * of bounds).  Errors: WF_EINVAL (host-side arguments), WF_EHIP. */
#define WF_BRIGGS_NOALLOC_MAX_CELLS 4194304
wf_status wf_briggs_weights_noalloc(const double* d_uvw_m, int64_t nrows, double freq_hz,
                                    wf_image_shape shape, double robust,
                                    const float* d_natural, const uint8_t* d_flags,
                                    float* d_out, void* hip_stream);

/* The four apply calls below return WF_EINVAL for a null handle or buffer, WF_ENOTSUP for
 * wf_forward / wf_adjoint on a holographic operator (it holds H_p only), and WF_EHIP when
 * a HIP call fails (work already queued on the stream may then be partial).  They
 * allocate no device memory. */

/* y = Phi x (eq. 3, eq. 6).  d_img: real FP32 [nchan][ny][nx];
 * d_vis: complex FP32 [total rows] in [chan][row] caller order. */
wf_status wf_forward(wf_op* op, const float* d_img, float* d_vis, void* hip_stream);

/* x = Phi^dag y = sum_p Z_p^dag F^dag G_p^dag y_p (the adjoint of eq. 6, the factors of
 * eq. 8 applied to data; Sect. 3.3).  d_vis: complex FP32 [total rows] in [chan][row]
 * caller order; d_img: complex FP32 [nchan][ny][nx]. */
wf_status wf_adjoint(wf_op* op, const float* d_vis, float* d_img, void* hip_stream);

/* Phi^dag Phi x (eq. 7-8): d_img real FP32 [nchan][ny][nx] -> d_out complex FP32
 * [nchan][ny][nx].  The sum over w-layers is accumulated in place on the device. */
wf_status wf_psf_apply(wf_op* op, const float* d_img, float* d_out, void* hip_stream);

/* Re{Phi^dag Phi x}, the quantity the forward-backward update uses (Sect. 2, eq. 4):
 * d_out real FP32 [nchan][ny][nx]. */
wf_status wf_psf_apply_re(wf_op* op, const float* d_img, float* d_out, void* hip_stream);

typedef struct {
  int32_t nchan;
  int32_t nbins;            /* P of this channel                                       */
  wf_strategy strategy;     /* strategy chosen by the decision tree                    */
  wf_store store;
  int32_t Kx, Ky;           /* grid sides (o nx, o ny)                                 */
  int32_t tile;             /* fused-kernel tile side                                  */
  int32_t p_wsclean;        /* ceil of eq. 5 over the field (search upper end)         */
  int32_t p_star;           /* minimiser of eq. 10                                      */
  int64_t nrows;            /* rows of this channel that were built (not flagged)      */
  int64_t ntaps;            /* stored values of G (K of eq. 9)                          */
  int64_t nwork;            /* work items of the fused kernel                           */
  double k_estimate;        /* planner's K(P) estimate at the chosen P                  */
  double mem_g_bytes;       /* device bytes of G (values + row metadata)                */
  double mem_model_bytes;   /* eq. 9 (GPU form) at the chosen P                         */
  double cost_model;        /* eq. 10 at the chosen P                                   */
  double capped_fraction;   /* rows whose kernel side was capped at smax               */
  double max_dropped_energy;/* largest per-row dropped kernel energy fraction           */
  double build_seconds;     /* wall time of the build of this channel                  */
  int32_t max_rows_per_item;/* rows per work item of the current split                 */
  int32_t branch;           /* branch that writes this channel's output                */
  double surrogate_fraction;/* rows whose residual kernel came from the network        */
  double mem_h_bytes;       /* device bytes of the holographic stencils (strategy (b))  */
  int64_t nflagged;         /* flagged rows of this channel (discarded)                 */
  double mem_transient_bytes;/* on-the-fly: value buffer of one branch (largest chunk)   */
  double value_pass_flops;  /* on-the-fly, rebuilt: FP64 flops of one apply's value pass
                               (two DFT sweeps of each residual kernel, 16 nk^3, and its
                               Kaiser-Bessel convolution, 4 J (n' T + T^2)); factorised:
                               FP32 flops of the convolution alone; else 0            */
  double mem_khat_bytes;    /* factorised on-the-fly: device bytes of the stored kernels,
                               their offsets and taps (included in mem_g_bytes); else 0 */
  int32_t otf_form;         /* on-the-fly: 1 rebuilt, 2 factorised; else 0             */
} wf_plan_info;

/* The planner alone, on the host (the compute-resource planning of Sect. 3.4, run by the
 * paper as a tool of its own before the build): for the rows uvw_m (host, [nrows][3]
 * metres) of one channel at freq_hz it evaluates eq. 5 (the search range), K(P) on the
 * planning subset, the GPU form of eq. 9 and eq. 10 for every P, and the decision tree
 * of Fig. 2, exactly as wf_build_operator does.  Fills nbins, strategy (WF_PRECOMP_G,
 * or WF_PRECOMP_H where no precomputed G fits: the build then settles (b) or (c) from
 * the exact holographic size), store, Kx, Ky, p_wsclean, p_star, nrows, k_estimate,
 * mem_model_bytes and cost_model of *out; other fields are zero.  centroids (may be
 * NULL): the ascending w-bin centroids of the chosen P, cap >= nbins.  Touches no
 * device.  WF_EINVAL on bad arguments (as wf_build_operator); WF_ENOTSUP when the
 * strategy option forces precomputed G and none fits. */
wf_status wf_plan(const double* uvw_m, int64_t nrows, double freq_hz, wf_image_shape shape,
                  uint64_t memory_budget_bytes, const wf_options* opt, wf_plan_info* out,
                  double* centroids, int32_t cap);

/* Plan and matrix statistics of channel chan (Sect. 3.4 quantities). */
wf_status wf_get_plan(const wf_op* op, int32_t chan, wf_plan_info* out);

/* Ascending w-bin centroids (w_p^stack, wavelengths) of channel chan; cap >= nbins. */
wf_status wf_get_centroids(const wf_op* op, int32_t chan, double* out, int32_t cap);

/* Per-bin row counts M_p of channel chan; cap >= nbins. */
wf_status wf_get_bin_rows(const wf_op* op, int32_t chan, int64_t* out, int32_t cap);

/* Diagnostic: one stored row of G for caller-order row `row` of channel chan, converted
 * to FP32.  Writes the patch side T, the patch origin (q_u0, q_v0) on the periodic grid
 * (in [0, Kx) x [0, Ky)), the bin, and T*T complex values (row-major [a_v][a_u]) into
 * host buffer vals (capacity cap complex values).  Synchronous. */
wf_status wf_get_row(const wf_op* op, int32_t chan, int64_t row, int32_t* T, int32_t* qu0,
                     int32_t* qv0, int32_t* bin, float* vals, int32_t cap);

/* Diagnostic: X_p = F Z_p x for channel chan and bin p, written as a complex FP32 grid
 * [Ky][Kx] (row-major, rows = v) into device buffer d_grid.  Asynchronous. */
wf_status wf_layer_grid(wf_op* op, int32_t chan, int32_t bin, const float* d_img,
                        float* d_grid, void* hip_stream);

/* Diagnostic timing: when enabled, every launch of kernel `kernel_id` (0 = the fused
 * G^dag G kernel, 1 = forward row FFT, 2 = forward column FFT, 3 = inverse column FFT,
 * 4 = inverse row FFT, 5 = the on-the-fly value pass of G) is bracketed by HIP events on its stream; wf_profile_read
 * returns the number of launches and their summed duration in ms (synchronising). */
wf_status wf_profile_enable(wf_op* op, int32_t kernel_id, int32_t enable);
wf_status wf_profile_read(wf_op* op, int32_t kernel_id, int64_t* launches, double* total_ms);

/* ------------------------------------------------------------------ batched form
 * The channels of a wideband operator are independent operators (Sect. 2; the paper
 * runs one worker pool per frequency).  An apply issues its (channel, bin) layers on
 * `branches` concurrent HIP streams forked from and joined back into the caller's
 * stream; each branch owns a set of work grids (2 Kx Ky + ny Kx complex FP32 values,
 * plus an nx ny accumulator when a single channel's bins are split over branches).
 * Channels are placed on branches largest first (by measured time after wf_autotune,
 * else by stored values and FFT work).  Results equal the one-branch apply up to the
 * order of FP32 additions. */

/* Set the number of branches (1..16).  Allocates the extra branches' grids; with one
 * channel and n > 1 the channel's bins are split over the branches and the partial sums
 * are added in the caller's stream.  Invalidates graphs captured earlier. */
wf_status wf_set_branches(wf_op* op, int32_t branches);

/* Layer-batched sweep (enable >= 1): every later apply (and every graph captured
 * afterwards) runs each stage as one launch over all (channel, bin) layers at once --
 * forward row FFTs, forward column FFTs, the de-gridding / gridding / fused G^dag G row
 * kernels as one persistent launch per (patch class, work-item tile) draining the items
 * of every layer from a device queue, inverse column FFTs, and inverse row FFTs that sum
 * each channel's layers in registers and write its image once.  enable = lanes (at most
 * 4, at most the channel count): the channels are cut into that many contiguous ranges
 * of about equal work, each running the stages above on a stream of its own; lane k
 * starts once lane k - 1 has issued its forward FFTs, so that one lane's row kernels run
 * beside the next lane's FFTs (the Sect. 2 worker pools per frequency; wf_autotune
 * times 1..3 lanes).  Holds the grids of every layer (2 Kx Ky + ny Kx complex FP32
 * values each) while enabled; WF_ENOMEM when they do not fit.  Needs Kx = 2 nx and
 * Ky = 2 ny in 2048 .. 16384 and a stored G for every channel (WF_ENOTSUP otherwise).
 * Latency stamps mark the completion of each channel's last image row.  Results equal
 * the branch apply up to the order of FP32 additions.  enable = 0 releases the sweep;
 * WF_EINVAL for enable < 0.  Synchronous; invalidates graphs captured earlier. */
wf_status wf_set_sweep(wf_op* op, int32_t enable);

typedef enum {
  WF_APPLY_FORWARD = 0,   /* wf_forward      */
  WF_APPLY_ADJOINT = 1,   /* wf_adjoint      */
  WF_APPLY_PSF = 2,       /* wf_psf_apply    */
  WF_APPLY_PSF_RE = 3     /* wf_psf_apply_re */
} wf_apply_kind;

typedef struct wf_graph wf_graph;

/* Capture one apply of `kind` with fixed device buffers d_in / d_out (as for the
 * matching apply call) into an instantiated HIP graph: all channels, bins, branches and
 * per-channel stamps of the sweep become one graph launch.  hip_stream must be a
 * created (non-NULL) stream; it is used for the capture only.  The graph refers to the
 * operator's grids: it must not run concurrently with another apply of the same
 * handle, and it becomes invalid (wf_graph_launch returns WF_EINVAL) after
 * wf_set_branches or wf_autotune.  Profiling is off inside the graph. */
wf_status wf_graph_capture(wf_op* op, wf_apply_kind kind, const float* d_in, float* d_out,
                           void* hip_stream, wf_graph** out);
/* Launch a captured apply on hip_stream (any stream of the operator's device). */
wf_status wf_graph_launch(wf_graph* g, void* hip_stream);
/* Count the nodes of a captured apply: *kernels = kernel launches, *total = all nodes
 * (kernels, event records and waits of the branch fork/join, copies).  Host-only query;
 * WF_EINVAL for a null graph or output pointer. */
wf_status wf_graph_nodes(const wf_graph* g, int64_t* kernels, int64_t* total);
/* Release a graph; graphs of a handle are destroyed before the handle itself. */
wf_status wf_graph_destroy(wf_graph* g);

/* Per-channel completion latency.  When enabled, every apply (eager or a graph captured
 * while enabled) writes the device wall clock at its start and after each channel's
 * last kernel.  wf_read_latency synchronises the device and writes, for the last apply
 * that ran, the milliseconds from its start to each channel's completion into host
 * ms[nchan] (cap >= nchan); channels without rows report their zero fill. */
wf_status wf_latency_enable(wf_op* op, int32_t enable);
wf_status wf_read_latency(wf_op* op, double* ms, int32_t cap);

typedef struct {
  int32_t branches;        /* branch count chosen (a sweep: its lane count)           */
  int32_t retuned_chans;   /* channels whose work-item size changed                   */
  double sweep_ms_before;  /* Re{Phi^dag Phi} sweep (all channels) before tuning      */
  double sweep_ms_after;   /* ... and after                                           */
  int32_t wide_tile_bins;  /* bins whose work items now cover 2 x 2 base tiles        */
} wf_tune_info;

/* Autotuner: by timing Re{Phi^dag Phi} applies on d_img (real FP32 [nchan][ny][nx])
 * into the caller's scratch d_out (same shape), choose per channel the rows per work
 * item (256, 512 or 1024) and per bin the work items' tile side (the base tile, or 2 x 2
 * base tiles where the LDS accumulator of such an item fits), from the fused kernel's
 * time on every bin under each combination; only the work-item split of the stored rows
 * and their patch words change, never their values.  Then, unless the operator runs as
 * a layer-batched sweep (wf_set_sweep, whose item lists are rebuilt instead), the branch
 * count (1, 2, 4, and 8 when nchan >= 8).  reps timed runs per candidate (>= 1).
 * Synchronous; invalidates graphs captured earlier. */
wf_status wf_autotune(wf_op* op, const float* d_img, float* d_out, void* hip_stream,
                      int32_t reps, wf_tune_info* info);

/* Work-item tile side per bin of channel chan (tiles[P], cap >= P): the grid block that
 * one work item of the fused, gridding and de-gridding kernels covers -- the operator's
 * tile, or twice it (2 x 2 base tiles).  wf_set_bin_tiles sets them (each entry the
 * tile or twice the tile; twice the tile only where the LDS accumulator fits, and for
 * strategy (a) channels; n = P) and re-splits the channel's rows, keeping its rows per
 * item; synchronous, invalidates graphs captured earlier.  Results equal the
 * base-tile split up to the order of FP32 additions. */
wf_status wf_get_bin_tiles(const wf_op* op, int32_t chan, int32_t* tiles, int32_t cap);
wf_status wf_set_bin_tiles(wf_op* op, int32_t chan, const int32_t* tiles, int32_t n);

/* ------------------------------------------------------------------ forward-backward
 * The operator's consumer (Sect. 2, eq. 4): x <- D(x + gamma (x_dirty - Re{Phi^dag Phi x}))
 * with x_dirty = Re{Phi^dag y}, here with the non-learned denoiser D(z) = max(z - gamma
 * lambda, 0), the prox of lambda ||x||_1 under positivity.  Images are real FP32
 * [nchan][ny][nx] device buffers; the library keeps two work images of that size (and a
 * complex one for the dirty image), allocated on first use. */

/* x_dirty = Re{Phi^dag y}; d_vis complex FP32 [total rows].  Not for holographic
 * operators (WF_ENOTSUP). */
wf_status wf_dirty_image(wf_op* op, const float* d_vis, float* d_dirty, void* hip_stream);
/* Largest eigenvalue of x -> Re{Phi^dag Phi x}, by `iters` power iterations from the
 * normalised all-ones image (Rayleigh quotient of the last iterate, a lower bound);
 * gamma < 2 / norm makes eq. 4 convergent.  Synchronous. */
wf_status wf_op_norm(wf_op* op, int32_t iters, double* norm, void* hip_stream);
/* `iters` forward-backward iterations on d_x in place (asynchronous). */
wf_status wf_fb_iterate(wf_op* op, const float* d_dirty, float* d_x, int32_t iters,
                        double gamma, double lambda, void* hip_stream);

/* ------------------------------------------------------------------ learned kernels
 * Not in the paper.  A multilayer perceptron predicts the thresholded residual-w kernel
 * of Sect. 3.1 (the w-projection kernel built from the tapered chirp, Fig. 1) so that
 * the build of G can skip the exact construction where the network is accurate; the
 * exact construction is the fallback and the judge.
 *  Inputs (WF_MLP_IN per row, FP32): w_proj (o L)^2 / 4, L / (4 degrees in radians),
 *    the row's u and v offsets from its nearest grid cell (cells, [-1/2, 1/2)), n_k / 15
 *    with n_k the uncapped kernel side of the bandwidth rule; L = nx cell (square field).
 *  Outputs (WF_MLP_OUT per row, FP32): the kernel centred in a 15 x 15 window,
 *    row-major over (s_v, s_u), (re, im) per tap, then the predicted log10 of the
 *    relative L2 error of those 450 outputs.
 *  Network: 5 -> 4 hidden layers of 256 with exact GELU -> 451, trained in FP32 (Adam)
 *    by the library's matrix-core kernels; inference in BF16 with FP32 accumulation
 *    (first layer in FP32).  Flat parameters: per layer W [in][out] row-major, then b.
 *  Loss of a batch of B rows: (1/B) sum [ |p - t|^2 over the 450 kernel outputs +
 *    (e - log10(max(r, 1e-8)))^2 ], r = |p - t| / |t| held constant; the error output
 *    trains its own weights only.
 * All pointers named d_* are device memory of the network's device. */
#define WF_MLP_IN 5
#define WF_MLP_OUT 451

/* Create a network with seeded uniform(+-1/sqrt(fan_in)) weights and zero biases on the
 * current device. */
wf_status wf_mlp_create(uint64_t seed, wf_mlp** out);
wf_status wf_mlp_destroy(wf_mlp* m);
/* Number of parameters (314,819). */
int64_t wf_mlp_num_params(void);
/* Copy the flat FP32 parameters to / from host memory (n = wf_mlp_num_params()).
 * Setting them resets the Adam state.  Synchronous. */
wf_status wf_mlp_get_params(const wf_mlp* m, float* host, int64_t n);
wf_status wf_mlp_set_params(wf_mlp* m, const float* host, int64_t n);

/* Training inputs d_x [n][WF_MLP_IN] and uncapped kernel sides d_nk [n] (may be NULL)
 * for examples (d_w: w_proj in wavelengths, d_L: field side nx cell, d_fu, d_fv: cell
 * offsets), all FP64 [n]; opt supplies alpha and the oversampling (NULL: defaults). */
wf_status wf_mlp_inputs(const double* d_w, const double* d_L, const double* d_fu,
                        const double* d_fv, int64_t n, const wf_options* opt, float* d_x,
                        int32_t* d_nk, void* hip_stream);
/* Training targets d_t [n][450]: the exact thresholded kernels (the construction the
 * operator build uses), centred in the 15 x 15 window; zeros where n_k > 15. */
wf_status wf_mlp_targets(const double* d_w, const double* d_L, int64_t n,
                         const wf_options* opt, float* d_t, void* hip_stream);

/* Loss and gradient of one batch (batch <= 65536 rows of d_x, d_t): writes the two loss
 * terms to d_loss[2] and, if d_grad is not NULL, the flat gradient [num_params]. */
wf_status wf_mlp_loss_grad(wf_mlp* m, const float* d_x, const float* d_t, int32_t batch,
                           float* d_grad, float* d_loss, void* hip_stream);
/* One Adam step (b1 0.9, b2 0.999, eps 1e-8) with the gradient of the last
 * wf_mlp_loss_grad call. */
wf_status wf_mlp_adam_step(wf_mlp* m, float lr, void* hip_stream);
/* Train over n examples for `epochs` epochs of floor(n / batch) minibatches each (a
 * seeded SplitMix64 shuffle per epoch), learning rate cosine-annealed from lr0 to
 * lr_end.  d_hist (may be NULL) receives per epoch the sums over its minibatches of the
 * two loss terms, [epochs][2].  Asynchronous on hip_stream apart from the shuffles. */
wf_status wf_mlp_train(wf_mlp* m, const float* d_x, const float* d_t, int64_t n,
                       int32_t batch, int32_t epochs, double lr0, double lr_end,
                       uint64_t seed, float* d_hist, void* hip_stream);
/* Outputs d_out [n][WF_MLP_OUT] for inputs d_x [n][WF_MLP_IN].  bf16 = 0: the FP32
 * training kernels; 1: the BF16 inference kernel with plain BF16 operands (relative
 * output error near 1e-3); 2: the BF16 inference kernel with split operands (high part
 * + BF16 residual, three BF16 products per step, FP32-level error) -- the form the
 * operator build uses. */
wf_status wf_mlp_infer(wf_mlp* m, const float* d_x, int64_t n, int32_t bf16,
                       float* d_out, void* hip_stream);

/* Release all device and host memory of the handle (synchronises its device). */
wf_status wf_destroy(wf_op* op);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* wf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WF_H */
