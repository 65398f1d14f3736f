/*
 * ara.h -- C ABI of the MI355X (gfx950) Aggregate Risk Analysis trial pass.
 *
 * The operation is the per-layer, per-trial simulation of Varghese & Barker,
 * "Are Clouds Ready to Accelerate Ad hoc Financial Simulations?", Section III
 * (the YET / ELT / Layer data model, Algorithm 1 and its four steps):
 *
 *   for every trial i of the Year Event Table (YET), for every event E of the
 *   trial in stored (time) order:
 *     l_j  = loss of E in ELT j of the layer, 0 if E is not in ELT j
 *     x_j  = min(max(l_j - r_j, 0), u_j)             per-ELT terms FT1
 *     e    = x_0 + x_1 + ... + x_{J-1}                combined event loss
 *     o    = min(max(e - FT2_1, 0), FT2_2)            occurrence terms FT2
 *     S   += o                                        cumulative loss of the trial
 *   YLT[i] = min(max(S - FT3_1, 0), FT3_2)            aggregate terms FT3
 *
 * Risk metrics read from the YLT (the paper names them without a formula):
 * for a return period of N years over T trials, k = floor(T / N) >= 1,
 * PML_N is the k-th largest year loss and TVaR_N the mean of the k largest.
 *
 * Conventions for every entry point:
 *   - Every function returns ara_status: ARA_OK (0) or a negative error code.
 *     Nothing throws across this boundary.  ara_last_error() returns a
 *     message for the last failing call on the calling thread.
 *   - "d_" pointers are device pointers (HIP device memory of the current
 *     device); "h_" pointers are host pointers.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Launches are asynchronous on that stream unless stated otherwise.
 *   - All floating-point outputs are IEEE binary64.
 *   - Host threads: calls may come from several threads at once, with two
 *     exceptions: a batch handle is used by one thread at a time, and no
 *     handle is destroyed while another call still uses it.  The library's
 *     per-device state (launch attributes, its set-up stream, the PML/TVaR
 *     scratch, whose calls on one device run one after another) is guarded.
 */
#ifndef ARA_H
#define ARA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ara_status;

#define ARA_OK 0
#define ARA_ERR_INVALID_ARG -1  /* null handle/pointer, bad size, bad enum */
#define ARA_ERR_EVENT_RANGE -2  /* an event ID outside [0, catalog_size) */
#define ARA_ERR_DUP_EVENT -3    /* the same event ID twice in one ELT (an ELT is a dictionary) */
#define ARA_ERR_VALUE -4        /* NaN, negative loss or term, or infinite retention/loss */
#define ARA_ERR_OOM -5          /* device or host allocation failed; no state was changed */
#define ARA_ERR_DEVICE -6       /* a HIP call failed */
#define ARA_ERR_RP -7           /* a return period leaves no tail trial (floor(T/N) < 1) */
#define ARA_ERR_UNSUPPORTED -8  /* a valid request the library does not handle (e.g. too many ELTs) */

#define ARA_MAX_ELTS 32         /* ELTs per layer; the paper's layers cover 3 to 30 */
#define ARA_MAX_BATCH 64        /* layers per batch, YLTs per ara_pml_tvar_many call */

typedef struct ara_yet_s *ara_yet;
typedef struct ara_layer_s *ara_layer;

/* Arithmetic of the trial pass.
 *   ARA_FP64  : losses, terms and sums in binary64.
 *   ARA_FP32C : losses and per-ELT / occurrence terms stored and applied in
 *               binary32; the cross-ELT sum and the per-trial cumulative sum
 *               are compensated binary32 (TwoSum pairs); the aggregate terms
 *               and the YLT are binary64.  (Section IV's single-precision
 *               optimisation, with compensated accumulation added.) */
typedef enum { ARA_FP64 = 0, ARA_FP32C = 1 } ara_precision;

/* Device layout of a layer's ELTs (Section IV discusses direct-access versus
 * compact tables).
 *   ARA_LAYOUT_DIRECT  : one dense catalogue-sized table per ELT, ELT-major
 *                        ([J][catalog]); J loads per event (the paper's choice).
 *   ARA_LAYOUT_SPARSE  : per-ELT event IDs sorted ascending with their losses;
 *                        a binary search per ELT per event.
 *   ARA_LAYOUT_COMPACT : a presence bitmap over the catalogue with per-word
 *                        ranks, and one row of J losses per event present in
 *                        any ELT of the layer (event-major).
 *   ARA_LAYOUT_FUSED   : the occurrence loss of every catalogue event,
 *                        o(E) = FT2(sum_j FT1_j(l_j(E))), computed once when
 *                        the layer is built (steps 1-3 depend on the event
 *                        only, not on the trial: occurrence terms apply to
 *                        each occurrence independently of the others), kept
 *                        as a catalogue-sized table, plus a bitmap of the
 *                        blocks of events whose o is non-zero that the trial
 *                        pass holds in LDS.  Same arithmetic, same order.
 *   ARA_LAYOUT_AUTO    : the library's choice (currently FUSED).
 * Every layout gives bitwise the same YLT for the same precision. */
typedef enum {
    ARA_LAYOUT_AUTO = 0,
    ARA_LAYOUT_DIRECT = 1,
    ARA_LAYOUT_SPARSE = 2,
    ARA_LAYOUT_COMPACT = 3,
    ARA_LAYOUT_FUSED = 4
} ara_layout;

/* Register a device-resident YET (Section III: trials of event IDs ordered by
 * time stamp; the time stamps themselves are not needed, only the order).
 *   d_event_ids     int32 [n_events], BORROWED: must stay valid and unchanged
 *                   until ara_destroy_yet.  16-byte alignment is faster but
 *                   not required.
 *   d_offsets       int64 [n_trials + 1] trial boundaries, d_offsets[0] == 0,
 *                   non-decreasing; trial i is d_event_ids[off[i] .. off[i+1]).
 *                   BORROWED like the IDs.  NULL means every trial holds
 *                   events_per_trial events (n_events = n_trials * events_per_trial).
 *   catalog_size    number of possible event IDs (1 .. 2^31-1).
 * Validates (one device pass, synchronous on hip_stream) that every ID lies in
 * [0, catalog_size) -> ARA_ERR_EVENT_RANGE, and that offsets are well formed
 * -> ARA_ERR_INVALID_ARG.  On success *out receives a handle owned by the
 * caller (free with ara_destroy_yet). */
ara_status ara_create_yet(const int32_t *d_event_ids, const int64_t *d_offsets, int64_t n_trials,
                          int64_t events_per_trial, int32_t catalog_size, void *hip_stream, ara_yet *out);

/* Build one layer (Section III: a set of ELTs with their FT1 terms, plus the
 * occurrence terms FT2 and aggregate terms FT3) in device memory.
 *   n_elts          1 .. ARA_MAX_ELTS, the ELTs in layer order (the order of
 *                   the cross-ELT sum).
 *   h_elt_ids       int32, all ELTs' event IDs concatenated in layer order;
 *                   ELT j has h_elt_sizes[j] entries (0 allowed), each in
 *                   [0, catalog_size) of the YET and unique within the ELT.
 *   h_elt_losses    binary64 losses, same layout; finite and >= 0.
 *   h_ret, h_lim    FT1 per ELT: retention (finite, >= 0) and limit (>= 0,
 *                   +INFINITY for none).
 *   occ_ret/occ_lim FT2 occurrence retention (finite, >= 0) / limit (>= 0 or +INF).
 *   agg_ret/agg_lim FT3 aggregate retention (finite, >= 0) / limit (>= 0 or +INF).
 *   precision       ara_precision; layout: ara_layout.
 * All host inputs are COPIED; the caller may free them on return.  Device
 * memory is owned by the layer until ara_destroy_layer.  The FUSED layout
 * stages the ELTs in a device buffer of the library (one per device, grown
 * to the largest layer's ELT bytes, plus 4 bytes per catalogue event for
 * FP32C, and kept until the process ends).  Synchronous.
 * Errors: ARA_ERR_INVALID_ARG, ARA_ERR_EVENT_RANGE, ARA_ERR_DUP_EVENT,
 * ARA_ERR_VALUE, ARA_ERR_UNSUPPORTED (n_elts > ARA_MAX_ELTS), ARA_ERR_OOM. */
ara_status ara_create_layer(ara_yet yet, int32_t n_elts, const int32_t *h_elt_ids, const double *h_elt_losses,
                            const int64_t *h_elt_sizes, const double *h_ret, const double *h_lim,
                            double occ_ret, double occ_lim, double agg_ret, double agg_lim,
                            int32_t precision, int32_t layout, ara_layer *out);

/* The trial pass of one layer over the whole YET (Algorithm 1 for one
 * layer): writes d_ylt[i] for every trial i.
 *   d_ylt   binary64 [n_trials], caller-owned device memory.
 * Asynchronous on hip_stream.  The result is deterministic: the same inputs
 * give bitwise the same YLT on every call. */
ara_status ara_run_layer(ara_yet yet, ara_layer layer, double *d_ylt, void *hip_stream);

/* The trial pass with per-event outputs (Section III: aggregate terms act on
 * the cumulative sum of occurrence losses, so the share of each occurrence in
 * the aggregate-net loss depends on the events before it).
 *   d_ylt        binary64 [n_trials] as in ara_run_layer (required).
 *   d_event_cum  binary64 [n_events] or NULL: S_k, the cumulative occurrence
 *                loss of the trial up to and including event k.
 *   d_event_net  binary64 [n_events] or NULL: A_k - A_{k-1} with
 *                A_k = min(max(S_k - FT3_1, 0), FT3_2), A_0 = 0; the
 *                increments of a trial add up to its year loss.
 * Per-event arrays are indexed like the YET's event IDs.  Asynchronous. */
ara_status ara_run_layer_events(ara_yet yet, ara_layer layer, double *d_ylt, double *d_event_cum,
                                double *d_event_net, void *hip_stream);

/* The trial pass with the loss on an occurrence basis as well: the largest
 * occurrence loss of each trial (the event losses net of the occurrence
 * terms, Section III step 3; 0 for an empty trial).  PML, TVaR and return
 * period losses on the occurrence basis follow from it with ara_pml_tvar as
 * they do from the YLT on the aggregate basis (Section III names these
 * metrics and return period losses as products of the analysis).
 *   d_ylt      binary64 [n_trials] as in ara_run_layer (required).
 *   d_max_occ  binary64 [n_trials], caller-owned device memory (required).
 * With ARA_FP64 layers d_max_occ holds exactly the largest of the binary64
 * occurrence losses; with ARA_FP32C, the largest binary32 one.  The YLT is
 * bitwise the one of ara_run_layer.  Asynchronous on hip_stream. */
ara_status ara_run_layer_max_occurrence(ara_yet yet, ara_layer layer, double *d_ylt, double *d_max_occ,
                                        void *hip_stream);

/* Several layers over one YET in one pass (Algorithm 1's loop over the
 * layers of a program, with the YET read once for all of them).
 *
 * A batch of up to 16 layers holds, per group of at most 4 of its layers
 * and per catalogue event, one dense record of the event's occurrence losses
 * in those layers, and LDS filters of the events with any non-zero loss:
 * one pass over the YET per group of 4 layers, gathering a record only for
 * events that pass the filters.  A larger batch, or a small one whose
 * groups' non-zero events cover too much of the catalogue for that to pay,
 * holds one 64-byte (FP64) or 32-byte (FP32C) record per catalogue event of
 * the layers in which its occurrence loss is non-zero and those losses, and
 * reads one record per trial-event in a single pass.  Either way the pass keeps one running sum
 * per (layer, lane), adding each layer's losses in the same order as the
 * single-layer pass.
 *   layers    1 .. ARA_MAX_BATCH layer handles, all built against this YET
 *             with ARA_LAYOUT_FUSED (or AUTO) and the same precision
 *             (else ARA_ERR_UNSUPPORTED / ARA_ERR_INVALID_ARG).  The batch
 *             copies what it needs: the layers may be destroyed afterwards.
 * ara_create_batch is synchronous; the batch owns its device memory.
 * ara_run_batch writes d_ylts[l] (binary64 [n_trials], caller-owned) for
 * every layer l of the batch; each is bitwise the YLT ara_run_layer gives
 * for that layer.  The launch shape (work-group size, work-groups per CU
 * and the number of 256-event chunks loaded per step) is chosen on the first
 * run by timing candidates (and remembered per precision, power-of-two layer
 * count or record width, and YET), then the pass is replayed from a HIP
 * graph captured once.  A capture that fails (a capture can be invalidated
 * from outside, e.g. by a synchronizing call another host thread makes
 * meanwhile) costs nothing but the graph: that run launches the pass directly, the next
 * run captures again, and after three failures in a row the batch launches
 * directly from then on.
 * Asynchronous on hip_stream. */
typedef struct ara_batch_s *ara_batch;
ara_status ara_create_batch(ara_yet yet, const ara_layer *layers, int32_t n_layers, ara_batch *out);
ara_status ara_run_batch(ara_batch batch, double *const *d_ylts, void *hip_stream);
size_t ara_batch_device_bytes(ara_batch batch);
/* Rebuild a batch's records for other layers (same YET and precision),
 * reusing its device memory (the overflow area grows when the new layers
 * need more entries).  Synchronous.  It first waits for the batch's last
 * ara_run_batch, on whatever stream that run was queued, so the caller need
 * not synchronise before it.  A captured graph is replayed only while the
 * tables it was captured with are unchanged (it is captured again after a
 * rebuild that moved them); once rebuilt with another number of layers, the
 * batch launches its pass directly instead (a server's batches change size
 * all the time).  A run queued on another stream than the batch's previous
 * run waits for that run.  After a failed rebuild the batch holds no valid
 * records: ara_run_batch returns ARA_ERR_INVALID_ARG until a rebuild
 * succeeds. */
ara_status ara_batch_rebuild(ara_batch batch, const ara_layer *layers, int32_t n_layers);
/* Launch shape chosen for the batch (0, 0 before its first run). */
ara_status ara_batch_launch_config(ara_batch batch, int32_t *threads, int32_t *wg_per_cu);
/* Number of 256-event chunks of a trial the batch's pass loads per step
 * (2, 4 or 8; for a dense batch, that of its first group of 4 layers), or
 * 1 for the pipelined record pass (one chunk per step, each chunk's ID,
 * record and overflow loads issued over the three steps before its sums),
 * chosen with the launch shape by timing candidates on the first run (0
 * before it).  The environment variable ARA_BATCH_LAUNCH =
 * "threads,wg_per_cu,group" forces a shape for the sparse record pass
 * (not remembered for later batches). */
ara_status ara_batch_launch_group(ara_batch batch, int32_t *group);
void ara_destroy_batch(ara_batch batch);

/* One-shot form: ara_create_batch + ara_run_batch + ara_destroy_batch
 * (synchronous; n_layers up to ARA_MAX_BATCH). */
ara_status ara_run_layers(ara_yet yet, const ara_layer *layers, double *const *d_ylts, int32_t n_layers,
                          void *hip_stream);

/* PML and TVaR of a YLT for n_rp return periods (years, > 0).  The paper
 * names Probable Maximum Loss and Tail Value-at-Risk as the risk metrics
 * derived from the YLT (Sections I and III) without defining them; here, on
 * the YLT's (aggregate) basis or on any per-trial loss array such as the
 * largest occurrence losses:
 *   d_ylt              binary64 [n_trials] device memory, n_trials in 1 .. 2^31-1,
 *                      no NaN (-> ARA_ERR_VALUE).
 *   h_return_periods   host [n_rp], 1 <= n_rp <= 16.
 *   h_pml, h_tvar      host [n_rp] outputs.
 * k = floor(n_trials / N) must be >= 1 (else ARA_ERR_RP).  PML is exactly the
 * k-th largest entry; TVaR is the binary64 mean of the k largest entries.
 * SYNCHRONOUS: returns once the results are on the host. */
ara_status ara_pml_tvar(const double *d_ylt, int64_t n_trials, const double *h_return_periods, int32_t n_rp,
                        double *h_pml, double *h_tvar, void *hip_stream);

/* A pool of ELTs resident on the device, from which layers are built on the
 * GPU (for ad hoc queries against a resident YET, the use the paper
 * motivates in Section I with real-time pricing: the ELTs are loaded once,
 * each query picks some of them and brings its own terms).
 *   h_elt_ids / h_elt_losses / h_elt_sizes  as for ara_create_layer (COPIED).
 *   precision   of every layer built from the pool.
 *   max_layers  number of layers from this pool that may exist at once; the
 *               pool allocates their fused tables up front ((catalog + 1)
 *               values + LDS filter each, plus a binary32 scratch of catalog
 *               entries for FP32C), which is the memory budget a server
 *               admits queries against.
 * Synchronous. */
typedef struct ara_pool_s *ara_pool;
ara_status ara_create_pool(ara_yet yet, int32_t n_elts, const int32_t *h_elt_ids, const double *h_elt_losses,
                           const int64_t *h_elt_sizes, int32_t precision, int32_t max_layers, ara_pool *out);
void ara_destroy_pool(ara_pool pool);  /* waits for the device; destroy the pool's layers first */
size_t ara_pool_device_bytes(ara_pool pool);
int32_t ara_pool_free_slots(ara_pool pool);  /* layer slots free now, -1 for NULL */

/* A fused layer (ARA_LAYOUT_FUSED, the pool's precision) of pool ELTs
 * h_elt_index[0 .. n_elts) in that order, with the given terms (as for
 * ara_create_layer).  Built on the GPU, ASYNCHRONOUSLY on hip_stream: work on
 * other streams through this library waits for the build.  Returns
 * ARA_ERR_OOM, with nothing changed, when every slot of the pool is taken.
 * ara_destroy_layer returns the slot at once, without waiting for the device:
 * the caller destroys such a layer only when no queued work still reads it
 * (or when that work is ordered before the slot's next build, e.g. on the
 * same stream).  The YLT is bitwise the one of the same layer built by
 * ara_create_layer. */
ara_status ara_create_layer_from_pool(ara_pool pool, int32_t n_elts, const int32_t *h_elt_index, const double *h_ret,
                                      const double *h_lim, double occ_ret, double occ_lim, double agg_ret,
                                      double agg_lim, void *hip_stream, ara_layer *out);

/* PML and TVaR of n_ylts YLTs of the same length at once (as ara_pml_tvar
 * for each): h_pml / h_tvar are [n_ylts][n_rp] row-major.  1 <= n_ylts <=
 * ARA_MAX_BATCH.  SYNCHRONOUS. */
ara_status ara_pml_tvar_many(const double *const *d_ylts, int32_t n_ylts, int64_t n_trials,
                             const double *h_return_periods, int32_t n_rp, double *h_pml, double *h_tvar,
                             void *hip_stream);

/* PML and TVaR as ara_pml_tvar_many, for callers that cannot allocate
 * memory or wait for the device (code being captured into a HIP graph, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same results, bitwise, but every scratch buffer lives in a static device
 * array of the library (about 2 MiB per GPU, held until the process ends)
 * and the results stay on the device.
 *   d_ylts, n_ylts, n_trials, h_return_periods, n_rp   as ara_pml_tvar_many,
 *               with n_ylts * n_rp <= ARA_NOALLOC_MAX_SEL (else
 *               ARA_ERR_UNSUPPORTED, nothing launched).
 *   d_pml, d_tvar   caller-owned device binary64 [n_ylts][n_rp], row-major;
 *               they must not overlap the YLTs.  A YLT holding NaN gets NaN
 *               for its PML and TVaR (the call cannot return ARA_ERR_VALUE:
 *               it does not wait for the device).
 * ASYNCHRONOUS on hip_stream; no device or host allocation, no memset node,
 * no synchronisation.  Every call on one GPU uses the same scratch: calls
 * whose work overlaps on the device (e.g. queued on two streams without an
 * order between them) race and give undefined results; calls ordered on one
 * stream are safe: a call that runs to its end leaves the scratch's flags
 * and histograms at zero for the next one (the first call on a device, and
 * a call after one that failed between its launches, clears them first).
 * Errors: as ara_pml_tvar_many, detected on the host before any launch. */
#define ARA_NOALLOC_MAX_SEL 128
ara_status ara_pml_tvar_many_noalloc(const double *const *d_ylts, int32_t n_ylts, int64_t n_trials,
                                     const double *h_return_periods, int32_t n_rp, double *d_pml, double *d_tvar,
                                     void *hip_stream);

/* Roll-up of year loss tables into programs, or of programs into a
 * portfolio.  Section III nests layers in programs and programs in a
 * portfolio and leaves their combination unstated; the reading here: group
 * g's year loss in a trial is the binary64 sum of the year losses in that
 * trial of the inputs l with h_group[l] == g, added in increasing l starting
 * from 0 (a group without inputs gets zeros).  Rolling the program tables up
 * again with every h_group entry 0 gives the portfolio.
 *   d_ylts    n_inputs device pointers to binary64 [n_trials] tables,
 *             1 <= n_inputs <= ARA_MAX_BATCH.
 *   h_group   host [n_inputs], each in 0 .. n_groups-1.
 *   n_groups  1 .. ARA_MAX_BATCH.
 *   n_trials  0 .. 2^31-1 (0: nothing to do; the table pointers may then be NULL).
 *   d_out     n_groups caller-owned device pointers to binary64 [n_trials];
 *             no output may overlap an input or another output
 *             (ARA_ERR_INVALID_ARG).
 * ASYNCHRONOUS on hip_stream; the inputs are read once. */
ara_status ara_rollup(const double *const *d_ylts, int32_t n_inputs, const int32_t *h_group, int32_t n_groups,
                      int64_t n_trials, double *const *d_out, void *hip_stream);

/* Device bytes a layer holds (for memory admission). */
size_t ara_layer_device_bytes(ara_layer layer);

/* Layout a layer was built with (after resolving ARA_LAYOUT_AUTO), its
 * precision and its ELT count, or -1 for a NULL handle. */
int32_t ara_layer_layout(ara_layer layer);
int32_t ara_layer_precision(ara_layer layer);
int32_t ara_layer_n_elts(ara_layer layer);

/* Free a handle (NULL is ignored).  Waits for the device to finish any work
 * that may still use it.  A YET must outlive the layers run against it. */
void ara_destroy_layer(ara_layer layer);
void ara_destroy_yet(ara_yet yet);

/* Message of the last non-OK status returned on the calling thread. */
const char *ara_last_error(void);

/* ABI version of this header: 1. */
int32_t ara_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ARA_H */
