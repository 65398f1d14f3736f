/*
 * CPU oracle for Aggregate Risk Analysis -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, float64 implementation of the trial pass of Varghese &
 * Barker, "Are Clouds Ready to Accelerate Ad hoc Financial Simulations?"
 * (Section III, Algorithm 1 and the four-step description that follows it).
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library; the product path never does.  It shares no code with
 * the GPU library.
 *
 * What it computes, per layer and per trial i of the YET (Section III):
 *   step 1  look up each event E of the trial in every ELT j of the layer;
 *           an event absent from an ELT has loss 0 (the direct-access table
 *           of Section IV holds zero for absent events);
 *   step 2  apply the ELT's terms FT1 = (retention r_j, limit u_j) as
 *           x_j = min(max(l_j - r_j, 0), u_j), and add the x_j over the ELTs
 *           of the layer, in layer order, into one event loss e
 *           (secondary uncertainty is taken as the identity);
 *   step 3  apply the occurrence terms FT2 to every event occurrence on its
 *           own: o = min(max(e - FT2_1, 0), FT2_2);
 *   step 4  add the o's in the trial's stored (time) order into the running
 *           aggregate S and apply the aggregate terms FT3 to it:
 *           A = min(max(S - FT3_1, 0), FT3_2).
 *   The year loss of the trial (its YLT entry) is A after the last event; an
 *   empty trial has year loss 0.  The optional per-event output is the
 *   increment of A that each occurrence causes, A_k - A_{k-1} with A_0 = 0:
 *   the part of the aggregate-net loss attributed to the k-th event, which
 *   is the quantity that depends on the order of prior events; the other
 *   optional per-event output is S itself after each event.
 *   The optional per-trial output occ_max is the largest occurrence loss o
 *   of the trial (0 for an empty trial): the loss on an occurrence basis,
 *   from which occurrence-basis PML/TVaR and return period losses follow
 *   the same way as from the YLT (the paper names return period losses
 *   among the reports derived from the analysis, Section III, without
 *   naming their basis: taking the per-trial largest occurrence loss as the
 *   occurrence basis is a reading).
 *
 * Readings of points the paper leaves open: the printed FT2/FT3 formulas
 * give max(.) a single argument, read as max(x - retention, 0); the event
 * loss is reset for every event (the text applies the occurrence terms to
 * each occurrence independently); FT1 is a retention/limit pair of the same
 * form as FT2/FT3.
 *
 * Lookups use one dense direct-access table per ELT (catalogue-sized, zero
 * for absent events), as the paper's implementations do (Section IV, data
 * structures).  Compile without fused multiply-add contraction.
 *
 * Status codes: 0 ok, -1 bad argument, -2 event ID outside the catalogue,
 * -3 duplicate event ID inside one ELT, -5 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double clamp_excess(double x, double retention, double limit)
{
    /* min(max(x - retention, 0), limit) */
    double v = x - retention;
    if (v < 0.0) v = 0.0;
    if (v > limit) v = limit;
    return v;
}

int oracle_run_layer(const int32_t *event_ids,      /* [n_events] */
                     const int64_t *offsets,        /* [n_trials+1] or NULL */
                     int64_t n_trials, int64_t events_per_trial,
                     int32_t catalog_size, int32_t n_elts,
                     const int32_t *elt_ids,        /* concatenated ELT event IDs */
                     const double *elt_losses,      /* concatenated ELT losses */
                     const int64_t *elt_sizes,      /* [n_elts] */
                     const double *ret, const double *lim,   /* FT1 per ELT */
                     double occ_ret, double occ_lim,         /* FT2 */
                     double agg_ret, double agg_lim,         /* FT3 */
                     int n_threads,
                     double *ylt,                   /* [n_trials] year losses */
                     double *occ_sum,               /* [n_trials] S before FT3, or NULL */
                     double *gross,                 /* [n_trials] sum of looked-up losses, or NULL */
                     double *event_cum,             /* [n_events] S after event k, or NULL */
                     double *event_net,             /* [n_events] A_k - A_{k-1}, or NULL */
                     double *occ_max)               /* [n_trials] largest o of the trial, or NULL */
{
    if (n_trials < 0 || n_elts < 0 || catalog_size < 0) return -1;
    if (!offsets && events_per_trial < 0) return -1;

    /* Pre-processing stage: one direct-access table per ELT. */
    size_t C = (size_t)catalog_size;
    double *table = NULL;
    if (n_elts > 0 && C > 0) {
        table = (double *)calloc((size_t)n_elts * C, sizeof(double));
        if (!table) return -5;
    }
    unsigned char *seen = (unsigned char *)calloc(C ? C : 1, 1);
    if (!seen) { free(table); return -5; }
    int64_t pos = 0;
    for (int32_t j = 0; j < n_elts; ++j) {
        memset(seen, 0, C ? C : 1);
        for (int64_t n = 0; n < elt_sizes[j]; ++n, ++pos) {
            int32_t e = elt_ids[pos];
            if (e < 0 || (size_t)e >= C) { free(table); free(seen); return -2; }
            if (seen[e]) { free(table); free(seen); return -3; }
            seen[e] = 1;
            table[(size_t)j * C + (size_t)e] = elt_losses[pos];
        }
    }
    free(seen);

    int bad = 0;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads) reduction(| : bad)
#endif
    for (int64_t i = 0; i < n_trials; ++i) {
        int64_t begin = offsets ? offsets[i] : i * events_per_trial;
        int64_t end = offsets ? offsets[i + 1] : (i + 1) * events_per_trial;
        double S = 0.0, G = 0.0, A_prev = 0.0, M = 0.0;
        for (int64_t k = begin; k < end; ++k) {
            int32_t E = event_ids[k];
            if (E < 0 || (size_t)E >= C) { bad = 1; break; }
            /* steps 1-2: lookup, per-ELT terms, accumulate across ELTs */
            double e = 0.0;
            for (int32_t j = 0; j < n_elts; ++j) {
                double l = table[(size_t)j * C + (size_t)E];
                G += l;
                e += clamp_excess(l, ret[j], lim[j]);
            }
            /* step 3: occurrence terms */
            double o = clamp_excess(e, occ_ret, occ_lim);
            if (o > M) M = o;
            /* step 4: cumulative sum within the trial, aggregate terms */
            S += o;
            if (event_cum) event_cum[k] = S;
            if (event_net) {
                double A = clamp_excess(S, agg_ret, agg_lim);
                event_net[k] = A - A_prev;
                A_prev = A;
            }
        }
        ylt[i] = clamp_excess(S, agg_ret, agg_lim);
        if (occ_sum) occ_sum[i] = S;
        if (gross) gross[i] = G;
        if (occ_max) occ_max[i] = M;
    }
    free(table);
    return bad ? -2 : 0;
}

int oracle_version(void) { return 2; }
