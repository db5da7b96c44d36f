/*
 * CPU oracle for the SVT linearized track fit -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct nested loops.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load this library; the
 * product path never calls it.  It shares no code, header or table with the
 * HIP library.
 *
 * What it computes (paper Sec. 2 and Sec. 2.1):
 *   - for every event, every road, every combination of one hit per layer
 *     (three nested loops: events, roads, combinations -- Sec. 2.1);
 *   - the linearized fit of Sec. 2, p_i = f_i . x + q_i, for all six rows of
 *     the sector's constant set: rows 0..2 are the track words (d0, phi,
 *     curvature), rows 3..5 the chi2 constraint components;
 *   - chi2 = y3^2 + y4^2 + y5^2 with integer additions and multiplications
 *     only (Sec. 2);
 *   - the chi2 cut (chi2 <= cut passes) and the best passing combination per
 *     road: smallest chi2, ties to the lowest combination index;
 *   - optionally the list of every passing combination (orc_list_passing).
 * Readings where the paper is silent: the fit input is one combination
 * x = (h0[i0], h1[i1], h2[i2], h3[i3], xft0, xft1); combinations are counted
 * lexicographically with layer 0 most significant; no shift or rounding is
 * applied anywhere (y exact in int32, chi2 exact in uint64).
 *
 * Accumulation is done in int64 and every fit row is asserted to fit int32
 * (the constant loader enforces the bound that guarantees it).
 */
#include <stdint.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_OK = 0, ORC_E_INVAL = -1, ORC_E_RANGE = -2 };

typedef struct {
    int64_t total_comb;
    int64_t total_pass;
    int32_t total_tracks;
    int32_t err_road;
    int32_t err_event;
    int32_t pad;
} orc_summary;

/* Bound that makes every fit row exact in int32: for every sector s and row k,
 * sum_j |A[s][k][j]| * 4095 + |b[s][k]| <= 2^31 - 1; the chi2 cut < 2^48. */
int orc_check_constants(int32_t n_sectors, const int32_t *coef, const int32_t *offset,
                        uint64_t chi2_cut)
{
    if (n_sectors < 1 || n_sectors > 256 || coef == NULL || offset == NULL)
        return ORC_E_INVAL;
    if (chi2_cut >= ((uint64_t)1 << 48))
        return ORC_E_RANGE;
    for (int s = 0; s < n_sectors; ++s) {
        for (int k = 0; k < 6; ++k) {
            int64_t bound = llabs((long long)offset[s * 6 + k]);
            for (int j = 0; j < 6; ++j)
                bound += llabs((long long)coef[(s * 6 + k) * 6 + j]) * 4095;
            if (bound > 2147483647LL)
                return ORC_E_RANGE;
        }
    }
    return ORC_OK;
}

static int bad_event(int32_t e, int32_t n_events, int32_t n_roads, const int32_t *ro)
{
    if (ro[e] < 0 || ro[e + 1] < ro[e] || ro[e + 1] > n_roads)
        return 1;
    if (e == 0 && ro[0] != 0)
        return 1;
    if (e == n_events - 1 && ro[n_events] != n_roads)
        return 1;
    return 0;
}

static int bad_road(int32_t r, int32_t n_roads, int32_t n_hits, int32_t n_sectors,
                    const uint8_t *sector, const uint8_t *nhits, const int32_t *hoff,
                    const int16_t *hits, const int16_t *xft)
{
    if (sector[r] >= n_sectors)
        return 1;
    int64_t total = 0;
    for (int l = 0; l < 4; ++l) {
        if (nhits[r * 4 + l] > 16)
            return 1;
        total += nhits[r * 4 + l];
    }
    if (hoff[r] < 0 || hoff[r + 1] > n_hits || (int64_t)hoff[r + 1] - hoff[r] != total)
        return 1;
    if (r == 0 && hoff[0] != 0)
        return 1;
    if (r == n_roads - 1 && hoff[n_roads] != n_hits)
        return 1;
    for (int i = 0; i < 2; ++i)
        if (xft[r * 2 + i] < 0 || xft[r * 2 + i] >= 4096)
            return 1;
    for (int32_t h = hoff[r]; h < hoff[r + 1]; ++h)
        if (hits[h] < 0 || hits[h] >= 4096)
            return 1;
    return 0;
}

/* One road: every combination, the six fit rows, chi2, cut, best. */
static void fit_road(int32_t r, const uint8_t *sector, const uint8_t *nhits, const int32_t *hoff,
                     const int16_t *hits, const int16_t *xft, const int32_t *coef,
                     const int32_t *offset, uint64_t cut, int32_t *ncomb, int32_t *npass,
                     int32_t *best, uint64_t *chi2, int32_t *params, uint8_t *hit_index)
{
    const int s = sector[r];
    const int n0 = nhits[r * 4 + 0], n1 = nhits[r * 4 + 1];
    const int n2 = nhits[r * 4 + 2], n3 = nhits[r * 4 + 3];
    /* layer-major hit lists */
    const int16_t *h0 = hits + hoff[r];
    const int16_t *h1 = h0 + n0;
    const int16_t *h2 = h1 + n1;
    const int16_t *h3 = h2 + n2;
    const int32_t *A = coef + s * 36;
    const int32_t *b = offset + s * 6;

    int32_t np = 0, bk = -1, k = 0;
    uint64_t bchi = UINT64_MAX;
    int32_t bp[3] = {0, 0, 0};
    uint8_t bh[4] = {0xFF, 0xFF, 0xFF, 0xFF};

    for (int i0 = 0; i0 < n0; ++i0)
        for (int i1 = 0; i1 < n1; ++i1)
            for (int i2 = 0; i2 < n2; ++i2)
                for (int i3 = 0; i3 < n3; ++i3, ++k) {
                    const int64_t x[6] = {h0[i0], h1[i1], h2[i2], h3[i3],
                                          xft[r * 2 + 0], xft[r * 2 + 1]};
                    int64_t y[6];
                    for (int row = 0; row < 6; ++row) {
                        int64_t acc = b[row];
                        for (int j = 0; j < 6; ++j)
                            acc += (int64_t)A[row * 6 + j] * x[j];
                        if (acc < INT32_MIN || acc > INT32_MAX) {
                            fprintf(stderr, "oracle: fit row outside int32\n");
                            abort();
                        }
                        y[row] = acc;
                    }
                    const uint64_t c2 = (uint64_t)(y[3] * y[3]) + (uint64_t)(y[4] * y[4]) +
                                        (uint64_t)(y[5] * y[5]);
                    if (c2 <= cut) {
                        ++np;
                        if (c2 < bchi) {
                            bchi = c2;
                            bk = k;
                            bp[0] = (int32_t)y[0];
                            bp[1] = (int32_t)y[1];
                            bp[2] = (int32_t)y[2];
                            bh[0] = (uint8_t)i0;
                            bh[1] = (uint8_t)i1;
                            bh[2] = (uint8_t)i2;
                            bh[3] = (uint8_t)i3;
                        }
                    }
                }
    ncomb[r] = n0 * n1 * n2 * n3;
    npass[r] = np;
    best[r] = bk;
    chi2[r] = bchi;
    memcpy(params + r * 3, bp, sizeof bp);
    memcpy(hit_index + r * 4, bh, sizeof bh);
}

/*
 * Fit a batch.  Layout: CSR events -> roads -> hits (see the HIP library's
 * header for the same contract stated independently).  Returns ORC_OK,
 * ORC_E_INVAL (malformed call) or ORC_E_RANGE (malformed data; the lowest
 * offending road / event go to the summary, results are then unspecified).
 * n_threads > 1 parallelizes the event loop with OpenMP (one event per task,
 * the event-parallel scheme the paper used on the many-core card).
 */
int orc_fit(int32_t n_events, int32_t n_roads, int32_t n_hits,
            const int32_t *road_offsets, const uint8_t *sector, const uint8_t *nhits,
            const int32_t *hit_offsets, const int16_t *hits, const int16_t *xft,
            int32_t n_sectors, const int32_t *coef, const int32_t *offset, uint64_t cut,
            int32_t *ncomb, int32_t *npass, int32_t *best, uint64_t *chi2, int32_t *params,
            uint8_t *hit_index, int32_t *ntracks, int64_t *comb_offsets, int32_t n_threads,
            orc_summary *summary)
{
    if (summary == NULL || road_offsets == NULL)
        return ORC_E_INVAL;
    memset(summary, 0, sizeof *summary);
    summary->err_road = -1;
    summary->err_event = -1;
    if (n_events < 0 || n_roads < 0 || n_hits < 0)
        return ORC_E_INVAL;
    if (n_events == 0 && n_roads != 0)
        return ORC_E_INVAL;
    if (n_roads == 0 && n_hits != 0)
        return ORC_E_INVAL;
    if (n_roads > 0 && (sector == NULL || nhits == NULL || hit_offsets == NULL || xft == NULL ||
                        ncomb == NULL || npass == NULL || best == NULL || chi2 == NULL ||
                        params == NULL || hit_index == NULL))
        return ORC_E_INVAL;
    if (n_hits > 0 && hits == NULL)
        return ORC_E_INVAL;
    if (n_events > 0 && ntracks == NULL)
        return ORC_E_INVAL;
    int rc = orc_check_constants(n_sectors, coef, offset, cut);
    if (rc != ORC_OK)
        return rc;

    /* validation first: the lowest offending event and road */
    for (int32_t e = 0; e < n_events; ++e)
        if (bad_event(e, n_events, n_roads, road_offsets)) {
            summary->err_event = e;
            break;
        }
    for (int32_t r = 0; r < n_roads; ++r)
        if (bad_road(r, n_roads, n_hits, n_sectors, sector, nhits, hit_offsets, hits, xft)) {
            summary->err_road = r;
            break;
        }
    if (summary->err_event >= 0 || summary->err_road >= 0)
        return ORC_E_RANGE;

    int64_t tot_comb = 0, tot_pass = 0, tot_trk = 0;
    int nt = n_threads > 1 ? n_threads : 1;
    (void)nt;
#pragma omp parallel for schedule(dynamic) num_threads(nt) reduction(+ : tot_comb, tot_pass, tot_trk)
    for (int32_t e = 0; e < n_events; ++e) {             /* loop on events */
        int32_t trk = 0;
        for (int32_t r = road_offsets[e]; r < road_offsets[e + 1]; ++r) {   /* loop on roads */
            fit_road(r, sector, nhits, hit_offsets, hits, xft, coef, offset, cut, ncomb, npass,
                     best, chi2, params, hit_index);      /* loop on combinations */
            tot_comb += ncomb[r];
            tot_pass += npass[r];
            trk += best[r] >= 0;
        }
        ntracks[e] = trk;
        tot_trk += trk;
    }
    if (comb_offsets != NULL) {
        int64_t acc = 0;
        for (int32_t r = 0; r < n_roads; ++r) {
            comb_offsets[r] = acc;
            acc += ncomb[r];
        }
        comb_offsets[n_roads] = acc;
    }
    summary->total_comb = tot_comb;
    summary->total_pass = tot_pass;
    summary->total_tracks = (int32_t)tot_trk;
    return ORC_OK;
}

/*
 * Every passing combination (chi2 <= cut) of every road, road by road and in
 * combination-index order within a road: the fit of Sec. 2 runs on all
 * combinations, and this keeps each one that passes instead of only the
 * best.  Plain nested loops as in fit_road.  offsets[n_roads + 1] receives
 * the exclusive running count of passing combinations per road; entries
 * [offsets[r], offsets[r + 1]) hold road r's combination index k, chi2 and
 * fit rows 0..2.  The arrays must hold `capacity` entries; returns ORC_OK,
 * ORC_E_INVAL, or ORC_E_RANGE for malformed data (as orc_fit) or when the
 * list does not fit (offsets are then complete, entries past capacity are
 * not written).
 */
int orc_list_passing(int32_t n_events, int32_t n_roads, int32_t n_hits,
                     const int32_t *road_offsets, const uint8_t *sector, const uint8_t *nhits,
                     const int32_t *hit_offsets, const int16_t *hits, const int16_t *xft,
                     int32_t n_sectors, const int32_t *coef, const int32_t *offset, uint64_t cut,
                     int64_t capacity, int64_t *offsets, int32_t *list_k, uint64_t *list_chi2,
                     int32_t *list_params, orc_summary *summary)
{
    if (summary == NULL || road_offsets == NULL || offsets == NULL || capacity < 0)
        return ORC_E_INVAL;
    memset(summary, 0, sizeof *summary);
    summary->err_road = -1;
    summary->err_event = -1;
    if (n_events < 0 || n_roads < 0 || n_hits < 0)
        return ORC_E_INVAL;
    if (n_roads > 0 && (sector == NULL || nhits == NULL || hit_offsets == NULL || xft == NULL))
        return ORC_E_INVAL;
    if (capacity > 0 && (list_k == NULL || list_chi2 == NULL || list_params == NULL))
        return ORC_E_INVAL;
    int rc = orc_check_constants(n_sectors, coef, offset, cut);
    if (rc != ORC_OK)
        return rc;
    for (int32_t e = 0; e < n_events; ++e)
        if (bad_event(e, n_events, n_roads, road_offsets)) {
            summary->err_event = e;
            break;
        }
    for (int32_t r = 0; r < n_roads; ++r)
        if (bad_road(r, n_roads, n_hits, n_sectors, sector, nhits, hit_offsets, hits, xft)) {
            summary->err_road = r;
            break;
        }
    if (summary->err_event >= 0 || summary->err_road >= 0)
        return ORC_E_RANGE;

    int64_t at = 0;   /* entries so far, in road order */
    for (int32_t r = 0; r < n_roads; ++r) {
        offsets[r] = at;
        const int s = sector[r];
        const int n0 = nhits[r * 4 + 0], n1 = nhits[r * 4 + 1];
        const int n2 = nhits[r * 4 + 2], n3 = nhits[r * 4 + 3];
        const int16_t *h0 = hits + hit_offsets[r];
        const int16_t *h1 = h0 + n0;
        const int16_t *h2 = h1 + n1;
        const int16_t *h3 = h2 + n2;
        const int32_t *A = coef + s * 36;
        const int32_t *b = offset + s * 6;
        int32_t k = 0;
        for (int i0 = 0; i0 < n0; ++i0)
            for (int i1 = 0; i1 < n1; ++i1)
                for (int i2 = 0; i2 < n2; ++i2)
                    for (int i3 = 0; i3 < n3; ++i3, ++k) {
                        const int64_t x[6] = {h0[i0], h1[i1], h2[i2], h3[i3],
                                              xft[r * 2 + 0], xft[r * 2 + 1]};
                        int64_t y[6];
                        for (int row = 0; row < 6; ++row) {
                            int64_t acc = b[row];
                            for (int j = 0; j < 6; ++j)
                                acc += (int64_t)A[row * 6 + j] * x[j];
                            if (acc < INT32_MIN || acc > INT32_MAX) {
                                fprintf(stderr, "oracle: fit row outside int32\n");
                                abort();
                            }
                            y[row] = acc;
                        }
                        const uint64_t c2 = (uint64_t)(y[3] * y[3]) + (uint64_t)(y[4] * y[4]) +
                                            (uint64_t)(y[5] * y[5]);
                        if (c2 <= cut) {
                            if (at < capacity) {
                                list_k[at] = k;
                                list_chi2[at] = c2;
                                list_params[at * 3 + 0] = (int32_t)y[0];
                                list_params[at * 3 + 1] = (int32_t)y[1];
                                list_params[at * 3 + 2] = (int32_t)y[2];
                            }
                            ++at;
                        }
                        summary->total_comb += 1;
                    }
    }
    offsets[n_roads] = at;
    summary->total_pass = at;
    return at > capacity ? ORC_E_RANGE : ORC_OK;
}

/*
 * Unpack (Sec. 2.1: the first of the three stages fills the data structures
 * from the input) of a packed word stream into the CSR batch layout.  The
 * stream format is this project's own stand-in (the SVT format is not
 * available): 32-bit words whose top two bits are a tag --
 *   3 event header (bits 29..0 zero): roads up to the next event header
 *     belong to this event;
 *   2 road header: bits 29..22 sector, bits 19..0 the hit counts of layers
 *     0..3 (5 bits each, layer 0 lowest, each <= 16), bits 21..20 zero;
 *   1 XFT word: bits 11..0 and 23..12 the two XFT words, bits 29..24 zero;
 *   0 hit word: bits 11..0 and 23..12 two hits in layer-major order (the
 *     second zero in a road's last word when its hit count is odd), bits
 *     29..24 zero.
 * A road is its header, its XFT word and ceil(hits / 2) hit words; the
 * stream starts with an event header.  A sequential parser: the first word
 * that does not fit (or n_words when the stream ends inside a road) goes to
 * *bad_word and the call returns ORC_E_RANGE.  counts[3] receives the
 * events, roads and hits; a well-formed stream larger than the capacities
 * returns ORC_E_RANGE with *bad_word = -1 (arrays then filled up to them).
 */
int orc_unpack_stream(const uint32_t *w, int64_t n_words, int32_t max_events, int32_t max_roads,
                      int32_t max_hits, int32_t *road_offsets, uint8_t *sector, uint8_t *nhits,
                      int32_t *hit_offsets, int16_t *hits, int16_t *xft, int64_t *counts,
                      int64_t *bad_word)
{
    if (counts == NULL || bad_word == NULL || n_words < 0 || (n_words > 0 && w == NULL) ||
        max_events < 0 || max_roads < 0 || max_hits < 0 || road_offsets == NULL ||
        hit_offsets == NULL)
        return ORC_E_INVAL;
    int64_t ne = 0, nr = 0, nh = 0;
    int64_t err = -1;        /* the first word that does not fit */
    *bad_word = -1;
    int64_t i = 0;
    int32_t road_hits = 0;
    while (i < n_words && err < 0) {
        const uint32_t v = w[i];
        const uint32_t tag = v >> 30;
        if (tag == 3) {                                   /* event header */
            if (v & 0x3FFFFFFFu) {
                err = i;
                break;
            }
            if (ne < max_events)
                road_offsets[ne] = (int32_t)nr;
            ++ne;
            ++i;
        } else if (tag == 2 && ne > 0) {                  /* road header, then XFT, then hits */
            const uint32_t cnt = v & 0xFFFFFu;
            const int n[4] = {(int)(cnt & 31u), (int)((cnt >> 5) & 31u), (int)((cnt >> 10) & 31u),
                              (int)((cnt >> 15) & 31u)};
            if ((v & 0x300000u) || n[0] > 16 || n[1] > 16 || n[2] > 16 || n[3] > 16) {
                err = i;
                break;
            }
            road_hits = n[0] + n[1] + n[2] + n[3];
            if (nr < max_roads) {
                sector[nr] = (uint8_t)((v >> 22) & 255u);
                for (int l = 0; l < 4; ++l)
                    nhits[nr * 4 + l] = (uint8_t)n[l];
                hit_offsets[nr] = (int32_t)nh;
            }
            if (i + 1 >= n_words) {
                err = n_words;                            /* ends before the XFT word */
                break;
            }
            const uint32_t x = w[i + 1];
            if ((x >> 30) != 1u || (x & 0x3F000000u)) {
                err = i + 1;
                break;
            }
            if (nr < max_roads) {
                xft[nr * 2 + 0] = (int16_t)(x & 0xFFFu);
                xft[nr * 2 + 1] = (int16_t)((x >> 12) & 0xFFFu);
            }
            i += 2;
            for (int32_t j = 0; j < road_hits; j += 2) {
                if (i >= n_words) {
                    err = n_words;                        /* ends inside the hits */
                    break;
                }
                const uint32_t h = w[i];
                const int two = j + 1 < road_hits;
                if ((h >> 30) != 0u || (h & 0x3F000000u) || (!two && (h & 0xFFF000u))) {
                    err = i;
                    break;
                }
                if (nh + j < max_hits)
                    hits[nh + j] = (int16_t)(h & 0xFFFu);
                if (two && nh + j + 1 < max_hits)
                    hits[nh + j + 1] = (int16_t)((h >> 12) & 0xFFFu);
                ++i;
            }
            if (err >= 0)
                break;
            nh += road_hits;
            ++nr;
        } else {
            err = i;                                      /* a word out of place */
        }
    }
    if (err >= 0) {
        *bad_word = err;
        counts[0] = ne;
        counts[1] = nr;
        counts[2] = nh;
        return ORC_E_RANGE;
    }
    if (ne <= max_events)
        road_offsets[ne] = (int32_t)nr;
    if (nr <= max_roads)
        hit_offsets[nr] = (int32_t)nh;
    counts[0] = ne;
    counts[1] = nr;
    counts[2] = nh;
    if (ne > max_events || nr > max_roads || nh > max_hits)
        return ORC_E_RANGE;
    return ORC_OK;
}

/* Number of threads OpenMP would use (for reporting the CPU baseline). */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
