/*
 * oracle.c -- plain, slow CPU reference for the length-bucketed word sort.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  The GPU library
 * never calls it, and the two share no code, header, table or helper.
 *
 * What the method computes (Alyasseri et al., "Parallelize Bubble and Merge
 * Sort Algorithms Using MPI", arXiv:1411.5283):
 *   - phase 2 of "Pre-processing" (section 3, Methodology): the words are put
 *     into one sub-array per character count, shorter words before longer
 *     ones; the size of each sub-array is the number of words of that length
 *     (Abstract);
 *   - phase 3 (same passage): each sub-array is put in alphabetical order by
 *     bubble sort;
 *   - bubble sort (section 2): compare each item with the next one, exchange
 *     them when they are out of order, and repeat whole passes until one pass
 *     makes no exchange;
 *   - the parallel form (sections 3.2 and 4, "MPI Implementation"): a
 *     sub-array is cut into chunks, each chunk is bubble-sorted on its own,
 *     and the sorted chunks are merged.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - alphabetic order is unsigned byte order (memcmp);
 *   - the exchange condition is strictly greater-than, so equal words are
 *     never exchanged and keep their input order (bubble sort is stable);
 *   - word length is the byte count offsets[i+1]-offsets[i]; lengths 0..32 are
 *     accepted, a longer word is an error;
 *   - output: perm[k] = index of the word at sorted position k, and
 *     bucket_offsets[L] = number of words shorter than L (34 entries, the last
 *     one equal to n).
 *
 * Every entry point takes host pointers.  Return codes: 0 ok, -1 invalid
 * argument (a null pointer, or offsets that decrease), -2 a word longer than
 * 32 bytes, -3 more words than the caller's output holds, -4 out of host
 * memory.
 *
 * Around the sort: oracle_tokenize is the first pre-processing phase (raw
 * text to the word list) and oracle_materialize writes the sorted words out
 * as text (section 4: the master merges the chunks and prints the result).
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LEN 32
#define ORC_NBUCKET (ORC_MAX_LEN + 1)

enum { ORC_OK = 0, ORC_INVALID = -1, ORC_TOO_LONG = -2, ORC_CAPACITY = -3, ORC_OOM = -4 };

/* Phase-1 check shared by every entry point: offsets non-decreasing, every
 * length at most ORC_MAX_LEN.  A decreasing offset outranks a long word. */
static int check_words(const uint32_t *offsets, uint32_t n)
{
    int too_long = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (offsets[i + 1] < offsets[i])
            return ORC_INVALID;
        if (offsets[i + 1] - offsets[i] > ORC_MAX_LEN)
            too_long = 1;
    }
    return too_long ? ORC_TOO_LONG : ORC_OK;
}

static uint32_t word_len(const uint32_t *offsets, uint32_t i)
{
    return offsets[i + 1] - offsets[i];
}

/* Phase 2 (section 3, Methodology; Abstract): one list per length, holding the
 * word indices of that length in ascending input order.  counts[L] is the
 * size of list L; lists are returned back to back in `lists`, list L starting
 * at start[L]. */
static void bucket_by_length(const uint32_t *offsets, uint32_t n,
                             uint32_t *counts, uint32_t *start, uint32_t *lists)
{
    uint32_t fill[ORC_NBUCKET];
    for (int L = 0; L < ORC_NBUCKET; ++L)
        counts[L] = 0;
    for (uint32_t i = 0; i < n; ++i)
        counts[word_len(offsets, i)] += 1;
    start[0] = 0;
    for (int L = 0; L < ORC_NBUCKET; ++L)
        start[L + 1] = start[L] + counts[L];
    for (int L = 0; L < ORC_NBUCKET; ++L)
        fill[L] = start[L];
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t L = word_len(offsets, i);
        lists[fill[L]] = i;
        fill[L] += 1;
    }
}

/* "Word a comes after word b" for two words of the same length L. */
static int word_after(const uint8_t *chars, const uint32_t *offsets,
                      uint32_t a, uint32_t b, uint32_t L)
{
    return memcmp(chars + offsets[a], chars + offsets[b], L) > 0;
}

/* Bubble sort (section 2) of the m word indices in v, all of length L: passes
 * over adjacent pairs, exchanging a pair when the first word is after the
 * second, until a pass makes no exchange.  Each pass leaves the largest
 * remaining word at the end, so the next pass may stop one place earlier. */
static void bubble_sort_words(const uint8_t *chars, const uint32_t *offsets,
                              uint32_t *v, uint32_t m, uint32_t L)
{
    uint32_t end = m;
    while (end > 1) {
        int swapped = 0;
        for (uint32_t j = 0; j + 1 < end; ++j) {
            if (word_after(chars, offsets, v[j], v[j + 1], L)) {
                uint32_t t = v[j];
                v[j] = v[j + 1];
                v[j + 1] = t;
                swapped = 1;
            }
        }
        if (!swapped)
            break;
        end -= 1;
    }
}

/* The sequential method: phase 2 then phase 3, then the lists concatenated in
 * length order (every shorter word ahead of every longer one, §3). */
int oracle_bubble(const uint8_t *chars, const uint32_t *offsets, uint32_t n,
                  uint32_t *perm, uint32_t *bucket_offsets)
{
    uint32_t counts[ORC_NBUCKET], start[ORC_NBUCKET + 1];
    if (!offsets || !bucket_offsets || (n && (!chars || !perm)))
        return ORC_INVALID;
    int rc = check_words(offsets, n);
    if (rc != ORC_OK)
        return rc;
    bucket_by_length(offsets, n, counts, start, perm);
    for (int L = 0; L < ORC_NBUCKET; ++L)
        bubble_sort_words(chars, offsets, perm + start[L], counts[L], (uint32_t)L);
    for (int L = 0; L <= ORC_NBUCKET; ++L)
        bucket_offsets[L] = start[L];
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * The parallel form of sections 3.2 and 4: each length list is cut into
 * chunks of `chunk` words (the last one shorter), each chunk is bubble-sorted
 * alone, and all sorted chunks of the list are merged.  The merge repeatedly
 * takes the smallest head among the chunks; on equal words it takes the
 * earliest chunk, whose words came earlier in the input.  The result must
 * equal oracle_bubble for every chunk size. */
int oracle_chunked(const uint8_t *chars, const uint32_t *offsets, uint32_t n,
                   uint32_t chunk, uint32_t *perm, uint32_t *bucket_offsets)
{
    uint32_t counts[ORC_NBUCKET], start[ORC_NBUCKET + 1];
    if (!offsets || !bucket_offsets || (n && (!chars || !perm)) || chunk == 0)
        return ORC_INVALID;
    int rc = check_words(offsets, n);
    if (rc != ORC_OK)
        return rc;
    uint32_t *lists = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!lists)
        return ORC_OOM;
    bucket_by_length(offsets, n, counts, start, lists);
    for (int L = 0; L < ORC_NBUCKET; ++L) {
        uint32_t *v = lists + start[L];
        uint32_t m = counts[L];
        uint32_t nchunks = (m + chunk - 1) / chunk;
        for (uint32_t c = 0; c < nchunks; ++c) {
            uint32_t lo = c * chunk;            /* < m, so no overflow */
            uint32_t len = (m - lo < chunk) ? m - lo : chunk;
            bubble_sort_words(chars, offsets, v + lo, len, (uint32_t)L);
        }
        /* merge: head[c] = next unread position of chunk c */
        uint32_t *head = (uint32_t *)malloc(sizeof(uint32_t) * (nchunks ? nchunks : 1));
        if (!head) {
            free(lists);
            return ORC_OOM;
        }
        for (uint32_t c = 0; c < nchunks; ++c)
            head[c] = c * chunk;
        for (uint32_t k = 0; k < m; ++k) {
            int64_t best = -1;
            for (uint32_t c = 0; c < nchunks; ++c) {
                uint64_t end = ((uint64_t)c + 1) * chunk;
                if (end > m)
                    end = m;
                if (head[c] >= end)
                    continue;
                if (best < 0 || word_after(chars, offsets, v[head[best]], v[head[c]], (uint32_t)L))
                    best = c;
            }
            perm[start[L] + k] = v[head[best]];
            head[best] += 1;
        }
        free(head);
    }
    free(lists);
    for (int L = 0; L <= ORC_NBUCKET; ++L)
        bucket_offsets[L] = start[L];
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * The slaves' step of section 4 alone: each length list is cut into chunks of
 * `chunk` words from its start (the last one shorter) and each chunk is
 * bubble-sorted on its own; the chunks are not merged.  perm holds the lists
 * in length order, each list's chunks one after another.  bucket_offsets as
 * in oracle_bubble. */
int oracle_chunks(const uint8_t *chars, const uint32_t *offsets, uint32_t n,
                  uint32_t chunk, uint32_t *perm, uint32_t *bucket_offsets)
{
    uint32_t counts[ORC_NBUCKET], start[ORC_NBUCKET + 1];
    if (!offsets || !bucket_offsets || (n && (!chars || !perm)) || chunk == 0)
        return ORC_INVALID;
    int rc = check_words(offsets, n);
    if (rc != ORC_OK)
        return rc;
    bucket_by_length(offsets, n, counts, start, perm);
    for (int L = 0; L < ORC_NBUCKET; ++L) {
        uint32_t *v = perm + start[L];
        for (uint32_t lo = 0; lo < counts[L]; lo += chunk) {
            uint32_t len = (counts[L] - lo < chunk) ? counts[L] - lo : chunk;
            bubble_sort_words(chars, offsets, v + lo, len, (uint32_t)L);
        }
    }
    for (int L = 0; L <= ORC_NBUCKET; ++L)
        bucket_offsets[L] = start[L];
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * The definition the method reaches: the unique ordering of the indices by
 * the total order key(i) = (length, bytes as unsigned, i).  A library sort
 * (qsort) serves as the step; the index in the key makes every key distinct,
 * so any correct sort gives the same permutation. */
struct def_ctx {
    const uint8_t *chars;
    const uint32_t *offsets;
};

static int def_cmp(const void *pa, const void *pb, void *arg)
{
    const struct def_ctx *c = (const struct def_ctx *)arg;
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    uint32_t la = word_len(c->offsets, a), lb = word_len(c->offsets, b);
    if (la != lb)
        return la < lb ? -1 : 1;
    int r = memcmp(c->chars + c->offsets[a], c->chars + c->offsets[b], la);
    if (r != 0)
        return r;
    return a < b ? -1 : (a > b ? 1 : 0);
}

int oracle_def(const uint8_t *chars, const uint32_t *offsets, uint32_t n,
               uint32_t *perm, uint32_t *bucket_offsets)
{
    if (!offsets || !bucket_offsets || (n && (!chars || !perm)))
        return ORC_INVALID;
    int rc = check_words(offsets, n);
    if (rc != ORC_OK)
        return rc;
    struct def_ctx c = {chars, offsets};
    for (uint32_t i = 0; i < n; ++i)
        perm[i] = i;
    qsort_r(perm, n, sizeof(uint32_t), def_cmp, &c);
    for (int L = 0; L <= ORC_NBUCKET; ++L)
        bucket_offsets[L] = 0;
    for (uint32_t i = 0; i < n; ++i)
        bucket_offsets[word_len(offsets, i) + 1] += 1;
    for (int L = 1; L <= ORC_NBUCKET; ++L)
        bucket_offsets[L] += bucket_offsets[L - 1];
    return ORC_OK;
}

/* Definitional rank of word i: the number of words whose key is smaller.
 * Lets a test check one output position of an input too large to sort here:
 * perm[oracle_rank(i)] must be i.  Offsets must already be valid. */
uint64_t oracle_rank(const uint8_t *chars, const uint32_t *offsets, uint32_t n, uint32_t i)
{
    struct def_ctx c = {chars, offsets};
    uint64_t r = 0;
    for (uint32_t j = 0; j < n; ++j)
        if (def_cmp(&j, &i, &c) < 0)
            r += 1;
    return r;
}

/* Number of words of each length 0..32: the sizes of the phase-2 lists
 * (Abstract: a sub-array's size is the number of words with that many
 * characters), for bucket checks at any size.  The same checks and return
 * codes as the sorts: offsets that decrease are -1, a word longer than 32
 * bytes is -2 (counts are then unspecified). */
int oracle_length_counts(const uint32_t *offsets, uint32_t n, uint64_t *counts)
{
    if (!offsets || !counts)
        return ORC_INVALID;
    const int rc = check_words(offsets, n);
    if (rc != ORC_OK)
        return rc;
    for (int L = 0; L < ORC_NBUCKET; ++L)
        counts[L] = 0;
    for (uint32_t i = 0; i < n; ++i)
        counts[offsets[i + 1] - offsets[i]] += 1;
    return ORC_OK;
}

/* ---------------------------------------------------------------- phase 1
 * First phase of "Pre-processing" (section 3): the special characters of the
 * text are removed.  Reading: words are the runs of bytes between ASCII
 * whitespace (tab, line feed, vertical tab, form feed, carriage return,
 * space); inside a run only the ASCII letters are kept, in order, and every
 * other byte (digit, punctuation, control, non-ASCII) is dropped without
 * splitting the run; a run left without letters is no word.  With flag bit 0
 * set, capitals become lower case.
 * Output: chars = the kept letters of all words back to back; offsets =
 * n_words+1 entries from 0 (out_offsets must hold max_words+1).  Returns 0,
 * or -3 when the text has more than max_words words. */
static int is_space(uint8_t c) { return c == ' ' || (c >= 9 && c <= 13); }
static int is_letter(uint8_t c) { return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z'); }

int oracle_tokenize(const uint8_t *text, uint64_t n_bytes, uint32_t flags, uint8_t *out_chars,
                    uint32_t *out_offsets, uint32_t max_words, uint32_t *n_words)
{
    uint32_t nw = 0, nc = 0;
    int started = 0;   /* the current run already holds a letter */
    for (uint64_t i = 0; i < n_bytes; ++i) {
        const uint8_t c = text[i];
        if (is_space(c)) {
            started = 0;
            continue;
        }
        if (!is_letter(c))
            continue;   /* a special character: removed */
        if (!started) {
            if (nw == max_words)
                return ORC_CAPACITY;
            out_offsets[nw++] = nc;
            started = 1;
        }
        out_chars[nc++] = (flags & 1u) && c <= 'Z' ? (uint8_t)(c + 32) : c;
    }
    out_offsets[nw] = nc;
    *n_words = nw;
    return ORC_OK;
}

/* ---------------------------------------------------------------- output
 * The sorted text (section 4: the merged result is printed): word perm[k]
 * for k = 0..n-1, each followed by the byte sep when 0 <= sep <= 255, back to
 * back when sep < 0.  out holds offsets[n]-offsets[0] bytes, plus n with a
 * separator.  perm must be a permutation of 0..n-1 and offsets must not
 * decrease; otherwise -1. */
int oracle_materialize(const uint8_t *chars, const uint32_t *offsets, uint32_t n,
                       const uint32_t *perm, int sep, uint8_t *out)
{
    if (n && (!offsets || !perm))
        return ORC_INVALID;
    for (uint32_t i = 0; i < n; ++i)
        if (offsets[i + 1] < offsets[i])
            return ORC_INVALID;
    uint8_t *seen = calloc(n ? n : 1, 1);
    if (!seen)
        return ORC_OOM;
    size_t pos = 0;
    int rc = ORC_OK;
    for (uint32_t k = 0; k < n; ++k) {
        const uint32_t i = perm[k];
        if (i >= n || seen[i]) {
            rc = ORC_INVALID;
            break;
        }
        seen[i] = 1;
        const uint32_t L = offsets[i + 1] - offsets[i];
        memcpy(out + pos, chars + offsets[i], L);
        pos += L;
        if (sep >= 0 && sep <= 255)
            out[pos++] = (uint8_t)sep;
    }
    free(seen);
    return rc;
}
