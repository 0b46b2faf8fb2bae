/*
 * CPU oracle for the sliding super point detector of
 * "Regain Sliding super point from distributed edge routers by GPU" (Jie Xu, 2018).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, literal model of the
 * paper's method.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the GPU product path never calls it and shares
 * no code, header, table or helper with it.
 *
 * What it follows (section / algorithm / equation of the paper):
 *   - Sliding estimator (Sec. 3.2): eta unsigned 16-bit distance recorders
 *     (DR) per estimator, initialised once to 65535; an update sets the DR
 *     chosen by H1(oip) to 0; at every slot boundary each DR below 65535 is
 *     increased by one; R_k is the number of DRs below k.
 *   - Linear estimator (Eq. 1): Est = -eta * ln(z0 / eta) with z0 = eta - R_k.
 *   - UnionSE (Alg. 1): per-DR maximum over a set of estimators.
 *   - RSEA + RHFG (Sec. 3.3, Eq. 2 and 3): r rows x 2^q columns of estimators;
 *     RHFG[0] is a tabulation hash; RHFG[i](cip) = ((cip >> shift_i) XOR
 *     RHFG[0](cip)) mod 2^q; B(i) = RHFG[i] XOR RHFG[0].
 *   - Update RSEA (Alg. 2): per pair, the DR H1(oip) of estimator
 *     RSEA[i, RHFG[i](cip)] is set to 0 for every row i.
 *   - Hot estimator threshold (Sec. 3.3): R_k >= eta * (1 - e^(-theta/eta)).
 *   - Regain SSP and IRSSP (Alg. 3 and 4): recursive growth of candidate
 *     tuples, one hot estimator per row, pruned by the B overlap test; at the
 *     last row the tuple's UnionSE is tested against the threshold and the host
 *     is extracted from the B(i).
 *   - Merge RSEA (Alg. 5): per-estimator union over the routers' RSEAs.
 *   - Distance recorder update (Sec. 4.3): +1 on every DR after reconstruction.
 *
 * Readings taken where the paper is silent, ambiguous or inconsistent (each is
 * listed with its justification in the design notes of the repository):
 *   R1  shift_i = (i-1)*delta for i = 1..r-1, so that B(1) holds the low q bits
 *       and (r-2)*delta + q >= key_bits is exactly the coverage condition.
 *   R2  the overlap test between consecutive rows is
 *       (B(i-1) >> delta) == (B(i) mod 2^(q-delta)), with B(j) = he_0 XOR he_j.
 *   R3  UnionSE inside the candidate check is the literal per-DR maximum; the
 *       router merge takes the per-DR minimum distance (most recent hit).
 *   R4  a tuple holds one hot estimator for each row 0..r-1; the terminal test
 *       runs once row r-1 has been added; r >= 3.
 *   R5  the real threshold is rounded up once: T = ceil(eta*(1-exp(-theta/eta)))
 *       in double; both the hot test and the final test use R >= T.
 *   R6  Est at saturation uses z0 = max(eta - R, 1).
 *   R10 reconstruction at the end of slot t sees DR = t - (last hit slot);
 *       aging follows.
 *   R12 the output is sorted by ip, one entry per ip with its maximum R.
 *   R13 a reconstructed value with any bit at or above key_bits set is dropped.
 *   R14 optional re-hash check (off = paper mode): drop x unless
 *       RHFG[0](x) == he_0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DR_MAX 65535u

typedef struct orc_rsea {
    uint32_t q, r, delta, eta, k, theta, key_bits, verify_rehash;
    uint32_t T;                     /* integer hot threshold (R5)            */
    uint32_t tab[2][4][256];        /* [0] RHFG[0], [1] H1 tabulation tables */
    uint16_t *dr;                   /* DR[r][2^q][eta]                       */
    /* products of the last close, kept for inspection */
    uint32_t *rk;                   /* R_k[r][2^q]                           */
    uint32_t *hse;                  /* HSE(i) lists, row i at hse + i*2^q    */
    uint32_t *hse_n;                /* |HSE(i)|                              */
    uint32_t *tuples;               /* candidate tuples reaching the final test, r words each */
    uint64_t n_tuples, cap_tuples;
    uint32_t *res_ip, *res_rk;      /* reported hosts (sorted, unique)       */
    double   *res_est;
    uint64_t n_res, cap_res;
} orc_rsea;

/* ---- hashing (Sec. 3.2 H1, Sec. 3.3 RHFG, Eq. 2) ---- */

static uint32_t tab_hash(const uint32_t t[4][256], uint32_t x)
{
    return t[0][x & 255u] ^ t[1][(x >> 8) & 255u] ^ t[2][(x >> 16) & 255u] ^ t[3][x >> 24];
}

static uint32_t rhfg0(const orc_rsea *s, uint32_t cip)
{
    return tab_hash(s->tab[0], cip) & ((1u << s->q) - 1u);
}

uint32_t orc_h1(const orc_rsea *s, uint32_t oip)
{
    return tab_hash(s->tab[1], oip) & (s->eta - 1u);
}

/* RHFG[i](cip) for i = 0..r-1 (Eq. 2 with reading R1). */
void orc_rhfg(const orc_rsea *s, uint32_t cip, uint32_t *cols)
{
    uint32_t h0 = rhfg0(s, cip);
    uint32_t qmask = (1u << s->q) - 1u;
    cols[0] = h0;
    for (uint32_t i = 1; i < s->r; i++) {
        uint32_t sh = (i - 1) * s->delta;
        uint32_t part = sh < 32 ? (cip >> sh) : 0u;
        cols[i] = (part ^ h0) & qmask;
    }
}

static uint16_t *se_ptr(const orc_rsea *s, uint32_t row, uint32_t col)
{
    return s->dr + (((uint64_t)row << s->q) + col) * (uint64_t)s->eta;
}

/* ---- life cycle ---- */

orc_rsea *orc_create(uint32_t q, uint32_t r, uint32_t delta, uint32_t eta, uint32_t k,
                     uint32_t theta, uint32_t key_bits, uint32_t verify_rehash,
                     const uint32_t *tables)
{
    orc_rsea *s = (orc_rsea *)calloc(1, sizeof(orc_rsea));
    if (!s) return NULL;
    s->q = q; s->r = r; s->delta = delta; s->eta = eta; s->k = k; s->theta = theta;
    s->key_bits = key_bits; s->verify_rehash = verify_rehash;
    memcpy(s->tab, tables, sizeof(s->tab));
    /* hot threshold (Sec. 3.3), rounded up once (R5) */
    s->T = (uint32_t)ceil((double)eta * (1.0 - exp(-(double)theta / (double)eta)));
    uint64_t n_se = (uint64_t)r << q;
    uint64_t n_dr = n_se * eta;
    s->dr = (uint16_t *)malloc(n_dr * sizeof(uint16_t));
    s->rk = (uint32_t *)calloc(n_se, sizeof(uint32_t));
    s->hse = (uint32_t *)calloc(n_se, sizeof(uint32_t));
    s->hse_n = (uint32_t *)calloc(r, sizeof(uint32_t));
    if (!s->dr || !s->rk || !s->hse || !s->hse_n) { free(s->dr); free(s->rk); free(s->hse); free(s->hse_n); free(s); return NULL; }
    /* every DR starts at its largest value, once (Sec. 3.2) */
    for (uint64_t i = 0; i < n_dr; i++) s->dr[i] = (uint16_t)DR_MAX;
    return s;
}

void orc_destroy(orc_rsea *s)
{
    if (!s) return;
    free(s->dr); free(s->rk); free(s->hse); free(s->hse_n); free(s->tuples);
    free(s->res_ip); free(s->res_rk); free(s->res_est);
    free(s);
}

uint32_t orc_threshold(const orc_rsea *s) { return s->T; }
uint16_t *orc_dr(orc_rsea *s) { return s->dr; }

/* ---- Alg. 2: update RSEA for each IP pair ---- */

void orc_scan(orc_rsea *s, const uint32_t *pairs, uint64_t n)
{
    uint32_t cols[64];
    for (uint64_t p = 0; p < n; p++) {
        uint32_t cip = pairs[2 * p], oip = pairs[2 * p + 1];
        uint32_t dridx = orc_h1(s, oip);
        orc_rhfg(s, cip, cols);
        for (uint32_t i = 0; i < s->r; i++)
            se_ptr(s, i, cols[i])[dridx] = 0;
    }
}

/* R_k of one estimator: DRs below k (Sec. 3.2). */
static uint32_t se_rk(const orc_rsea *s, const uint16_t *se)
{
    uint32_t n = 0;
    for (uint32_t d = 0; d < s->eta; d++) n += se[d] < s->k;
    return n;
}

/* ---- Alg. 3 / Alg. 4: regain sliding super points ---- */

static int push_tuple(orc_rsea *s, const uint32_t *ct)
{
    if (s->n_tuples == s->cap_tuples) {
        uint64_t nc = s->cap_tuples ? 2 * s->cap_tuples : 1024;
        uint32_t *nt = (uint32_t *)realloc(s->tuples, nc * s->r * sizeof(uint32_t));
        if (!nt) return -1;
        s->tuples = nt; s->cap_tuples = nc;
    }
    memcpy(s->tuples + s->n_tuples * s->r, ct, s->r * sizeof(uint32_t));
    s->n_tuples++;
    return 0;
}

static int push_result(orc_rsea *s, uint32_t ip, uint32_t rk)
{
    if (s->n_res == s->cap_res) {
        uint64_t nc = s->cap_res ? 2 * s->cap_res : 256;
        uint32_t *a = (uint32_t *)realloc(s->res_ip, nc * sizeof(uint32_t));
        if (!a) return -1;
        s->res_ip = a;
        uint32_t *b = (uint32_t *)realloc(s->res_rk, nc * sizeof(uint32_t));
        if (!b) return -1;
        s->res_rk = b;
        double *c = (double *)realloc(s->res_est, nc * sizeof(double));
        if (!c) return -1;
        s->res_est = c;
        s->cap_res = nc;
    }
    s->res_ip[s->n_res] = ip; s->res_rk[s->n_res] = rk; s->n_res++;
    return 0;
}

/* Extract the host from B(1..r-1) (Eq. 3): B(i) holds q bits of the host
 * starting at bit (i-1)*delta; overlapping bits agree once the overlap tests
 * have passed, so OR-ing the shifted B(i) assembles the host. */
uint64_t orc_extract(const orc_rsea *s, const uint32_t *ct)
{
    uint64_t x = 0;
    for (uint32_t i = 1; i < s->r; i++)
        x |= (uint64_t)(ct[0] ^ ct[i]) << ((i - 1) * s->delta);
    return x;
}

/* Overlap test between rows i-1 and i of a tuple (reading R2), i >= 2. */
static int overlap_ok(const orc_rsea *s, const uint32_t *ct, uint32_t i)
{
    uint32_t m = (1u << (s->q - s->delta)) - 1u;
    return ((ct[0] ^ ct[i - 1]) >> s->delta) == ((ct[0] ^ ct[i]) & m);
}

/* Pin helper: for every host in [lo, hi), hash it with RHFG, check that its
 * own tuple passes every overlap test and that extraction returns the host.
 * Returns the number of hosts that fail (0 when the hashes are invertible). */
uint64_t orc_roundtrip_failures(const orc_rsea *s, uint64_t lo, uint64_t hi, uint64_t stride)
{
    uint32_t ct[64];
    uint64_t bad = 0;
    if (stride == 0) stride = 1;
    for (uint64_t x = lo; x < hi; x += stride) {
        orc_rhfg(s, (uint32_t)x, ct);
        int ok = 1;
        for (uint32_t i = 2; i < s->r; i++) ok &= overlap_ok(s, ct, i);
        if (!ok || orc_extract(s, ct) != (x & 0xFFFFFFFFull)) bad++;
    }
    return bad;
}

/* Terminal step of IRSSP: the tuple holds one hot estimator per row. */
static int final_test(orc_rsea *s, const uint32_t *ct, uint16_t *use)
{
    uint64_t x = orc_extract(s, ct);
    if (s->key_bits < 64 && (x >> s->key_bits) != 0) return 0;        /* R13 */
    if (push_tuple(s, ct)) return -1;
    if (s->verify_rehash && rhfg0(s, (uint32_t)x) != ct[0]) return 0; /* R14 */
    /* UnionSE over the tuple (Alg. 1): per-DR maximum, starting from 0 */
    for (uint32_t d = 0; d < s->eta; d++) use[d] = 0;
    for (uint32_t i = 0; i < s->r; i++) {
        const uint16_t *se = se_ptr(s, i, ct[i]);
        for (uint32_t d = 0; d < s->eta; d++)
            if (use[d] < se[d]) use[d] = se[d];
    }
    uint32_t R = se_rk(s, use);
    if (R >= s->T) return push_result(s, (uint32_t)x, R);
    return 0;
}

/* IRSSP: ct[0..len-1] is filled; try every hot estimator of row `len`. */
static int irssp(orc_rsea *s, uint32_t *ct, uint32_t len, uint16_t *use)
{
    const uint32_t *h = s->hse + ((uint64_t)len << s->q);
    for (uint32_t a = 0; a < s->hse_n[len]; a++) {
        ct[len] = h[a];
        if (!overlap_ok(s, ct, len)) continue;      /* B(len-1) against B(len) */
        int rc = (len == s->r - 1) ? final_test(s, ct, use) : irssp(s, ct, len + 1, use);
        if (rc) return rc;
    }
    return 0;
}

static int cmp_ip_then_rk_desc(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

/* Reconstruction at the end of a slot (Alg. 3 and 4).  Fills R_k, the hot
 * lists, the candidate tuples and the reported hosts.  Returns the number of
 * reported hosts, or -1 on allocation failure. */
int64_t orc_reconstruct(orc_rsea *s)
{
    uint64_t n_col = 1ull << s->q;
    s->n_tuples = 0;
    s->n_res = 0;
    /* R_k of every estimator and the hot lists HSE(i), in column order */
    for (uint32_t i = 0; i < s->r; i++) {
        s->hse_n[i] = 0;
        for (uint64_t c = 0; c < n_col; c++) {
            uint32_t R = se_rk(s, se_ptr(s, i, (uint32_t)c));
            s->rk[((uint64_t)i << s->q) + c] = R;
            if (R >= s->T) s->hse[((uint64_t)i << s->q) + s->hse_n[i]++] = (uint32_t)c;
        }
    }
    uint16_t *use = (uint16_t *)malloc(s->eta * sizeof(uint16_t));
    if (!use) return -1;
    /* Alg. 3: every pair from HSE(0) x HSE(1), grown over HSE(2..r-1) */
    uint32_t ct[64];
    int rc = 0;
    for (uint32_t a = 0; a < s->hse_n[0] && !rc; a++)
        for (uint32_t b = 0; b < s->hse_n[1] && !rc; b++) {
            ct[0] = s->hse[a];
            ct[1] = s->hse[((uint64_t)1 << s->q) + b];
            rc = irssp(s, ct, 2, use);
        }
    free(use);
    if (rc) return -1;
    /* R12: one entry per ip with its largest R, ascending ip */
    if (s->n_res) {
        uint64_t *key = (uint64_t *)malloc(s->n_res * sizeof(uint64_t));
        if (!key) return -1;
        for (uint64_t i = 0; i < s->n_res; i++)
            key[i] = ((uint64_t)s->res_ip[i] << 32) | (uint32_t)(0xFFFFFFFFu - s->res_rk[i]);
        qsort(key, s->n_res, sizeof(uint64_t), cmp_ip_then_rk_desc);
        uint64_t m = 0;
        for (uint64_t i = 0; i < s->n_res; i++) {
            uint32_t ip = (uint32_t)(key[i] >> 32);
            if (m && s->res_ip[m - 1] == ip) continue;
            s->res_ip[m] = ip;
            s->res_rk[m] = 0xFFFFFFFFu - (uint32_t)key[i];
            m++;
        }
        free(key);
        s->n_res = m;
        /* Eq. 1 with z0 = eta - R (R6: z0 at least 1) */
        for (uint64_t i = 0; i < m; i++) {
            double z0 = (double)s->eta - (double)s->res_rk[i];
            if (z0 < 1.0) z0 = 1.0;
            s->res_est[i] = -(double)s->eta * log(z0 / (double)s->eta);
        }
    }
    return (int64_t)s->n_res;
}

/* Sec. 4.3: after reconstruction every DR below its maximum grows by one. */
void orc_age(orc_rsea *s)
{
    uint64_t n_dr = ((uint64_t)s->r << s->q) * s->eta;
    for (uint64_t i = 0; i < n_dr; i++)
        if (s->dr[i] < DR_MAX) s->dr[i]++;
}

/* End of slot: reconstruct (skipped for a router that only advances), then
 * age.  Returns the number of reported hosts, or -1 on failure. */
int64_t orc_close(orc_rsea *s, int advance_only)
{
    int64_t n = 0;
    if (advance_only) { s->n_tuples = 0; s->n_res = 0; }
    else n = orc_reconstruct(s);
    orc_age(s);
    return n;
}

/* ---- inspection ---- */

uint64_t orc_results(const orc_rsea *s, uint32_t *ip, uint32_t *rk, double *est, uint64_t cap)
{
    uint64_t n = s->n_res < cap ? s->n_res : cap;
    for (uint64_t i = 0; i < n; i++) { ip[i] = s->res_ip[i]; rk[i] = s->res_rk[i]; est[i] = s->res_est[i]; }
    return s->n_res;
}

void orc_rk(const orc_rsea *s, uint32_t *out)
{
    memcpy(out, s->rk, ((uint64_t)s->r << s->q) * sizeof(uint32_t));
}

/* HSE lists: counts[r]; lists packed row after row into out (capacity r*2^q). */
void orc_hse(const orc_rsea *s, uint32_t *counts, uint32_t *out)
{
    uint64_t o = 0;
    for (uint32_t i = 0; i < s->r; i++) {
        counts[i] = s->hse_n[i];
        if (s->hse_n[i]) memcpy(out + o, s->hse + ((uint64_t)i << s->q), s->hse_n[i] * sizeof(uint32_t));
        o += s->hse_n[i];
    }
}

uint64_t orc_tuples(const orc_rsea *s, uint32_t *out, uint64_t cap)
{
    uint64_t n = s->n_tuples < cap ? s->n_tuples : cap;
    if (n) memcpy(out, s->tuples, n * s->r * sizeof(uint32_t));   /* out may be NULL when cap is 0 */
    return s->n_tuples;
}

/* Canonical state: DR where DR < k (inside the window), else 0xFFFF. */
void orc_canonical(const orc_rsea *s, uint16_t *out)
{
    uint64_t n_dr = ((uint64_t)s->r << s->q) * s->eta;
    for (uint64_t i = 0; i < n_dr; i++) out[i] = s->dr[i] < s->k ? s->dr[i] : 0xFFFFu;
}

/* ---- Alg. 5: merge the routers' RSEAs into the global one (reading R3) ---- */

int orc_merge(orc_rsea *g, orc_rsea *const *routers, uint32_t n)
{
    for (uint32_t j = 0; j < n; j++) {
        const orc_rsea *s = routers[j];
        if (s->q != g->q || s->r != g->r || s->eta != g->eta || s->delta != g->delta ||
            memcmp(s->tab, g->tab, sizeof(g->tab)) != 0)
            return -1;
    }
    uint64_t n_dr = ((uint64_t)g->r << g->q) * g->eta;
    for (uint64_t i = 0; i < n_dr; i++) {
        uint16_t v = (uint16_t)DR_MAX;
        for (uint32_t j = 0; j < n; j++)
            if (routers[j]->dr[i] < v) v = routers[j]->dr[i];
        g->dr[i] = v;
    }
    return 0;
}

/* ---- pins: forward brute force over a range of hosts ----
 * Every x in [x_lo, x_hi) whose r estimators are all hot and whose UnionSE
 * passes the threshold, on the current DRs (call it before aging).  This
 * enumerates hosts forward through the hashes instead of inverting them.
 * Returns the count; writes up to cap (ip, R) entries in ascending ip order,
 * or returns UINT64_MAX on allocation failure. */
uint64_t orc_bruteforce(const orc_rsea *s, uint64_t x_lo, uint64_t x_hi,
                        uint32_t *ip, uint32_t *rk, uint64_t cap)
{
    uint32_t cols[64];
    uint64_t n = 0;
    uint64_t n_se = (uint64_t)s->r << s->q;
    uint16_t *use = (uint16_t *)malloc(s->eta * sizeof(uint16_t));
    uint8_t *hot = (uint8_t *)malloc(n_se);
    if (!use || !hot) { free(use); free(hot); return UINT64_MAX; }
    for (uint64_t e = 0; e < n_se; e++) hot[e] = se_rk(s, s->dr + e * s->eta) >= s->T;
    for (uint64_t x = x_lo; x < x_hi; x++) {
        orc_rhfg(s, (uint32_t)x, cols);
        uint32_t i;
        for (i = 0; i < s->r; i++)
            if (!hot[((uint64_t)i << s->q) + cols[i]]) break;
        if (i < s->r) continue;
        for (uint32_t d = 0; d < s->eta; d++) use[d] = 0;
        for (i = 0; i < s->r; i++) {
            const uint16_t *se = se_ptr(s, i, cols[i]);
            for (uint32_t d = 0; d < s->eta; d++) if (use[d] < se[d]) use[d] = se[d];
        }
        uint32_t R = se_rk(s, use);
        if (R >= s->T) {
            if (n < cap) { ip[n] = (uint32_t)x; rk[n] = R; }
            n++;
        }
    }
    free(use);
    free(hot);
    return n;
}
