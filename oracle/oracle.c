/*
 * CPU oracle for the projected Hamiltonian of a selected-CI determinant set.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU path: it is the plain, slow definition that the GPU path is checked
 * against.
 *
 * What it computes (paper Sec. 2.2, the Hamiltonian preceding Step 1, and
 * Step 3):
 *   H = E_core + sum_{PQ} h_PQ a+_P a_Q
 *              + 1/2 sum_{PQRS} <PQ|RS> a+_P a+_Q a_S a_R
 * over spin-orbitals P = (p, sigma), with h_PQ = h_pq delta(sP,sQ) and the
 * physicists' integral <PQ|RS> = (pr|qs) delta(sP,sR) delta(sQ,sS) built from
 * the chemists' (pq|rs) that callers supply.  The determinant |x> with the
 * 2*norb-bit occupation string x = (sigma_alpha, sigma_beta) of Sec. 2.1 is
 * prod_{P occupied, ascending} a+_P |vac>, alpha spin-orbitals 0..norb-1 first,
 * then beta spin-orbitals norb..2norb-1.
 *
 * Everything is done by applying the operators one at a time to the bit
 * string, right to left, with the sign (-1)^(number of occupied spin-orbitals
 * below the one acted on) counted by a plain loop.  Matrix elements
 * [H_B]_ij = <x_i|H|x_j> (Step 3) are read off the expansion of H|x_j> in the
 * determinants of B, looked up in a hash map.  No Slater-Condon rule is used.
 *
 * Selection steps around Step 3 (paper Sec. 2.2, Steps 1' and 2), from the
 * expansion of H|x> over all determinants, not only those of B:
 *   classical expansion (Eq. 2): every y not in B with <y|H|x> != 0 for some
 *     x among the n_top determinants of B with the largest |c_i|;
 *   PT2 importance (Eq. 3): s(x) = |<x|H|Psi_0>|^2 / |E_0 - H_xx| with
 *     <x|H|Psi_0> = sum_i c_i <x|H|x_i>.
 *
 * Reduced density matrices (used as dE/dh and dE/d(pq|rs)):
 *   rdm1[p,q]     = sum_s     <c| a+_{p s} a_{q s} |c>
 *   rdm2[p,q,r,s] = sum_{s t} <c| a+_{p s} a+_{r t} a_{s t} a_{q s} |c>
 * so that E = E_core + sum h_pq rdm1[p,q] + 1/2 sum (pq|rs) rdm2[p,q,r,s]
 * for a normalized c.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- strings */

/* Occupation of spin-orbital P in string x (0 or 1). */
static int occupied(uint64_t x, int P) { return (int)((x >> P) & 1u); }

/* Number of occupied spin-orbitals strictly below P, counted one by one. */
static int count_below(uint64_t x, int P)
{
    int n = 0;
    for (int Q = 0; Q < P; ++Q) n += occupied(x, Q);
    return n;
}

/* a_P acting on *x: returns 0 if P is empty, else the sign, and clears P. */
static int annihilate(uint64_t *x, int P)
{
    if (!occupied(*x, P)) return 0;
    int sign = (count_below(*x, P) % 2) ? -1 : 1;
    *x &= ~((uint64_t)1 << P);
    return sign;
}

/* a+_P acting on *x: returns 0 if P is occupied, else the sign, and sets P. */
static int create(uint64_t *x, int P)
{
    if (occupied(*x, P)) return 0;
    int sign = (count_below(*x, P) % 2) ? -1 : 1;
    *x |= ((uint64_t)1 << P);
    return sign;
}

/* ---------------------------------------------------------------- handle */

typedef struct {
    int norb, na, nb;
    int64_t ndet;
    uint64_t *x;          /* 2norb-bit strings, caller order */
    double *h;            /* norb^2 */
    double *eri;          /* norb^4, chemists' (pq|rs) */
    double ecore;
    int64_t cap;          /* hash table size (power of two) */
    uint64_t *hkey;
    int64_t *hval;        /* -1 = empty */
    /* results of the last or_rows() call */
    int64_t nrows;
    int64_t *rowptr;
    int64_t *col;
    double *val;
    int8_t *etype, *orb, *sign;   /* orb: 4 per entry */
} oracle_t;

static uint64_t mix64(uint64_t k)
{
    k ^= k >> 33; k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

static int64_t lookup(const oracle_t *o, uint64_t key)
{
    uint64_t m = (uint64_t)o->cap - 1;
    uint64_t s = mix64(key) & m;
    for (;;) {
        if (o->hval[s] < 0) return -1;
        if (o->hkey[s] == key) return o->hval[s];
        s = (s + 1) & m;
    }
}

static double eri_at(const oracle_t *o, int p, int q, int r, int s)
{
    int n = o->norb;
    return o->eri[(((int64_t)p * n + q) * n + r) * n + s];
}

/*
 * Create the oracle.  *status: 0 ok, 1 bad arguments, 2 duplicate
 * determinant, 3 wrong electron count or stray bits.
 */
void *or_create(int norb, int na, int nb, const double *h, const double *eri, double ecore,
                int64_t ndet, const uint64_t *alpha, const uint64_t *beta, int *status)
{
    *status = 1;
    if (norb < 1 || norb > 32 || ndet < 0) return NULL;
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    o->norb = norb; o->na = na; o->nb = nb; o->ndet = ndet; o->ecore = ecore;
    o->x = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(ndet > 0 ? ndet : 1));
    size_t n2 = (size_t)norb * norb, n4 = n2 * n2;
    o->h = (double *)malloc(sizeof(double) * n2);
    o->eri = (double *)malloc(sizeof(double) * n4);
    memcpy(o->h, h, sizeof(double) * n2);
    memcpy(o->eri, eri, sizeof(double) * n4);
    o->cap = 1;
    while (o->cap < 2 * ndet + 2) o->cap <<= 1;
    o->hkey = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)o->cap);
    o->hval = (int64_t *)malloc(sizeof(int64_t) * (size_t)o->cap);
    for (int64_t s = 0; s < o->cap; ++s) o->hval[s] = -1;
    for (int64_t i = 0; i < ndet; ++i) {
        uint64_t a = alpha[i], b = beta[i];
        int ca = 0, cb = 0;
        for (int p = 0; p < 64; ++p) {
            if ((a >> p) & 1u) { if (p >= norb) { *status = 3; goto fail; } ++ca; }
            if ((b >> p) & 1u) { if (p >= norb) { *status = 3; goto fail; } ++cb; }
        }
        if (ca != na || cb != nb) { *status = 3; goto fail; }
        uint64_t x = a | (b << norb);
        o->x[i] = x;
        uint64_t m = (uint64_t)o->cap - 1;
        uint64_t s = mix64(x) & m;
        while (o->hval[s] >= 0) {
            if (o->hkey[s] == x) { *status = 2; goto fail; }
            s = (s + 1) & m;
        }
        o->hkey[s] = x;
        o->hval[s] = i;
    }
    *status = 0;
    return o;
fail:
    free(o->x); free(o->h); free(o->eri); free(o->hkey); free(o->hval); free(o);
    return NULL;
}

static void free_rows(oracle_t *o)
{
    free(o->rowptr); free(o->col); free(o->val); free(o->etype); free(o->orb); free(o->sign);
    o->rowptr = NULL; o->col = NULL; o->val = NULL; o->etype = NULL; o->orb = NULL; o->sign = NULL;
    o->nrows = 0;
}

void or_destroy(void *handle)
{
    oracle_t *o = (oracle_t *)handle;
    if (!o) return;
    free_rows(o);
    free(o->x); free(o->h); free(o->eri); free(o->hkey); free(o->hval); free(o);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------- H applied to |x> */

typedef struct {
    double *acc;      /* ndet accumulators */
    int64_t *stamp;   /* last row that touched each accumulator */
    int64_t *touched; /* list of touched determinant indices */
    int64_t ntouched;
} scratch_t;

static void touch(const oracle_t *o, scratch_t *w, int64_t row, uint64_t y, double coeff)
{
    int64_t j = lookup(o, y);
    if (j < 0) return;
    if (w->stamp[j] != row) {
        w->stamp[j] = row;
        w->acc[j] = 0.0;
        w->touched[w->ntouched++] = j;
    }
    w->acc[j] += coeff;
}

/* Expand H|x_i> over B: afterwards w->acc[j] = <x_j|H|x_i> for every touched j. */
static void apply_h(const oracle_t *o, scratch_t *w, int64_t i)
{
    const int n = o->norb, n2 = 2 * n;
    const uint64_t x = o->x[i];
    w->ntouched = 0;
    /* constant term */
    touch(o, w, i, x, o->ecore);
    /* one-body: h_PQ a+_P a_Q, same spin */
    for (int Q = 0; Q < n2; ++Q) {
        uint64_t y1 = x;
        int s1 = annihilate(&y1, Q);
        if (!s1) continue;
        for (int P = 0; P < n2; ++P) {
            if ((P < n) != (Q < n)) continue;              /* delta(sP, sQ) */
            uint64_t y2 = y1;
            int s2 = create(&y2, P);
            if (!s2) continue;
            touch(o, w, i, y2, s1 * s2 * o->h[(P % n) * n + (Q % n)]);
        }
    }
    /* two-body: 1/2 <PQ|RS> a+_P a+_Q a_S a_R with <PQ|RS> = (pr|qs) */
    for (int R = 0; R < n2; ++R) {
        uint64_t y1 = x;
        int s1 = annihilate(&y1, R);
        if (!s1) continue;
        for (int S = 0; S < n2; ++S) {
            uint64_t y2 = y1;
            int s2 = annihilate(&y2, S);
            if (!s2) continue;
            for (int Q = 0; Q < n2; ++Q) {
                if ((Q < n) != (S < n)) continue;          /* delta(sQ, sS) */
                uint64_t y3 = y2;
                int s3 = create(&y3, Q);
                if (!s3) continue;
                for (int P = 0; P < n2; ++P) {
                    if ((P < n) != (R < n)) continue;      /* delta(sP, sR) */
                    uint64_t y4 = y3;
                    int s4 = create(&y4, P);
                    if (!s4) continue;
                    double g = eri_at(o, P % n, R % n, Q % n, S % n);
                    touch(o, w, i, y4, 0.5 * s1 * s2 * s3 * s4 * g);
                }
            }
        }
    }
}

static scratch_t *scratch_new(const oracle_t *o)
{
    scratch_t *w = (scratch_t *)malloc(sizeof(scratch_t));
    size_t nd = (size_t)(o->ndet > 0 ? o->ndet : 1);
    w->acc = (double *)malloc(sizeof(double) * nd);
    w->stamp = (int64_t *)malloc(sizeof(int64_t) * nd);
    w->touched = (int64_t *)malloc(sizeof(int64_t) * nd);
    for (size_t j = 0; j < nd; ++j) w->stamp[j] = -1;
    w->ntouched = 0;
    return w;
}

static void scratch_free(scratch_t *w)
{
    free(w->acc); free(w->stamp); free(w->touched); free(w);
}

/* Difference between x_i (bra) and x_j (ket): holes are spin-orbitals occupied in
 * x_j and empty in x_i, particles the reverse.  Returns the number of holes. */
/* ------------------------------------------- H applied to any determinant */

/* Amplitudes of H|x> keyed by determinant (open addressing), insertion order kept. */
typedef struct {
    int64_t cap;
    uint64_t *key;
    double *amp;
    int8_t *used;
    int64_t *order;
    int64_t n;
} ampmap_t;

static ampmap_t *ampmap_new(int64_t want)
{
    ampmap_t *m = (ampmap_t *)malloc(sizeof(ampmap_t));
    m->cap = 1;
    while (m->cap < 2 * want + 2) m->cap <<= 1;
    m->key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)m->cap);
    m->amp = (double *)malloc(sizeof(double) * (size_t)m->cap);
    m->used = (int8_t *)calloc((size_t)m->cap, 1);
    m->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)m->cap);
    m->n = 0;
    return m;
}

static void ampmap_free(ampmap_t *m)
{
    free(m->key); free(m->amp); free(m->used); free(m->order); free(m);
}

static void ampmap_clear(ampmap_t *m)
{
    for (int64_t k = 0; k < m->n; ++k) m->used[m->order[k]] = 0;
    m->n = 0;
}

static void ampmap_add(ampmap_t *m, uint64_t y, double v)
{
    uint64_t mask = (uint64_t)m->cap - 1;
    uint64_t s = mix64(y) & mask;
    while (m->used[s] && m->key[s] != y) s = (s + 1) & mask;
    if (!m->used[s]) {
        m->used[s] = 1;
        m->key[s] = y;
        m->amp[s] = 0.0;
        m->order[m->n++] = (int64_t)s;
    }
    m->amp[s] += v;
}

/* Number of determinants H|x> can reach (x itself, singles, doubles): the map size. */
static int64_t reach_bound(const oracle_t *o)
{
    int64_t n = o->norb, a = o->na, b = o->nb;
    int64_t sa = a * (n - a), sb = b * (n - b);
    int64_t daa = (a * (a - 1) / 2) * ((n - a) * (n - a - 1) / 2);
    int64_t dbb = (b * (b - 1) / 2) * ((n - b) * (n - b - 1) / 2);
    return 1 + sa + sb + daa + dbb + sa * sb;
}

/* Expand H|x> over all determinants: afterwards m holds <y|H|x> for every y
 * some term of H produces from x (the same operator-by-operator rules as
 * apply_h, without the restriction to B). */
static void expand_h(const oracle_t *o, uint64_t x, ampmap_t *m)
{
    const int n = o->norb, n2 = 2 * n;
    ampmap_clear(m);
    ampmap_add(m, x, o->ecore);
    for (int Q = 0; Q < n2; ++Q) {
        uint64_t y1 = x;
        int s1 = annihilate(&y1, Q);
        if (!s1) continue;
        for (int P = 0; P < n2; ++P) {
            if ((P < n) != (Q < n)) continue;
            uint64_t y2 = y1;
            int s2 = create(&y2, P);
            if (!s2) continue;
            ampmap_add(m, y2, s1 * s2 * o->h[(P % n) * n + (Q % n)]);
        }
    }
    for (int R = 0; R < n2; ++R) {
        uint64_t y1 = x;
        int s1 = annihilate(&y1, R);
        if (!s1) continue;
        for (int S = 0; S < n2; ++S) {
            uint64_t y2 = y1;
            int s2 = annihilate(&y2, S);
            if (!s2) continue;
            for (int Q = 0; Q < n2; ++Q) {
                if ((Q < n) != (S < n)) continue;
                uint64_t y3 = y2;
                int s3 = create(&y3, Q);
                if (!s3) continue;
                for (int P = 0; P < n2; ++P) {
                    if ((P < n) != (R < n)) continue;
                    uint64_t y4 = y3;
                    int s4 = create(&y4, P);
                    if (!s4) continue;
                    ampmap_add(m, y4, 0.5 * s1 * s2 * s3 * s4 * eri_at(o, P % n, R % n, Q % n, S % n));
                }
            }
        }
    }
}

/*
 * PT2 importance of candidate determinants (Eq. 3): for each (alpha, beta)
 * the numerator <x|H|Psi_0> = sum_i c_i <x_i|H|x> (c in caller order; the
 * diagonal term is included when x lies in B), the diagonal element H_xx and
 * the score numer^2 / |e0 - H_xx| (IEEE division).  absnum (may be NULL)
 * receives sum_i |c_i <x_i|H|x>|, the scale of the numerator's rounding.
 */
void or_pt2(void *handle, const double *c, double e0, int64_t ncand, const uint64_t *ca,
            const uint64_t *cb, double *numer, double *hxx, double *score, double *absnum)
{
    const oracle_t *o = (const oracle_t *)handle;
    const int64_t bound = reach_bound(o);
#pragma omp parallel
    {
        ampmap_t *m = ampmap_new(bound);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < ncand; ++t) {
            const uint64_t x = ca[t] | (cb[t] << o->norb);
            expand_h(o, x, m);
            double num = 0.0, d = 0.0, anum = 0.0;
            for (int64_t k = 0; k < m->n; ++k) {
                const int64_t s = m->order[k];
                if (m->key[s] == x) d = m->amp[s];
                const int64_t j = lookup(o, m->key[s]);
                if (j >= 0) {
                    num += c[j] * m->amp[s];
                    anum += fabs(c[j] * m->amp[s]);
                }
            }
            if (absnum) absnum[t] = anum;
            numer[t] = num;
            hxx[t] = d;
            score[t] = num * num / fabs(e0 - d);
        }
        ampmap_free(m);
    }
}

typedef struct {
    double mag;
    int64_t idx;
} magidx_t;

static int cmp_mag_desc(const void *a, const void *b)
{
    const magidx_t *x = (const magidx_t *)a, *y = (const magidx_t *)b;
    if (x->mag > y->mag) return -1;
    if (x->mag < y->mag) return 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/*
 * Classical expansion (Eq. 2).  top[0..ntop) receives the caller indices of
 * the ntop determinants with the largest |c_i| (ties: lower index first).
 * The distinct y not in B with <y|H|x> != 0 for some chosen x are written
 * in ascending (alpha, beta) order, at most cap of them; returns how many
 * there are.
 */
int64_t or_expand(void *handle, const double *c, int64_t ntop, int32_t *top, int64_t cap, uint64_t *out_a,
                  uint64_t *out_b)
{
    const oracle_t *o = (const oracle_t *)handle;
    if (ntop > o->ndet) ntop = o->ndet;
    magidx_t *mi = (magidx_t *)malloc(sizeof(magidx_t) * (size_t)(o->ndet > 0 ? o->ndet : 1));
    for (int64_t i = 0; i < o->ndet; ++i) {
        mi[i].mag = fabs(c[i]);
        mi[i].idx = i;
    }
    qsort(mi, (size_t)o->ndet, sizeof(magidx_t), cmp_mag_desc);
    for (int64_t t = 0; t < ntop; ++t) top[t] = (int32_t)mi[t].idx;
    const int64_t bound = reach_bound(o);
    const uint64_t lowmask = ((uint64_t)1 << o->norb) - 1;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(ntop * bound + 1));
    int64_t nk = 0;
    ampmap_t *m = ampmap_new(bound);
    for (int64_t t = 0; t < ntop; ++t) {
        expand_h(o, o->x[mi[t].idx], m);
        for (int64_t k = 0; k < m->n; ++k) {
            const int64_t s = m->order[k];
            if (m->amp[s] == 0.0 || lookup(o, m->key[s]) >= 0) continue;
            const uint64_t y = m->key[s];
            keys[nk++] = ((y & lowmask) << o->norb) | (y >> o->norb);  /* (alpha, beta) order */
        }
    }
    ampmap_free(m);
    qsort(keys, (size_t)nk, sizeof(uint64_t), cmp_u64);
    int64_t nu = 0;
    for (int64_t k = 0; k < nk; ++k)
        if (nu == 0 || keys[k] != keys[nu - 1]) keys[nu++] = keys[k];
    for (int64_t k = 0; k < nu && k < cap; ++k) {
        out_a[k] = keys[k] >> o->norb;
        out_b[k] = keys[k] & lowmask;
    }
    free(keys);
    free(mi);
    return nu;
}

static int differences(const oracle_t *o, uint64_t xi, uint64_t xj, int *holes, int *parts)
{
    int nh = 0, np_ = 0;
    for (int P = 0; P < 2 * o->norb; ++P) {
        int oi = occupied(xi, P), oj = occupied(xj, P);
        if (oj && !oi) { if (nh < 4) holes[nh] = P; ++nh; }
        if (oi && !oj) { if (np_ < 4) parts[np_] = P; ++np_; }
    }
    return nh;
}

/*
 * Excitation class of the pair (x_i <- x_j) and the sign of the canonical
 * operator string that maps x_j onto x_i:
 *   single q->p           : a+_p a_q                       (type 1 alpha, 2 beta)
 *   same-spin double      : a+_p1 a+_p2 a_h2 a_h1, h1<h2, p1<p2 (type 3 alpha, 4 beta)
 *   opposite-spin double  : a+_pa a+_pb a_hb a_ha          (type 5)
 * orb[] receives spatial indices (h1, h2, p1, p2); for type 5 h1/p1 are the
 * alpha hole/particle and h2/p2 the beta ones; unused entries are -1.
 */
static void classify(const oracle_t *o, uint64_t xi, uint64_t xj, int8_t *etype,
                     int8_t *orb, int8_t *sgn)
{
    int n = o->norb;
    int holes[4], parts[4];
    int deg = differences(o, xi, xj, holes, parts);
    uint64_t y = xj;
    int s = 1;
    orb[0] = orb[1] = orb[2] = orb[3] = -1;
    if (deg == 1) {
        s *= annihilate(&y, holes[0]);
        s *= create(&y, parts[0]);
        *etype = (holes[0] < n) ? 1 : 2;
        orb[0] = (int8_t)(holes[0] % n); orb[2] = (int8_t)(parts[0] % n);
    } else if (deg == 2) {
        /* holes[] and parts[] come out ascending in spin-orbital order, so alpha first */
        int same = ((holes[0] < n) == (holes[1] < n));
        if (same) {
            s *= annihilate(&y, holes[0]);
            s *= annihilate(&y, holes[1]);
            s *= create(&y, parts[1]);
            s *= create(&y, parts[0]);
            *etype = (holes[0] < n) ? 3 : 4;
        } else {
            /* holes[0], parts[0] are alpha; holes[1], parts[1] beta */
            s *= annihilate(&y, holes[0]);
            s *= annihilate(&y, holes[1]);
            s *= create(&y, parts[1]);
            s *= create(&y, parts[0]);
            *etype = 5;
        }
        orb[0] = (int8_t)(holes[0] % n); orb[1] = (int8_t)(holes[1] % n);
        orb[2] = (int8_t)(parts[0] % n); orb[3] = (int8_t)(parts[1] % n);
    } else {
        *etype = 0;
        s = 0;
    }
    if (s != 0 && y != xi) s = 0;   /* cannot happen for deg 1/2 */
    *sgn = (int8_t)s;
}

/*
 * Rows rows[0..nrows) of H_B by operator application.  Each row lists the
 * diagonal first, then every other determinant reached from x_i, ascending.
 * Results stay inside the handle (or_rows_total / or_rows_export).
 * Returns the total number of stored entries.
 */
static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int64_t or_rows(void *handle, int64_t nrows, const int64_t *rows)
{
    oracle_t *o = (oracle_t *)handle;
    free_rows(o);
    o->nrows = nrows;
    int64_t *cnt = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    int64_t **rc = (int64_t **)calloc((size_t)nrows + 1, sizeof(int64_t *));
    double **rv = (double **)calloc((size_t)nrows + 1, sizeof(double *));
#pragma omp parallel
    {
        scratch_t *w = scratch_new(o);
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t i = rows[r];
            apply_h(o, w, i);
            /* H_ij = <x_i|H|x_j> = <x_j|H|x_i> for real symmetric integrals;
             * H|x_i> therefore lists row i. */
            qsort(w->touched, (size_t)w->ntouched, sizeof(int64_t), cmp_i64);
            int64_t m = w->ntouched;
            rc[r] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
            rv[r] = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
            int64_t t = 0;
            rc[r][t] = i; rv[r][t] = 0.0; ++t;      /* diagonal first */
            for (int64_t a = 0; a < m; ++a) {
                int64_t j = w->touched[a];
                if (j == i) { rv[r][0] = w->acc[j]; continue; }
                rc[r][t] = j; rv[r][t] = w->acc[j]; ++t;
            }
            cnt[r] = t;
        }
        scratch_free(w);
    }
    o->rowptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nrows + 1));
    o->rowptr[0] = 0;
    for (int64_t r = 0; r < nrows; ++r) o->rowptr[r + 1] = o->rowptr[r] + cnt[r];
    int64_t tot = o->rowptr[nrows];
    size_t tt = (size_t)(tot > 0 ? tot : 1);
    o->col = (int64_t *)malloc(sizeof(int64_t) * tt);
    o->val = (double *)malloc(sizeof(double) * tt);
    o->etype = (int8_t *)malloc(tt);
    o->orb = (int8_t *)malloc(4 * tt);
    o->sign = (int8_t *)malloc(tt);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t b = o->rowptr[r];
        uint64_t xi = o->x[rows[r]];
        for (int64_t t = 0; t < cnt[r]; ++t) {
            o->col[b + t] = rc[r][t];
            o->val[b + t] = rv[r][t];
            if (t == 0) {
                o->etype[b] = 0; o->sign[b] = 1;
                o->orb[4 * b] = o->orb[4 * b + 1] = o->orb[4 * b + 2] = o->orb[4 * b + 3] = -1;
            } else {
                classify(o, xi, o->x[rc[r][t]], &o->etype[b + t], &o->orb[4 * (b + t)],
                         &o->sign[b + t]);
            }
        }
        free(rc[r]); free(rv[r]);
    }
    free(rc); free(rv); free(cnt);
    return tot;
}

void or_rows_export(void *handle, int64_t *rowptr, int64_t *col, double *val, int8_t *etype,
                    int8_t *orb, int8_t *sgn)
{
    oracle_t *o = (oracle_t *)handle;
    int64_t tot = o->rowptr[o->nrows];
    memcpy(rowptr, o->rowptr, sizeof(int64_t) * ((size_t)o->nrows + 1));
    if (col) memcpy(col, o->col, sizeof(int64_t) * (size_t)tot);
    if (val) memcpy(val, o->val, sizeof(double) * (size_t)tot);
    if (etype) memcpy(etype, o->etype, (size_t)tot);
    if (orb) memcpy(orb, o->orb, 4 * (size_t)tot);
    if (sgn) memcpy(sgn, o->sign, (size_t)tot);
}

/* S[r, :] = sum_j <x_rows[r]|H|x_j> X[j, :] for a k-column block X (ndet x k, row-major).
 * Returns the number of (row, determinant) pairs with a stored element, diagonal included. */
int64_t or_sigma_rows(void *handle, int64_t nrows, const int64_t *rows, int k, const double *X,
                      double *S)
{
    oracle_t *o = (oracle_t *)handle;
    int64_t pairs = 0;
#pragma omp parallel reduction(+ : pairs)
    {
        scratch_t *w = scratch_new(o);
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; ++r) {
            apply_h(o, w, rows[r]);
            for (int c = 0; c < k; ++c) {
                double s = 0.0;
                for (int64_t a = 0; a < w->ntouched; ++a) {
                    int64_t j = w->touched[a];
                    s += w->acc[j] * X[j * k + c];
                }
                S[r * k + c] = s;
            }
            pairs += w->ntouched;
        }
        scratch_free(w);
    }
    return pairs;
}

/* --------------------------------------------------------------- RDMs */

/* rdm1 (norb^2) and rdm2 (norb^4) of the vector c, operator by operator. */
void or_rdm12(void *handle, const double *c, double *rdm1, double *rdm2)
{
    oracle_t *o = (oracle_t *)handle;
    const int n = o->norb, n2 = 2 * n;
    const size_t N2 = (size_t)n * n, N4 = N2 * N2;
    memset(rdm1, 0, sizeof(double) * N2);
    memset(rdm2, 0, sizeof(double) * N4);
    int nt = or_num_threads();
    double *p1 = (double *)calloc((size_t)nt * N2, sizeof(double));
    double *p2 = (double *)calloc((size_t)nt * N4, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g1 = p1 + (size_t)tid * N2, *g2 = p2 + (size_t)tid * N4;
#pragma omp for schedule(dynamic, 8)
        for (int64_t j = 0; j < o->ndet; ++j) {
            const uint64_t x = o->x[j];
            if (c[j] == 0.0) continue;
            /* a+_{p s} a_{q s} */
            for (int Q = 0; Q < n2; ++Q) {
                uint64_t y1 = x;
                int s1 = annihilate(&y1, Q);
                if (!s1) continue;
                for (int P = 0; P < n2; ++P) {
                    if ((P < n) != (Q < n)) continue;
                    uint64_t y2 = y1;
                    int s2 = create(&y2, P);
                    if (!s2) continue;
                    int64_t i = lookup(o, y2);
                    if (i < 0) continue;
                    g1[(P % n) * n + (Q % n)] += s1 * s2 * c[i] * c[j];
                }
            }
            /* a+_{p s} a+_{r t} a_{s t} a_{q s}: spin-orbitals P=(p,s), R=(r,t), S=(s,t), Q=(q,s) */
            for (int Q = 0; Q < n2; ++Q) {
                uint64_t y1 = x;
                int s1 = annihilate(&y1, Q);
                if (!s1) continue;
                for (int S = 0; S < n2; ++S) {
                    uint64_t y2 = y1;
                    int s2 = annihilate(&y2, S);
                    if (!s2) continue;
                    for (int R = 0; R < n2; ++R) {
                        if ((R < n) != (S < n)) continue;
                        uint64_t y3 = y2;
                        int s3 = create(&y3, R);
                        if (!s3) continue;
                        for (int P = 0; P < n2; ++P) {
                            if ((P < n) != (Q < n)) continue;
                            uint64_t y4 = y3;
                            int s4 = create(&y4, P);
                            if (!s4) continue;
                            int64_t i = lookup(o, y4);
                            if (i < 0) continue;
                            size_t at = (((size_t)(P % n) * n + (Q % n)) * n + (R % n)) * n + (S % n);
                            g2[at] += s1 * s2 * s3 * s4 * c[i] * c[j];
                        }
                    }
                }
            }
        }
    }
    for (int t = 0; t < nt; ++t) {
        for (size_t a = 0; a < N2; ++a) rdm1[a] += p1[(size_t)t * N2 + a];
        for (size_t a = 0; a < N4; ++a) rdm2[a] += p2[(size_t)t * N4 + a];
    }
    free(p1); free(p2);
}

/* Selected rdm2 elements idx[4e..4e+3] = (p, q, r, s), one pass over B each. */
void or_rdm2_elements(void *handle, const double *c, int64_t nel, const int32_t *idx, double *out)
{
    oracle_t *o = (oracle_t *)handle;
    const int n = o->norb;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < nel; ++e) {
        int p = idx[4 * e], q = idx[4 * e + 1], r = idx[4 * e + 2], s = idx[4 * e + 3];
        double acc = 0.0;
        for (int64_t j = 0; j < o->ndet; ++j) {
            if (c[j] == 0.0) continue;
            for (int sg = 0; sg < 2; ++sg) {
                for (int tg = 0; tg < 2; ++tg) {
                    uint64_t y = o->x[j];
                    int sgn = annihilate(&y, q + sg * n);
                    if (!sgn) continue;
                    sgn *= annihilate(&y, s + tg * n);
                    if (!sgn) continue;
                    sgn *= create(&y, r + tg * n);
                    if (!sgn) continue;
                    sgn *= create(&y, p + sg * n);
                    if (!sgn) continue;
                    int64_t i = lookup(o, y);
                    if (i < 0) continue;
                    acc += sgn * c[i] * c[j];
                }
            }
        }
        out[e] = acc;
    }
}
