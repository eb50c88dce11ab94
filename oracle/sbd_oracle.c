/*
 * CPU FP64 oracle for selected-basis diagonalisation.  TEST INFRASTRUCTURE
 * ONLY: the tests, the smoke check and the CPU-baseline leg of the benchmark
 * call it; the product path never does.  It shares no code with the HIP path.
 *
 * What it computes (paper Sec. II):
 *   H_ij = <Phi_i|H|Phi_j> over the selected determinants (Eq. 1), with the
 *   second-quantised Hamiltonian of Eq. 3 (one-electron h_pq, two-electron
 *   (pq|rs)), nonzero only for 0-, 1- and 2-electron excitations (Slater-Condon
 *   rules, Eq. 4), and the matrix-free action y = H x (Eq. 4, Sec. II-A).
 *
 * Readings of the paper fixed here:
 *   - (pq|rs) is the chemists' integral; the two-body operator is
 *     1/2 sum (pq|rs) a+_p a+_r a_s a_q over spin orbitals with spin conserved
 *     on each (pq) and (rs) pair.  (Eq. 3 prints the operator order that goes
 *     with physicists' <pq|rs>; this reading is pinned by the tests.)
 *   - A determinant is the product of alpha creators (ascending orbital) and
 *     then beta creators (ascending) on the vacuum, i.e. a 2*norb spin-orbital
 *     string with alpha orbitals first: spin orbital P < norb is alpha orbital
 *     P, P >= norb is beta orbital P - norb.
 *   - Half-bitstrings: bit p of a uint64 is spatial orbital p.  The basis is
 *     the Cartesian product of the sorted alpha and beta string lists with
 *     determinant index ia*nb + ib (Sec. III-B, task loop).
 *
 * Everything is written the plain way: matrix elements come from the generic
 * spin-orbital Slater-Condon rules applied to two determinants (the role of
 * the paper's Hij(DetI, DetJ)), phases from applying annihilators/creators
 * right to left, excitation tables from a brute-force comparison of every
 * pair of strings.  Built with -O2 -ffp-contract=off; OpenMP only splits
 * independent bra rows.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_ERR -1

typedef struct {
    uint64_t w[2]; /* w[0]: alpha occupations, w[1]: beta occupations */
} det_t;

typedef struct {
    int norb;
    const double* h;   /* norb x norb row-major */
    const double* eri; /* norb^4, (pq|rs) at ((p*n+q)*n+r)*n+s */
    double e_core;
} ham_t;

static inline int popc(uint64_t x) { return __builtin_popcountll(x); }
static inline uint64_t below(int p) { return p >= 64 ? ~0ull : ((1ull << p) - 1ull); }

/* Number of occupied spin orbitals with index lower than spin orbital P. */
static int occupied_below(const det_t* d, int norb, int P) {
    if (P < norb) return popc(d->w[0] & below(P));
    return popc(d->w[0]) + popc(d->w[1] & below(P - norb));
}

static inline int spin_of(int norb, int P) { return P < norb ? 0 : 1; }
static inline int orb_of(int norb, int P) { return P < norb ? P : P - norb; }

/* a_P |d>: returns 0 if P is empty, otherwise the phase (+1/-1) and clears P. */
static int annihilate(det_t* d, int norb, int P) {
    int s = spin_of(norb, P), p = orb_of(norb, P);
    if (!((d->w[s] >> p) & 1ull)) return 0;
    int ph = (occupied_below(d, norb, P) & 1) ? -1 : 1;
    d->w[s] &= ~(1ull << p);
    return ph;
}

/* a+_P |d>: returns 0 if P is occupied, otherwise the phase and sets P. */
static int create(det_t* d, int norb, int P) {
    int s = spin_of(norb, P), p = orb_of(norb, P);
    if ((d->w[s] >> p) & 1ull) return 0;
    int ph = (occupied_below(d, norb, P) & 1) ? -1 : 1;
    d->w[s] |= (1ull << p);
    return ph;
}

static inline double h1(const ham_t* H, int p, int q) { return H->h[p * H->norb + q]; }
static inline double g2(const ham_t* H, int p, int q, int r, int s) {
    size_t n = (size_t)H->norb;
    return H->eri[((p * n + q) * n + r) * n + s];
}

/* Spin-orbital integrals: zero unless spins match on each pair. */
static double h_so(const ham_t* H, int P, int Q) {
    int n = H->norb;
    if (spin_of(n, P) != spin_of(n, Q)) return 0.0;
    return h1(H, orb_of(n, P), orb_of(n, Q));
}
static double g_so(const ham_t* H, int P, int Q, int R, int S) {
    int n = H->norb;
    if (spin_of(n, P) != spin_of(n, Q) || spin_of(n, R) != spin_of(n, S)) return 0.0;
    return g2(H, orb_of(n, P), orb_of(n, Q), orb_of(n, R), orb_of(n, S));
}

static int list_occ(const det_t* d, int norb, int* occ) {
    int k = 0;
    for (int P = 0; P < 2 * norb; ++P) {
        int s = spin_of(norb, P), p = orb_of(norb, P);
        if ((d->w[s] >> p) & 1ull) occ[k++] = P;
    }
    return k;
}

/* Spin orbitals set in a but not in b, ascending. */
static int list_diff(const det_t* a, const det_t* b, int norb, int* out, int cap) {
    int k = 0;
    for (int P = 0; P < 2 * norb; ++P) {
        int s = spin_of(norb, P), p = orb_of(norb, P);
        if (((a->w[s] >> p) & 1ull) && !((b->w[s] >> p) & 1ull)) {
            if (k < cap) out[k] = P;
            ++k;
        }
    }
    return k;
}

/*
 * <I|H|J> by the Slater-Condon rules on spin orbitals (Eq. 4):
 *   same determinant:  E_core + sum_P h_PP + sum_{P<Q} [(PP|QQ) - (PQ|QP)]
 *   one difference  :  s * [h_AP + sum_{K in J} ((AP|KK) - (AK|KP))]
 *   two differences :  s * [(AP|BQ) - (AQ|BP)]
 * where P(,Q) are the spin orbitals occupied in J but not I, A(,B) those
 * occupied in I but not J, and s is the phase with
 *   a+_A a_P |J> = s |I>   or   a+_A a+_B a_Q a_P |J> = s |I>.
 */
static double hij(const ham_t* H, const det_t* I, const det_t* J) {
    int n = H->norb;
    int nd = popc(I->w[0] ^ J->w[0]) + popc(I->w[1] ^ J->w[1]);
    if (nd == 0) {
        int occ[128];
        int no = list_occ(I, n, occ);
        double e = H->e_core;
        for (int x = 0; x < no; ++x) e += h_so(H, occ[x], occ[x]);
        for (int x = 0; x < no; ++x)
            for (int y = x + 1; y < no; ++y) {
                int P = occ[x], Q = occ[y];
                e += g_so(H, P, P, Q, Q) - g_so(H, P, Q, Q, P);
            }
        return e;
    }
    if (nd == 2) {
        int P, A;
        if (list_diff(J, I, n, &P, 1) != 1 || list_diff(I, J, n, &A, 1) != 1) return 0.0;
        det_t t = *J;
        int s = annihilate(&t, n, P);
        s *= create(&t, n, A);
        if (s == 0 || t.w[0] != I->w[0] || t.w[1] != I->w[1]) return 0.0;
        double v = h_so(H, A, P);
        int occ[128];
        int no = list_occ(J, n, occ);
        for (int x = 0; x < no; ++x) {
            int K = occ[x];
            v += g_so(H, A, P, K, K) - g_so(H, A, K, K, P);
        }
        return s * v;
    }
    if (nd == 4) {
        int PQ[2], AB[2];
        if (list_diff(J, I, n, PQ, 2) != 2 || list_diff(I, J, n, AB, 2) != 2) return 0.0;
        int P = PQ[0], Q = PQ[1], A = AB[0], B = AB[1];
        det_t t = *J;
        int s = annihilate(&t, n, P);
        s *= annihilate(&t, n, Q);
        s *= create(&t, n, B);
        s *= create(&t, n, A);
        if (s == 0 || t.w[0] != I->w[0] || t.w[1] != I->w[1]) return 0.0;
        return s * (g_so(H, A, P, B, Q) - g_so(H, A, Q, B, P));
    }
    return 0.0;
}

/* ------------------------------------------------------------------ */
/* Exported API (called through ctypes by oracle/__init__.py)          */
/* ------------------------------------------------------------------ */

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/* Sort ascending as unsigned integers and drop duplicates; returns new count. */
int64_t orc_sort_unique(uint64_t* s, int64_t n) {
    if (n <= 0) return 0;
    qsort(s, (size_t)n, sizeof(uint64_t), cmp_u64);
    int64_t k = 1;
    for (int64_t i = 1; i < n; ++i)
        if (s[i] != s[k - 1]) s[k++] = s[i];
    return k;
}

/*
 * Excitation table of one spin by brute force over all pairs (bra I, ket J)
 * of same-spin strings: popcount(I^J) == 2 is a single, == 4 a double.
 * kind = 1 (singles) or 2 (doubles).  Row I lists its kets J in ascending
 * index order.  For a single, orbs[2e..] = (i, a) with i in J\I annihilated and
 * a in I\J created; for a double orbs[4e..] = (i, j, a, b), i<j in J\I and
 * a<b in I\J.  sign = phase of a+_a a_i |J> (single) or a+_a a+_b a_j a_i |J>
 * (double), applied right to left on the one-spin string.
 * Call with J == NULL to obtain row_ptr only.
 */
int orc_exc_table(const uint64_t* s, int64_t n, int norb, int kind,
                  int64_t* row_ptr, int32_t* J, uint8_t* orbs, int8_t* sign) {
    if (kind != 1 && kind != 2) return ORC_ERR;
    int want = 2 * kind;
    row_ptr[0] = 0;
    for (int64_t I = 0; I < n; ++I) {
        int64_t c = 0;
        for (int64_t K = 0; K < n; ++K)
            if (popc(s[I] ^ s[K]) == want) ++c;
        row_ptr[I + 1] = row_ptr[I] + c;
    }
    if (!J) return ORC_OK;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t I = 0; I < n; ++I) {
        int64_t e = row_ptr[I];
        for (int64_t K = 0; K < n; ++K) {
            uint64_t bra = s[I], ket = s[K];
            if (popc(bra ^ ket) != want) continue;
            int ann[2], cre[2], na = 0, nc = 0;
            for (int p = 0; p < norb; ++p) {
                if (((ket >> p) & 1ull) && !((bra >> p) & 1ull)) ann[na++] = p;
                if (((bra >> p) & 1ull) && !((ket >> p) & 1ull)) cre[nc++] = p;
            }
            /* one-spin string as a determinant with only the alpha word used */
            det_t t = {{ket, 0ull}};
            int ph;
            if (kind == 1) {
                ph = annihilate(&t, norb, ann[0]);
                ph *= create(&t, norb, cre[0]);
                orbs[2 * e + 0] = (uint8_t)ann[0];
                orbs[2 * e + 1] = (uint8_t)cre[0];
            } else {
                ph = annihilate(&t, norb, ann[0]);
                ph *= annihilate(&t, norb, ann[1]);
                ph *= create(&t, norb, cre[1]);
                ph *= create(&t, norb, cre[0]);
                orbs[4 * e + 0] = (uint8_t)ann[0];
                orbs[4 * e + 1] = (uint8_t)ann[1];
                orbs[4 * e + 2] = (uint8_t)cre[0];
                orbs[4 * e + 3] = (uint8_t)cre[1];
            }
            J[e] = (int32_t)K;
            sign[e] = (int8_t)ph;
            ++e;
        }
    }
    return ORC_OK;
}

typedef struct {
    const uint64_t* a;
    const uint64_t* b;
    int64_t na, nb;
    /* same-spin neighbour tables (singles and doubles) per spin */
    const int64_t *a1p, *a2p, *b1p, *b2p;
    const int32_t *a1J, *a2J, *b1J, *b2J;
} basis_t;

static inline det_t mkdet(const basis_t* B, int64_t ia, int64_t ib) {
    det_t d = {{B->a[ia], B->b[ib]}};
    return d;
}

/*
 * (H x)_I for one bra I = (ia, ib) and nvec vectors ([v][det], N per vector),
 * written to acc[v].  The sum runs over I itself and its Slater-Condon
 * neighbourhood N(I) (Eq. 4): (Ja, ib) for Ja an alpha single/double of ia,
 * (ia, Jb) likewise for beta, and (Ja, Jb) for an alpha single Ja times a beta
 * single Jb.  Every matrix element comes from hij().
 */
static void sigma_row(const ham_t* H, const basis_t* B, int64_t ia, int64_t ib,
                      int nvec, const double* x, int64_t N, double* acc) {
    det_t I = mkdet(B, ia, ib);
    int64_t bra = ia * B->nb + ib;
    for (int v = 0; v < nvec; ++v) acc[v] = 0.0;
    double d = hij(H, &I, &I);
    for (int v = 0; v < nvec; ++v) acc[v] += d * x[v * N + bra];
    const int64_t* ap[2] = {B->a1p, B->a2p};
    const int32_t* aJ[2] = {B->a1J, B->a2J};
    for (int k = 0; k < 2; ++k)
        for (int64_t e = ap[k][ia]; e < ap[k][ia + 1]; ++e) {
            int64_t ja = aJ[k][e];
            det_t J = mkdet(B, ja, ib);
            double hv = hij(H, &I, &J);
            int64_t ket = ja * B->nb + ib;
            for (int v = 0; v < nvec; ++v) acc[v] += hv * x[v * N + ket];
        }
    const int64_t* bp[2] = {B->b1p, B->b2p};
    const int32_t* bJ[2] = {B->b1J, B->b2J};
    for (int k = 0; k < 2; ++k)
        for (int64_t e = bp[k][ib]; e < bp[k][ib + 1]; ++e) {
            int64_t jb = bJ[k][e];
            det_t J = mkdet(B, ia, jb);
            double hv = hij(H, &I, &J);
            int64_t ket = ia * B->nb + jb;
            for (int v = 0; v < nvec; ++v) acc[v] += hv * x[v * N + ket];
        }
    for (int64_t ea = B->a1p[ia]; ea < B->a1p[ia + 1]; ++ea) {
        int64_t ja = B->a1J[ea];
        for (int64_t eb = B->b1p[ib]; eb < B->b1p[ib + 1]; ++eb) {
            int64_t jb = B->b1J[eb];
            det_t J = mkdet(B, ja, jb);
            double hv = hij(H, &I, &J);
            int64_t ket = ja * B->nb + jb;
            for (int v = 0; v < nvec; ++v) acc[v] += hv * x[v * N + ket];
        }
    }
}

static void fill_basis(basis_t* B, const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb,
                       const int64_t* a1p, const int32_t* a1J, const int64_t* a2p, const int32_t* a2J,
                       const int64_t* b1p, const int32_t* b1J, const int64_t* b2p, const int32_t* b2J) {
    B->a = a; B->b = b; B->na = na; B->nb = nb;
    B->a1p = a1p; B->a1J = a1J; B->a2p = a2p; B->a2J = a2J;
    B->b1p = b1p; B->b1J = b1J; B->b2p = b2p; B->b2J = b2J;
}

/* Full sigma: y = H x for nvec vectors ([v][ia*nb+ib]). */
int orc_sigma(int norb, const double* h, const double* eri, double e_core,
              const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb,
              const int64_t* a1p, const int32_t* a1J, const int64_t* a2p, const int32_t* a2J,
              const int64_t* b1p, const int32_t* b1J, const int64_t* b2p, const int32_t* b2J,
              int nvec, const double* x, double* y) {
    if (nvec < 1 || nvec > 64) return ORC_ERR;
    ham_t H = {norb, h, eri, e_core};
    basis_t B;
    fill_basis(&B, a, na, b, nb, a1p, a1J, a2p, a2J, b1p, b1J, b2p, b2J);
    int64_t N = na * nb;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ia = 0; ia < na; ++ia)
        for (int64_t ib = 0; ib < nb; ++ib) {
            double acc[64];
            sigma_row(&H, &B, ia, ib, nvec, x, N, acc);
            for (int v = 0; v < nvec; ++v) y[v * N + ia * nb + ib] = acc[v];
        }
    return ORC_OK;
}

/* sigma at selected determinant indices only: y[k] = (H x)_{idx[k]} (one vector). */
int orc_sigma_at(int norb, const double* h, const double* eri, double e_core,
                 const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb,
                 const int64_t* a1p, const int32_t* a1J, const int64_t* a2p, const int32_t* a2J,
                 const int64_t* b1p, const int32_t* b1J, const int64_t* b2p, const int32_t* b2J,
                 const double* x, const int64_t* idx, int64_t nidx, double* y) {
    ham_t H = {norb, h, eri, e_core};
    basis_t B;
    fill_basis(&B, a, na, b, nb, a1p, a1J, a2p, a2J, b1p, b1J, b2p, b2J);
    int64_t N = na * nb;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nidx; ++k) {
        int64_t I = idx[k];
        double acc[1];
        sigma_row(&H, &B, I / nb, I % nb, 1, x, N, acc);
        y[k] = acc[0];
    }
    return ORC_OK;
}

/*
 * Componentwise magnitude bound at selected determinants:
 * y[k] = sum_J |H_IJ - shift delta_IJ| |x_J| for I = idx[k] (one vector).  The
 * same neighbourhood walk as sigma, with every element and vector entry taken
 * in absolute value; it bounds the rounding error of any summation order of
 * (H - shift) x (u * z_I * y[k] to first order, z_I terms in row I).
 */
int orc_sigma_abs_at(int norb, const double* h, const double* eri, double e_core,
                     const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb,
                     const int64_t* a1p, const int32_t* a1J, const int64_t* a2p, const int32_t* a2J,
                     const int64_t* b1p, const int32_t* b1J, const int64_t* b2p, const int32_t* b2J,
                     const double* x, double shift, const int64_t* idx, int64_t nidx, double* y) {
    ham_t H = {norb, h, eri, e_core};
    basis_t B;
    fill_basis(&B, a, na, b, nb, a1p, a1J, a2p, a2J, b1p, b1J, b2p, b2J);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nidx; ++k) {
        const int64_t ia = idx[k] / nb, ib = idx[k] % nb;
        det_t I = mkdet(&B, ia, ib);
        double acc = fabs(hij(&H, &I, &I) - shift) * fabs(x[idx[k]]);
        const int64_t* ap[2] = {B.a1p, B.a2p};
        const int32_t* aJ[2] = {B.a1J, B.a2J};
        const int64_t* bp[2] = {B.b1p, B.b2p};
        const int32_t* bJ[2] = {B.b1J, B.b2J};
        for (int t = 0; t < 2; ++t) {
            for (int64_t e = ap[t][ia]; e < ap[t][ia + 1]; ++e) {
                det_t J = mkdet(&B, aJ[t][e], ib);
                acc += fabs(hij(&H, &I, &J)) * fabs(x[aJ[t][e] * nb + ib]);
            }
            for (int64_t e = bp[t][ib]; e < bp[t][ib + 1]; ++e) {
                det_t J = mkdet(&B, ia, bJ[t][e]);
                acc += fabs(hij(&H, &I, &J)) * fabs(x[ia * nb + bJ[t][e]]);
            }
        }
        for (int64_t ea = B.a1p[ia]; ea < B.a1p[ia + 1]; ++ea)
            for (int64_t eb = B.b1p[ib]; eb < B.b1p[ib + 1]; ++eb) {
                det_t J = mkdet(&B, B.a1J[ea], B.b1J[eb]);
                acc += fabs(hij(&H, &I, &J)) * fabs(x[(int64_t)B.a1J[ea] * nb + B.b1J[eb]]);
            }
        y[k] = acc;
    }
    return ORC_OK;
}

/* Diagonal H_II for every determinant. */
int orc_diag(int norb, const double* h, const double* eri, double e_core,
             const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb, double* d) {
    ham_t H = {norb, h, eri, e_core};
#pragma omp parallel for schedule(static)
    for (int64_t ia = 0; ia < na; ++ia)
        for (int64_t ib = 0; ib < nb; ++ib) {
            det_t I = {{a[ia], b[ib]}};
            d[ia * nb + ib] = hij(&H, &I, &I);
        }
    return ORC_OK;
}

/*
 * Dense H over the basis by brute force over ALL determinant pairs (no
 * excitation tables): out[i*N + j] = <Phi_i|H|Phi_j>.  Small N only.
 */
int orc_dense_h(int norb, const double* h, const double* eri, double e_core,
                const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb, double* out) {
    ham_t H = {norb, h, eri, e_core};
    int64_t N = na * nb;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < N; ++i) {
        det_t I = {{a[i / nb], b[i % nb]}};
        for (int64_t j = 0; j < N; ++j) {
            det_t J = {{a[j / nb], b[j % nb]}};
            out[i * N + j] = hij(&H, &I, &J);
        }
    }
    return ORC_OK;
}

/* Single matrix element between determinants (ia,ib) and (ja,jb) given as strings. */
double orc_hij(int norb, const double* h, const double* eri, double e_core,
               uint64_t Ia, uint64_t Ib, uint64_t Ja, uint64_t Jb) {
    ham_t H = {norb, h, eri, e_core};
    det_t I = {{Ia, Ib}}, J = {{Ja, Jb}};
    return hij(&H, &I, &J);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Full-bitstring bases (Sec. II-F, Sec. III-F): an arbitrary list of  */
/* determinants, each one packed spin-orbital string (alpha word,      */
/* beta word), not a Cartesian product of alpha and beta strings.      */
/* ------------------------------------------------------------------ */

static int cmp_det(const void* a, const void* b) {
    const uint64_t* x = (const uint64_t*)a;
    const uint64_t* y = (const uint64_t*)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

/* Sort determinants (2 words each: alpha, beta) by alpha string, then beta
 * string, ascending; remove duplicates; return the unique count. */
int64_t orc_full_sort_unique(uint64_t* d, int64_t n) {
    if (n <= 0) return 0;
    qsort(d, (size_t)n, 2 * sizeof(uint64_t), cmp_det);
    int64_t k = 1;
    for (int64_t i = 1; i < n; ++i)
        if (cmp_det(d + 2 * i, d + 2 * (k - 1)) != 0) {
            d[2 * k] = d[2 * i];
            d[2 * k + 1] = d[2 * i + 1];
            ++k;
        }
    return k;
}

/*
 * Connections of a determinant list by brute force over every pair: J is a
 * neighbour of I (I != J) when the two differ by one or two electrons, i.e.
 * popcount(I ^ J) over both words is 2 or 4 (the Slater-Condon neighbourhood,
 * Eq. 4).  CSR rows sorted by J; deg = electrons moved (1 or 2).  With J and
 * deg NULL only the row pointers are written.
 */
int orc_full_connections(const uint64_t* d, int64_t n, int64_t* rp, int32_t* J, int8_t* deg) {
    rp[0] = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            int x = popc(d[2 * i] ^ d[2 * j]) + popc(d[2 * i + 1] ^ d[2 * j + 1]);
            c += (j != i && (x == 2 || x == 4));
        }
        rp[i + 1] = c;
    }
    for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
    if (!J && !deg) return ORC_OK;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = rp[i];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            int x = popc(d[2 * i] ^ d[2 * j]) + popc(d[2 * i + 1] ^ d[2 * j + 1]);
            if (x == 2 || x == 4) {
                if (J) J[c] = (int32_t)j;
                if (deg) deg[c] = (int8_t)(x / 2);
                ++c;
            }
        }
    }
    return ORC_OK;
}

/* y = H x over a determinant list (nvec vectors, [v][I]), from its connections. */
int orc_full_sigma(int norb, const double* h, const double* eri, double e_core,
                   const uint64_t* d, int64_t n, const int64_t* rp, const int32_t* J,
                   int nvec, const double* x, double* y) {
    if (nvec < 1) return ORC_ERR;
    ham_t H = {norb, h, eri, e_core};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        det_t I = {{d[2 * i], d[2 * i + 1]}};
        double hd = hij(&H, &I, &I);
        for (int v = 0; v < nvec; ++v) y[v * n + i] = hd * x[v * n + i];
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int64_t j = J[e];
            det_t K = {{d[2 * j], d[2 * j + 1]}};
            double hv = hij(&H, &I, &K);
            for (int v = 0; v < nvec; ++v) y[v * n + i] += hv * x[v * n + j];
        }
    }
    return ORC_OK;
}

/* y_I = sum_J H_IJ x_J for the rows I = idx[0..m) only (one vector): each
 * row's neighbours are found by comparing it with every determinant of the
 * list (for spot checks of lists too large for the all-pairs connections). */
int orc_full_sigma_rows(int norb, const double* h, const double* eri, double e_core,
                        const uint64_t* d, int64_t n, const int64_t* idx, int64_t m,
                        const double* x, double* y) {
    ham_t H = {norb, h, eri, e_core};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < m; ++r) {
        const int64_t i = idx[r];
        det_t I = {{d[2 * i], d[2 * i + 1]}};
        double acc = hij(&H, &I, &I) * x[i];
        for (int64_t j = 0; j < n; ++j) {
            int nd = popc(d[2 * i] ^ d[2 * j]) + popc(d[2 * i + 1] ^ d[2 * j + 1]);
            if (j == i || (nd != 2 && nd != 4)) continue;
            det_t K = {{d[2 * j], d[2 * j + 1]}};
            acc += hij(&H, &I, &K) * x[j];
        }
        y[r] = acc;
    }
    return ORC_OK;
}

/* Diagonal H_II of a determinant list. */
int orc_full_diag(int norb, const double* h, const double* eri, double e_core,
                  const uint64_t* d, int64_t n, double* out) {
    ham_t H = {norb, h, eri, e_core};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        det_t I = {{d[2 * i], d[2 * i + 1]}};
        out[i] = hij(&H, &I, &I);
    }
    return ORC_OK;
}

/* Dense H over every pair of a determinant list (no connection lists). */
int orc_full_dense_h(int norb, const double* h, const double* eri, double e_core,
                     const uint64_t* d, int64_t n, double* out) {
    ham_t H = {norb, h, eri, e_core};
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        det_t I = {{d[2 * i], d[2 * i + 1]}};
        for (int64_t j = 0; j < n; ++j) {
            det_t K = {{d[2 * j], d[2 * j + 1]}};
            out[i * n + j] = hij(&H, &I, &K);
        }
    }
    return ORC_OK;
}
