/*
 * Serial tree Riccati recursion (see oracle_lqr.c for the problem and the
 * method), written once for a floating type REAL and included by
 * oracle_lqr.c for double and for long double.  The including file defines
 * REAL, SQRT, CHOL, CHOL_SOLVE and LQR.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
/* Cholesky H = L L^T in place (lower triangle).  Returns 0 on failure. */
static int CHOL(int n, REAL* H)
{
    for (int j = 0; j < n; ++j) {
        REAL d = H[j * n + j];
        for (int k = 0; k < j; ++k) d -= H[j * n + k] * H[j * n + k];
        if (!(d > 0.0) || !isfinite((double)d)) return 0;
        d = SQRT(d);
        H[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            REAL s = H[i * n + j];
            for (int k = 0; k < j; ++k) s -= H[i * n + k] * H[j * n + k];
            H[i * n + j] = s / d;
        }
    }
    return 1;
}

/* Solve (L L^T) z = y in place for one right-hand side. */
static void CHOL_SOLVE(int n, const REAL* L, REAL* y)
{
    for (int i = 0; i < n; ++i) {
        REAL s = y[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
        y[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        REAL s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * y[k];
        y[i] = s / L[i * n + i];
    }
}

static int LQR(int N, int nx, int nu, const int* parent,
               const REAL* A, const REAL* B, const REAL* c,
               const REAL* Q, const REAL* R, const REAL* M,
               const REAL* q, const REAL* r, const REAL* x0,
               REAL* x, REAL* u, REAL* lam,
               REAL* K, REAL* k, REAL* P, REAL* p, int* bad_node)
{
    if (N <= 0 || nx <= 0 || nu <= 0 || !parent) return ORC_ERR_INVALID_ARG;
    if (parent[0] != -1) return ORC_ERR_TOPOLOGY;
    for (int i = 1; i < N; ++i)
        if (parent[i] < 0 || parent[i] >= i) return ORC_ERR_TOPOLOGY;

    const int nn = nx * nx, nm = nx * nu, mm = nu * nu;
    /* children lists (CSR) in increasing node order */
    int* cnt = calloc((size_t)N + 1, sizeof(int));
    int* kids = malloc(sizeof(int) * (size_t)(N > 1 ? N - 1 : 1));
    int* fill = calloc((size_t)N, sizeof(int));
    REAL* H = malloc(sizeof(REAL) * mm);
    REAL* G = malloc(sizeof(REAL) * nm);
    REAL* g = malloc(sizeof(REAL) * nu);
    REAL* W = malloc(sizeof(REAL) * nn);
    REAL* w = malloc(sizeof(REAL) * nx);
    REAL* s = malloc(sizeof(REAL) * nx);
    REAL* PA = malloc(sizeof(REAL) * nn);
    REAL* PB = malloc(sizeof(REAL) * nm);
    REAL* col = malloc(sizeof(REAL) * nu);
    int status = ORC_OK;

    for (int i = 1; i < N; ++i) cnt[parent[i] + 1]++;
    for (int i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    for (int i = 1; i < N; ++i) kids[cnt[parent[i]] + fill[parent[i]]++] = i;

    /* backward: every child has a larger index than its parent */
    for (int n = N - 1; n >= 0 && status == ORC_OK; --n) {
        REAL* Pn = P + (size_t)n * nn;
        REAL* pn = p + (size_t)n * nx;
        REAL* Kn = K + (size_t)n * nm;
        REAL* kn = k + (size_t)n * nu;
        if (cnt[n + 1] == cnt[n]) {             /* leaf */
            memcpy(Pn, Q + (size_t)n * nn, sizeof(REAL) * nn);
            memcpy(pn, q + (size_t)n * nx, sizeof(REAL) * nx);
            memset(Kn, 0, sizeof(REAL) * nm);
            memset(kn, 0, sizeof(REAL) * nu);
            continue;
        }
        memcpy(H, R + (size_t)n * mm, sizeof(REAL) * mm);
        memcpy(G, M + (size_t)n * nm, sizeof(REAL) * nm);
        memcpy(g, r + (size_t)n * nu, sizeof(REAL) * nu);
        memcpy(W, Q + (size_t)n * nn, sizeof(REAL) * nn);
        memcpy(w, q + (size_t)n * nx, sizeof(REAL) * nx);
        for (int e = cnt[n]; e < cnt[n + 1]; ++e) {
            const int j = kids[e];
            const REAL* Pj = P + (size_t)j * nn;
            const REAL* pj = p + (size_t)j * nx;
            const REAL* Aj = A + (size_t)j * nn;
            const REAL* Bj = B + (size_t)j * nm;
            const REAL* cj = c + (size_t)j * nx;
            for (int a = 0; a < nx; ++a) {
                REAL acc = pj[a];
                for (int b = 0; b < nx; ++b) acc += Pj[a * nx + b] * cj[b];
                s[a] = acc;
                for (int b = 0; b < nx; ++b) {
                    REAL t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Pj[a * nx + l] * Aj[l * nx + b];
                    PA[a * nx + b] = t;
                }
                for (int b = 0; b < nu; ++b) {
                    REAL t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Pj[a * nx + l] * Bj[l * nu + b];
                    PB[a * nu + b] = t;
                }
            }
            for (int a = 0; a < nu; ++a) {
                for (int b = 0; b < nu; ++b) {
                    REAL t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Bj[l * nu + a] * PB[l * nu + b];
                    H[a * nu + b] += t;
                }
                for (int b = 0; b < nx; ++b) {
                    REAL t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Bj[l * nu + a] * PA[l * nx + b];
                    G[a * nx + b] += t;
                }
                REAL t = 0.0;
                for (int l = 0; l < nx; ++l) t += Bj[l * nu + a] * s[l];
                g[a] += t;
            }
            for (int a = 0; a < nx; ++a) {
                for (int b = 0; b < nx; ++b) {
                    REAL t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Aj[l * nx + a] * PA[l * nx + b];
                    W[a * nx + b] += t;
                }
                REAL t = 0.0;
                for (int l = 0; l < nx; ++l) t += Aj[l * nx + a] * s[l];
                w[a] += t;
            }
        }
        if (!CHOL(nu, H)) {
            status = ORC_ERR_NOT_PD;
            if (bad_node) *bad_node = n;
            break;
        }
        /* K = -H^{-1} G column by column, k = -H^{-1} g */
        for (int b = 0; b < nx; ++b) {
            for (int a = 0; a < nu; ++a) col[a] = G[a * nx + b];
            CHOL_SOLVE(nu, H, col);
            for (int a = 0; a < nu; ++a) Kn[a * nx + b] = -col[a];
        }
        for (int a = 0; a < nu; ++a) col[a] = g[a];
        CHOL_SOLVE(nu, H, col);
        for (int a = 0; a < nu; ++a) kn[a] = -col[a];
        for (int a = 0; a < nx; ++a) {
            for (int b = 0; b < nx; ++b) {
                REAL t = W[a * nx + b];
                for (int l = 0; l < nu; ++l) t += G[l * nx + a] * Kn[l * nx + b];
                Pn[a * nx + b] = t;
            }
            REAL t = w[a];
            for (int l = 0; l < nu; ++l) t += G[l * nx + a] * kn[l];
            pn[a] = t;
        }
        for (int a = 0; a < nx; ++a)
            for (int b = a + 1; b < nx; ++b) {
                REAL m = 0.5 * (Pn[a * nx + b] + Pn[b * nx + a]);
                Pn[a * nx + b] = m;
                Pn[b * nx + a] = m;
            }
    }

    if (status == ORC_OK) {
        /* forward rollout in increasing node order */
        memcpy(x, x0, sizeof(REAL) * nx);
        for (int n = 0; n < N; ++n) {
            const REAL* xn = x + (size_t)n * nx;
            REAL* un = u + (size_t)n * nu;
            const REAL* Pn = P + (size_t)n * nn;
            const REAL* pn = p + (size_t)n * nx;
            REAL* ln = lam + (size_t)n * nx;
            for (int a = 0; a < nx; ++a) {
                REAL t = pn[a];
                for (int b = 0; b < nx; ++b) t += Pn[a * nx + b] * xn[b];
                ln[a] = t;
            }
            if (cnt[n + 1] == cnt[n]) {
                memset(un, 0, sizeof(REAL) * nu);
                continue;
            }
            const REAL* Kn = K + (size_t)n * nm;
            const REAL* kn = k + (size_t)n * nu;
            for (int a = 0; a < nu; ++a) {
                REAL t = kn[a];
                for (int b = 0; b < nx; ++b) t += Kn[a * nx + b] * xn[b];
                un[a] = t;
            }
            for (int e = cnt[n]; e < cnt[n + 1]; ++e) {
                const int j = kids[e];
                const REAL* Aj = A + (size_t)j * nn;
                const REAL* Bj = B + (size_t)j * nm;
                const REAL* cj = c + (size_t)j * nx;
                REAL* xj = x + (size_t)j * nx;
                for (int a = 0; a < nx; ++a) {
                    REAL t = cj[a];
                    for (int b = 0; b < nx; ++b) t += Aj[a * nx + b] * xn[b];
                    for (int b = 0; b < nu; ++b) t += Bj[a * nu + b] * un[b];
                    xj[a] = t;
                }
            }
        }
    }

    free(cnt); free(kids); free(fill); free(H); free(G); free(g); free(W); free(w);
    free(s); free(PA); free(PB); free(col);
    return status;
}
