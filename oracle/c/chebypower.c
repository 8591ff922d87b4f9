/* FP64 CPU reference of ChebyPower (Alg. 3) and PwMethod (Alg. 1) in plain C.
 *
 * TEST INFRASTRUCTURE ONLY: this is part of the oracle the GPU library is
 * checked against (large graphs, where the Python oracle is too slow).  It
 * shares no code with the library.  Plain loops in the paper's order; the
 * only parallelism is an OpenMP split of the node loop of each step, which
 * does not change any sum (every output element is summed serially over
 * its row, in CSR order).
 *
 *   (P r)(v) = sum_{u in N(v)} r(u) / d_u          P = A D^{-1}  (Sec. 2.1)
 *   Alg. 3:  y = c_0 e_s; r_0 = e_s; r_1 = P e_s;
 *            for k = 1 .. K-1: y += c_k r_k; r_{k+1} = 2 P r_k - r_{k-1};
 *            y += c_K r_K.
 *   Alg. 1:  y = 0; r = e_s; for k = 0 .. N-1: y += zeta_k r; r = P r.
 *
 * oracle_chebypower_multi runs Alg. 3 for B sources side by side: column j
 * of the [n][B] row-major matrices is source j's r_k, with its own K_j and
 * coefficients.  Each column's additions are exactly those of
 * oracle_chebypower, in the same order; the columns only share the pass
 * over the CSR.  oracle_pwmethod_multi does the same for Alg. 1.
 *
 * oracle_ppr_residual_multi evaluates Def. 3's fixed-point equation on B
 * given vectors: for column j, ||alpha e_s + (1 - alpha) P y - y||_1.
 * Because ||P||_1 = 1, ||(I - (1 - alpha) P)^{-1}||_1 = 1 / alpha, so this
 * norm divided by alpha bounds ||pi_s - y||_1 without a reference vector.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static int g_verbose = 0;
void oracle_set_verbose(int v) { g_verbose = v; }

static void apply_P(int64_t n, const int64_t* rp, const int32_t* ci, const double* inv_d, const double* r,
                    double* out) {
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    double acc = 0.0;
    for (int64_t q = rp[v]; q < rp[v + 1]; ++q) acc += r[ci[q]] * inv_d[ci[q]];
    out[v] = acc;
  }
}

static double* inverse_degrees(int64_t n, const int64_t* rp) {
  double* inv_d = (double*)malloc(sizeof(double) * (size_t)n);
  if (!inv_d) return NULL;
#pragma omp parallel for
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = rp[v + 1] - rp[v];
    inv_d[v] = d > 0 ? 1.0 / (double)d : 0.0;
  }
  return inv_d;
}

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int oracle_chebypower(int64_t n, const int64_t* rp, const int32_t* ci, int64_t s, const double* c, int32_t K,
                      double* y) {
  if (n < 1 || s < 0 || s >= n || K < 1 || !rp || !ci || !c || !y) return -1;
  double* inv_d = inverse_degrees(n, rp);
  double* r_prev = (double*)calloc((size_t)n, sizeof(double));
  double* r_cur = (double*)calloc((size_t)n, sizeof(double));
  double* r_next = (double*)malloc(sizeof(double) * (size_t)n);
  if (!inv_d || !r_prev || !r_cur || !r_next) {
    free(inv_d); free(r_prev); free(r_cur); free(r_next);
    return -2;
  }
  memset(y, 0, sizeof(double) * (size_t)n);
  y[s] = c[0];            /* y = c_0 e_s */
  r_prev[s] = 1.0;        /* r_0 = e_s   */
  apply_P(n, rp, ci, inv_d, r_prev, r_cur); /* r_1 = P e_s */
  for (int32_t k = 1; k < K; ++k) {
    const double ck = c[k];
#pragma omp parallel for
    for (int64_t v = 0; v < n; ++v) y[v] += ck * r_cur[v];
    apply_P(n, rp, ci, inv_d, r_cur, r_next);
#pragma omp parallel for
    for (int64_t v = 0; v < n; ++v) r_next[v] = 2.0 * r_next[v] - r_prev[v];
    double* t = r_prev;
    r_prev = r_cur;
    r_cur = r_next;
    r_next = t;
    if (g_verbose) {
      fprintf(stderr, "[oracle] Alg. 3 step %d/%d\n", k, K - 1);
      fflush(stderr);
    }
  }
  const double cK = c[K];
#pragma omp parallel for
  for (int64_t v = 0; v < n; ++v) y[v] += cK * r_cur[v];
  free(inv_d); free(r_prev); free(r_cur); free(r_next);
  return 0;
}

int oracle_pwmethod(int64_t n, const int64_t* rp, const int32_t* ci, int64_t s, const double* zeta, int32_t N,
                    double* y) {
  if (n < 1 || s < 0 || s >= n || N < 1 || !rp || !ci || !zeta || !y) return -1;
  double* inv_d = inverse_degrees(n, rp);
  double* r = (double*)calloc((size_t)n, sizeof(double));
  double* r2 = (double*)malloc(sizeof(double) * (size_t)n);
  if (!inv_d || !r || !r2) {
    free(inv_d); free(r); free(r2);
    return -2;
  }
  memset(y, 0, sizeof(double) * (size_t)n);
  r[s] = 1.0;
  for (int32_t k = 0; k < N; ++k) {
    const double zk = zeta[k];
#pragma omp parallel for
    for (int64_t v = 0; v < n; ++v) y[v] += zk * r[v];
    apply_P(n, rp, ci, inv_d, r, r2);
    double* t = r;
    r = r2;
    r2 = t;
  }
  free(inv_d); free(r); free(r2);
  return 0;
}

/* P applied to the B columns of r ([n][B] row-major) at once. */
static void apply_P_multi(int64_t n, int32_t B, const int64_t* rp, const int32_t* ci, const double* inv_d,
                          const double* r, double* out) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v) {
    double* o = out + (size_t)v * (size_t)B;
    for (int32_t j = 0; j < B; ++j) o[j] = 0.0;
    for (int64_t q = rp[v]; q < rp[v + 1]; ++q) {
      const int64_t u = ci[q];
      const double w = inv_d[u];
      const double* ru = r + (size_t)u * (size_t)B;
      for (int32_t j = 0; j < B; ++j) o[j] += ru[j] * w;
    }
  }
}

/* Alg. 3 for B sources: src[j], K[j] >= 1, coefficients c[j * ldc + k] for
 * k = 0..K[j] (ldc >= max K + 1); Y is [n][B] row-major. */
int oracle_chebypower_multi(int64_t n, const int64_t* rp, const int32_t* ci, int32_t B, const int64_t* src,
                            const double* c, int32_t ldc, const int32_t* K, double* Y) {
  if (n < 1 || B < 1 || !rp || !ci || !src || !c || !K || !Y) return -1;
  int32_t Kmax = 0;
  for (int32_t j = 0; j < B; ++j) {
    if (src[j] < 0 || src[j] >= n || K[j] < 1 || K[j] + 1 > ldc) return -1;
    if (K[j] > Kmax) Kmax = K[j];
  }
  const size_t nb = (size_t)n * (size_t)B;
  double* inv_d = inverse_degrees(n, rp);
  double* r_prev = (double*)calloc(nb, sizeof(double));
  double* r_cur = (double*)calloc(nb, sizeof(double));
  double* r_next = (double*)malloc(sizeof(double) * nb);
  if (!inv_d || !r_prev || !r_cur || !r_next) {
    free(inv_d); free(r_prev); free(r_cur); free(r_next);
    return -2;
  }
  memset(Y, 0, sizeof(double) * nb);
  for (int32_t j = 0; j < B; ++j) {
    Y[(size_t)src[j] * B + j] = c[(size_t)j * ldc];  /* y = c_0 e_s */
    r_prev[(size_t)src[j] * B + j] = 1.0;            /* r_0 = e_s   */
  }
  apply_P_multi(n, B, rp, ci, inv_d, r_prev, r_cur); /* r_1 = P e_s */
  for (int32_t k = 1; k <= Kmax; ++k) {
    /* y += c_k r_k for the columns that still have a term k */
#pragma omp parallel for
    for (int64_t v = 0; v < n; ++v)
      for (int32_t j = 0; j < B; ++j)
        if (k <= K[j]) Y[(size_t)v * B + j] += c[(size_t)j * ldc + k] * r_cur[(size_t)v * B + j];
    if (k == Kmax) break;
    apply_P_multi(n, B, rp, ci, inv_d, r_cur, r_next);
#pragma omp parallel for
    for (int64_t i = 0; i < (int64_t)nb; ++i) r_next[i] = 2.0 * r_next[i] - r_prev[i];
    double* t = r_prev;
    r_prev = r_cur;
    r_cur = r_next;
    r_next = t;
    if (g_verbose) {
      fprintf(stderr, "[oracle] Alg. 3 x%d step %d/%d\n", B, k, Kmax - 1);
      fflush(stderr);
    }
  }
  free(inv_d); free(r_prev); free(r_cur); free(r_next);
  return 0;
}

/* Alg. 1 for B sources: src[j], N[j] >= 1, weights zeta[j * ldz + k] for
 * k = 0..N[j]-1 (ldz >= max N); Y is [n][B] row-major. */
int oracle_pwmethod_multi(int64_t n, const int64_t* rp, const int32_t* ci, int32_t B, const int64_t* src,
                          const double* zeta, int32_t ldz, const int32_t* N, double* Y) {
  if (n < 1 || B < 1 || !rp || !ci || !src || !zeta || !N || !Y) return -1;
  int32_t Nmax = 0;
  for (int32_t j = 0; j < B; ++j) {
    if (src[j] < 0 || src[j] >= n || N[j] < 1 || N[j] > ldz) return -1;
    if (N[j] > Nmax) Nmax = N[j];
  }
  const size_t nb = (size_t)n * (size_t)B;
  double* inv_d = inverse_degrees(n, rp);
  double* r = (double*)calloc(nb, sizeof(double));
  double* r2 = (double*)malloc(sizeof(double) * nb);
  if (!inv_d || !r || !r2) {
    free(inv_d); free(r); free(r2);
    return -2;
  }
  memset(Y, 0, sizeof(double) * nb);
  for (int32_t j = 0; j < B; ++j) r[(size_t)src[j] * B + j] = 1.0; /* r = e_s */
  for (int32_t k = 0; k < Nmax; ++k) {
    /* y += zeta_k r for the columns that still have a term k */
#pragma omp parallel for
    for (int64_t v = 0; v < n; ++v)
      for (int32_t j = 0; j < B; ++j)
        if (k < N[j]) Y[(size_t)v * B + j] += zeta[(size_t)j * ldz + k] * r[(size_t)v * B + j];
    if (k == Nmax - 1) break;
    apply_P_multi(n, B, rp, ci, inv_d, r, r2); /* r = P r */
    double* t = r;
    r = r2;
    r2 = t;
    if (g_verbose) {
      fprintf(stderr, "[oracle] Alg. 1 x%d step %d/%d\n", B, k + 1, Nmax - 1);
      fflush(stderr);
    }
  }
  free(inv_d); free(r); free(r2);
  return 0;
}

/* res[j] = || alpha[j] e_{src[j]} + (1 - alpha[j]) P y_j - y_j ||_1 for the B
 * columns y_j of Y ([n][B] row-major, double).  One pass over the CSR; the
 * l1 sum of each column is taken in node order. */
int oracle_ppr_residual_multi(int64_t n, const int64_t* rp, const int32_t* ci, int32_t B, const int64_t* src,
                              const double* alpha, const double* Y, double* res) {
  if (n < 1 || B < 1 || !rp || !ci || !src || !alpha || !Y || !res) return -1;
  for (int32_t j = 0; j < B; ++j)
    if (src[j] < 0 || src[j] >= n || !(alpha[j] > 0.0 && alpha[j] < 1.0)) return -1;
  const size_t nb = (size_t)n * (size_t)B;
  double* inv_d = inverse_degrees(n, rp);
  double* py = (double*)malloc(sizeof(double) * nb);
  if (!inv_d || !py) {
    free(inv_d); free(py);
    return -2;
  }
  apply_P_multi(n, B, rp, ci, inv_d, Y, py);
  for (int32_t j = 0; j < B; ++j) {
    double acc = 0.0;
    for (int64_t v = 0; v < n; ++v) {
      double e = (1.0 - alpha[j]) * py[(size_t)v * B + j] - Y[(size_t)v * B + j];
      if (v == src[j]) e += alpha[j];
      acc += e < 0.0 ? -e : e;
    }
    res[j] = acc;
  }
  free(inv_d); free(py);
  return 0;
}

/* Threads of the OpenMP loops from here on (t <= 0: back to the count the
 * process started with, e.g. from OMP_NUM_THREADS). */
void oracle_set_threads(int t) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  extern int omp_get_max_threads(void);
  static int initial = 0;
  if (!initial) initial = omp_get_max_threads();
  omp_set_num_threads(t > 0 ? t : initial);
#else
  (void)t;
#endif
}

int oracle_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
