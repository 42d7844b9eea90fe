/*
 * Oracle: a plain, single-threaded FP64 CPU implementation of the
 * Schwarz-preconditioned restarted GMRES solve of a 3x3-block Jacobian.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check
 * and the benchmark's CPU-baseline leg may load this library.  It shares no
 * code, header, table or helper with the GPU implementation; it is written
 * for readability, not speed.
 *
 * Paper: Jackson, Taroni, Ponting, "A Two-Level Variant of Additive Schwarz
 * Preconditioning for Use in Reservoir Simulation" (arXiv:1401.7227).
 *
 *   problem        Section 2: r = b - A x with b = R and A = -J; unknowns
 *                  grouped per cell into 3-vectors, 3x3 sub-matrices
 *                  (Section 1).
 *   classical AS   eq. (3.3)-(3.4): B^-1 = sum_i R_i^T A_i^-1 R_i,
 *                  A_i = R_i A R_i^T, R_i restricts to subdomain i.
 *   two-level      Section 4, eq. (4.1): R_i keeps subdomain i and
 *                  coarsens everything else (near field shared with
 *                  neighbours, far field shared by all), coarsening by
 *                  summation of matrix elements (Appendix B, eq. (B.3)).
 *                  Combination (4.2)-(4.5): keep each subdomain's own rows,
 *                  discard the coarse solution (restricted AS).
 *   local solver   Section 2: block ILU(0), 3x3 pivots inverted directly;
 *                  Section 6 generalises the exact local solve of Section 5
 *                  to such incomplete factorisations.  Exact mode = dense
 *                  Gaussian elimination (Section 5).
 *   accelerator    Section 2: GMRES; here restarted, right-preconditioned,
 *                  modified Gram-Schmidt, Givens rotations.
 *
 * Readings where the paper is silent (overlap, box geometry, ordering inside
 * A_i, per-component lumping of 3-unknown cells, GMRES details) are listed in
 * the design notes of the repository; the code below states each one where
 * it is used.
 *
 * Status codes: 0 ok, 1 not converged, -1 invalid input, -2 out of memory,
 * -3 singular pivot, -4 non-finite input.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_INVALID (-1)
#define OR_OOM (-2)
#define OR_SINGULAR (-3)
#define OR_NONFINITE (-4)

#define KIND_NONE 0
#define KIND_CLASSICAL 1
#define KIND_TWO_LEVEL 2

#define COMBINE_ADDITIVE 0
#define COMBINE_RESTRICTED 1

#define LOCAL_ILU0 0
#define LOCAL_EXACT 1

/* Outside cells in the two-level form (Section 5 compares the three):
 * near and far fields, the near field only (far cells dropped, in effect
 * additive Schwarz with coarsened overlap) or the far field only (every
 * outside cell lumped into far boxes). */
#define FIELD_NEAR_FAR 0
#define FIELD_NEAR 1
#define FIELD_FAR 2

/* Global coarse-grid correction added to the Schwarz preconditioner:
 * eq. (3.5)-(3.6) (added to the local solves) or eq. (3.7)-(3.8) (applied
 * after them to the remaining residual). */
#define COARSE_NONE 0
#define COARSE_ADDITIVE 1
#define COARSE_TWO_STAGE 2

static char g_err[512];

const char *or_last_error(void) { return g_err; }

static void set_err(const char *msg, long a) {
  snprintf(g_err, sizeof g_err, "%s (%ld)", msg, a);
}

/* ------------------------------------------------------------------ */
/* The matrix A: BSR with 3x3 row-major blocks on an nx*ny*nz grid,    */
/* cell c = (ix*ny + iy)*nz + iz.                                       */
/* ------------------------------------------------------------------ */
typedef struct {
  int nx, ny, nz, N;
  const int *rp;      /* N+1 */
  const int *ci;      /* nnzb */
  const double *v;    /* 9*nnzb */
} Mat;

/* y = A x (x, y of length 3N). */
void or_spmv(int N, const int *rp, const int *ci, const double *v,
             const double *x, double *y) {
  for (int r = 0; r < N; r++) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int e = rp[r]; e < rp[r + 1]; e++) {
      const double *B = v + 9 * (size_t)e;
      const double *xc = x + 3 * (size_t)ci[e];
      s0 += B[0] * xc[0] + B[1] * xc[1] + B[2] * xc[2];
      s1 += B[3] * xc[0] + B[4] * xc[1] + B[5] * xc[2];
      s2 += B[6] * xc[0] + B[7] * xc[1] + B[8] * xc[2];
    }
    y[3 * (size_t)r] = s0;
    y[3 * (size_t)r + 1] = s1;
    y[3 * (size_t)r + 2] = s2;
  }
}

static int check_matrix(const Mat *A) {
  if (A->nx < 1 || A->ny < 1 || A->nz < 1 || A->N != A->nx * A->ny * A->nz) {
    set_err("grid does not match the number of block rows", A->N);
    return OR_INVALID;
  }
  if (A->rp[0] != 0) { set_err("row_ptr[0] must be 0", A->rp[0]); return OR_INVALID; }
  for (int r = 0; r < A->N; r++) {
    if (A->rp[r + 1] < A->rp[r]) { set_err("row_ptr not monotone at row", r); return OR_INVALID; }
    int has_diag = 0;
    for (int e = A->rp[r]; e < A->rp[r + 1]; e++) {
      int c = A->ci[e];
      if (c < 0 || c >= A->N) { set_err("column out of range in row", r); return OR_INVALID; }
      if (e > A->rp[r] && A->ci[e - 1] >= c) { set_err("columns not strictly increasing in row", r); return OR_INVALID; }
      if (c == r) has_diag = 1;
      for (int k = 0; k < 9; k++)
        if (!isfinite(A->v[9 * (size_t)e + k])) { set_err("non-finite matrix value in row", r); return OR_NONFINITE; }
    }
    if (!has_diag) { set_err("missing diagonal block in row", r); return OR_INVALID; }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* 3x3 block helpers                                                    */
/* ------------------------------------------------------------------ */

/* C = A * B */
static void mul33(const double *A, const double *B, double *C) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

/* y -= A x (3-vectors) */
static void submv(const double *A, const double *x, double *y) {
  for (int i = 0; i < 3; i++) y[i] -= A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}

/* Inverse of a 3x3 block by Gauss-Jordan elimination with partial
 * pivoting.  Returns 0 on success, -1 if a pivot is exactly zero or the
 * result is not finite (the singular-pivot error of the setup). */
static int inv33(const double *A, double *Ainv) {
  double a[3][6];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      a[i][j] = A[3 * i + j];
      a[i][3 + j] = (i == j) ? 1.0 : 0.0;
    }
  for (int c = 0; c < 3; c++) {
    int p = c;
    for (int r = c + 1; r < 3; r++)
      if (fabs(a[r][c]) > fabs(a[p][c])) p = r;
    if (!(fabs(a[p][c]) > 0.0)) return -1;
    if (p != c)
      for (int j = 0; j < 6; j++) { double t = a[c][j]; a[c][j] = a[p][j]; a[p][j] = t; }
    double piv = a[c][c];
    for (int j = 0; j < 6; j++) a[c][j] /= piv;
    for (int r = 0; r < 3; r++) {
      if (r == c) continue;
      double f = a[r][c];
      if (f != 0.0)
        for (int j = 0; j < 6; j++) a[r][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      Ainv[3 * i + j] = a[i][3 + j];
      if (!isfinite(Ainv[3 * i + j])) return -1;
    }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Preconditioner data                                                  */
/* ------------------------------------------------------------------ */
typedef struct {
  int n;          /* block rows of A_i: fine rows first, then coarse rows */
  int nfine;      /* fine rows (cells of the overlapping subdomain F_i)  */
  int ncoarse;    /* coarse rows (lumped groups of outside cells)        */
  int *cell;      /* [nfine] global cell of each fine row, increasing     */
  int *owned;     /* [nfine] 1 if the cell belongs to this subdomain     */
  int *label;     /* [N] row of A_i that each global cell maps to, -1 none */
  int *rp, *ci;   /* CSR pattern of A_i (columns increasing)              */
  double *a;      /* [9*nnz] assembled A_i = R_i A R_i^T                  */
  double *f;      /* [9*nnz] ILU(0) factors: L below the diagonal (unit   */
                  /* diagonal implied), U above, D^-1 on the diagonal     */
  double *lu;     /* exact mode: dense LU of A_i, (3n)^2                  */
  int *piv;       /* exact mode: row pivots                               */
} Sub;

typedef struct {
  int kind, combine, local;
  int sx, sy, overlap;
  int near[3], far[3];
  int field;
  int N, nsub;
  Sub *sub;
  int *owner;     /* [N] subdomain owning each cell */
  /* global coarse-grid correction */
  int coarse;
  int cbox[3];    /* coarse box size */
  int nC;         /* coarse variables (boxes of the global box grid) */
  int *cvar;      /* [N] coarse variable of each cell */
  double *clu;    /* dense LU of A_C = R_C A R_C^T, (3 nC)^2 */
  int *cpiv;
  Mat A;          /* the matrix (the caller keeps its arrays alive) */
} Precond;

void or_precond_free(Precond *P);

/* Balanced split of n columns into k parts: the first (n mod k) parts get
 * one extra column.  Returns the part of column i. */
static int split_part(int n, int k, int i) {
  int base = n / k, rem = n % k;
  int big = rem * (base + 1);
  if (i < big) return i / (base + 1);
  return rem + (i - big) / base;
}

/* Undirected adjacency of A's block graph (pattern of A plus its
 * transpose), used for the algebraic overlap. */
typedef struct { int *ptr, *idx; } Graph;

static int build_graph(const Mat *A, Graph *G) {
  int N = A->N;
  int *deg = calloc((size_t)N, sizeof(int));
  if (!deg) return OR_OOM;
  for (int r = 0; r < N; r++)
    for (int e = A->rp[r]; e < A->rp[r + 1]; e++) {
      int c = A->ci[e];
      if (c == r) continue;
      deg[r]++;
      deg[c]++;
    }
  G->ptr = malloc(((size_t)N + 1) * sizeof(int));
  size_t tot = 0;
  for (int r = 0; r < N; r++) tot += deg[r];
  G->idx = malloc((tot ? tot : 1) * sizeof(int));
  if (!G->ptr || !G->idx) { free(deg); return OR_OOM; }
  G->ptr[0] = 0;
  for (int r = 0; r < N; r++) G->ptr[r + 1] = G->ptr[r] + deg[r];
  memset(deg, 0, (size_t)N * sizeof(int));
  for (int r = 0; r < N; r++)
    for (int e = A->rp[r]; e < A->rp[r + 1]; e++) {
      int c = A->ci[e];
      if (c == r) continue;
      G->idx[G->ptr[r] + deg[r]++] = c;
      G->idx[G->ptr[c] + deg[c]++] = r;
    }
  free(deg);
  return OR_OK;
}

static int box_index(int ix, int iy, int iz, const int C[3], int ny, int nz) {
  int nby = (ny + C[1] - 1) / C[1], nbz = (nz + C[2] - 1) / C[2];
  return ((ix / C[0]) * nby + iy / C[1]) * nbz + iz / C[2];
}

/* Labels of subdomain s: fine cells get 0..nfine-1 in increasing global
 * order; for the two-level form the remaining cells are lumped.
 * Region of an outside cell: "near" if its owner shares a face with s in
 * the sx*sy subdomain grid, else "far".  A coarse variable is a non-empty
 * (near box intersect near region) or (far box intersect far region); near
 * variables are numbered first by box index, then far variables by box
 * index, all after the fine rows (the layout of eq. (4.4)). */
static int make_labels(const Mat *A, const Precond *P, const Graph *G, int s, Sub *S) {
  int N = A->N;
  int *dist = malloc((size_t)N * sizeof(int));
  int *queue = malloc((size_t)N * sizeof(int));
  S->label = malloc((size_t)N * sizeof(int));
  if (!dist || !queue || !S->label) { free(dist); free(queue); return OR_OOM; }
  for (int c = 0; c < N; c++) dist[c] = -1;
  int qh = 0, qt = 0;
  for (int c = 0; c < N; c++)
    if (P->owner[c] == s) { dist[c] = 0; queue[qt++] = c; }
  /* breadth-first growth by graph distance up to the overlap */
  while (qh < qt) {
    int c = queue[qh++];
    if (dist[c] >= P->overlap) continue;
    for (int e = G->ptr[c]; e < G->ptr[c + 1]; e++) {
      int d = G->idx[e];
      if (dist[d] < 0) { dist[d] = dist[c] + 1; queue[qt++] = d; }
    }
  }
  int nfine = 0;
  for (int c = 0; c < N; c++) {
    if (dist[c] >= 0) S->label[c] = nfine++;
    else S->label[c] = -1;
  }
  S->nfine = nfine;
  S->cell = malloc((size_t)(nfine ? nfine : 1) * sizeof(int));
  S->owned = malloc((size_t)(nfine ? nfine : 1) * sizeof(int));
  if (!S->cell || !S->owned) { free(dist); free(queue); return OR_OOM; }
  for (int c = 0; c < N; c++)
    if (S->label[c] >= 0) {
      S->cell[S->label[c]] = c;
      S->owned[S->label[c]] = (P->owner[c] == s);
    }
  S->ncoarse = 0;
  if (P->kind == KIND_TWO_LEVEL) {
    int px = s / P->sy, py = s % P->sy;
    int nny = A->ny, nnz = A->nz;
    int nbn = ((A->nx + P->near[0] - 1) / P->near[0]) * ((nny + P->near[1] - 1) / P->near[1]) *
              ((nnz + P->near[2] - 1) / P->near[2]);
    int nbf = ((A->nx + P->far[0] - 1) / P->far[0]) * ((nny + P->far[1] - 1) / P->far[1]) *
              ((nnz + P->far[2] - 1) / P->far[2]);
    int *near_id = malloc((size_t)nbn * sizeof(int));
    int *far_id = malloc((size_t)nbf * sizeof(int));
    /* region code per cell: 0 fine, 1 near, 2 far */
    if (!near_id || !far_id) { free(near_id); free(far_id); free(dist); free(queue); return OR_OOM; }
    for (int k = 0; k < nbn; k++) near_id[k] = -1;
    for (int k = 0; k < nbf; k++) far_id[k] = -1;
    for (int c = 0; c < N; c++) {
      if (S->label[c] >= 0) continue;
      int o = P->owner[c];
      int ox = o / P->sy, oy = o % P->sy;
      int is_near = (abs(ox - px) + abs(oy - py)) == 1 && P->field != FIELD_FAR;
      int ix = c / (nny * nnz), iy = (c / nnz) % nny, iz = c % nnz;
      if (is_near) near_id[box_index(ix, iy, iz, P->near, nny, nnz)] = 0;
      else if (P->field != FIELD_NEAR) far_id[box_index(ix, iy, iz, P->far, nny, nnz)] = 0;
    }
    int next = nfine;
    for (int k = 0; k < nbn; k++) if (near_id[k] == 0) near_id[k] = next++;
    for (int k = 0; k < nbf; k++) if (far_id[k] == 0) far_id[k] = next++;
    S->ncoarse = next - nfine;
    for (int c = 0; c < N; c++) {
      if (S->label[c] >= 0) continue;
      int o = P->owner[c];
      int ox = o / P->sy, oy = o % P->sy;
      int is_near = (abs(ox - px) + abs(oy - py)) == 1 && P->field != FIELD_FAR;
      int ix = c / (nny * nnz), iy = (c / nnz) % nny, iz = c % nnz;
      if (is_near) S->label[c] = near_id[box_index(ix, iy, iz, P->near, nny, nnz)];
      else if (P->field != FIELD_NEAR) S->label[c] = far_id[box_index(ix, iy, iz, P->far, nny, nnz)];
      /* near field only: far cells stay unlabelled (dropped) */
    }
    free(near_id);
    free(far_id);
  }
  S->n = S->nfine + S->ncoarse;
  free(dist);
  free(queue);
  return OR_OK;
}

/* A_i = R_i A R_i^T: entry (u, v) is the 3x3 sum of A_ab over all cells a
 * labelled u and b labelled v (eq. (3.4) for selection, eq. (B.3) for
 * lumping, applied per unknown component).  Cells without a label (outside
 * a classical subdomain) are dropped.  The pattern is every (u, v) reached
 * by a structural entry of A. */
static int assemble(const Mat *A, Sub *S) {
  int N = A->N, n = S->n;
  /* cells of each label, in increasing cell order */
  int *cnt = calloc((size_t)n + 1, sizeof(int));
  int *members = malloc((size_t)N * sizeof(int));
  double *acc = calloc((size_t)9 * n, sizeof(double));
  int *mark = malloc((size_t)n * sizeof(int));
  int *cols = malloc((size_t)n * sizeof(int));
  if (!cnt || !members || !acc || !mark || !cols) goto oom;
  for (int c = 0; c < N; c++) if (S->label[c] >= 0) cnt[S->label[c] + 1]++;
  for (int u = 0; u < n; u++) cnt[u + 1] += cnt[u];
  {
    int *fill = malloc((size_t)n * sizeof(int));
    if (!fill) goto oom;
    memcpy(fill, cnt, (size_t)n * sizeof(int));
    for (int c = 0; c < N; c++) if (S->label[c] >= 0) members[fill[S->label[c]]++] = c;
    free(fill);
  }
  for (int u = 0; u < n; u++) mark[u] = -1;
  /* first pass: pattern sizes */
  S->rp = malloc(((size_t)n + 1) * sizeof(int));
  if (!S->rp) goto oom;
  S->rp[0] = 0;
  for (int u = 0; u < n; u++) {
    int nc = 0;
    for (int m = cnt[u]; m < cnt[u + 1]; m++) {
      int a = members[m];
      for (int e = A->rp[a]; e < A->rp[a + 1]; e++) {
        int v = S->label[A->ci[e]];
        if (v < 0) continue;
        if (mark[v] != u) { mark[v] = u; nc++; }
      }
    }
    S->rp[u + 1] = S->rp[u] + nc;
  }
  int nnz = S->rp[n];
  S->ci = malloc((size_t)(nnz ? nnz : 1) * sizeof(int));
  S->a = malloc((size_t)9 * (nnz ? nnz : 1) * sizeof(double));
  if (!S->ci || !S->a) goto oom;
  for (int u = 0; u < n; u++) mark[u] = -1;
  /* second pass: accumulate each row densely, then emit sorted columns */
  for (int u = 0; u < n; u++) {
    int nc = 0;
    for (int m = cnt[u]; m < cnt[u + 1]; m++) {
      int a = members[m];
      for (int e = A->rp[a]; e < A->rp[a + 1]; e++) {
        int v = S->label[A->ci[e]];
        if (v < 0) continue;
        if (mark[v] != u) {
          mark[v] = u;
          cols[nc++] = v;
          memset(acc + 9 * (size_t)v, 0, 9 * sizeof(double));
        }
        for (int k = 0; k < 9; k++) acc[9 * (size_t)v + k] += A->v[9 * (size_t)e + k];
      }
    }
    /* insertion sort of the (short) column list */
    for (int i = 1; i < nc; i++) {
      int t = cols[i], j = i - 1;
      while (j >= 0 && cols[j] > t) { cols[j + 1] = cols[j]; j--; }
      cols[j + 1] = t;
    }
    for (int i = 0; i < nc; i++) {
      int e = S->rp[u] + i;
      S->ci[e] = cols[i];
      memcpy(S->a + 9 * (size_t)e, acc + 9 * (size_t)cols[i], 9 * sizeof(double));
    }
  }
  free(cnt); free(members); free(acc); free(mark); free(cols);
  return OR_OK;
oom:
  free(cnt); free(members); free(acc); free(mark); free(cols);
  return OR_OOM;
}

/* Block ILU(0) on the pattern of A_i in the row (IKJ) form: for each row i,
 * for each k < i in the row in increasing order: L_ik = a_ik D_k^-1, then
 * a_ij -= L_ik U_kj for every j > k that is in both row k and row i.  The
 * updated diagonal is the pivot D_i; its inverse is stored in its place. */
static int ilu0(Sub *S, int *bad_row) {
  int n = S->n;
  int nnz = S->rp[n];
  S->f = malloc((size_t)9 * (nnz ? nnz : 1) * sizeof(double));
  int *pos = malloc((size_t)(n ? n : 1) * sizeof(int));
  int *diag = malloc((size_t)(n ? n : 1) * sizeof(int));
  if (!S->f || !pos || !diag) { free(pos); free(diag); return OR_OOM; }
  memcpy(S->f, S->a, (size_t)9 * nnz * sizeof(double));
  for (int i = 0; i < n; i++) {
    pos[i] = -1;
    diag[i] = -1;
    for (int e = S->rp[i]; e < S->rp[i + 1]; e++) if (S->ci[e] == i) diag[i] = e;
    if (diag[i] < 0) { *bad_row = i; free(pos); free(diag); return OR_SINGULAR; }
  }
  double L[9], t[9];
  for (int i = 0; i < n; i++) {
    for (int e = S->rp[i]; e < S->rp[i + 1]; e++) pos[S->ci[e]] = e;
    for (int e = S->rp[i]; e < S->rp[i + 1]; e++) {
      int k = S->ci[e];
      if (k >= i) break;
      mul33(S->f + 9 * (size_t)e, S->f + 9 * (size_t)diag[k], L);
      memcpy(S->f + 9 * (size_t)e, L, sizeof L);
      for (int ek = diag[k] + 1; ek < S->rp[k + 1]; ek++) {
        int j = S->ci[ek];
        int ej = pos[j];
        if (ej < 0) continue;
        mul33(L, S->f + 9 * (size_t)ek, t);
        for (int q = 0; q < 9; q++) S->f[9 * (size_t)ej + q] -= t[q];
      }
    }
    double Dinv[9];
    if (inv33(S->f + 9 * (size_t)diag[i], Dinv) != 0) {
      *bad_row = i; free(pos); free(diag); return OR_SINGULAR;
    }
    memcpy(S->f + 9 * (size_t)diag[i], Dinv, sizeof Dinv);
    for (int e = S->rp[i]; e < S->rp[i + 1]; e++) pos[S->ci[e]] = -1;
  }
  free(pos);
  free(diag);
  return OR_OK;
}

/* Exact local solver (Section 5): dense LU with partial pivoting of the
 * scalar 3n x 3n matrix A_i. */
/* Dense LU with partial pivoting of the m x m row-major matrix M, in
 * place (P M = L U, unit L below the diagonal); piv[c] is the row swapped
 * with row c at step c.  bad receives the failing column on a zero pivot. */
static int lu_factor(double *M, int *piv, int m, int *bad) {
  for (int c = 0; c < m; c++) {
    int p = c;
    for (int r = c + 1; r < m; r++) if (fabs(M[(size_t)r * m + c]) > fabs(M[(size_t)p * m + c])) p = r;
    piv[c] = p;
    if (!(fabs(M[(size_t)p * m + c]) > 0.0)) { *bad = c; return OR_SINGULAR; }
    if (p != c)
      for (int j = 0; j < m; j++) { double t = M[(size_t)c * m + j]; M[(size_t)c * m + j] = M[(size_t)p * m + j]; M[(size_t)p * m + j] = t; }
    for (int r = c + 1; r < m; r++) {
      double f = M[(size_t)r * m + c] / M[(size_t)c * m + c];
      M[(size_t)r * m + c] = f;
      if (f != 0.0)
        for (int j = c + 1; j < m; j++) M[(size_t)r * m + j] -= f * M[(size_t)c * m + j];
    }
  }
  return OR_OK;
}

/* x <- M^-1 x with the factors of lu_factor. */
static void lu_solve(const double *M, const int *piv, int m, double *x) {
  /* the factorisation swapped whole rows, so P A = L U: permute first */
  for (int c = 0; c < m; c++) {
    int p = piv[c];
    if (p != c) { double t = x[c]; x[c] = x[p]; x[p] = t; }
  }
  for (int c = 0; c < m; c++)
    for (int r = c + 1; r < m; r++) x[r] -= M[(size_t)r * m + c] * x[c];
  for (int r = m - 1; r >= 0; r--) {
    double s = x[r];
    for (int j = r + 1; j < m; j++) s -= M[(size_t)r * m + j] * x[j];
    x[r] = s / M[(size_t)r * m + r];
  }
}

static int dense_lu(Sub *S, int *bad_row) {
  int m = 3 * S->n;
  size_t mm = (size_t)m * (size_t)m;
  S->lu = calloc(mm ? mm : 1, sizeof(double));
  S->piv = malloc((size_t)(m ? m : 1) * sizeof(int));
  if (!S->lu || !S->piv) return OR_OOM;
  for (int u = 0; u < S->n; u++)
    for (int e = S->rp[u]; e < S->rp[u + 1]; e++) {
      int v = S->ci[e];
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
          S->lu[(size_t)(3 * u + i) * m + 3 * v + j] = S->a[9 * (size_t)e + 3 * i + j];
    }
  int bad = 0;
  int st = lu_factor(S->lu, S->piv, m, &bad);
  if (st != OR_OK) *bad_row = bad / 3;
  return st;
}

/* Solve A_i xh = rh with the subdomain's local solver. */
static void local_solve(const Precond *P, const Sub *S, const double *rh, double *xh) {
  int n = S->n;
  if (P->local == LOCAL_EXACT) {
    memcpy(xh, rh, (size_t)3 * n * sizeof(double));
    lu_solve(S->lu, S->piv, 3 * n, xh);
    return;
  }
  /* forward: y_i = rh_i - sum_{k<i} L_ik y_k (unit lower) */
  for (int i = 0; i < n; i++) {
    double y[3] = {rh[3 * i], rh[3 * i + 1], rh[3 * i + 2]};
    for (int e = S->rp[i]; e < S->rp[i + 1]; e++) {
      int k = S->ci[e];
      if (k >= i) break;
      submv(S->f + 9 * (size_t)e, xh + 3 * (size_t)k, y);
    }
    xh[3 * i] = y[0]; xh[3 * i + 1] = y[1]; xh[3 * i + 2] = y[2];
  }
  /* backward: x_i = D_i^-1 (y_i - sum_{j>i} U_ij x_j) */
  for (int i = n - 1; i >= 0; i--) {
    double t[3] = {xh[3 * i], xh[3 * i + 1], xh[3 * i + 2]};
    const double *Dinv = NULL;
    for (int e = S->rp[i]; e < S->rp[i + 1]; e++) {
      int j = S->ci[e];
      if (j < i) continue;
      if (j == i) { Dinv = S->f + 9 * (size_t)e; continue; }
      submv(S->f + 9 * (size_t)e, xh + 3 * (size_t)j, t);
    }
    for (int q = 0; q < 3; q++)
      xh[3 * i + q] = Dinv[3 * q] * t[0] + Dinv[3 * q + 1] * t[1] + Dinv[3 * q + 2] * t[2];
  }
}

/* Restriction R_i r: fine rows copy the cell's 3 values, coarse rows sum
 * the values of their cells per component (eq. (B.2)). */
static void restrict_vec(const Sub *S, int N, const double *r, double *rh) {
  memset(rh, 0, (size_t)3 * S->n * sizeof(double));
  for (int i = 0; i < S->nfine; i++) {
    size_t c = (size_t)S->cell[i];
    rh[3 * i] = r[3 * c];
    rh[3 * i + 1] = r[3 * c + 1];
    rh[3 * i + 2] = r[3 * c + 2];
  }
  if (S->ncoarse == 0) return;
  for (int c = 0; c < N; c++) {
    int u = S->label[c];
    if (u < S->nfine) continue;
    rh[3 * u] += r[3 * (size_t)c];
    rh[3 * u + 1] += r[3 * (size_t)c + 1];
    rh[3 * u + 2] += r[3 * (size_t)c + 2];
  }
}

typedef struct {
  int kind, combine, sx, sy, overlap;
  int near[3], far[3];
  int local;
  int field;
  int coarse;
  int cbox[3];
} or_opts;

/* The global coarse operator of eq. (3.5)-(3.6): R_C sums the cells of each
 * box of a global box grid (per unknown component, as the lumping of
 * Appendix B), A_C = R_C A R_C^T is the 3x3-block matrix of the box sums of
 * A's blocks, factorised densely (the coarse problem is solved exactly). */
static int coarse_setup(Precond *P) {
  const Mat *A = &P->A;
  int N = A->N, ny = A->ny, nz = A->nz;
  int nbx = (A->nx + P->cbox[0] - 1) / P->cbox[0], nby = (ny + P->cbox[1] - 1) / P->cbox[1],
      nbz = (nz + P->cbox[2] - 1) / P->cbox[2];
  P->nC = nbx * nby * nbz;  /* boxes clipped at the boundary are never empty */
  P->cvar = malloc((size_t)N * sizeof(int));
  int m = 3 * P->nC;
  P->clu = calloc((size_t)m * m, sizeof(double));
  P->cpiv = malloc((size_t)m * sizeof(int));
  if (!P->cvar || !P->clu || !P->cpiv) return OR_OOM;
  for (int c = 0; c < N; c++) {
    int ix = c / (ny * nz), iy = (c / nz) % ny, iz = c % nz;
    P->cvar[c] = box_index(ix, iy, iz, P->cbox, ny, nz);
  }
  for (int a = 0; a < N; a++)
    for (int e = A->rp[a]; e < A->rp[a + 1]; e++) {
      int U = P->cvar[a], V = P->cvar[A->ci[e]];
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) P->clu[(size_t)(3 * U + i) * m + 3 * V + j] += A->v[9 * (size_t)e + 3 * i + j];
    }
  int bad = 0;
  int st = lu_factor(P->clu, P->cpiv, m, &bad);
  if (st == OR_SINGULAR) snprintf(g_err, sizeof g_err, "singular coarse operator at coarse row %d", bad / 3);
  return st;
}

/* z += R_C^T A_C^-1 R_C r: box sums of r, the coarse solve, and the coarse
 * value given back to every cell of its box. */
static int coarse_correct(const Precond *P, const double *r, double *z) {
  int N = P->N, m = 3 * P->nC;
  double *xc = calloc((size_t)m, sizeof(double));
  if (!xc) return OR_OOM;
  for (int c = 0; c < N; c++)
    for (int q = 0; q < 3; q++) xc[3 * P->cvar[c] + q] += r[3 * (size_t)c + q];
  lu_solve(P->clu, P->cpiv, m, xc);
  for (int c = 0; c < N; c++)
    for (int q = 0; q < 3; q++) z[3 * (size_t)c + q] += xc[3 * P->cvar[c] + q];
  free(xc);
  return OR_OK;
}

int or_precond_setup(int nx, int ny, int nz, const int *rp, const int *ci, const double *v,
                     const or_opts *o, Precond **out) {
  g_err[0] = 0;
  *out = NULL;
  Mat A = {nx, ny, nz, nx * ny * nz, rp, ci, v};
  int st = check_matrix(&A);
  if (st != OR_OK) return st;
  if (o->kind < KIND_NONE || o->kind > KIND_TWO_LEVEL || o->combine < 0 || o->combine > 1 ||
      o->local < 0 || o->local > 1 || o->field < FIELD_NEAR_FAR || o->field > FIELD_FAR ||
      o->coarse < COARSE_NONE || o->coarse > COARSE_TWO_STAGE ||
      (o->coarse != COARSE_NONE && (o->kind == KIND_NONE || o->cbox[0] < 1 || o->cbox[1] < 1 || o->cbox[2] < 1))) {
    set_err("bad preconditioner option", o->kind);
    return OR_INVALID;
  }
  Precond *P = calloc(1, sizeof(Precond));
  if (!P) return OR_OOM;
  P->kind = o->kind; P->combine = o->combine; P->local = o->local;
  P->sx = o->sx; P->sy = o->sy; P->overlap = o->overlap;
  memcpy(P->near, o->near, sizeof P->near);
  memcpy(P->far, o->far, sizeof P->far);
  P->field = o->field;
  P->coarse = o->coarse;
  memcpy(P->cbox, o->cbox, sizeof P->cbox);
  P->A = A;
  P->N = A.N;
  if (P->kind == KIND_NONE) { *out = P; return OR_OK; }
  if (o->sx < 1 || o->sy < 1 || o->sx > nx || o->sy > ny || o->overlap < 0) {
    set_err("bad subdomain split or overlap", o->sx);
    free(P);
    return OR_INVALID;
  }
  if (P->kind == KIND_TWO_LEVEL)
    for (int d = 0; d < 3; d++)
      if (o->near[d] < 1 || o->far[d] < 1) { set_err("bad coarsening box", d); free(P); return OR_INVALID; }
  P->nsub = o->sx * o->sy;
  P->owner = malloc((size_t)A.N * sizeof(int));
  P->sub = calloc((size_t)P->nsub, sizeof(Sub));
  if (!P->owner || !P->sub) { or_precond_free(P); return OR_OOM; }
  for (int c = 0; c < A.N; c++) {
    int ix = c / (ny * nz), iy = (c / nz) % ny;
    P->owner[c] = split_part(nx, o->sx, ix) * o->sy + split_part(ny, o->sy, iy);
  }
  Graph G = {0, 0};
  st = build_graph(&A, &G);
  if (st != OR_OK) { free(G.ptr); free(G.idx); or_precond_free(P); return st; }
  for (int s = 0; s < P->nsub && st == OR_OK; s++) {
    Sub *S = &P->sub[s];
    st = make_labels(&A, P, &G, s, S);
    if (st == OR_OK) st = assemble(&A, S);
    if (st == OR_OK) {
      int bad = -1;
      st = (P->local == LOCAL_EXACT) ? dense_lu(S, &bad) : ilu0(S, &bad);
      if (st == OR_SINGULAR) {
        int cellrow = (bad >= 0 && bad < S->nfine) ? S->cell[bad] : -1;
        snprintf(g_err, sizeof g_err,
                 "singular pivot in subdomain %d, local block row %d (global cell %d)", s, bad, cellrow);
      }
    }
  }
  free(G.ptr);
  free(G.idx);
  if (st == OR_OK && P->coarse != COARSE_NONE) st = coarse_setup(P);
  if (st != OR_OK) { or_precond_free(P); return st; }
  *out = P;
  return OR_OK;
}

void or_precond_free(Precond *P) {
  if (!P) return;
  if (P->sub)
    for (int s = 0; s < P->nsub; s++) {
      Sub *S = &P->sub[s];
      free(S->cell); free(S->owned); free(S->label); free(S->rp); free(S->ci);
      free(S->a); free(S->f); free(S->lu); free(S->piv);
    }
  free(P->sub);
  free(P->owner);
  free(P->cvar);
  free(P->clu);
  free(P->cpiv);
  free(P);
}

/* z = B^-1 r.
 *   additive   (3.3): z = sum_i R_i^T A_i^-1 R_i r over the fine rows of
 *              each subdomain, contributions summed in subdomain order;
 *   restricted (4.2): z = sum_i P_i (A_i^-1 R_i r), each cell taking the
 *              value from its owning subdomain; the coarse part of the
 *              local solution is discarded;
 * then, with a global coarse grid, z += B_C^-1 r (eq. (3.5)) or
 * z += B_C^-1 (r - A z) (eq. (3.8)), B_C^-1 = R_C^T A_C^-1 R_C (eq. (3.6)). */
int or_precond_apply(const Precond *P, const double *r, double *z) {
  int N = P->N;
  if (P->kind == KIND_NONE) { memcpy(z, r, (size_t)3 * N * sizeof(double)); return OR_OK; }
  memset(z, 0, (size_t)3 * N * sizeof(double));
  for (int s = 0; s < P->nsub; s++) {
    const Sub *S = &P->sub[s];
    double *rh = malloc((size_t)3 * S->n * sizeof(double) + 1);
    double *xh = malloc((size_t)3 * S->n * sizeof(double) + 1);
    if (!rh || !xh) { free(rh); free(xh); return OR_OOM; }
    restrict_vec(S, N, r, rh);
    local_solve(P, S, rh, xh);
    for (int i = 0; i < S->nfine; i++) {
      if (P->combine == COMBINE_RESTRICTED && !S->owned[i]) continue;
      int c = S->cell[i];
      z[3 * (size_t)c] += xh[3 * i];
      z[3 * (size_t)c + 1] += xh[3 * i + 1];
      z[3 * (size_t)c + 2] += xh[3 * i + 2];
    }
    free(rh);
    free(xh);
  }
  if (P->coarse == COARSE_ADDITIVE) return coarse_correct(P, r, z);  /* eq. (3.5) */
  if (P->coarse == COARSE_TWO_STAGE) {                               /* eq. (3.8) */
    size_t n = (size_t)3 * N;
    double *az = malloc(n * sizeof(double));
    if (!az) return OR_OOM;
    or_spmv(N, P->A.rp, P->A.ci, P->A.v, z, az);
    for (size_t k = 0; k < n; k++) az[k] = r[k] - az[k];  /* (I - A B_AS^-1) r */
    int st = coarse_correct(P, az, z);
    free(az);
    return st;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Accessors for tests                                                  */
/* ------------------------------------------------------------------ */
int or_precond_nsub(const Precond *P) { return P->nsub; }

void or_sub_sizes(const Precond *P, int s, int *n, int *nfine, int *ncoarse, int *nnz) {
  const Sub *S = &P->sub[s];
  *n = S->n; *nfine = S->nfine; *ncoarse = S->ncoarse; *nnz = S->rp[S->n];
}

/* Copies out labels [N], fine cells [nfine], owned flags [nfine], the CSR
 * pattern, assembled values and ILU(0) factors (factors only in ILU mode). */
void or_sub_export(const Precond *P, int s, int *label, int *cell, int *owned, int *rp, int *ci,
                   double *a, double *f) {
  const Sub *S = &P->sub[s];
  int nnz = S->rp[S->n];
  if (label) memcpy(label, S->label, (size_t)P->N * sizeof(int));
  if (cell) memcpy(cell, S->cell, (size_t)S->nfine * sizeof(int));
  if (owned) memcpy(owned, S->owned, (size_t)S->nfine * sizeof(int));
  if (rp) memcpy(rp, S->rp, ((size_t)S->n + 1) * sizeof(int));
  if (ci) memcpy(ci, S->ci, (size_t)nnz * sizeof(int));
  if (a) memcpy(a, S->a, (size_t)9 * nnz * sizeof(double));
  if (f && S->f) memcpy(f, S->f, (size_t)9 * nnz * sizeof(double));
}

/* Local solve of subdomain s on a local right-hand side (length 3n). */
void or_sub_solve(const Precond *P, int s, const double *rh, double *xh) {
  local_solve(P, &P->sub[s], rh, xh);
}

/* ------------------------------------------------------------------ */
/* Restarted right-preconditioned GMRES(m)                              */
/* ------------------------------------------------------------------ */
typedef struct {
  int iters, cycles;
  double rel_res_true, rel_res_est;
} or_info;

static double dot(const double *a, const double *b, size_t n) {
  double s = 0;
  for (size_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

/* Solves A x = b from the initial guess in x.  One iteration is one
 * Arnoldi step.  A cycle ends when the Givens residual estimate reaches
 * rtol*||b||, at m steps, at a happy breakdown (h_{j+1,j} <= 1e-14 times
 * the norm of A z_j) or at the iteration limit; then x += B^-1 (V y) and
 * the true residual b - A x is recomputed.  fixed_iters > 0 runs exactly
 * that many steps with no convergence test (for comparisons at equal
 * iteration counts).  hist (optional, max_iters+1 entries) receives the
 * estimated relative residual after each step. */
int or_gmres(int nx, int ny, int nz, const int *rp, const int *ci, const double *v, const Precond *P,
             const double *b, double *x, int m, double rtol, int max_iters, int fixed_iters,
             or_info *info, double *hist) {
  g_err[0] = 0;
  int N = nx * ny * nz;
  size_t n = (size_t)3 * N;
  Mat A = {nx, ny, nz, N, rp, ci, v};
  memset(info, 0, sizeof *info);
  if (m < 1 || max_iters < 1 || fixed_iters < 0 || !(rtol >= 0)) { set_err("bad solver option", m); return OR_INVALID; }
  for (size_t i = 0; i < n; i++)
    if (!isfinite(b[i]) || !isfinite(x[i])) { set_err("non-finite b or x0 at unknown", (long)i); return OR_NONFINITE; }
  (void)A;
  double *V = malloc((size_t)(m + 1) * n * sizeof(double));
  double *H = calloc((size_t)(m + 1) * m, sizeof(double));
  double *cs = malloc((size_t)m * sizeof(double)), *sn = malloc((size_t)m * sizeof(double));
  double *g = malloc((size_t)(m + 1) * sizeof(double)), *y = malloc((size_t)m * sizeof(double));
  double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double)), *w = malloc(n * sizeof(double));
  if (!V || !H || !cs || !sn || !g || !y || !r || !z || !w) {
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(r); free(z); free(w);
    return OR_OOM;
  }
#define HH(i, j) H[(size_t)(i) * m + (j)]
  double bnorm = sqrt(dot(b, b, n));
  int status = OR_NOT_CONVERGED;
  if (bnorm == 0.0 && fixed_iters == 0) {
    memset(x, 0, n * sizeof(double));
    info->rel_res_true = info->rel_res_est = 0.0;
    status = OR_OK;
    goto done;
  }
  double scale = bnorm > 0 ? bnorm : 1.0;
  double tol = rtol * bnorm;
  or_spmv(N, rp, ci, v, x, r);
  for (size_t i = 0; i < n; i++) r[i] = b[i] - r[i];
  double beta = sqrt(dot(r, r, n));
  info->rel_res_true = info->rel_res_est = beta / scale;
  if (hist) hist[0] = beta / scale;
  if (fixed_iters == 0 && beta <= tol) { status = OR_OK; goto done; }
  int limit = fixed_iters > 0 ? fixed_iters : max_iters;
  while (1) {
    if (beta == 0.0) { status = OR_OK; break; }
    info->cycles++;
    for (size_t i = 0; i < n; i++) V[i] = r[i] / beta;
    for (int i = 0; i <= m; i++) g[i] = 0.0;
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; j++) {
      double *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
      int st = or_precond_apply(P, vj, z);
      if (st != OR_OK) { status = st; goto done; }
      or_spmv(N, rp, ci, v, z, w);
      info->iters++;
      double w0 = sqrt(dot(w, w, n));
      for (int i = 0; i <= j; i++) {
        const double *vi = V + (size_t)i * n;
        double h = dot(w, vi, n);
        HH(i, j) = h;
        for (size_t q = 0; q < n; q++) w[q] -= h * vi[q];
      }
      double hn = sqrt(dot(w, w, n));
      HH(j + 1, j) = hn;
      for (int i = 0; i < j; i++) {
        double t = cs[i] * HH(i, j) + sn[i] * HH(i + 1, j);
        HH(i + 1, j) = -sn[i] * HH(i, j) + cs[i] * HH(i + 1, j);
        HH(i, j) = t;
      }
      double rho = hypot(HH(j, j), HH(j + 1, j));
      if (rho == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
      else { cs[j] = HH(j, j) / rho; sn[j] = HH(j + 1, j) / rho; }
      HH(j, j) = rho;
      HH(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      info->rel_res_est = fabs(g[j + 1]) / scale;
      if (hist) hist[info->iters] = info->rel_res_est;
      if (hn <= 1e-14 * w0) break;                              /* happy breakdown */
      if (fixed_iters == 0 && fabs(g[j + 1]) <= tol) break;     /* converged estimate */
      if (info->iters >= limit) break;
      for (size_t q = 0; q < n; q++) vn[q] = w[q] / hn;
    }
    /* y = R^-1 g, x += B^-1 (V y) */
    for (int i = k - 1; i >= 0; i--) {
      double s = g[i];
      for (int j = i + 1; j < k; j++) s -= HH(i, j) * y[j];
      y[i] = s / HH(i, i);
    }
    memset(w, 0, n * sizeof(double));
    for (int i = 0; i < k; i++) {
      const double *vi = V + (size_t)i * n;
      for (size_t q = 0; q < n; q++) w[q] += y[i] * vi[q];
    }
    int st = or_precond_apply(P, w, z);
    if (st != OR_OK) { status = st; goto done; }
    for (size_t q = 0; q < n; q++) x[q] += z[q];
    or_spmv(N, rp, ci, v, x, r);
    for (size_t q = 0; q < n; q++) r[q] = b[q] - r[q];
    beta = sqrt(dot(r, r, n));
    info->rel_res_true = beta / scale;
    if (fixed_iters > 0) {
      if (info->iters >= fixed_iters) { status = OR_OK; break; }
    } else if (beta <= tol) { status = OR_OK; break; }
    if (info->iters >= limit) { status = OR_NOT_CONVERGED; break; }
  }
done:
#undef HH
  free(V); free(H); free(cs); free(sn); free(g); free(y); free(r); free(z); free(w);
  return status;
}
