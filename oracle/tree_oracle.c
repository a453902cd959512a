/*
 * tree_oracle.c -- CPU FP64 reference for the octree evaluation of the (screened) GWN
 * (Sec. 5.2 "Octree Traversal", after the fast winding numbers of Barill et al. 2018).
 *
 * TEST INFRASTRUCTURE ONLY, like dwg_oracle.c: plain recursive code, double precision,
 * OpenMP over independent queries. Shares nothing with the GPU library.
 *
 * Octree. The root cell is the cube [lo, lo + ext]^3 with lo = the per-axis minimum of the
 * points and ext = the largest per-axis extent. A point's cell at the deepest level D = 21
 * has integer coordinates c = floor((x - lo) * (2^D / ext)) clamped to [0, 2^D - 1]
 * (double arithmetic; ext == 0 puts every point in cell 0); its Morton code interleaves
 * the bits of (cx, cy, cz) with x the most significant of each triple. Points are ordered
 * by (code, index). A node is a non-empty cell; it is a leaf when it holds at most
 * `leaf` points or sits at level D, otherwise its non-empty children (in Morton order)
 * are nodes. A cell whose points all lie in one child cell is not a node of its own: it
 * holds exactly the points of that child, so every summary below and every decision of
 * the traversal would be the same for both; the deepest cell of such a chain is kept.
 * Nodes are numbered in depth-first pre-order.
 *
 * Node summary (Sec. 5.2): area A = sum a_j; mass centre c.m = sum a_j p_j / A (the first
 * point of the node when A == 0); r = the largest |p_j - c.m|; moment M = sum a_j n_j (the
 * area-weighted normal); dmax = the largest kernel radius max(delta_j, eps) in the node.
 *
 * Traversal of a query q from the root: a node whose centre is close, |q - c.m| <= crit,
 * is opened (its children visited, or its points summed one by one with the modified
 * kernel when it is a leaf); otherwise the node counts as one dipole M at c.m.
 * crit = max(beta r, r + dmax). The paper's criterion is beta r with beta = 2.3; the
 * second term keeps every point of a far node outside its own clamp radius, so that the
 * far-field dipole uses the kernel the point would have used (reading of the paper, which
 * evaluates at octree leaves rather than at the points).
 * A query is flagged when | |q - c.m| - crit | <= 1e-7 crit for a visited node (an FP32 or
 * differently ordered FP64 evaluation may decide the other way) or when a leaf pair sits
 * on a clamp boundary as in orc_gwn.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define TREE_DEPTH 21

typedef struct {
  int64_t start, end; /* range in the sorted order */
  int level, leaf, nchild;
  int64_t child[8];
  int64_t skip; /* pre-order index of the next node after this subtree */
  double area, cm[3], r, dmax, M[3];
} tnode;

typedef struct {
  uint64_t code;
  int64_t idx;
} tkey;

typedef struct {
  tnode* nodes;
  int64_t count, cap;
  const uint64_t* code; /* sorted codes */
  int leaf;
} tbuild;

static int cmp_key(const void* a, const void* b) {
  const tkey* x = (const tkey*)a;
  const tkey* y = (const tkey*)b;
  if (x->code != y->code) return x->code < y->code ? -1 : 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

static uint64_t spread21(uint64_t v) {
  uint64_t out = 0;
  for (int b = 0; b < TREE_DEPTH; ++b)
    if ((v >> b) & 1u) out |= (uint64_t)1 << (3 * b);
  return out;
}

static int64_t new_node(tbuild* t) {
  if (t->count == t->cap) {
    t->cap = t->cap ? 2 * t->cap : 1024;
    t->nodes = (tnode*)realloc(t->nodes, (size_t)t->cap * sizeof(tnode));
  }
  memset(&t->nodes[t->count], 0, sizeof(tnode));
  return t->count++;
}

/* true when every point of [s, e) lies in the same cell of level `level` */
static int one_cell(const tbuild* t, int64_t s, int64_t e, int level) {
  const int sh = 3 * (TREE_DEPTH - level);
  return (t->code[s] >> sh) == (t->code[e - 1] >> sh);
}

static int64_t build(tbuild* t, int64_t s, int64_t e, int level) {
  while (e - s > t->leaf && level < TREE_DEPTH && one_cell(t, s, e, level + 1)) ++level;
  const int64_t k = new_node(t);
  t->nodes[k].start = s;
  t->nodes[k].end = e;
  t->nodes[k].level = level;
  if (e - s <= t->leaf || level == TREE_DEPTH) {
    t->nodes[k].leaf = 1;
  } else {
    const int sh = 3 * (TREE_DEPTH - level - 1);
    int64_t i = s;
    for (int digit = 0; digit < 8; ++digit) {
      int64_t j = i;
      while (j < e && (int)((t->code[j] >> sh) & 7u) == digit) ++j;
      if (j > i) {
        const int64_t c = build(t, i, j, level + 1);
        tnode* nk = &t->nodes[k]; /* re-fetch: build() may have moved the array */
        nk->child[nk->nchild++] = c;
      }
      i = j;
    }
  }
  t->nodes[k].skip = t->count;
  return k;
}

/* Sorted order (perm) and the node list; returns the node count, or -1. */
static int64_t tree_build(const double* P, int64_t n, int leaf, int64_t* perm, tnode** nodes_out) {
  if (n < 1 || leaf < 1) return -1;
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = hi[d] = P[d * n];
    for (int64_t i = 1; i < n; ++i) {
      const double v = P[d * n + i];
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  }
  double ext = hi[0] - lo[0];
  if (hi[1] - lo[1] > ext) ext = hi[1] - lo[1];
  if (hi[2] - lo[2] > ext) ext = hi[2] - lo[2];
  const double cells = (double)((uint64_t)1 << TREE_DEPTH);
  tkey* key = (tkey*)malloc((size_t)n * sizeof(tkey));
  for (int64_t i = 0; i < n; ++i) {
    uint64_t c[3] = {0, 0, 0};
    if (ext > 0.0) {
      const double scale = cells / ext;
      for (int d = 0; d < 3; ++d) {
        double f = floor((P[d * n + i] - lo[d]) * scale);
        if (f < 0.0) f = 0.0;
        if (f > cells - 1.0) f = cells - 1.0;
        c[d] = (uint64_t)f;
      }
    }
    key[i].code = (spread21(c[0]) << 2) | (spread21(c[1]) << 1) | spread21(c[2]);
    key[i].idx = i;
  }
  qsort(key, (size_t)n, sizeof(tkey), cmp_key);
  uint64_t* code = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  for (int64_t i = 0; i < n; ++i) {
    code[i] = key[i].code;
    perm[i] = key[i].idx;
  }
  free(key);
  tbuild t = {NULL, 0, 0, code, leaf};
  build(&t, 0, n, 0);
  free(code);
  *nodes_out = t.nodes;
  return t.count;
}

/* Plain recursive octree: perm [n] (sorted position -> index); info [cap][4] = (start, end,
 * level, skip) in pre-order. Returns the node count (entries beyond cap are not written). */
int64_t orc_octree(const double* P, int64_t n, int leaf, int64_t* perm, int64_t* info, int64_t cap) {
  tnode* nodes = NULL;
  const int64_t cnt = tree_build(P, n, leaf, perm, &nodes);
  if (cnt < 0) return -1;
  for (int64_t k = 0; k < cnt && k < cap; ++k) {
    info[4 * k + 0] = nodes[k].start;
    info[4 * k + 1] = nodes[k].end;
    info[4 * k + 2] = nodes[k].level;
    info[4 * k + 3] = nodes[k].skip;
  }
  free(nodes);
  return cnt;
}

typedef struct {
  double s, c;
} nsum;
static inline void nadd(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static inline double nval(const nsum* a) { return a->s + a->c; }

typedef struct {
  nsum w, g[3];
} acc4;

/* One dipole of moment mv (= a n, or a node's M) at offset d = p - q with kernel radius
 * floor (0 for a far node): the w and grad w terms of orc_gwn's definition. */
static void dipole(acc4* a, double dx, double dy, double dz, const double mv[3], double floor_r, double s,
                   int want_grad) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (r2 == 0.0) return;
  const double r = sqrt(r2);
  const double rho = r > floor_r ? r : floor_r;
  const double sr = s * r;
  const double E = exp(-sr);
  const double c = dx * mv[0] + dy * mv[1] + dz * mv[2];
  const double rho3 = rho * rho * rho;
  const double k = 1.0 / (4.0 * M_PI);
  nadd(&a->w, k * E * (1.0 + sr) * c / rho3);
  if (want_grad) {
    const double coef = (rho == r ? 3.0 * (1.0 + sr) / r2 : 0.0) + s * s;
    const double f = k * E / rho3;
    nadd(&a->g[0], f * (coef * c * dx - (1.0 + sr) * mv[0]));
    nadd(&a->g[1], f * (coef * c * dy - (1.0 + sr) * mv[1]));
    nadd(&a->g[2], f * (coef * c * dz - (1.0 + sr) * mv[2]));
  }
}

typedef struct {
  const tnode* nodes;
  const int64_t* perm;
  const double *P, *N, *A, *D;
  int64_t n;
  double s, eps, beta;
  int want_grad;
} tctx;

/* work[0] counts the visited nodes, work[1] the far nodes taken as one dipole, work[2] the
 * source pairs summed at leaves, work[3] the sources inside the far nodes. */
static void visit(const tctx* c, int64_t k, const double q[3], acc4* acc, int32_t* flag, int64_t work[4]) {
  const tnode* nd = &c->nodes[k];
  ++work[0];
  const double dx = nd->cm[0] - q[0], dy = nd->cm[1] - q[1], dz = nd->cm[2] - q[2];
  const double dist = sqrt(dx * dx + dy * dy + dz * dz);
  double crit = c->beta * nd->r;
  if (nd->r + nd->dmax > crit) crit = nd->r + nd->dmax;
  if (crit > 0.0 && fabs(dist - crit) <= 1e-7 * crit) *flag = 1;
  if (dist > crit) {
    dipole(acc, dx, dy, dz, nd->M, 0.0, c->s, c->want_grad);
    ++work[1];
    work[3] += nd->end - nd->start;
    return;
  }
  if (nd->leaf) {
    const int64_t n = c->n;
    work[2] += nd->end - nd->start;
    for (int64_t t = nd->start; t < nd->end; ++t) {
      const int64_t j = c->perm[t];
      double fl = c->D ? c->D[j] : 0.0;
      if (c->eps > fl) fl = c->eps;
      const double px = c->P[j] - q[0], py = c->P[n + j] - q[1], pz = c->P[2 * n + j] - q[2];
      const double r = sqrt(px * px + py * py + pz * pz);
      if (fl > 0.0 && fabs(r - fl) <= 1e-6 * fl) *flag = 1;
      const double mv[3] = {c->A[j] * c->N[j], c->A[j] * c->N[n + j], c->A[j] * c->N[2 * n + j]};
      dipole(acc, px, py, pz, mv, fl, c->s, c->want_grad);
    }
    return;
  }
  for (int i = 0; i < nd->nchild; ++i) visit(c, nd->child[i], q, acc, flag, work);
}

/* Octree-approximated w, grad w (may be NULL), flags and per-query work [m][4] (visited
 * nodes, far dipoles, leaf pairs, sources inside the far nodes; may be NULL) at m queries. Arguments as orc_gwn plus beta
 * (> 0) and leaf (>= 1). */
int orc_tree_gwn(const double* P, const double* Nrm, const double* A, const double* D, int64_t n,
                 const double* Q, int64_t m, double lambda, double eps, double beta, int leaf, double* w,
                 double* g, int32_t* flag, int64_t* work) {
  if (!P || !Nrm || !A || !Q || !w || n < 1 || m < 0 || !(lambda >= 0.0) || !(eps >= 0.0) || !(beta > 0.0) ||
      leaf < 1)
    return -1;
  int64_t* perm = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  tnode* nodes = NULL;
  const int64_t cnt = tree_build(P, n, leaf, perm, &nodes);
  /* node summaries straight from their points */
  int64_t k;
#pragma omp parallel for schedule(dynamic, 64)
  for (k = 0; k < cnt; ++k) {
    tnode* nd = &nodes[k];
    nsum a = {0, 0}, ap[3] = {{0, 0}, {0, 0}, {0, 0}}, mm[3] = {{0, 0}, {0, 0}, {0, 0}};
    double dmax = 0.0;
    for (int64_t t = nd->start; t < nd->end; ++t) {
      const int64_t j = perm[t];
      nadd(&a, A[j]);
      for (int d = 0; d < 3; ++d) {
        nadd(&ap[d], A[j] * P[d * n + j]);
        nadd(&mm[d], A[j] * Nrm[d * n + j]);
      }
      double fl = D ? D[j] : 0.0;
      if (eps > fl) fl = eps;
      if (fl > dmax) dmax = fl;
    }
    nd->area = nval(&a);
    for (int d = 0; d < 3; ++d) {
      nd->cm[d] = nd->area != 0.0 ? nval(&ap[d]) / nd->area : P[d * n + perm[nd->start]];
      nd->M[d] = nval(&mm[d]);
    }
    double r = 0.0;
    for (int64_t t = nd->start; t < nd->end; ++t) {
      const int64_t j = perm[t];
      const double ex = P[j] - nd->cm[0], ey = P[n + j] - nd->cm[1], ez = P[2 * n + j] - nd->cm[2];
      const double dd = sqrt(ex * ex + ey * ey + ez * ez);
      if (dd > r) r = dd;
    }
    nd->r = r;
    nd->dmax = dmax;
  }
  const tctx c = {nodes, perm, P, Nrm, A, D, n, sqrt(lambda), eps, beta, g != NULL};
  int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
  for (i = 0; i < m; ++i) {
    const double q[3] = {Q[i], Q[m + i], Q[2 * m + i]};
    acc4 acc;
    memset(&acc, 0, sizeof acc);
    int32_t fl = 0;
    int64_t wk[4] = {0, 0, 0, 0};
    visit(&c, 0, q, &acc, &fl, wk);
    w[i] = nval(&acc.w);
    if (g)
      for (int d = 0; d < 3; ++d) g[d * m + i] = nval(&acc.g[d]);
    if (flag) flag[i] = fl;
    if (work)
      for (int d = 0; d < 4; ++d) work[4 * i + d] = wk[d];
  }
  free(nodes);
  free(perm);
  return 0;
}
