/*
 * oracle.c - plain single-threaded CPU oracle (see oracle.h).
 *
 * TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU-baseline leg
 * use it.  Built with gcc -O2 -ffp-contract=off so that no multiply-add is fused except
 * the explicit fmaf calls; fmaf is correctly rounded.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

float oracle_fK(float v, uint32_t K) {
  for (uint32_t k = 0; k < K; ++k) v = fmaf(v, 0.999f, 0.001f);
  return v;
}

void oracle_gather(const uint8_t* image, uint64_t row_bytes, const int64_t* rows, uint64_t n,
                   uint8_t* out) {
  for (uint64_t i = 0; i < n; ++i)
    memcpy(out + i * row_bytes, image + (uint64_t)rows[i] * row_bytes, row_bytes);
}

static inline const float* table_row(const uint8_t* image, uint64_t rows, uint32_t dim,
                                     uint32_t t, int64_t r) {
  const uint64_t table_bytes = rows * (uint64_t)dim * sizeof(float);
  return (const float*)(image + (uint64_t)t * table_bytes +
                        (uint64_t)r * dim * sizeof(float));
}

void oracle_embbag_forward(const uint8_t* image, uint64_t rows, uint32_t dim, uint32_t T,
                           const int64_t* idx, const int64_t* off, uint64_t B, uint32_t K,
                           const int64_t* bags, uint64_t nbags, float* out) {
  const uint64_t n = bags ? nbags : B * T;
  for (uint64_t k = 0; k < n; ++k) {
    const uint64_t g = bags ? (uint64_t)bags[k] : k;
    const uint32_t t = (uint32_t)(g % T);
    for (uint32_t d = 0; d < dim; ++d) {
      float acc = 0.0f;
      for (int64_t j = off[g]; j < off[g + 1]; ++j)
        acc = acc + oracle_fK(table_row(image, rows, dim, t, idx[j])[d], K);
      out[k * dim + d] = acc;
    }
  }
}

typedef struct {
  uint64_t row; /* global row: t * rows + r */
  uint64_t pos; /* lookup position j */
  uint64_t bag;
} occ_t;

static int cmp_occ(const void* a, const void* b) {
  const occ_t* x = (const occ_t*)a;
  const occ_t* y = (const occ_t*)b;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  return (x->pos > y->pos) - (x->pos < y->pos);
}

uint64_t oracle_embbag_backward_sgd(uint8_t* image, uint64_t rows, uint32_t dim, uint32_t T,
                                    const int64_t* idx, const int64_t* off, uint64_t B,
                                    const float* grad_out, float lr) {
  const uint64_t nbag = B * T;
  const uint64_t n = (uint64_t)off[nbag];
  if (n == 0) return 0;
  occ_t* occ = (occ_t*)malloc(n * sizeof(occ_t));
  for (uint64_t g = 0; g < nbag; ++g)
    for (int64_t j = off[g]; j < off[g + 1]; ++j) {
      occ[j].row = (g % T) * rows + (uint64_t)idx[j];
      occ[j].pos = (uint64_t)j;
      occ[j].bag = g;
    }
  qsort(occ, n, sizeof(occ_t), cmp_occ);
  float* grad = (float*)malloc(dim * sizeof(float));
  uint64_t unique = 0;
  for (uint64_t s = 0; s < n;) {
    uint64_t e = s;
    while (e < n && occ[e].row == occ[s].row) ++e;
    for (uint32_t d = 0; d < dim; ++d) {
      float g = 0.0f;
      for (uint64_t i = s; i < e; ++i) g = g + grad_out[occ[i].bag * dim + d];
      grad[d] = g;
    }
    float* w = (float*)(image + occ[s].row * (uint64_t)dim * sizeof(float));
    for (uint32_t d = 0; d < dim; ++d) w[d] = fmaf(-lr, grad[d], w[d]);
    ++unique;
    s = e;
  }
  free(grad);
  free(occ);
  return unique;
}

void oracle_bfs(const int64_t* row_ptr, const int32_t* col, uint64_t V, int64_t src,
                int32_t* level) {
  for (uint64_t v = 0; v < V; ++v) level[v] = -1;
  if (src < 0 || (uint64_t)src >= V) return;
  int32_t* cur = (int32_t*)malloc(V * sizeof(int32_t));
  int32_t* nxt = (int32_t*)malloc(V * sizeof(int32_t));
  uint64_t ncur = 1, nnxt;
  cur[0] = (int32_t)src;
  level[src] = 0;
  for (int32_t L = 0; ncur > 0; ++L) {
    nnxt = 0;
    for (uint64_t i = 0; i < ncur; ++i) {
      const int32_t v = cur[i];
      for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
        const int32_t u = col[k];
        if (level[u] == -1) {
          level[u] = L + 1;
          nxt[nnxt++] = u;
        }
      }
    }
    int32_t* t = cur;
    cur = nxt;
    nxt = t;
    ncur = nnxt;
  }
  free(cur);
  free(nxt);
}

int oracle_bfs_validate(const int64_t* row_ptr, const int32_t* col, uint64_t V, int64_t src,
                        const int32_t* level) {
  if (src < 0 || (uint64_t)src >= V || level[src] != 0) return 1;
  uint8_t* has_parent = (uint8_t*)calloc(V, 1);
  int bad = 0;
  for (uint64_t u = 0; u < V && !bad; ++u) {
    if (level[u] < -1) bad = 2;
    if (level[u] < 0) continue;
    for (int64_t k = row_ptr[u]; k < row_ptr[u + 1]; ++k) {
      const int32_t v = col[k];
      if (level[v] < 0 || level[v] > level[u] + 1) {
        bad = 2;
        break;
      }
      if (level[v] == level[u] + 1) has_parent[v] = 1;
    }
  }
  for (uint64_t v = 0; v < V && !bad; ++v)
    if (level[v] > 0 && !has_parent[v]) bad = 3;
  free(has_parent);
  return bad;
}

void oracle_spmv(const int64_t* row_ptr, const int32_t* col, const float* val, const float* x,
                 uint64_t r0, uint64_t r1, float* y) {
  for (uint64_t i = r0; i < r1; ++i) {
    float acc = 0.0f;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) acc = fmaf(val[k], x[col[k]], acc);
    y[i - r0] = acc;
  }
}

struct oracle_clock {
  uint32_t sets, assoc;
  uint8_t* valid;
  uint8_t* ref;
  uint8_t* dirty;
  uint64_t* tag;
  uint32_t* hand;
  uint64_t hits, misses, wb_evict, wb_flush;
};

oracle_clock* oracle_clock_new(uint32_t sets, uint32_t assoc) {
  oracle_clock* c = (oracle_clock*)calloc(1, sizeof(oracle_clock));
  const uint64_t n = (uint64_t)sets * assoc;
  c->sets = sets;
  c->assoc = assoc;
  c->valid = (uint8_t*)calloc(n, 1);
  c->ref = (uint8_t*)calloc(n, 1);
  c->dirty = (uint8_t*)calloc(n, 1);
  c->tag = (uint64_t*)calloc(n, sizeof(uint64_t));
  c->hand = (uint32_t*)calloc(sets, sizeof(uint32_t));
  return c;
}

void oracle_clock_free(oracle_clock* c) {
  if (!c) return;
  free(c->valid);
  free(c->ref);
  free(c->dirty);
  free(c->tag);
  free(c->hand);
  free(c);
}

int oracle_clock_access(oracle_clock* c, uint64_t line_id, int write, int32_t* way) {
  const uint32_t s = (uint32_t)(line_id % c->sets);
  const uint64_t base = (uint64_t)s * c->assoc;
  for (uint32_t w = 0; w < c->assoc; ++w) {
    if (c->valid[base + w] && c->tag[base + w] == line_id) {
      c->ref[base + w] = 1;
      if (write) c->dirty[base + w] = 1;
      c->hits++;
      if (way) *way = (int32_t)w;
      return 1;
    }
  }
  c->misses++;
  uint32_t h = c->hand[s];
  for (;;) {
    const uint64_t i = base + h;
    if (!c->valid[i] || c->ref[i] == 0) break;
    c->ref[i] = 0;
    h = (h + 1) % c->assoc;
  }
  const uint64_t v = base + h;
  if (c->valid[v] && c->dirty[v]) c->wb_evict++;
  c->valid[v] = 1;
  c->tag[v] = line_id;
  c->ref[v] = 1;
  c->dirty[v] = write ? 1 : 0;
  c->hand[s] = (h + 1) % c->assoc;
  if (way) *way = (int32_t)h;
  return 0;
}

void oracle_clock_run(oracle_clock* c, const uint64_t* lines, const uint8_t* writes, uint64_t n,
                      uint8_t* hit, int32_t* way) {
  for (uint64_t i = 0; i < n; ++i) {
    int32_t w = -1;
    int h = oracle_clock_access(c, lines[i], writes ? writes[i] : 0, &w);
    if (hit) hit[i] = (uint8_t)h;
    if (way) way[i] = w;
  }
}

uint64_t oracle_clock_flush(oracle_clock* c) {
  const uint64_t n = (uint64_t)c->sets * c->assoc;
  uint64_t k = 0;
  for (uint64_t i = 0; i < n; ++i)
    if (c->valid[i] && c->dirty[i]) {
      c->dirty[i] = 0;
      ++k;
    }
  c->wb_flush += k;
  return k;
}

void oracle_clock_counters(const oracle_clock* c, uint64_t* counters) {
  counters[0] = c->hits;
  counters[1] = c->misses;
  counters[2] = c->wb_evict;
  counters[3] = c->wb_flush;
}

void oracle_clock_state(const oracle_clock* c, int64_t* tags, uint8_t* dirty) {
  const uint64_t n = (uint64_t)c->sets * c->assoc;
  for (uint64_t i = 0; i < n; ++i) {
    tags[i] = c->valid[i] ? (int64_t)c->tag[i] : -1;
    if (dirty) dirty[i] = c->dirty[i];
  }
}

double oracle_eq1(double ctc) {
  if (ctc < 0.0) return NAN;
  return ctc <= 1.0 ? 1.0 + ctc : 1.0 + 1.0 / ctc;
}

/* ---- interleaving over several devices (Sec. 4.3) */
void oracle_stripe_split(const uint8_t* logical, uint64_t units, uint64_t unit_bytes, uint32_t n,
                         uint8_t* const* devs) {
  for (uint64_t u = 0; u < units; ++u) {
    const uint32_t d = (uint32_t)(u % n);
    const uint64_t k = u / n;
    memcpy(devs[d] + k * unit_bytes, logical + u * unit_bytes, unit_bytes);
  }
}

void oracle_write_units(uint8_t* image, uint64_t unit_bytes, const uint64_t* lines, uint64_t k,
                        const uint8_t* src) {
  for (uint64_t i = 0; i < k; ++i) memcpy(image + lines[i] * unit_bytes, src + i * unit_bytes, unit_bytes);
}
