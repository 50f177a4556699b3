// graph_host.cpp -- host preparation of the streamed graph (Section 3.1):
// the in-edge CSR ("CSC") of the input, cut into pages of consecutive
// destination vertices with their incoming edges and no destination array.
// Each page also carries its degree-bin lists so the GPU can load-balance a
// page without any device-side preprocessing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <thread>

#include "engine.hpp"

namespace sr {

int host_threads() {
  unsigned t = std::thread::hardware_concurrency();
  if (const char *e = getenv("OMP_NUM_THREADS")) t = (unsigned)atoi(e);
  if (const char *e = getenv("SR_HOST_THREADS")) t = (unsigned)atoi(e);
  if (t < 1) t = 1;
  if (t > 32) t = 32;
  return (int)t;
}

template <class F>
static void parallel_for(int64_t n, int T, F f, int64_t min_n = 4096) {
  if (T <= 1 || n < min_n) { f(0, 0, n); return; }
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t) {
    int64_t lo = n * t / T, hi = n * (t + 1) / T;
    th.emplace_back([=, &f] { f(t, lo, hi); });
  }
  for (auto &x : th) x.join();
}


uint64_t graph_bytes(const sr_graph *g) {
  return 4ull * ((uint64_t)g->n + 1) + 4ull * (uint64_t)g->m * (g->weighted ? 2 : 1);
}

// Transpose (and optionally symmetrize) the out-edge CSR into in-edges.
// Counting sort by destination with per-thread cursors over contiguous
// source ranges, so every in-row lists its sources in increasing order and
// the result does not depend on the thread count.
// Vertex order for SR_LOAD_REORDER: new ids by descending in-degree (plus
// out-degree when the graph is symmetrized), ties by old id; a counting
// sort over the degrees. Fills rank (old -> new) and perm (new -> old) and
// the out-CSR of the relabeled graph, each row's heads sorted (weights
// follow their arcs).
void relabel_by_degree(int32_t n, const int64_t *ro, const int32_t *ci, const uint32_t *wi, bool symmetrize,
                       std::vector<int32_t> &rank, std::vector<int32_t> &perm, std::vector<int64_t> &ro2,
                       std::vector<int32_t> &ci2, std::vector<uint32_t> &w2) {
  const int64_t m = ro[n];
  std::vector<int64_t> deg((size_t)n, 0);
  for (int64_t e = 0; e < m; ++e) deg[ci[e]]++;
  if (symmetrize)
    for (int32_t u = 0; u < n; ++u) deg[u] += ro[u + 1] - ro[u];
  int64_t maxd = 0;
  for (int32_t v = 0; v < n; ++v) maxd = std::max(maxd, deg[v]);
  std::vector<int64_t> start((size_t)maxd + 2, 0);  // bucket d holds vertices of degree d
  for (int32_t v = 0; v < n; ++v) start[(size_t)(maxd - deg[v]) + 1]++;
  for (int64_t d = 0; d <= maxd; ++d) start[(size_t)d + 1] += start[(size_t)d];
  perm.assign((size_t)n, 0);
  rank.assign((size_t)n, 0);
  for (int32_t v = 0; v < n; ++v) {
    const int64_t p = start[(size_t)(maxd - deg[v])]++;
    perm[(size_t)p] = v;
    rank[(size_t)v] = (int32_t)p;
  }
  ro2.assign((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) ro2[(size_t)i + 1] = ro2[(size_t)i] + (ro[perm[i] + 1] - ro[perm[i]]);
  ci2.assign((size_t)m, 0);
  if (wi) w2.assign((size_t)m, 0);
  const int T = host_threads();
  parallel_for(n, T, [&](int, int64_t lo, int64_t hi) {
    std::vector<std::pair<int32_t, uint32_t>> row;
    for (int64_t i = lo; i < hi; ++i) {
      const int32_t u = perm[i];
      row.clear();
      for (int64_t e = ro[u]; e < ro[u + 1]; ++e) row.push_back({rank[ci[e]], wi ? wi[e] : 0u});
      std::sort(row.begin(), row.end());
      int64_t k = ro2[i];
      for (auto &x : row) {
        ci2[k] = x.first;
        if (wi) w2[k] = x.second;
        ++k;
      }
    }
  }, 1);
}

sr_status build_in_csr(sr_graph *g, const int64_t *ro, const int32_t *ci, const uint32_t *wi,
                       bool symmetrize) {
  const int32_t n = g->n;
  const int64_t m_in = ro[n];
  const int T = host_threads();
  g->outdeg.resize(n);
  for (int32_t u = 0; u < n; ++u) g->outdeg[u] = (int32_t)(ro[u + 1] - ro[u]);

  // arcs to place: u->v for every input arc, plus v->u when symmetrizing
  std::vector<std::vector<int32_t>> cnt(T, std::vector<int32_t>());
  for (auto &c : cnt) c.assign((size_t)n, 0);
  parallel_for(n, T, [&](int t, int64_t lo, int64_t hi) {
    auto &c = cnt[t];
    for (int64_t u = lo; u < hi; ++u)
      for (int64_t e = ro[u]; e < ro[u + 1]; ++e) {
        c[ci[e]]++;
        if (symmetrize) c[u]++;
      }
  });
  std::vector<int64_t> start((size_t)n + 1, 0);
  {
    std::vector<int64_t> tot((size_t)n, 0);
    parallel_for(n, T, [&](int, int64_t lo, int64_t hi) {
      for (int64_t v = lo; v < hi; ++v) {
        int64_t s = 0;
        for (int t = 0; t < T; ++t) s += cnt[t][v];
        tot[v] = s;
      }
    });
    for (int32_t v = 0; v < n; ++v) start[v + 1] = start[v] + tot[v];
    parallel_for(n, T, [&](int, int64_t lo, int64_t hi) {
      for (int64_t v = lo; v < hi; ++v) {
        int64_t cur = 0;
        for (int t = 0; t < T; ++t) { int32_t c0 = cnt[t][v]; cnt[t][v] = (int32_t)cur; cur += c0; }
      }
    });
  }
  const int64_t arcs = start[n];
  if (arcs > INT32_MAX) return g->ctx->fail(SR_EINVAL, "more than 2^31-1 in-edges: int32 page offsets overflow");
  std::vector<int32_t> src((size_t)arcs);
  std::vector<uint32_t> w(wi ? (size_t)arcs : 0);
  parallel_for(n, T, [&](int t, int64_t lo, int64_t hi) {
    auto &c = cnt[t];
    for (int64_t u = lo; u < hi; ++u)
      for (int64_t e = ro[u]; e < ro[u + 1]; ++e) {
        int32_t v = ci[e];
        int64_t pos = start[v] + c[v]++;
        src[pos] = (int32_t)u;
        if (wi) w[pos] = wi[e];
        if (symmetrize) {
          int64_t p2 = start[u] + c[u]++;
          src[p2] = v;
          if (wi) w[p2] = wi[e];
        }
      }
  });
  cnt.clear();
  cnt.shrink_to_fit();
  if (!symmetrize) {
    // rows already list sources in increasing order (sources visited in order)
    g->in_off = std::move(start);
    g->in_src = std::move(src);
    g->in_w = std::move(w);
    g->m = m_in;
    return SR_OK;
  }
  // Symmetrized rows interleave both directions: sort each row by source and
  // drop repeated sources, keeping the smallest weight.
  std::vector<int64_t> keep((size_t)n + 1, 0);
  parallel_for(n, T, [&](int, int64_t lo, int64_t hi) {
    std::vector<uint64_t> tmp;
    for (int64_t v = lo; v < hi; ++v) {
      int64_t a = start[v], b = start[v + 1];
      tmp.resize((size_t)(b - a));
      for (int64_t i = a; i < b; ++i)
        tmp[i - a] = ((uint64_t)(uint32_t)src[i] << 32) | (wi ? w[i] : 0u);
      std::sort(tmp.begin(), tmp.end());
      int64_t k = 0;
      for (size_t i = 0; i < tmp.size(); ++i) {
        if (k > 0 && (tmp[i] >> 32) == (uint64_t)(uint32_t)src[a + k - 1]) continue;
        src[a + k] = (int32_t)(tmp[i] >> 32);
        if (wi) w[a + k] = (uint32_t)tmp[i];
        ++k;
      }
      keep[v] = k;
    }
  });
  g->in_off.assign((size_t)n + 1, 0);
  for (int32_t v = 0; v < n; ++v) g->in_off[v + 1] = g->in_off[v] + keep[v];
  const int64_t m2 = g->in_off[n];
  g->in_src.resize((size_t)m2);
  if (wi) g->in_w.resize((size_t)m2);
  parallel_for(n, T, [&](int, int64_t lo, int64_t hi) {
    for (int64_t v = lo; v < hi; ++v) {
      std::memcpy(&g->in_src[g->in_off[v]], &src[start[v]], sizeof(int32_t) * (size_t)keep[v]);
      if (wi) std::memcpy(&g->in_w[g->in_off[v]], &w[start[v]], sizeof(uint32_t) * (size_t)keep[v]);
    }
  });
  g->m = m2;
  return SR_OK;
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

static char *alloc_page_buffer(sr_ctx *ctx, uint64_t bytes) {
  if (ctx->host_only) return (char *)std::aligned_alloc(256, align256(bytes));
  void *p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
  return (char *)p;
}

static void free_page_buffer(sr_ctx *ctx, char *p) {
  if (!p) return;
  if (ctx->host_only) std::free(p);
  else (void)hipHostFree(p);
}

void free_pages(sr_graph *g) {
  for (auto &p : g->pages) {
    free_page_buffer(g->ctx, p.host);
    free_page_buffer(g->ctx, p.split);
  }
  g->pages.clear();
}

bool split_eligible(const sr_graph *g) {
  return g->weighted ? g->packed : (int64_t)g->n <= ((int64_t)1 << 24);
}

// Section offsets of a page's split-width image (see PageHeader) for mh
// narrow and mt wide in-edges among its first `lead` vertices; returns its size.
static uint64_t split_layout(const sr_graph *g, const PageHeader &h, int32_t lead, int64_t mh, int64_t mt,
                             PageHeader &s) {
  s = h;
  s.split = 1;
  // an unweighted graph's wide in-edges need only their id: n <= 2^24 for
  // every split image, so 3 bytes hold it
  s.wide3 = g->weighted ? 0 : 1;
  uint64_t o = sizeof(PageHeader);
  s.off_tiles = o;   o = align256(o + 8ull * (uint64_t)h.n_tiles);
  s.off_chunks = o;  o = align256(o + sizeof(Chunk) * (uint64_t)h.n_chunks);
  s.off_heavy = o;   o = align256(o + sizeof(Heavy) * (uint64_t)h.n_heavy);
  s.off_tbase = o;   o = align256(o + 8ull * (uint64_t)h.n_tiles_edges);
  s.off_hside = o;   o = align256(o + 16ull * (uint64_t)h.n_heavy);
  s.off_vpk = o;     o = align256(o + 4ull * (uint64_t)lead);
  s.off_hsrc = o;    o = align256(o + 2ull * (uint64_t)mh);
  s.off_src = o;     o = align256(o + (s.wide3 ? 3ull * (uint64_t)mt + 8ull : 4ull * (uint64_t)mt));
  s.off_w = o;       o = o + (g->weighted ? (uint64_t)mh : 0ull);
  s.off_offsets = 0;  // none: tile bases and vertex entries replace them
  s.off_bins = 0;
  s.bytes_lead = s.bytes_unweighted = s.bytes_weighted = s.bytes_total = o;
  s.w_bytes = 0;
  return o;
}

static int32_t lead_vertices(const PageHeader &h) { return (int32_t)((h.bytes_lead - h.off_offsets) / 4) - 1; }

void size_split_pages(sr_graph *g) {
  const int32_t P = (int32_t)g->pages.size();
  if (P == 0 || g->pages[0].narrow >= 0) return;
  const int T = std::min<int>(host_threads(), std::max<int32_t>(P, 1));
  parallel_for(P, T > 0 ? T : 1, [&](int, int64_t lo, int64_t hi) {
    for (int64_t p = lo; p < hi; ++p) {
      Page &pg = g->pages[p];
      const int32_t vb = pg.hdr.v_begin, lead = lead_vertices(pg.hdr);
      int64_t mh = 0;
      for (int64_t e = g->in_off[vb]; e < g->in_off[vb + lead]; ++e) mh += (uint32_t)g->in_src[e] < NARROW_LIMIT;
      const int64_t mt = (g->in_off[vb + lead] - g->in_off[vb]) - mh;
      PageHeader s;
      pg.split_bytes = split_layout(g, pg.hdr, lead, mh, mt, s);
      pg.narrow = mh;
    }
  }, 1);
}

uint64_t estimate_split_bytes(const sr_graph *g) {
  constexpr int64_t STRIDE = 1024;
  uint64_t total = 0;
  for (const Page &pg : g->pages) {
    const int32_t vb = pg.hdr.v_begin, lead = lead_vertices(pg.hdr);
    const int64_t e0 = g->in_off[vb], e1 = g->in_off[vb + lead];
    int64_t hit = 0, seen = 0;
    for (int64_t e = e0; e < e1; e += STRIDE, ++seen) hit += (uint32_t)g->in_src[e] < NARROW_LIMIT;
    const int64_t mh = seen ? (int64_t)((double)hit / (double)seen * (double)(e1 - e0)) : 0;
    PageHeader s;
    total += split_layout(g, pg.hdr, lead, mh, (e1 - e0) - mh, s);
  }
  return total;
}

// Split-width image of one page (see PageHeader): the sections the min
// programs read, with each vertex's in-edges from sources below
// NARROW_LIMIT stored as u16 ids (and u8 weights) ahead of the others, and
// tile-relative edge ends in place of the offsets.
static sr_status split_page(sr_graph *g, Page &pg) {
  const PageHeader &h = pg.hdr;
  const int32_t vb = h.v_begin;
  const int64_t eb = g->in_off[vb];
  const int32_t lead = lead_vertices(h);
  // narrow in-edges before each vertex (page-local), and their total
  std::vector<int32_t> nbefore((size_t)lead + 1);
  int64_t mh = 0;
  for (int32_t i = 0; i < lead; ++i) {
    nbefore[i] = (int32_t)mh;
    for (int64_t e = g->in_off[vb + i]; e < g->in_off[vb + i + 1]; ++e) mh += (uint32_t)g->in_src[e] < NARROW_LIMIT;
  }
  nbefore[lead] = (int32_t)mh;
  auto ebefore = [&](int32_t i) { return (int32_t)(g->in_off[vb + i] - eb); };
  const int64_t mt = (int64_t)ebefore(lead) - mh;
  const int32_t nte = h.n_tiles_edges;
  PageHeader s;
  const uint64_t o = split_layout(g, h, lead, mh, mt, s);
  if (pg.narrow >= 0 && (pg.narrow != mh || pg.split_bytes != o)) return SR_EINVAL;  // sizing disagrees
  char *buf = alloc_page_buffer(g->ctx, align256(o));
  if (!buf) return SR_ENOMEM;
  // the gaps between sections are never used; entries of vertices outside
  // the tiles with in-edges are read only by lanes whose result is dropped
  std::memset(buf + s.off_vpk, 0, 4ull * (uint64_t)lead);
  std::memcpy(buf + s.off_tiles, pg.host + h.off_tiles, 8ull * (uint64_t)h.n_tiles);
  std::memcpy(buf + s.off_chunks, pg.host + h.off_chunks, sizeof(Chunk) * (uint64_t)h.n_chunks);
  std::memcpy(buf + s.off_heavy, pg.host + h.off_heavy, sizeof(Heavy) * (uint64_t)h.n_heavy);
  const int32_t *tiles = (const int32_t *)(pg.host + h.off_tiles);
  const Heavy *heavy = (const Heavy *)(pg.host + h.off_heavy);
  int32_t *tbase = (int32_t *)(buf + s.off_tbase);
  int32_t *hside = (int32_t *)(buf + s.off_hside);
  uint32_t *vpk = (uint32_t *)(buf + s.off_vpk);
  for (int32_t k = 0; k < nte; ++k) {
    const int32_t t0 = tiles[2 * k], t1 = tiles[2 * k + 1];
    tbase[2 * k] = ebefore(t0);
    tbase[2 * k + 1] = nbefore[t0];
    for (int32_t i = t0; i < t1; ++i) {
      const uint32_t ne = (uint32_t)(nbefore[i + 1] - nbefore[t0]);
      const uint32_t we = (uint32_t)((ebefore(i + 1) - nbefore[i + 1]) - (ebefore(t0) - nbefore[t0]));
      if (ne > 0xFFFFu || we > 0xFFFFu) { free_page_buffer(g->ctx, buf); return SR_EINVAL; }
      vpk[i] = ne | we << 16;
    }
  }
  for (int32_t k = 0; k < h.n_heavy; ++k) {
    const int32_t v = heavy[k].vl;
    hside[4 * k] = ebefore(v);
    hside[4 * k + 1] = nbefore[v];
    hside[4 * k + 2] = nbefore[v + 1] - nbefore[v];
    hside[4 * k + 3] = ebefore(v + 1) - ebefore(v);
    vpk[v] = (uint32_t)k;
  }
  uint16_t *hsrc = (uint16_t *)(buf + s.off_hsrc);
  uint32_t *words = (uint32_t *)(buf + s.off_src);
  uint8_t *ids3 = (uint8_t *)(buf + s.off_src);
  if (s.wide3) std::memset(ids3 + 3ull * (uint64_t)mt, 0, 8);
  uint8_t *hw = (uint8_t *)(buf + s.off_w);
  int64_t nh = 0, nt = 0;
  for (int64_t e = eb; e < g->in_off[vb + lead]; ++e) {
    // per vertex the narrow edges land in order in hsrc, the wide in words
    const uint32_t u = (uint32_t)g->in_src[e];
    const uint32_t w = g->weighted ? g->in_w[e] : 0u;
    if (u < NARROW_LIMIT) {
      hsrc[nh] = (uint16_t)u;
      if (g->weighted) hw[nh] = (uint8_t)w;
      nh++;
    } else if (s.wide3) {
      ids3[3 * nt] = (uint8_t)u;
      ids3[3 * nt + 1] = (uint8_t)(u >> 8);
      ids3[3 * nt + 2] = (uint8_t)(u >> 16);
      nt++;
    } else {
      words[nt++] = u | (g->weighted ? w << 24 : 0u);
    }
  }
  std::memcpy(buf, &s, sizeof(PageHeader));
  pg.split = buf;
  pg.shdr = s;
  pg.narrow = mh;
  pg.split_bytes = o;
  return SR_OK;
}

sr_status build_split_pages(sr_graph *g) {
  if (!g->pages.empty() && g->pages[0].split) return SR_OK;
  if (!split_eligible(g)) return g->ctx->fail(SR_EINVAL, "graph has no split-width pages");
  const int32_t P = (int32_t)g->pages.size();
  std::vector<sr_status> st((size_t)P, SR_OK);
  const int T = std::min<int>(host_threads(), std::max<int32_t>(P, 1));
  parallel_for(P, T > 0 ? T : 1, [&](int, int64_t lo, int64_t hi) {
    for (int64_t p = lo; p < hi; ++p) st[p] = split_page(g, g->pages[p]);
  }, 1);
  for (int32_t p = 0; p < P; ++p) {
    if (st[p] != SR_OK) {
      for (auto &pg : g->pages) { free_page_buffer(g->ctx, pg.split); pg.split = nullptr; }
      return g->ctx->fail(st[p], st[p] == SR_ENOMEM ? "split page allocation failed"
                                                    : "split page image disagrees with its sizing");
    }
  }
  return SR_OK;
}

// Fill one page buffer for destination range [vb, ve).
static void fill_page(const sr_graph *g, int32_t vb, int32_t ve, Page &pg) {
  PageHeader &h = pg.hdr;
  const int64_t eb = g->in_off[vb];
  const int32_t np = ve - vb;
  const int64_t mp = g->in_off[ve] - eb;
  char *buf = pg.host;
  std::memcpy(buf, &h, sizeof(PageHeader));
  int32_t *off = (int32_t *)(buf + h.off_offsets);
  for (int32_t i = 0; i <= np; ++i) off[i] = (int32_t)(g->in_off[vb + i] - eb);
  int32_t *bins = (int32_t *)(buf + h.off_bins);
  int32_t cur[NBINS];
  for (int b = 0; b < NBINS; ++b) cur[b] = h.bin_start[b];
  Chunk *ch = (Chunk *)(buf + h.off_chunks);
  Heavy *hv = (Heavy *)(buf + h.off_heavy);
  int32_t nch = 0, nhv = 0;
  for (int32_t i = 0; i < np; ++i) {
    int64_t d = g->in_off[vb + i + 1] - g->in_off[vb + i];
    if (d == 0) { bins[cur[BIN_ZERO]++] = i; continue; }
    if (d > HEAVY) {
      int32_t count = (int32_t)((d + CHUNK - 1) / CHUNK);
      int32_t first = nch;
      hv[nhv].vl = i;
      hv[nhv].first_count = (int32_t)((uint32_t)first | ((uint32_t)count << 20));
      nhv++;
      for (int32_t c = 0; c < count; ++c) {
        Chunk k;
        k.vl = i;
        k.e_begin = off[i] + c * CHUNK;
        k.e_end = (int32_t)std::min<int64_t>(off[i] + (int64_t)(c + 1) * CHUNK, off[i + 1]);
        k.first_count = (int32_t)((uint32_t)first | ((uint32_t)count << 20));
        ch[nch++] = k;
      }
      continue;
    }
    int b = d >= 64 ? BIN_WAVE : 31 - __builtin_clz((uint32_t)d);
    bins[cur[b]++] = i;
  }
  {
    // tiles with in-edges first, then the tiles of zero in-degree vertices
    int32_t *tl = (int32_t *)(buf + h.off_tiles);
    std::vector<int32_t> empty;
    int32_t nt = 0, tv = 0, t0 = 0;
    int64_t te = 0;
    bool open = false;
    auto close = [&](int32_t end) {
      if (te > 0) { tl[2 * nt] = t0; tl[2 * nt + 1] = end; nt++; }
      else { empty.push_back(t0); empty.push_back(end); }
      open = false;
    };
    for (int32_t i = 0; i < np; ++i) {
      int64_t d = g->in_off[vb + i + 1] - g->in_off[vb + i];
      if (d > HEAVY) {
        if (open) close(i);
        continue;
      }
      if (open && (tv + 1 > TILE_V || te + d > h.tile_e)) close(i);
      if (!open) { open = true; t0 = i; tv = 0; te = 0; }
      tv++; te += d;
    }
    if (open) close(np);
    for (size_t k = 0; k < empty.size(); ++k) tl[2 * nt + k] = empty[k];
  }
  if (h.packed) {
    uint32_t *words = (uint32_t *)(buf + h.off_src);
    for (int64_t e = 0; e < mp; ++e) words[e] = (uint32_t)g->in_src[eb + e] | g->in_w[eb + e] << 24;
  } else {
    std::memcpy(buf + h.off_src, &g->in_src[eb], sizeof(int32_t) * (size_t)mp);
    if (h.w_bytes == 4) std::memcpy(buf + h.off_w, &g->in_w[eb], sizeof(uint32_t) * (size_t)mp);
  }
}

// Header (sizes, bin counts, section offsets) of the page [vb, ve).
static PageHeader page_header(const sr_graph *g, int32_t vb, int32_t ve) {
  PageHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = PAGE_MAGIC;
  h.v_begin = vb;
  h.n_p = ve - vb;
  h.m_p = g->in_off[ve] - g->in_off[vb];
  int32_t chunks = 0, heavy = 0, maxd = 0;
  for (int32_t v = vb; v < ve; ++v) {
    int64_t d = g->in_off[v + 1] - g->in_off[v];
    maxd = std::max<int32_t>(maxd, (int32_t)d);
    if (d == 0) { h.bin_count[BIN_ZERO]++; continue; }
    if (d > HEAVY) { heavy++; chunks += (int32_t)((d + CHUNK - 1) / CHUNK); continue; }
    int b = d >= 64 ? BIN_WAVE : 31 - __builtin_clz((uint32_t)d);
    h.bin_count[b]++;
  }
  h.bin_count[BIN_CHUNK] = chunks;
  h.n_chunks = chunks;
  h.n_heavy = heavy;
  h.max_indeg = maxd;
  int32_t s = 0;
  for (int b = 0; b < NBINS; ++b) {
    if (b == BIN_CHUNK) continue;
    h.bin_start[b] = s;
    s += h.bin_count[b];
  }
  h.packed = g->weighted && g->packed ? 1 : 0;
  h.w_bytes = g->weighted && !g->packed ? 4 : 0;
  h.tile_e = TILE_E;
  uint64_t o = sizeof(PageHeader);
  // tiles: greedy runs of consecutive non-heavy vertices; `lead` counts the
  // leading vertices whose offsets the min programs read (every vertex of a
  // tile with in-edges, every heavy vertex)
  int32_t lead = 0;
  {
    int32_t nt = 0, ne = 0, tv = 0;
    int64_t te = 0;
    bool open = false;
    auto close = [&](int32_t end) {
      nt++;
      if (te > 0) { ne++; lead = std::max(lead, end - vb); }
      open = false;
    };
    for (int32_t v = vb; v < ve; ++v) {
      int64_t d = g->in_off[v + 1] - g->in_off[v];
      if (d > HEAVY) { if (open) close(v); lead = std::max(lead, v + 1 - vb); continue; }
      if (open && (tv + 1 > TILE_V || te + d > h.tile_e)) close(v);
      if (!open) { open = true; tv = 0; te = 0; }
      tv++; te += d;
    }
    if (open) close(ve);
    h.n_tiles = nt;
    h.n_tiles_edges = ne;
  }
  h.off_tiles = o;   o = align256(o + 8ull * (uint64_t)h.n_tiles);
  h.off_chunks = o;  o = align256(o + sizeof(Chunk) * (uint64_t)chunks);
  h.off_heavy = o;   o = align256(o + sizeof(Heavy) * (uint64_t)heavy);
  h.off_src = o;     o = align256(o + 4ull * (uint64_t)h.m_p);
  // offsets after the edge words, so a min program's prefix can end at the
  // last vertex it reads (zero in-degree vertices gather up at the end of
  // the order under degree numbering)
  h.off_offsets = o; o = align256(o + 4ull * ((uint64_t)h.n_p + 1));
  h.bytes_lead = h.off_offsets + 4ull * ((uint64_t)lead + 1);
  h.bytes_unweighted = o;
  h.off_w = o;
  o = align256(o + (uint64_t)h.w_bytes * (uint64_t)h.m_p);
  h.bytes_weighted = o;
  h.off_bins = o;    o = align256(o + 4ull * (uint64_t)s);
  h.bytes_total = o;
  return h;
}

// Streamed bytes of the vertices [0, v): one offset per vertex and one edge
// word per in-edge (plus a separate u32 weight when weights are not packed).
// With equal_edges the cost is the in-edge count alone.
static uint64_t stream_cost(const sr_graph *g, int32_t v, bool equal_edges = false) {
  if (equal_edges) return (uint64_t)g->in_off[v];
  const uint64_t eb = (g->weighted && !g->packed) ? 8 : 4;
  return 4ull * (uint64_t)v + eb * (uint64_t)g->in_off[v];
}

// Split into nparts contiguous destination ranges of about equal streamed
// bytes (or equal in-edge counts): boundary i is the first vertex whose
// prefix cost reaches ceil(i * total / nparts); a vertex never straddles two
// pages, and empty ranges (a vertex heavier than a share) are dropped.
static std::vector<int32_t> split_bounds(const sr_graph *g, int32_t nparts, bool equal_edges = false) {
  std::vector<int32_t> bounds;
  bounds.push_back(0);
  const uint64_t total = stream_cost(g, g->n, equal_edges);
  for (int32_t i = 1; i < nparts; ++i) {
    const uint64_t target = (total * (uint64_t)i + nparts - 1) / (uint64_t)nparts;
    int32_t lo = 0, hi = g->n;  // smallest b with stream_cost(b) >= target
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      if (stream_cost(g, mid, equal_edges) >= target) hi = mid; else lo = mid + 1;
    }
    if (lo > bounds.back() && lo < g->n) bounds.push_back(lo);
  }
  bounds.push_back(g->n);
  return bounds;
}

int32_t auto_parts(const sr_graph *g, uint64_t slot_bytes, bool equal_edges) {
  const uint64_t total = stream_cost(g, g->n);
  int32_t P = (int32_t)std::max<uint64_t>(1, (total + slot_bytes - 1) / std::max<uint64_t>(slot_bytes, 1));
  while (P < g->n) {
    const std::vector<int32_t> b = split_bounds(g, P, equal_edges);
    uint64_t mx = 0;
    for (size_t i = 0; i + 1 < b.size(); ++i) {
      const PageHeader h = page_header(g, b[i], b[i + 1]);
      const uint64_t sc = ((8ull * (uint64_t)std::max<int32_t>(h.n_chunks, 1)) + 255) & ~255ull;
      mx = std::max(mx, h.bytes_weighted + sc);
    }
    if (mx <= slot_bytes) return P;
    P = P + std::max<int32_t>(1, P / 16);
  }
  return -1;
}

sr_status make_pages(sr_graph *g, int32_t nparts, bool equal_edges) {
  if (nparts < 1) return g->ctx->fail(SR_EINVAL, "num_parts must be >= 1");
  if (nparts > g->n) nparts = g->n;
  const std::vector<int32_t> bounds = split_bounds(g, nparts, equal_edges);
  free_pages(g);
  const int32_t P = (int32_t)bounds.size() - 1;
  g->pages.resize(P);
  for (int32_t p = 0; p < P; ++p) {
    g->pages[p].hdr = page_header(g, bounds[p], bounds[p + 1]);
    if ((uint32_t)g->pages[p].hdr.n_chunks >= (1u << 20))
      return g->ctx->fail(SR_EINVAL, "page has too many heavy-vertex chunks; use more parts");
    if (g->pages[p].hdr.max_indeg > CHUNK * 4095)
      return g->ctx->fail(SR_EINVAL, "in-degree above 8.3M is not supported");
    g->pages[p].bytes = g->pages[p].hdr.bytes_total;
    g->pages[p].host = alloc_page_buffer(g->ctx, g->pages[p].bytes);
    if (!g->pages[p].host) {
      free_pages(g);
      return g->ctx->fail(SR_ENOMEM, "page buffer allocation failed");
    }
  }
  const int T = std::min<int>(host_threads(), P);
  parallel_for(P, T > 0 ? T : 1, [&](int, int64_t lo, int64_t hi) {
    for (int64_t p = lo; p < hi; ++p) fill_page(g, bounds[p], bounds[p + 1], g->pages[p]);
  }, 2);
  g->nparts = P;
  g->equal_edges = equal_edges;
  return SR_OK;
}

}  // namespace sr
