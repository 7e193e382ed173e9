// bvh.cpp -- host construction of the bounding-volume hierarchy the GPU
// traverses, and a host self-check of it.
//
// Binned surface-area heuristic (Wald 2007) over triangle centroids, all
// three axes, built top-down as a two-wide tree; the upper levels run on
// several host threads and the result is emitted in depth-first order, so
// the output does not depend on the thread count.  Build depth is bounded by
// kMaxDepth - 1 by switching to object-median splits when the remaining
// depth budget gets tight.  The tree is then collapsed into four-wide nodes
// with 8-bit child boxes quantised outward in the node's frame.
//
// Optionally, before the build, the references with the largest boxes are
// split (early split clipping, Ernst & Greiner, "Early split clipping for
// bounding volume hierarchies", RT 2007): a reference is cut at the middle of
// its box's longest axis and each half is bounded by the part of the
// triangle inside it, so long diagonal triangles (walls, ground) get several
// tight boxes instead of one loose one.  A triangle may then sit in several
// leaves; the closest hit is the same, since every test of it gives the same
// (t, original id).
#include "bvh.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <memory>
#include <queue>
#include <thread>

namespace rr {
namespace {

struct Box {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  void grow(const Box& b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], b.lo[a]);
      hi[a] = std::max(hi[a], b.hi[a]);
    }
  }
  void grow(const float* p) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
  double area() const {
    double e[3];
    for (int a = 0; a < 3; ++a) e[a] = hi[a] > lo[a] ? (double)hi[a] - lo[a] : 0.0;
    return 2.0 * (e[0] * e[1] + e[1] * e[2] + e[2] * e[0]);
  }
  bool empty() const { return !(lo[0] <= hi[0]); }
};

struct Ref {
  Box box;
  float c[3];
  uint32_t id;
};

// Bounds of the part of triangle (p0, p1, p2) inside box r, rounded outward
// to float; false if that part is empty.  Sutherland-Hodgman in float64.
bool clipped_bounds(const double p[3][3], const double rlo[3], const double rhi[3], Box& out) {
  double poly[16][3], tmp[16][3];
  int n = 3;
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) poly[i][a] = p[i][a];
  for (int a = 0; a < 3 && n > 0; ++a) {
    for (int side = 0; side < 2 && n > 0; ++side) {
      const double c = side ? rhi[a] : rlo[a];
      auto inside = [&](const double* v) { return side ? v[a] <= c : v[a] >= c; };
      int m = 0;
      for (int i = 0; i < n; ++i) {
        const double* u = poly[i];
        const double* v = poly[(i + 1) % n];
        const bool iu = inside(u), iv = inside(v);
        if (iu && m < 16) {
          for (int q = 0; q < 3; ++q) tmp[m][q] = u[q];
          ++m;
        }
        if (iu != iv && m < 16) {
          const double s = (c - u[a]) / (v[a] - u[a]);
          for (int q = 0; q < 3; ++q) tmp[m][q] = u[q] + s * (v[q] - u[q]);
          tmp[m][a] = c;
          ++m;
        }
      }
      n = m;
      for (int i = 0; i < n; ++i)
        for (int q = 0; q < 3; ++q) poly[i][q] = tmp[i][q];
    }
  }
  if (n == 0) return false;
  out = Box();
  for (int i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      float lo = (float)poly[i][a], hi = lo;
      if ((double)lo > poly[i][a]) lo = std::nextafter(lo, -INFINITY);
      if ((double)hi < poly[i][a]) hi = std::nextafter(hi, INFINITY);
      out.lo[a] = std::min(out.lo[a], lo);
      out.hi[a] = std::max(out.hi[a], hi);
    }
  }
  return true;
}

struct BNode {
  Box box;
  std::unique_ptr<BNode> l, r;
  uint32_t begin = 0, count = 0;  // leaf range in the ref array
  uint32_t span = 0;              // references below an inner node (from begin)
  uint32_t plan = 0;              // cost-optimal collapse: index of the node's Plan
  std::vector<Ref> items;         // spatial-split build: a leaf's references until they are gathered
  bool leaf() const { return !l; }
};

// Binned SAH with spatial splits (after Stich, Friedrich and Dietrich,
// "Spatial splits in bounding volume hierarchies", HPG 2009).  Next to the
// object split over centroid bins, a node whose two object-split halves
// overlap also tries splitting space at the planes of bins over its box: a
// reference that straddles the plane goes to both sides, each copy bounded by
// the part of its triangle on that side (clipped_bounds), so large triangles
// stop inflating the boxes of the small ones around them.  The split with the
// lower surface-area cost wins while the node's allowance of extra references
// lasts; what a split does not use passes to the two children in proportion
// to their sizes, so the tree does not depend on the thread count.  Each
// subtree keeps its references in vectors of its own; gather() lays them out
// depth-first into one array afterwards.
constexpr double kSpatialOverlap = 1e-5;  // of the scene box's area

struct SpatialBuilder {
  const float* V;
  const uint32_t* F;
  uint32_t max_leaf, bins;
  int par_depth;
  double min_overlap;  // overlap area of the object split that starts a spatial search

  void tri(uint32_t id, double p[3][3]) const {
    for (int v = 0; v < 3; ++v) {
      const float* q = V + 3 * (size_t)F[3 * (size_t)id + v];
      for (int a = 0; a < 3; ++a) p[v][a] = q[a];
    }
  }

  // bounds of the part of r's triangle inside r.box with lo <= x_a <= hi
  bool chop(const Ref& r, int a, double lo, double hi, Box& out) const {
    double rlo[3], rhi[3];
    for (int q = 0; q < 3; ++q) {
      rlo[q] = r.box.lo[q];
      rhi[q] = r.box.hi[q];
    }
    rlo[a] = std::max(rlo[a], lo);
    rhi[a] = std::min(rhi[a], hi);
    if (rlo[a] > rhi[a]) return false;
    double p[3][3];
    tri(r.id, p);
    if (!clipped_bounds(p, rlo, rhi, out)) return false;
    for (int q = 0; q < 3; ++q) {  // never wider than the reference
      out.lo[q] = std::max(out.lo[q], r.box.lo[q]);
      out.hi[q] = std::min(out.hi[q], r.box.hi[q]);
    }
    return !out.empty();
  }

  static void set_centroid(Ref& r) {
    for (int a = 0; a < 3; ++a) r.c[a] = 0.5f * (r.box.lo[a] + r.box.hi[a]);
  }

  std::unique_ptr<BNode> make_leaf(std::vector<Ref>& v, const Box& box) {
    auto nd = std::make_unique<BNode>();
    nd->box = box;
    nd->count = (uint32_t)v.size();
    nd->items = std::move(v);
    return nd;
  }

  // bin of coordinate x among `bins` bins of width w from lo
  int bin_of(double x, double lo, double w) const {
    int b = (int)((x - lo) / w);
    return std::min<int>(std::max(b, 0), (int)bins - 1);
  }

  std::unique_ptr<BNode> build(std::vector<Ref> v, int depth, int64_t allow) {
    const uint32_t n = (uint32_t)v.size();
    Box box, cb;
    for (const Ref& r : v) {
      box.grow(r.box);
      cb.grow(r.c);
    }
    if (n <= 1) return make_leaf(v, box);
    int budget = 0;
    while ((1ull << budget) < (uint64_t)((n + max_leaf - 1) / max_leaf)) ++budget;
    bool median = depth + budget >= kMaxDepth - 1;
    std::vector<Ref> L, R;
    int64_t used = 0;
    if (!median) {
      // object split: binned SAH over centroids, all three axes
      double best = INFINITY;
      int best_axis = -1, best_bin = -1;
      for (int a = 0; a < 3; ++a) {
        const float ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0.0f)) continue;
        std::vector<Box> bb(bins);
        std::vector<uint32_t> cnt(bins, 0);
        const double k = (double)bins / ext;
        for (const Ref& r : v) {
          int bi = std::min<int>(std::max((int)((r.c[a] - cb.lo[a]) * k), 0), (int)bins - 1);
          bb[bi].grow(r.box);
          cnt[bi]++;
        }
        std::vector<double> rarea(bins, 0.0);
        std::vector<uint32_t> rcnt(bins, 0);
        Box acc;
        uint32_t c = 0;
        for (int i = (int)bins - 1; i > 0; --i) {
          acc.grow(bb[i]);
          c += cnt[i];
          rarea[i] = acc.empty() ? 0.0 : acc.area();
          rcnt[i] = c;
        }
        Box lacc;
        uint32_t lc = 0;
        for (uint32_t i = 0; i + 1 < bins; ++i) {
          lacc.grow(bb[i]);
          lc += cnt[i];
          if (lc == 0 || rcnt[i + 1] == 0) continue;
          const double cost = lacc.area() * lc + rarea[i + 1] * rcnt[i + 1];
          if (cost < best) {
            best = cost;
            best_axis = a;
            best_bin = (int)i;
          }
        }
      }
      // the object split's halves and their overlap
      Box ol, orr;
      if (best_axis >= 0) {
        const int a = best_axis;
        const double k = (double)bins / (cb.hi[a] - cb.lo[a]);
        for (const Ref& r : v) {
          const int bi = std::min<int>(std::max((int)((r.c[a] - cb.lo[a]) * k), 0), (int)bins - 1);
          (bi <= best_bin ? ol : orr).grow(r.box);
        }
      }
      double overlap = 0.0;
      if (best_axis >= 0) {
        Box ov;
        for (int a = 0; a < 3; ++a) {
          ov.lo[a] = std::max(ol.lo[a], orr.lo[a]);
          ov.hi[a] = std::min(ol.hi[a], orr.hi[a]);
        }
        overlap = ov.empty() ? 0.0 : ov.area();
      }
      // spatial split: bins over the node box, straddling references chopped
      double sbest = INFINITY;
      int s_axis = -1, s_bin = -1;
      if (allow > 0 && (best_axis < 0 || overlap > min_overlap)) {
        for (int a = 0; a < 3; ++a) {
          const double lo = box.lo[a], ext = (double)box.hi[a] - lo;
          if (!(ext > 0.0)) continue;
          const double w = ext / bins;
          std::vector<Box> bb(bins);
          std::vector<uint32_t> ent(bins, 0), ex(bins, 0);
          // the references a plane would copy are counted before any is cut:
          // an axis where every plane copies more than the allowance is
          // skipped (long triangles crossing the whole node would otherwise
          // be clipped into every bin at every level for nothing)
          for (const Ref& r : v) {
            ent[bin_of(r.box.lo[a], lo, w)]++;
            ex[bin_of(r.box.hi[a], lo, w)]++;
          }
          int64_t open = 0, least = INT64_MAX;
          for (uint32_t i = 0; i + 1 < bins; ++i) {
            open += (int64_t)ent[i] - (int64_t)ex[i];  // references that start at or left of bin i and end right of it
            least = std::min(least, open);
          }
          if (least > allow) continue;
          for (const Ref& r : v) {
            const int b0 = bin_of(r.box.lo[a], lo, w), b1 = bin_of(r.box.hi[a], lo, w);
            if (b0 == b1) {
              bb[b0].grow(r.box);
            } else {
              for (int k = b0; k <= b1; ++k) {
                Box part;
                const double plo = k == b0 ? -INFINITY : lo + k * w;
                const double phi = k == b1 ? INFINITY : lo + (k + 1) * w;
                if (chop(r, a, plo, phi, part)) bb[k].grow(part);
              }
            }
          }
          std::vector<double> rarea(bins, 0.0);
          std::vector<uint32_t> rcnt(bins, 0);
          Box acc;
          uint32_t c = 0;
          for (int i = (int)bins - 1; i > 0; --i) {
            acc.grow(bb[i]);
            c += ex[i];
            rarea[i] = acc.empty() ? 0.0 : acc.area();
            rcnt[i] = c;
          }
          Box lacc;
          uint32_t lc = 0;
          for (uint32_t i = 0; i + 1 < bins; ++i) {
            lacc.grow(bb[i]);
            lc += ent[i];
            const uint32_t rc = rcnt[i + 1];
            if (lc == 0 || rc == 0 || lc >= n || rc >= n) continue;
            if ((int64_t)lc + rc - n > allow) continue;
            const double cost = lacc.area() * lc + rarea[i + 1] * rc;
            if (cost < sbest) {
              sbest = cost;
              s_axis = a;
              s_bin = (int)i;
            }
          }
        }
      }
      const double parea = box.area();
      const double cost = std::min(best, sbest);
      const double split_cost = parea > 0.0 ? 1.0 + cost / parea : INFINITY;
      if (n <= max_leaf && ((best_axis < 0 && s_axis < 0) || (double)n <= split_cost)) return make_leaf(v, box);
      if (s_axis >= 0 && sbest < best) {
        const int a = s_axis;
        const double lo = box.lo[a], w = ((double)box.hi[a] - lo) / bins;
        const double x = lo + (s_bin + 1) * w;
        for (const Ref& r : v) {
          const int b0 = bin_of(r.box.lo[a], lo, w), b1 = bin_of(r.box.hi[a], lo, w);
          if (b1 <= s_bin) {
            L.push_back(r);
          } else if (b0 > s_bin) {
            R.push_back(r);
          } else {
            Box lb, rb;
            const bool hl = chop(r, a, -INFINITY, x, lb), hr = chop(r, a, x, INFINITY, rb);
            if (hl) {
              Ref q = r;
              q.box = lb;
              set_centroid(q);
              L.push_back(q);
            }
            if (hr) {
              Ref q = r;
              q.box = rb;
              set_centroid(q);
              R.push_back(q);
            }
            if (!hl && !hr) L.push_back(r);
          }
        }
        if (L.empty() || R.empty()) {
          L.clear();
          R.clear();
        } else {
          used = (int64_t)L.size() + (int64_t)R.size() - n;
        }
      }
      if (L.empty() && best_axis >= 0) {
        const int a = best_axis;
        const double k = (double)bins / (cb.hi[a] - cb.lo[a]);
        for (const Ref& r : v) {
          const int bi = std::min<int>(std::max((int)((r.c[a] - cb.lo[a]) * k), 0), (int)bins - 1);
          (bi <= best_bin ? L : R).push_back(r);
        }
        if (L.empty() || R.empty()) {
          L.clear();
          R.clear();
        }
      }
      if (L.empty()) median = true;
    }
    if (L.empty()) {
      if (n <= max_leaf && !median) return make_leaf(v, box);
      int a = 0;
      for (int q = 1; q < 3; ++q)
        if (cb.hi[q] - cb.lo[q] > cb.hi[a] - cb.lo[a]) a = q;
      const uint32_t mid = n / 2;
      std::nth_element(v.begin(), v.begin() + mid, v.end(), [&](const Ref& x, const Ref& y) {
        return x.c[a] < y.c[a] || (x.c[a] == y.c[a] && x.id < y.id);
      });
      if (n <= max_leaf && budget == 0) return make_leaf(v, box);
      L.assign(v.begin(), v.begin() + mid);
      R.assign(v.begin() + mid, v.end());
    }
    v.clear();
    v.shrink_to_fit();
    auto nd = std::make_unique<BNode>();
    nd->box = box;
    const int64_t rest = std::max<int64_t>(allow - used, 0);
    const int64_t al = (int64_t)((double)rest * (double)L.size() / (double)(L.size() + R.size()));
    const int64_t ar = rest - al;
    if (depth < par_depth && n > 4096) {
      auto fut = std::async(std::launch::async,
                            [this, &L, depth, al] { return build(std::move(L), depth + 1, al); });
      nd->r = build(std::move(R), depth + 1, ar);
      nd->l = fut.get();
    } else {
      nd->l = build(std::move(L), depth + 1, al);
      nd->r = build(std::move(R), depth + 1, ar);
    }
    return nd;
  }

  // depth-first layout of the leaves' references; sets begin / count / span
  static void gather(BNode* n, std::vector<Ref>& out) {
    n->begin = (uint32_t)out.size();
    if (n->leaf()) {
      out.insert(out.end(), n->items.begin(), n->items.end());
      n->count = (uint32_t)n->items.size();
      std::vector<Ref>().swap(n->items);
      return;
    }
    gather(n->l.get(), out);
    gather(n->r.get(), out);
    n->span = (uint32_t)out.size() - n->begin;
  }
};

// Four-wide collapse plan of one build node (cost-optimal mode): cover[j-1]
// is the least expected cost of the subtree as at most j entries of a wide
// node; the subtree is one entry if cl[j-1] == 0, else its left child takes
// cl[j-1] entries and its right child cr[j-1].  As a wide node of its own,
// the left child takes wide_l of the four entries; as one entry it is a leaf
// if as_leaf.
struct Plan {
  float cover[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  uint8_t cl[4] = {0, 0, 0, 0}, cr[4] = {0, 0, 0, 0};
  uint8_t wide_l = 2;
  bool as_leaf = false;
};

struct Builder {
  std::vector<Ref>& refs;
  uint32_t max_leaf, bins;
  int par_depth;

  static int ceil_log2(uint64_t x) {
    int k = 0;
    while ((1ull << k) < x) ++k;
    return k;
  }

  std::unique_ptr<BNode> make_leaf(uint32_t b, uint32_t n, const Box& box) {
    auto nd = std::make_unique<BNode>();
    nd->box = box;
    nd->begin = b;
    nd->count = n;
    return nd;
  }

  // depth = depth of the inner node this call may create
  std::unique_ptr<BNode> build(uint32_t b, uint32_t e, int depth) {
    uint32_t n = e - b;
    Box box, cb;
    for (uint32_t i = b; i < e; ++i) {
      box.grow(refs[i].box);
      cb.grow(refs[i].c);
    }
    if (n <= 1) return make_leaf(b, n, box);
    int budget = ceil_log2((n + max_leaf - 1) / max_leaf);
    bool median = depth + budget >= kMaxDepth - 1;
    uint32_t mid = b;
    if (!median) {
      // binned SAH over all three axes
      double best = INFINITY;
      int best_axis = -1, best_bin = -1;
      for (int a = 0; a < 3; ++a) {
        float ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0.0f)) continue;
        std::vector<Box> bb(bins);
        std::vector<uint32_t> cnt(bins, 0);
        double k = (double)bins / ext;
        for (uint32_t i = b; i < e; ++i) {
          int bi = (int)((refs[i].c[a] - cb.lo[a]) * k);
          bi = std::min<int>(std::max(bi, 0), bins - 1);
          bb[bi].grow(refs[i].box);
          cnt[bi]++;
        }
        std::vector<double> rarea(bins, 0.0);
        std::vector<uint32_t> rcnt(bins, 0);
        Box acc;
        uint32_t c = 0;
        for (int i = bins - 1; i > 0; --i) {
          acc.grow(bb[i]);
          c += cnt[i];
          rarea[i] = acc.empty() ? 0.0 : acc.area();
          rcnt[i] = c;
        }
        Box lacc;
        uint32_t lc = 0;
        for (uint32_t i = 0; i + 1 < bins; ++i) {
          lacc.grow(bb[i]);
          lc += cnt[i];
          if (lc == 0 || rcnt[i + 1] == 0) continue;
          double cost = lacc.area() * lc + rarea[i + 1] * rcnt[i + 1];
          if (cost < best) {
            best = cost;
            best_axis = a;
            best_bin = (int)i;
          }
        }
      }
      double parea = box.area();
      double split_cost = parea > 0.0 ? 1.0 + best / parea : INFINITY;
      if (n <= max_leaf && (best_axis < 0 || (double)n <= split_cost)) return make_leaf(b, n, box);
      if (best_axis >= 0) {
        int a = best_axis;
        double k = (double)bins / (cb.hi[a] - cb.lo[a]);
        auto it = std::partition(refs.begin() + b, refs.begin() + e, [&](const Ref& r) {
          int bi = (int)((r.c[a] - cb.lo[a]) * k);
          bi = std::min<int>(std::max(bi, 0), bins - 1);
          return bi <= best_bin;
        });
        mid = (uint32_t)(it - refs.begin());
      } else {
        median = true;  // all centroids coincide
      }
    }
    if (median || mid == b || mid == e) {
      if (n <= max_leaf && !median) return make_leaf(b, n, box);
      int a = 0;
      for (int q = 1; q < 3; ++q)
        if (cb.hi[q] - cb.lo[q] > cb.hi[a] - cb.lo[a]) a = q;
      mid = b + n / 2;
      std::nth_element(refs.begin() + b, refs.begin() + mid, refs.begin() + e,
                       [&](const Ref& x, const Ref& y) {
                         return x.c[a] < y.c[a] || (x.c[a] == y.c[a] && x.id < y.id);
                       });
      if (n <= max_leaf && budget == 0) return make_leaf(b, n, box);
    }
    auto nd = std::make_unique<BNode>();
    nd->box = box;
    nd->begin = b;  // an inner node's references are [b, e) too
    nd->span = n;
    if (depth < par_depth && n > 4096) {
      auto fut = std::async(std::launch::async, [&, b, mid, depth] { return build(b, mid, depth + 1); });
      nd->r = build(mid, e, depth + 1);
      nd->l = fut.get();
    } else {
      nd->l = build(b, mid, depth + 1);
      nd->r = build(mid, e, depth + 1);
    }
    return nd;
  }
};

// Collapses the two-wide build tree into four-wide quantised nodes.  Which
// build nodes become wide nodes, leaves or opened entries is chosen either
// greedily (each output node takes the two children of a build node and
// repeatedly opens its largest-area inner child until it has four children)
// or, by default, by the dynamic program of the surface-area cost over the
// build tree (as in Ylitie, Karras and Laine, HPG 2017, for eight-wide
// trees): the expected cost of a wide node is kWideNodeCost times its area,
// that of a leaf kLeafRefCost times its area per reference, and every build
// node's cheapest cover by one to four entries is found bottom-up.  Children
// are emitted after their parent (preorder), so child indices exceed
// parents'.
struct Flattener4 {
  // relative cost of one node step (four box tests, the sort and the stack)
  // and of one triangle test, per unit of box area
  static constexpr double kWideNodeCost = 1.0;
  static constexpr double kLeafRefCost = 0.3;

  const std::vector<Ref>& refs;
  const std::vector<float4>& tri3;
  const std::vector<float4>& aux0;
  BuiltBvh& out;
  float pad;
  double root_area;
  uint32_t leaf_max = 0;  // > 0: a subtree with at most this many references becomes one leaf
  bool optimal = true;    // cost-optimal collapse (else greedy)
  std::vector<Plan> plans;  // cost-optimal collapse: one per build node

  static uint32_t refs_of(const BNode* k) { return k->leaf() ? k->count : k->span; }
  bool is_leaf(const BNode* k) const {
    if (optimal) return k->leaf() || plans[k->plan].as_leaf;
    return k->leaf() || (leaf_max && k->span <= leaf_max);
  }

  // bottom-up cover costs of the cost-optimal collapse (costs in float: only
  // their order matters)
  void plan(BNode* n) {
    n->plan = (uint32_t)plans.size();
    plans.emplace_back();
    const float area = n->box.empty() ? 0.0f : n->box.area();
    if (n->leaf()) {
      Plan& P = plans[n->plan];
      const float c = (float)kLeafRefCost * (float)n->count * area;
      for (int j = 0; j < 4; ++j) P.cover[j] = c;
      P.as_leaf = true;
      return;
    }
    BNode* l = n->l.get();
    BNode* r = n->r.get();
    plan(l);
    plan(r);
    const Plan& L = plans[l->plan];
    const Plan& Rr = plans[r->plan];
    Plan P;
    // as a wide node: the two children share its four entries
    float wide = INFINITY;
    for (int k = 1; k <= 3; ++k) {
      const float c = L.cover[k - 1] + Rr.cover[4 - k - 1];
      if (c < wide) {
        wide = c;
        P.wide_l = (uint8_t)k;
      }
    }
    wide += (float)kWideNodeCost * area;
    const float as_leaf =
        (leaf_max && n->span <= leaf_max) ? (float)kLeafRefCost * (float)n->span * area : INFINITY;
    P.as_leaf = as_leaf <= wide;
    P.cover[0] = std::min(as_leaf, wide);
    for (int j = 2; j <= 4; ++j) {
      P.cover[j - 1] = P.cover[j - 2];
      P.cl[j - 1] = P.cl[j - 2];
      P.cr[j - 1] = P.cr[j - 2];
      for (int k = 1; k < j; ++k) {
        const float c = L.cover[k - 1] + Rr.cover[j - k - 1];
        if (c < P.cover[j - 1]) {
          P.cover[j - 1] = c;
          P.cl[j - 1] = (uint8_t)k;
          P.cr[j - 1] = (uint8_t)(j - k);
        }
      }
    }
    plans[n->plan] = P;
  }

  // the entries of a subtree covered by at most j entries, in order
  void gather(const BNode* n, int j, std::vector<const BNode*>& kids) const {
    const Plan& P = plans[n->plan];
    if (P.cl[j - 1] == 0) {
      kids.push_back(n);
      return;
    }
    gather(n->l.get(), P.cl[j - 1], kids);
    gather(n->r.get(), P.cr[j - 1], kids);
  }

  static void quantise_axis(float lo, float hi, float& origin, uint32_t& ebyte) {
    origin = lo;
    double ext = (double)hi - (double)lo;
    // smallest e with ext <= 255 * 2^e, so every child fits in 8 bits
    // a node with no box at all (every child empty) keeps step 1, so its
    // inverted empty slots stay far from any ray's interval
    int e = 0;
    if (ext > 0.0) {
      std::frexp(ext / 255.0, &e);
      while (e > -126 && ext <= 255.0 * std::ldexp(1.0, e - 1)) --e;
      while (ext > 255.0 * std::ldexp(1.0, e)) ++e;
      e = std::max(e, -126);
    }
    ebyte = (uint32_t)(e + 127);
  }

  uint32_t leaf_ref(const BNode* b, int32_t* ref, uint32_t* count) {
    if (refs_of(b) == 0) {
      *ref = kEmpty;
      *count = 0;
      return 0;
    }
    uint32_t start = (uint32_t)(out.tris.size() / 3);
    uint32_t kept = 0;
    for (uint32_t i = 0; i < refs_of(b); ++i) {
      uint32_t id = refs[b->begin + i].id;
      bool dup = false;  // split references of one triangle in the same leaf
      for (uint32_t k = 0; k < i; ++k) dup = dup || refs[b->begin + k].id == id;
      if (dup) continue;
      ++kept;
      out.tris.push_back(tri3[3 * id + 0]);
      out.tris.push_back(tri3[3 * id + 1]);
      out.tris.push_back(tri3[3 * id + 2]);
    }
    out.n_leaves++;
    if (root_area > 0.0) out.sah_cost += b->box.area() / root_area * kept;
    *ref = leaf_ref_encode(start, kept);
    *count = kept;
    return 0;
  }

  // Writes wide node idx (allocated by the caller) for build node b and,
  // below it, its subtree; returns the worst-case stack need of the subtree.
  // A node's leaf triangles are appended before any of its inner children
  // is emitted, and its inner children take consecutive indices (siblings
  // share cache lines and pages).
  uint32_t emit(const BNode* b, uint32_t depth, uint32_t idx) {
    std::vector<const BNode*> kids;
    if (optimal) {
      const uint8_t wl = plans[b->plan].wide_l;
      gather(b->l.get(), wl, kids);
      gather(b->r.get(), 4 - wl, kids);
    } else {
      kids = {b->l.get(), b->r.get()};
    }
    while (!optimal && kids.size() < 4) {
      // open the largest child that has children, those too big for a leaf first
      int best = -1;
      double ba = -1.0;
      bool big = false;
      for (size_t i = 0; i < kids.size(); ++i) {
        if (kids[i]->leaf()) continue;
        const bool kb = !is_leaf(kids[i]);
        if ((kb && !big) || ((kb == big) && kids[i]->box.area() > ba)) {
          ba = kids[i]->box.area();
          best = (int)i;
          big = kb;
        }
      }
      if (best < 0) break;
      const BNode* o = kids[(size_t)best];
      kids[(size_t)best] = o->l.get();
      kids.insert(kids.begin() + best + 1, o->r.get());
    }
    out.max_depth = std::max(out.max_depth, depth);
    if (root_area > 0.0) out.sah_cost += b->box.area() / root_area;
    // padded child boxes and the node frame
    float clo[4][3], chi[4][3];
    float nlo[3] = {INFINITY, INFINITY, INFINITY}, nhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (size_t j = 0; j < kids.size(); ++j) {
      const Box& cb = kids[j]->box;
      for (int a = 0; a < 3; ++a) {
        clo[j][a] = cb.empty() ? 0.0f : cb.lo[a] - pad;
        chi[j][a] = cb.empty() ? 0.0f : cb.hi[a] + pad;
        if (!cb.empty()) {
          nlo[a] = std::min(nlo[a], clo[j][a]);
          nhi[a] = std::max(nhi[a], chi[j][a]);
        }
      }
    }
    for (int a = 0; a < 3; ++a)
      if (!(nlo[a] <= nhi[a])) nlo[a] = nhi[a] = 0.0f;
    float origin[3];
    uint32_t eb[3];
    for (int a = 0; a < 3; ++a) quantise_axis(nlo[a], nhi[a], origin[a], eb[a]);
    uint32_t qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
    int32_t ref[4] = {kEmpty, kEmpty, kEmpty, kEmpty};
    uint32_t need_max = 0, n_kids = 0;
    for (size_t j = 0; j < kids.size(); ++j) {
      const BNode* k = kids[j];
      for (int a = 0; a < 3; ++a) {
        double sc = std::ldexp(1.0, (int)eb[a] - 127);
        double lo = std::floor(((double)clo[j][a] - (double)origin[a]) / sc);
        double hi = std::ceil(((double)chi[j][a] - (double)origin[a]) / sc);
        uint32_t ql = (uint32_t)std::min(255.0, std::max(0.0, lo));
        uint32_t qh = (uint32_t)std::min(255.0, std::max(0.0, hi));
        qlo[a] |= ql << (8 * j);
        qhi[a] |= qh << (8 * j);
      }
      if (is_leaf(k)) {
        uint32_t cnt;
        leaf_ref(k, &ref[j], &cnt);
        if (cnt) ++n_kids;
      }
    }
    // the inner children: one block of consecutive indices, then their subtrees
    uint32_t n_inner = 0;
    for (size_t j = 0; j < kids.size(); ++j) n_inner += is_leaf(kids[j]) ? 0u : 1u;
    const uint32_t base = (uint32_t)out.nodes.size();
    out.nodes.resize(out.nodes.size() + n_inner);
    for (size_t j = 0, k = 0; j < kids.size(); ++j) {
      if (is_leaf(kids[j])) continue;
      const uint32_t child = base + (uint32_t)k++;
      ref[j] = (int32_t)child;
      uint32_t need = emit(kids[j], depth + 1, child);
      need_max = std::max(need_max, need);
      ++n_kids;
    }
    invert_empty_slots(ref, qlo, qhi);
    Node4 nd{};
    uint32_t ebits = eb[0] | (eb[1] << 8) | (eb[2] << 16);
    float ebf;
    std::memcpy(&ebf, &ebits, 4);
    nd.w0 = float4{origin[0], origin[1], origin[2], ebf};
    nd.w1 = uint4{qlo[0], qhi[0], qlo[1], qhi[1]};
    nd.w2 = uint4{qlo[2], qhi[2], 0u, 0u};
    nd.w3 = int4{ref[0], ref[1], ref[2], ref[3]};
    out.nodes[idx] = nd;
    // every hit child but the nearest is pushed (leaves too); the deepest
    // inner child adds its own need on top
    return (n_kids ? n_kids - 1 : 0) + need_max;
  }
};

// Collapses the two-wide build tree into eight-wide quantised nodes.  Each
// output node opens its largest-area inner children until it has eight; the
// children are placed in slots by the corner of the node box they lie toward
// (greedy on the score sum_a sign_a(slot) * (child centre - node centre)_a),
// inner children get consecutive node indices and leaf children consecutive
// triangles.
struct Flattener8 {
  const std::vector<Ref>& refs;
  const std::vector<float4>& tri3;
  BuiltBvh& out;
  float pad;
  double root_area;
  uint32_t leaf_max;  // a subtree with at most this many references becomes one leaf

  static uint32_t refs_of(const BNode* k) { return k->leaf() ? k->count : k->span; }
  bool is_leaf(const BNode* k) const { return k->leaf() || k->span <= leaf_max; }

  // returns the stack need (groups) of the subtree below node `idx`
  uint32_t fill(const BNode* b, uint32_t idx, uint32_t depth) {
    std::vector<const BNode*> kids{b->l.get(), b->r.get()};
    while (kids.size() < 8) {
      // open the largest child that has children: first those too big for a
      // leaf, then leaf-sized ones, which splits them into smaller leaves
      int best = -1;
      double ba = -1.0;
      bool big = false;
      for (size_t i = 0; i < kids.size(); ++i) {
        if (kids[i]->leaf()) continue;
        const bool kb = !is_leaf(kids[i]);
        if ((kb && !big) || ((kb == big) && kids[i]->box.area() > ba)) {
          ba = kids[i]->box.area();
          best = (int)i;
          big = kb;
        }
      }
      if (best < 0) break;
      const BNode* o = kids[(size_t)best];
      kids[(size_t)best] = o->l.get();
      kids.insert(kids.begin() + best + 1, o->r.get());
    }
    kids.erase(std::remove_if(kids.begin(), kids.end(), [](const BNode* k) { return refs_of(k) == 0; }),
               kids.end());
    out.max_depth = std::max(out.max_depth, depth);
    if (root_area > 0.0) out.sah_cost += b->box.area() / root_area;
    // slots by octant
    const BNode* slot[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    {
      double c[3];
      for (int a = 0; a < 3; ++a) c[a] = 0.5 * ((double)b->box.lo[a] + (double)b->box.hi[a]);
      std::vector<bool> used(kids.size(), false);
      for (size_t round = 0; round < kids.size(); ++round) {
        double best = -INFINITY;
        int bk = -1, bs = -1;
        for (size_t j = 0; j < kids.size(); ++j) {
          if (used[j]) continue;
          double kc[3];
          for (int a = 0; a < 3; ++a) kc[a] = 0.5 * ((double)kids[j]->box.lo[a] + (double)kids[j]->box.hi[a]) - c[a];
          for (int s = 0; s < 8; ++s) {
            if (slot[s]) continue;
            double sc = 0.0;
            for (int a = 0; a < 3; ++a) sc += ((s >> a) & 1) ? kc[a] : -kc[a];
            if (sc > best) {
              best = sc;
              bk = (int)j;
              bs = s;
            }
          }
        }
        used[(size_t)bk] = true;
        slot[bs] = kids[(size_t)bk];
      }
    }
    // padded child boxes and the node frame
    float clo[8][3], chi[8][3];
    float nlo[3] = {INFINITY, INFINITY, INFINITY}, nhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int s = 0; s < 8; ++s) {
      if (!slot[s]) continue;
      const Box& cb = slot[s]->box;
      for (int a = 0; a < 3; ++a) {
        clo[s][a] = cb.empty() ? 0.0f : cb.lo[a] - pad;
        chi[s][a] = cb.empty() ? 0.0f : cb.hi[a] + pad;
        if (!cb.empty()) {
          nlo[a] = std::min(nlo[a], clo[s][a]);
          nhi[a] = std::max(nhi[a], chi[s][a]);
        }
      }
    }
    for (int a = 0; a < 3; ++a)
      if (!(nlo[a] <= nhi[a])) nlo[a] = nhi[a] = 0.0f;
    float origin[3];
    uint32_t eb[3];
    for (int a = 0; a < 3; ++a) Flattener4::quantise_axis(nlo[a], nhi[a], origin[a], eb[a]);
    uint32_t qlo[3][2] = {}, qhi[3][2] = {};
    for (int s = 0; s < 8; ++s) {
      if (!slot[s]) continue;
      for (int a = 0; a < 3; ++a) {
        double sc = std::ldexp(1.0, (int)eb[a] - 127);
        double lo = std::floor(((double)clo[s][a] - (double)origin[a]) / sc);
        double hi = std::ceil(((double)chi[s][a] - (double)origin[a]) / sc);
        uint32_t ql = (uint32_t)std::min(255.0, std::max(0.0, lo));
        uint32_t qh = (uint32_t)std::min(255.0, std::max(0.0, hi));
        qlo[a][s >> 2] |= ql << (8 * (s & 3));
        qhi[a][s >> 2] |= qh << (8 * (s & 3));
      }
    }
    // inner children: consecutive nodes in slot order
    uint32_t imask = 0, n_inner = 0;
    for (int s = 0; s < 8; ++s)
      if (slot[s] && !is_leaf(slot[s])) {
        imask |= 1u << s;
        ++n_inner;
      }
    const uint32_t first = (uint32_t)out.nodes8.size();
    out.nodes8.resize(first + n_inner);
    // leaf children: consecutive triangles in slot order
    const uint32_t first_tri = (uint32_t)(out.tris.size() / 3);
    uint32_t leafmask = 0, meta[2] = {0, 0};
    for (int s = 0; s < 8; ++s) {
      if (!slot[s] || !is_leaf(slot[s])) continue;
      const BNode* k = slot[s];
      const uint32_t offset = (uint32_t)(out.tris.size() / 3) - first_tri;
      uint32_t kept = 0;
      for (uint32_t i = 0; i < refs_of(k); ++i) {
        uint32_t id = refs[k->begin + i].id;
        bool dup = false;  // split references of one triangle in the same leaf
        for (uint32_t q = 0; q < i; ++q) dup = dup || refs[k->begin + q].id == id;
        if (dup) continue;
        ++kept;
        out.tris.push_back(tri3[3 * id + 0]);
        out.tris.push_back(tri3[3 * id + 1]);
        out.tris.push_back(tri3[3 * id + 2]);
      }
      out.n_leaves++;
      if (root_area > 0.0) out.sah_cost += k->box.area() / root_area * kept;
      leafmask |= 1u << s;
      meta[s >> 2] |= (((kept - 1u) << 5) | offset) << (8 * (s & 3));
    }
    Node8 nd{};
    uint32_t ebits = eb[0] | (eb[1] << 8) | (eb[2] << 16) | (imask << 24);
    float ebf;
    std::memcpy(&ebf, &ebits, 4);
    nd.w0 = float4{origin[0], origin[1], origin[2], ebf};
    nd.w1 = uint4{first, first_tri | (leafmask << 24), meta[0], meta[1]};
    nd.w2 = uint4{qlo[0][0], qlo[0][1], qhi[0][0], qhi[0][1]};
    nd.w3 = uint4{qlo[1][0], qlo[1][1], qhi[1][0], qhi[1][1]};
    nd.w4 = uint4{qlo[2][0], qlo[2][1], qhi[2][0], qhi[2][1]};
    out.nodes8[idx] = nd;
    uint32_t need = 0, rank = 0;
    for (int s = 0; s < 8; ++s)
      if ((imask >> s) & 1u) need = std::max(need, fill(slot[s], first + rank++, depth + 1));
    // descending into a child pushes at most this node's remaining group
    return need + (n_inner > 1 ? 1u : 0u);
  }
};

uint32_t depth_of(const BNode* b) {
  if (b->leaf()) return 0;
  return 1 + std::max(depth_of(b->l.get()), depth_of(b->r.get()));
}

inline uint32_t fbits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}
inline float bitsf(uint32_t u) {
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

}  // namespace

void build_bvh(const float* V, const uint32_t* F, uint32_t nt, const uint16_t* M,
               const BvhBuildOptions& opt, BuiltBvh& out) {
  auto t0 = std::chrono::steady_clock::now();
  out = BuiltBvh();
  out.n_tris = nt;
  std::vector<float4> tri3((size_t)nt * 3);
  std::vector<float4> aux0(nt);
  std::vector<Ref> refs;
  refs.reserve(nt);
  Box scene;
  float mag = 1.0f;
  for (uint32_t j = 0; j < nt; ++j) {
    const float* p0 = V + 3 * (size_t)F[3 * (size_t)j + 0];
    const float* p1 = V + 3 * (size_t)F[3 * (size_t)j + 1];
    const float* p2 = V + 3 * (size_t)F[3 * (size_t)j + 2];
    float e1[3], e2[3], n[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = p1[a] - p0[a];
      e2[a] = p2[a] - p0[a];
    }
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    float nn = dot3(n[0], n[1], n[2], n[0], n[1], n[2]);
    tri3[3 * (size_t)j + 0] = float4{p0[0], p0[1], p0[2], bitsf(j)};
    tri3[3 * (size_t)j + 1] = float4{e1[0], e1[1], e1[2], 0.0f};
    tri3[3 * (size_t)j + 2] = float4{e2[0], e2[1], e2[2], 0.0f};
    if (!(nn > 0.0f)) continue;  // zero-area: no normal, never hit
    float len = std::sqrt(nn);
    aux0[j] = float4{n[0] / len, n[1] / len, n[2] / len, bitsf((uint32_t)M[j])};
    Ref r;
    r.box.grow(p0);
    r.box.grow(p1);
    r.box.grow(p2);
    for (int a = 0; a < 3; ++a) {
      r.c[a] = 0.5f * (r.box.lo[a] + r.box.hi[a]);
      mag = std::max(mag, std::max(std::fabs(r.box.lo[a]), std::fabs(r.box.hi[a])));
    }
    r.id = j;
    scene.grow(r.box);
    refs.push_back(r);
  }
  out.n_hittable = (uint32_t)refs.size();
  if (opt.split_pct > 0 && !refs.empty()) {
    // largest boxes first; a reference is split while the budget lasts and
    // its box is larger than the mean triangle box
    double mean = 0.0;
    for (const Ref& r : refs) mean += r.box.area();
    mean /= (double)refs.size();
    const size_t budget = refs.size() + (size_t)((uint64_t)refs.size() * std::min(opt.split_pct, 200u) / 100u);
    struct Cell {
      double lo[3], hi[3];
    };
    std::vector<Cell> region(refs.size());  // the cell each reference is clipped to
    for (size_t i = 0; i < refs.size(); ++i)
      for (int a = 0; a < 3; ++a) {
        region[i].lo[a] = refs[i].box.lo[a];
        region[i].hi[a] = refs[i].box.hi[a];
      }
    auto cmp = [&](uint32_t x, uint32_t y) {
      const double ax = refs[x].box.area(), ay = refs[y].box.area();
      return ax < ay || (ax == ay && x > y);
    };
    std::priority_queue<uint32_t, std::vector<uint32_t>, decltype(cmp)> heap(cmp);
    for (uint32_t i = 0; i < (uint32_t)refs.size(); ++i) heap.push(i);
    while (refs.size() < budget && !heap.empty()) {
      const uint32_t i = heap.top();
      if (!(refs[i].box.area() > mean)) break;
      heap.pop();
      const uint32_t id = refs[i].id;
      double p[3][3];
      for (int v = 0; v < 3; ++v) {
        const float* q = V + 3 * (size_t)F[3 * (size_t)id + v];
        for (int a = 0; a < 3; ++a) p[v][a] = q[a];
      }
      const Box tb = refs[i].box;
      int ax = 0;
      for (int a = 1; a < 3; ++a)
        if (tb.hi[a] - tb.lo[a] > tb.hi[ax] - tb.lo[ax]) ax = a;
      const double c = 0.5 * ((double)tb.lo[ax] + (double)tb.hi[ax]);
      Cell lc, rc;
      for (int a = 0; a < 3; ++a) {
        lc.lo[a] = rc.lo[a] = std::max(region[i].lo[a], (double)tb.lo[a]);
        lc.hi[a] = rc.hi[a] = std::min(region[i].hi[a], (double)tb.hi[a]);
      }
      lc.hi[ax] = c;
      rc.lo[ax] = c;
      Box lb, rb;
      const bool hl = clipped_bounds(p, lc.lo, lc.hi, lb), hr = clipped_bounds(p, rc.lo, rc.hi, rb);
      if (!hl || !hr) continue;  // degenerate cut: keep the reference as it is
      for (int a = 0; a < 3; ++a) {  // never wider than the reference itself
        lb.lo[a] = std::max(lb.lo[a], tb.lo[a]);
        lb.hi[a] = std::min(lb.hi[a], tb.hi[a]);
        rb.lo[a] = std::max(rb.lo[a], tb.lo[a]);
        rb.hi[a] = std::min(rb.hi[a], tb.hi[a]);
      }
      // the two cells share the cut exactly (float64), so together they keep
      // every point of the triangle the parent cell held
      Ref r2 = refs[i];
      refs[i].box = lb;
      r2.box = rb;
      for (int a = 0; a < 3; ++a) {
        refs[i].c[a] = 0.5f * (lb.lo[a] + lb.hi[a]);
        r2.c[a] = 0.5f * (rb.lo[a] + rb.hi[a]);
      }
      region[i] = lc;
      refs.push_back(r2);
      region.push_back(rc);
      heap.push(i);
      heap.push((uint32_t)refs.size() - 1);
    }
  }
  out.n_refs = (uint32_t)refs.size();
  out.pad = mag * (1.0f / 262144.0f);  // 2^-18 of the largest coordinate
  for (int a = 0; a < 3; ++a) {
    out.lo[a] = scene.empty() ? 0.0f : scene.lo[a];
    out.hi[a] = scene.empty() ? 0.0f : scene.hi[a];
  }
  unsigned hw = std::thread::hardware_concurrency();
  unsigned th = opt.threads ? opt.threads : (hw ? hw : 1);
  int par_depth = 0;
  while ((1u << par_depth) < th && par_depth < 8) ++par_depth;
  // the eight-wide collapse forms its own leaves (subtrees of at most
  // max_leaf references), so its binary tree goes down to single triangles
  const bool merge = opt.width == 8 || opt.merge_leaves;
  const uint32_t leaf2 = merge ? 1u : std::max(1u, opt.max_leaf);
  Builder bld{refs, leaf2, std::max(4u, opt.bins), par_depth};
  std::unique_ptr<BNode> root;
  uint32_t n = (uint32_t)refs.size();
  if (n >= 2 && opt.spatial_pct > 0) {
    const double ra = scene.empty() ? 0.0 : scene.area();
    SpatialBuilder sb{V, F, leaf2, std::max(4u, opt.bins), par_depth, kSpatialOverlap * ra};
    const int64_t allow = (int64_t)((uint64_t)n * std::min(opt.spatial_pct, 200u) / 100u);
    root = sb.build(std::move(refs), 0, allow);
    refs.clear();
    SpatialBuilder::gather(root.get(), refs);
    n = (uint32_t)refs.size();
    out.n_refs = n;
  } else if (n >= 2) {
    root = bld.build(0, n, 0);
  }
  if (!root || root->leaf()) {
    // the root must be an inner node: hang everything (0 or 1 triangle, or
    // one leaf) under it next to an empty leaf
    auto r = std::make_unique<BNode>();
    Box box;
    for (uint32_t i = 0; i < n; ++i) box.grow(refs[i].box);
    r->box = box;
    r->l = bld.make_leaf(0, n, box);
    r->r = bld.make_leaf(n, 0, Box());
    root = std::move(r);
  }
  out.max_depth2 = depth_of(root.get()) - 1;
  out.width = opt.width == 8 ? 8u : 4u;
  if (out.width == 8) {
    Flattener8 fl{refs, tri3, out, out.pad, root->box.empty() ? 0.0 : root->box.area(), opt.max_leaf};
    out.nodes8.resize(1);
    out.max_stack = fl.fill(root.get(), 0, 0);
  } else {
    Flattener4 fl{refs, tri3, aux0, out, out.pad, root->box.empty() ? 0.0 : root->box.area(),
                  merge ? std::max(1u, opt.max_leaf) : 0u, opt.collapse != 1};
    if (fl.optimal) {
      fl.plans.reserve(2 * (size_t)n + 2);
      fl.plan(root.get());
    }
    out.nodes.resize(1);
    out.max_stack = fl.emit(root.get(), 0, 0);
  }
  out.aux = std::move(aux0);
  auto t1 = std::chrono::steady_clock::now();
  out.build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
}

// ---------------------------------------------------------------- host traversal
namespace {
inline void leaf_test(const BuiltBvh& b, uint32_t start, uint32_t count, const float o[3],
                      const float d[3], int32_t excl, float& best_t, int32_t& best,
                      uint32_t& best_orig) {
  for (uint32_t k = 0; k < count; ++k) {
    uint32_t li = start + k;
    const float4& a = b.tris[3 * (size_t)li + 0];
    if ((int32_t)fbits(a.w) == excl) continue;
    const float4& e1 = b.tris[3 * (size_t)li + 1];
    const float4& e2 = b.tris[3 * (size_t)li + 2];
    float t;
    if (!ray_tri(o[0], o[1], o[2], d[0], d[1], d[2], a.x, a.y, a.z, e1.x, e1.y, e1.z, e2.x, e2.y,
                 e2.z, best_t, t))
      continue;
    uint32_t orig = fbits(a.w);
    if (best < 0 || t < best_t || (t == best_t && orig < best_orig)) {
      best_t = t;
      best = (int32_t)li;
      best_orig = orig;
    }
  }
}
}  // namespace

int32_t host_traverse(const BuiltBvh& b, const float o[3], const float d[3], float tmax,
                      int32_t excl, float* t_out) {
  RayBox rb;
  ray_box_setup(o[0], o[1], o[2], d[0], d[1], d[2], rb);
  float best_t = tmax;
  int32_t best = -1;
  uint32_t best_orig = 0xffffffffu;
  int32_t stack[kStack + kSpill];
  int sp = 0;
  int32_t cur = 0;
  for (;;) {
    if (cur == kEmpty) {
      if (sp == 0) break;
      cur = stack[--sp];
    }
    if (cur < 0) {  // a leaf
      leaf_test(b, leaf_start(cur), leaf_count(cur), o, d, excl, best_t, best, best_orig);
      cur = kEmpty;
      continue;
    }
    const Node4& nd = b.nodes[(size_t)cur];
    float tn[4];
    uint32_t mask = node4_boxes(nd.w0, nd.w1, nd.w2, nd.w3, rb, best_t, tn);
    const int32_t ref[4] = {nd.w3.x, nd.w3.y, nd.w3.z, nd.w3.w};
    float key[4];
    int32_t val[4];
    for (int j = 0; j < 4; ++j) {
      bool h = (mask >> j) & 1u;
      key[j] = h ? tn[j] : INFINITY;
      val[j] = h ? ref[j] : kEmpty;
    }
    // near to far (5 compare-exchanges); misses sink to the end
    const int pairs[5][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}, {1, 2}};
    for (auto& pr : pairs)
      if (key[pr[1]] < key[pr[0]]) {
        std::swap(key[pr[0]], key[pr[1]]);
        std::swap(val[pr[0]], val[pr[1]]);
      }
    for (int j = 3; j >= 1; --j) {
      if (val[j] == kEmpty) continue;
      if (sp >= kStack + kSpill) return -2;  // exceeds the bound computed at build time
      stack[sp++] = val[j];
    }
    cur = val[0];
  }
  if (t_out) *t_out = best_t;
  return best;
}

// Eight-wide traversal on the host: the same node-group stack (first inner
// child, hit slots in octant order, inner-slot mask) the GPU kernel keeps.
int32_t host_traverse8(const BuiltBvh& b, const float o[3], const float d[3], float tmax,
                       int32_t excl, float* t_out) {
  RayBox rb;
  ray_box_setup(o[0], o[1], o[2], d[0], d[1], d[2], rb);
  const uint32_t oct = ray_octant(rb);
  float best_t = tmax;
  int32_t best = -1;
  uint32_t best_orig = 0xffffffffu;
  uint32_t gs_base[kMaxDepth + 2], gs_mask[kMaxDepth + 2];
  int sp = 0;
  uint32_t g_base = 0, g_mask = 0;  // current group: (first child, order bits | imask << 8)
  int32_t cur = 0;
  for (;;) {
    if (cur < 0) {
      if ((g_mask & 0xffu) == 0) {
        if (sp == 0) break;
        --sp;
        g_base = gs_base[sp];
        g_mask = gs_mask[sp];
      }
      const uint32_t i = (uint32_t)__builtin_ctz(g_mask & 0xffu);
      g_mask &= ~(1u << i);
      const uint32_t s = i ^ oct, im = g_mask >> 8;
      cur = (int32_t)(g_base + (uint32_t)__builtin_popcount(im & ((1u << s) - 1u)));
    }
    const Node8& nd = b.nodes8[(size_t)cur];
    const uint32_t hits = node8_boxes(nd, rb, best_t);
    const uint32_t im = fbits(nd.w0.w) >> 24, lm = nd.w1.y >> 24;
    for (int s = 0; s < 8; ++s) {
      if (!((hits & lm) >> s & 1u)) continue;
      const uint32_t meta = ((s < 4 ? nd.w1.z : nd.w1.w) >> (8 * (s & 3))) & 0xffu;
      leaf_test(b, (nd.w1.y & 0xffffffu) + (meta & 31u), (meta >> 5) + 1u, o, d, excl, best_t, best,
                best_orig);
    }
    const uint32_t inner = hits & im;
    if (inner) {
      if (g_mask & 0xffu) {
        if (sp >= kMaxDepth + 2) return -2;
        gs_base[sp] = g_base;
        gs_mask[sp] = g_mask;
        ++sp;
      }
      g_base = nd.w1.x;
      g_mask = octant_order(inner, oct) | (im << 8);
    }
    cur = -1;
  }
  if (t_out) *t_out = best_t;
  return best;
}

int32_t host_brute(const BuiltBvh& b, const float o[3], const float d[3], float tmax,
                   int32_t excl, float* t_out) {
  float best_t = tmax;
  int32_t best = -1;
  uint32_t best_orig = 0xffffffffu;
  leaf_test(b, 0, (uint32_t)(b.tris.size() / 3), o, d, excl, best_t, best, best_orig);
  if (t_out) *t_out = best_t;
  return best;
}

uint64_t bvh_selfcheck(const BuiltBvh& b, uint32_t n_rays, uint64_t seed) {
  // xorshift64* for ray sampling; rays start inside the scene bounds
  uint64_t s = seed * 0x9E3779B97F4A7C15ull + 1;
  auto next = [&]() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return (double)((s * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
  };
  float diag = 0.0f;
  for (int a = 0; a < 3; ++a) diag += (b.hi[a] - b.lo[a]) * (b.hi[a] - b.lo[a]);
  float tmax = 2.0f * std::sqrt(diag) + 1.0f;
  uint64_t bad = 0;
  uint32_t nl = (uint32_t)(b.tris.size() / 3);
  for (uint32_t r = 0; r < n_rays; ++r) {
    float o[3], d[3];
    for (int a = 0; a < 3; ++a) o[a] = (float)(b.lo[a] + (b.hi[a] - b.lo[a]) * next());
    double x, y, z, q;
    do {
      x = 2 * next() - 1;
      y = 2 * next() - 1;
      z = 2 * next() - 1;
      q = x * x + y * y + z * z;
    } while (q > 1.0 || q < 1e-6);
    q = std::sqrt(q);
    d[0] = (float)(x / q);
    d[1] = (float)(y / q);
    d[2] = (float)(z / q);
    int32_t excl = (nl && (r & 3) == 0) ? (int32_t)fbits(b.tris[3 * (size_t)(next() * nl)].w) : -1;
    float ta, tb;
    int32_t ha = b.width == 8 ? host_traverse8(b, o, d, tmax, excl, &ta) : host_traverse(b, o, d, tmax, excl, &ta);
    int32_t hb = host_brute(b, o, d, tmax, excl, &tb);
    uint32_t oa = ha >= 0 ? fbits(b.tris[3 * (size_t)ha].w) : 0xffffffffu;
    uint32_t ob = hb >= 0 ? fbits(b.tris[3 * (size_t)hb].w) : 0xffffffffu;
    if (oa != ob || ha == -2) ++bad;
  }
  return bad;
}

}  // namespace rr
