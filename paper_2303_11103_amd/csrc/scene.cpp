// Host-side scene preparation: triangle records, face grouping and a binned
// SAH bounding volume hierarchy laid out for the GPU traversal kernels.
//
// The paper models surfaces as triangle meshes whose primitives are
// intersected by rays (Sec. II) and identifies candidate paths by ordered
// lists of primitives (Sec. II-B).  Here a primitive of a candidate is a face:
// a maximal set of triangles in one plane with one material, since the image
// method depends only on the plane and the material of each interaction.
#include "scene.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

namespace rt {
namespace {

struct Box {
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const double* p) {
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], p[i]);
            hi[i] = std::max(hi[i], p[i]);
        }
    }
    void grow(const Box& b) {
        for (int i = 0; i < 3; ++i) {
            lo[i] = std::min(lo[i], b.lo[i]);
            hi[i] = std::max(hi[i], b.hi[i]);
        }
    }
    double area() const {
        double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        if (!(dx >= 0) || !(dy >= 0) || !(dz >= 0)) return 0.0;
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

struct Prim {
    Box box;
    double c[3];
    int32_t tri;
};

struct BuildNode {
    Box box;
    int32_t left = -1, right = -1;  // BuildNode indices, -1 for leaves
    int32_t first = 0, count = 0;   // leaf range in prims
};

class Builder {
public:
    // depth_bound: the binary tree gets no deeper than this; subtrees that
    // would exceed it are split at object medians
    Builder(std::vector<Prim>& prims, int depth_bound) : prims_(prims), bound_(depth_bound) {}

    int32_t build(int32_t first, int32_t count, int depth) {
        int32_t id = (int32_t)nodes_.size();
        nodes_.emplace_back();
        Box b, cb;
        for (int32_t i = first; i < first + count; ++i) {
            b.grow(prims_[i].box);
            cb.grow(prims_[i].c);
        }
        nodes_[id].box = b;
        max_depth_ = std::max(max_depth_, depth);
        if (count <= 2) return leaf(id, first, count);
        int force_median = (depth + (int)std::ceil(std::log2((double)count)) >= bound_ - 1);
        int axis = 0;
        double ext[3];
        for (int i = 0; i < 3; ++i) ext[i] = cb.hi[i] - cb.lo[i];
        if (ext[1] > ext[axis]) axis = 1;
        if (ext[2] > ext[axis]) axis = 2;
        int32_t mid = -1;
        if (!force_median && ext[axis] > 0.0) mid = sah_split(first, count, cb, b, count <= kMaxLeaf);
        if (mid == -2) return leaf(id, first, count);
        if (mid < 0) {  // object median along the widest centroid axis
            mid = first + count / 2;
            std::nth_element(prims_.begin() + first, prims_.begin() + mid, prims_.begin() + first + count,
                             [axis](const Prim& x, const Prim& y) {
                                 return x.c[axis] < y.c[axis] || (x.c[axis] == y.c[axis] && x.tri < y.tri);
                             });
        }
        int32_t l = build(first, mid - first, depth + 1);
        int32_t r = build(mid, first + count - mid, depth + 1);
        nodes_[id].left = l;
        nodes_[id].right = r;
        return id;
    }

    std::vector<BuildNode>& nodes() { return nodes_; }
    int max_depth() const { return max_depth_; }

private:
    int32_t leaf(int32_t id, int32_t first, int32_t count) {
        nodes_[id].first = first;
        nodes_[id].count = count;
        return id;
    }

    // Binned SAH, count / 8 bins per axis clamped to [16, 128] (large nodes,
    // where a coarse split costs most, get fine bins), plus one partition by
    // primitive size.  Returns the split position, -2 when a leaf is cheaper
    // (only allowed when count <= kMaxLeaf), -1 when no valid split exists.
    int32_t sah_split(int32_t first, int32_t count, const Box& cb, const Box& b, bool leaf_ok) {
        constexpr int kMaxBins = 128;
        const int kBins = std::min(kMaxBins, std::max(16, count / 8));
        constexpr double kTrav = 1.0, kIsect = 1.5;
        double best = INFINITY;
        int best_axis = -1, best_bin = -1;
        for (int ax = 0; ax < 3; ++ax) {
            double lo = cb.lo[ax], ext = cb.hi[ax] - cb.lo[ax];
            if (!(ext > 0.0)) continue;
            Box bins[kMaxBins];
            int cnt[kMaxBins] = {0};
            for (int32_t i = first; i < first + count; ++i) {
                int k = (int)((prims_[i].c[ax] - lo) / ext * kBins);
                k = std::min(std::max(k, 0), kBins - 1);
                bins[k].grow(prims_[i].box);
                cnt[k]++;
            }
            double right_area[kMaxBins];
            int right_cnt[kMaxBins];
            Box acc;
            int n = 0;
            for (int k = kBins - 1; k > 0; --k) {
                acc.grow(bins[k]);
                n += cnt[k];
                right_area[k] = acc.area();
                right_cnt[k] = n;
            }
            Box lacc;
            int ln = 0;
            for (int k = 0; k < kBins - 1; ++k) {
                lacc.grow(bins[k]);
                ln += cnt[k];
                if (ln == 0 || right_cnt[k + 1] == 0) continue;
                double cost = lacc.area() * ln + right_area[k + 1] * right_cnt[k + 1];
                if (cost < best) {
                    best = cost;
                    best_axis = ax;
                    best_bin = k;
                }
            }
        }
        // candidate: the primitives whose own box has at least a quarter of the
        // node's surface area apart from the others (a large ground polygon
        // otherwise inflates every node on its way down to a leaf)
        const double parent_area = b.area();
        int n_large = 0;
        Box large_box, small_box;
        for (int32_t i = first; i < first + count; ++i) {
            if (prims_[i].box.area() >= 0.25 * parent_area) {
                ++n_large;
                large_box.grow(prims_[i].box);
            } else {
                small_box.grow(prims_[i].box);
            }
        }
        bool size_split = false;
        if (n_large > 0 && n_large < count) {
            const double cost = large_box.area() * n_large + small_box.area() * (count - n_large);
            if (cost < best) {
                best = cost;
                size_split = true;
            }
        }
        if (best_axis < 0 && !size_split) return -1;
        double split_cost = kTrav + kIsect * best / std::max(parent_area, 1e-300);
        if (leaf_ok && kIsect * count <= split_cost) return -2;
        if (size_split) {
            auto it = std::partition(prims_.begin() + first, prims_.begin() + first + count,
                                     [&](const Prim& p) { return p.box.area() >= 0.25 * parent_area; });
            return (int32_t)(it - prims_.begin());
        }
        double lo = cb.lo[best_axis], ext = cb.hi[best_axis] - cb.lo[best_axis];
        auto it = std::partition(prims_.begin() + first, prims_.begin() + first + count, [&](const Prim& p) {
            int k = (int)((p.c[best_axis] - lo) / ext * kBins);
            k = std::min(std::max(k, 0), kBins - 1);
            return k <= best_bin;
        });
        int32_t mid = (int32_t)(it - prims_.begin());
        if (mid == first || mid == first + count) return -1;
        return mid;
    }

    std::vector<Prim>& prims_;
    int bound_;
    std::vector<BuildNode> nodes_;
    int max_depth_ = 0;
};

float round_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = std::nextafter(f, -INFINITY);
    return f;
}
float round_up(double x) {
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

void cross(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
double norm(const double* a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

// Wedges for first-order diffraction.  Mesh edges are matched by their two
// vertex positions; an edge is a wedge when exactly two triangles of two
// different faces share it, it does not lie on the ground (both vertices at
// the lowest z of the scene), and the interior angle alpha between the faces'
// half-planes (taken as the smaller one: convex solids) is below pi - 1e-6.
// The edge runs from the first to the second vertex as they appear in the
// lower-indexed triangle; the 0-face is the face with the smaller id.
void extract_wedges(const float* V, const int32_t* F, int64_t nt, const int32_t* tri_mat, HostScene& out) {
    using P3 = std::array<double, 3>;
    auto vert = [&](int32_t i) { return P3{(double)V[3 * i], (double)V[3 * i + 1], (double)V[3 * i + 2]}; };
    double zmin = INFINITY;
    struct Use {
        int64_t tri;
        P3 third, p, q;
    };
    std::map<std::pair<P3, P3>, std::vector<Use>> edges;
    for (int64_t k = 0; k < nt; ++k) {
        for (int i = 0; i < 3; ++i) {
            const P3 p = vert(F[3 * k + i]), q = vert(F[3 * k + (i + 1) % 3]), r = vert(F[3 * k + (i + 2) % 3]);
            zmin = std::min(zmin, p[2]);
            edges[p < q ? std::make_pair(p, q) : std::make_pair(q, p)].push_back(Use{k, r, p, q});
        }
    }
    auto sub = [](const P3& a, const P3& b) { return P3{a[0] - b[0], a[1] - b[1], a[2] - b[2]}; };
    auto dotp = [](const P3& a, const P3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    auto into = [&](const P3& a, const P3& e, const P3& v) {
        P3 w = sub(v, a);
        const double d = dotp(w, e);
        for (int i = 0; i < 3; ++i) w[i] -= d * e[i];
        const double l = std::sqrt(dotp(w, w));
        return P3{w[0] / l, w[1] / l, w[2] / l};
    };
    std::vector<std::pair<Wedge, P3>> ws;  // wedge and its second vertex (the sort key)
    for (const auto& kv : edges) {
        const auto& u = kv.second;
        if (u.size() != 2) continue;
        const int32_t f1 = out.face_of_input[u[0].tri], f2 = out.face_of_input[u[1].tri];
        if (f1 == f2) continue;
        const P3 a = u[0].p, b = u[0].q;
        if (a[2] <= zmin && b[2] <= zmin) continue;
        const P3 d = sub(b, a);
        const double len = std::sqrt(dotp(d, d));
        const P3 e{d[0] / len, d[1] / len, d[2] / len};
        const P3 u1 = into(a, e, u[0].third), u2 = into(a, e, u[1].third);
        const double alpha = std::acos(std::min(1.0, std::max(-1.0, dotp(u1, u2))));
        if (alpha >= M_PI - 1e-6) continue;
        const bool first0 = f1 < f2;
        const P3 t0 = first0 ? u1 : u2, tn = first0 ? u2 : u1;
        P3 n0{e[1] * t0[2] - e[2] * t0[1], e[2] * t0[0] - e[0] * t0[2], e[0] * t0[1] - e[1] * t0[0]};
        if (dotp(n0, tn) > 0.0)
            for (double& x : n0) x = -x;
        Wedge w{};
        for (int i = 0; i < 3; ++i) {
            w.a[i] = a[i];
            w.e[i] = e[i];
            w.t0[i] = t0[i];
            w.n0[i] = n0[i];
        }
        w.len = len;
        w.n = 2.0 - alpha / M_PI;
        w.face0 = first0 ? f1 : f2;
        w.facen = first0 ? f2 : f1;
        w.mat0 = tri_mat[first0 ? u[0].tri : u[1].tri];
        w.matn = tri_mat[first0 ? u[1].tri : u[0].tri];
        ws.emplace_back(w, b);
    }
    std::sort(ws.begin(), ws.end(), [](const std::pair<Wedge, P3>& x, const std::pair<Wedge, P3>& y) {
        if (x.first.face0 != y.first.face0) return x.first.face0 < y.first.face0;
        if (x.first.facen != y.first.facen) return x.first.facen < y.first.facen;
        for (int i = 0; i < 3; ++i)
            if (x.first.a[i] != y.first.a[i]) return x.first.a[i] < y.first.a[i];
        return x.second < y.second;
    });
    out.wedges.clear();
    for (const auto& w : ws) out.wedges.push_back(w.first);
}

}  // namespace

int build_scene(const float* V, int64_t nv, const int32_t* F, int64_t nt, const int32_t* tri_mat, int32_t nm,
                HostScene& out, std::string& err) {
    auto t0 = std::chrono::steady_clock::now();
    if (nt <= 0 || nt >= (int64_t(1) << 26)) {
        err = "number of triangles must be in [1, 2^26)";
        return -1;
    }
    double max_abs = 0.0;
    for (int64_t i = 0; i < 3 * nv; ++i) {
        if (!std::isfinite(V[i])) {
            err = "vertex coordinate " + std::to_string(i / 3) + " is not finite";
            return -1;
        }
        max_abs = std::max(max_abs, (double)std::fabs(V[i]));
    }
    out = HostScene();
    out.max_abs = std::max(max_abs, 64.0);
    out.pad = out.max_abs * std::ldexp(1.0, -20);

    // ---- triangle records and canonical planes (fp64 from exact float inputs)
    std::vector<Tri> tri(nt);
    std::vector<Shade> shade(nt);
    std::vector<Prim> prims(nt);
    std::vector<double> offs(nt);
    for (int64_t k = 0; k < nt; ++k) {
        int32_t i0 = F[3 * k], i1 = F[3 * k + 1], i2 = F[3 * k + 2];
        if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= nv || i1 >= nv || i2 >= nv) {
            err = "triangle " + std::to_string(k) + " has a vertex index outside [0, nv)";
            return -1;
        }
        if (tri_mat[k] < 0 || tri_mat[k] >= nm) {
            err = "triangle " + std::to_string(k) + " has a material index outside [0, nm)";
            return -1;
        }
        double p0[3], p1[3], p2[3];
        for (int i = 0; i < 3; ++i) {
            p0[i] = V[3 * i0 + i];
            p1[i] = V[3 * i1 + i];
            p2[i] = V[3 * i2 + i];
        }
        Tri& t = tri[k];
        for (int i = 0; i < 3; ++i) {
            t.v0[i] = p0[i];
            t.e1[i] = p1[i] - p0[i];
            t.e2[i] = p2[i] - p0[i];
        }
        t.thr = 1e-12 * norm(t.e1) * norm(t.e2);
        t.orig = (int32_t)k;
        double n[3];
        cross(t.e1, t.e2, n);
        double a = norm(n);
        if (!(a > 0.0)) {
            err = "triangle " + std::to_string(k) + " has zero area";
            return -1;
        }
        for (int i = 0; i < 3; ++i) n[i] /= a;
        int first = 0;
        while (first < 2 && !(std::fabs(n[first]) > 1e-6)) ++first;
        if (n[first] < 0)
            for (int i = 0; i < 3; ++i) n[i] = -n[i];
        for (int i = 0; i < 3; ++i) shade[k].n[i] = n[i];
        shade[k].mat = tri_mat[k];
        offs[k] = n[0] * p0[0] + n[1] * p0[1] + n[2] * p0[2];
        Prim& p = prims[k];
        p.box.grow(p0);
        p.box.grow(p1);
        p.box.grow(p2);
        for (int i = 0; i < 3; ++i) p.c[i] = (p0[i] + p1[i] + p2[i]) / 3.0;
        p.tri = (int32_t)k;
    }

    // ---- faces: (material, rint(n * 2^30), rint(c * 2^30)), numbered by first triangle
    const double q = std::ldexp(1.0, 30);
    std::map<std::tuple<int32_t, int64_t, int64_t, int64_t, int64_t>, int32_t> ids;
    out.face_of_input.resize(nt);
    std::vector<int32_t> face_first;
    for (int64_t k = 0; k < nt; ++k) {
        auto key = std::make_tuple(tri_mat[k], (int64_t)std::nearbyint(shade[k].n[0] * q),
                                   (int64_t)std::nearbyint(shade[k].n[1] * q),
                                   (int64_t)std::nearbyint(shade[k].n[2] * q), (int64_t)std::nearbyint(offs[k] * q));
        auto it = ids.find(key);
        int32_t f;
        if (it == ids.end()) {
            f = (int32_t)ids.size();
            ids.emplace(key, f);
            face_first.push_back((int32_t)k);
        } else {
            f = it->second;
        }
        out.face_of_input[k] = f;
        tri[k].face = f;
        shade[k].face = f;
    }
    out.num_faces = (int32_t)face_first.size();

    // ---- BVH.  The traversal kernels keep kStackEntries stack entries per
    // lane in LDS and need a slower variant with a private-memory overflow for
    // deeper trees, so a tree whose worst-case stack need exceeds that is
    // rebuilt with a tighter depth bound (deep, thin SAH branches become
    // balanced median splits) while the bound stays above log2(nt) + 2.
    const std::vector<Prim> prims_in = prims;
    std::vector<int32_t> new_of_old;
    const int min_bound = (int)std::ceil(std::log2((double)nt)) + 2;
    // Attempts: the SAH tree collapsed by opening the child of largest area;
    // then collapsed by opening the tallest child, which spends the four slots
    // on the deepest paths; then that with tighter depth bounds.
    for (int attempt = 0, bound = kMaxDepth;; ++attempt, bound -= attempt >= 2 ? 2 : 0) {
        const bool by_height = attempt >= 1;
        prims = prims_in;
        Builder builder(prims, bound);
        builder.build(0, (int32_t)nt, 0);
        auto& bn = builder.nodes();
        // subtree heights (children follow their parent in build order)
        std::vector<int> height(bn.size(), 0);
        for (size_t i = bn.size(); i-- > 0;)
            if (bn[i].left >= 0) height[i] = 1 + std::max(height[bn[i].left], height[bn[i].right]);
        out.depth = builder.max_depth();
        if (out.depth > kMaxDepth + 1) {
            err = "BVH build tree deeper than expected";
            return -1;
        }

        // reorder triangles by leaf order
        out.tris.resize(nt);
        out.shades.resize(nt);
        new_of_old.assign(nt, 0);
        for (int64_t i = 0; i < nt; ++i) {
            out.tris[i] = tri[prims[i].tri];
            out.shades[i] = shade[prims[i].tri];
            new_of_old[prims[i].tri] = (int32_t)i;
        }

        // Collapse the binary build tree into a 4-wide tree: a node adopts up to
        // four descendants by repeatedly opening the inner child with the largest
        // surface area.  Nodes are numbered breadth first, so the first ones are
        // the top levels, which the kernels stage in LDS.
        const double p = out.pad;
        auto set_box = [&](Node& g, int slot, const Box& B) {
            g.bx[0][slot] = round_down(B.lo[0] - p);
            g.bx[1][slot] = round_up(B.hi[0] + p);
            g.bx[2][slot] = round_down(B.lo[1] - p);
            g.bx[3][slot] = round_up(B.hi[1] + p);
            g.bz[0][slot] = round_down(B.lo[2] - p);
            g.bz[1][slot] = round_up(B.hi[2] + p);
        };
        auto empty_slot = [&](Node& g, int slot) {
            g.bx[0][slot] = g.bx[2][slot] = g.bz[0][slot] = INFINITY;
            g.bx[1][slot] = g.bx[3][slot] = g.bz[1][slot] = -INFINITY;
            g.child[slot] = kEmptyChild;
        };
        auto gather = [&](int32_t b) {
            std::vector<int32_t> kids;
            if (bn[b].left < 0) {
                kids.push_back(b);  // a root leaf becomes the only child of the root
                return kids;
            }
            kids = {bn[b].left, bn[b].right};
            while (kids.size() < 4) {
                int best = -1;
                double score = -1.0;
                for (int i = 0; i < (int)kids.size(); ++i) {
                    const BuildNode& c = bn[kids[i]];
                    // by height: the tallest subtree (ties: the largest area)
                    const double sc = by_height ? height[kids[i]] + c.box.area() / (1.0 + bn[0].box.area())
                                                : c.box.area();
                    if (c.left >= 0 && sc > score) {
                        score = sc;
                        best = i;
                    }
                }
                if (best < 0) break;
                int32_t open = kids[best];
                kids.erase(kids.begin() + best);
                kids.insert(kids.begin() + best, bn[open].right);
                kids.insert(kids.begin() + best, bn[open].left);
            }
            return kids;
        };
        {
            std::vector<int32_t> order = {0};            // build nodes that become GPU nodes, BFS order
            std::vector<std::vector<int32_t>> kids_of;
            std::vector<int32_t> gpu_of(bn.size(), -1);
            gpu_of[0] = 0;
            for (size_t h = 0; h < order.size(); ++h) {
                std::vector<int32_t> kids = gather(order[h]);
                for (int32_t c : kids) {
                    if (bn[c].left >= 0 && c != order[h]) {
                        gpu_of[c] = (int32_t)order.size();
                        order.push_back(c);
                    }
                }
                kids_of.push_back(kids);
            }
            out.nodes.resize(order.size());
            std::vector<int> need(order.size(), 0);
            for (size_t h = 0; h < order.size(); ++h) {
                Node& g = out.nodes[h];
                std::memset(&g, 0, sizeof(Node));
                const auto& kids = kids_of[h];
                for (int slot = 0; slot < 4; ++slot) {
                    if (slot >= (int)kids.size()) {
                        empty_slot(g, slot);
                        continue;
                    }
                    const BuildNode& c = bn[kids[slot]];
                    set_box(g, slot, c.box);
                    g.child[slot] = (c.left < 0 || kids[slot] == order[h]) ? make_leaf(c.first, c.count) : gpu_of[kids[slot]];
                }
            }
            // worst-case stack: along any root-to-leaf path, a visit pushes all but one child
            for (size_t h = order.size(); h-- > 0;) {
                int deepest = 0, n = 0;
                for (int slot = 0; slot < 4; ++slot) {
                    int32_t c = out.nodes[h].child[slot];
                    if (c == kEmptyChild) continue;
                    ++n;
                    if (c >= 0) deepest = std::max(deepest, need[c]);
                }
                need[h] = (n - 1) + deepest;
            }
            out.stack_need = need[0] + 1;
        }
        out.depth_bound = bound;
        out.collapse_by_height = by_height;
        if (out.stack_need <= kStackEntries || (attempt >= 1 && bound - 2 < min_bound)) break;
    }
    if (out.stack_need > kStackEntries + kStackOverflow) {  // 64 entries in all
        err = "BVH needs a deeper traversal stack than " + std::to_string(kStackEntries + kStackOverflow);
        return -1;
    }

    // ---- faces with their triangles (reordered indices)
    out.faces.resize(out.num_faces);
    std::vector<int32_t> cnt(out.num_faces, 0);
    for (int64_t k = 0; k < nt; ++k) cnt[out.face_of_input[k]]++;
    int32_t acc = 0;
    for (int32_t f = 0; f < out.num_faces; ++f) {
        Face& fc = out.faces[f];
        int32_t k = face_first[f];
        for (int i = 0; i < 3; ++i) {
            fc.n[i] = shade[k].n[i];
            fc.q[i] = tri[k].v0[i];
        }
        fc.mat = tri_mat[k];
        fc.first = acc;
        fc.count = cnt[f];
        fc.pad = 0;
        acc += cnt[f];
    }
    out.face_tris.resize(nt);
    std::vector<int32_t> fill(out.num_faces, 0);
    for (int64_t k = 0; k < nt; ++k) {
        int32_t f = out.face_of_input[k];
        out.face_tris[out.faces[f].first + fill[f]++] = new_of_old[k];
    }
    extract_wedges(V, F, nt, tri_mat, out);
    out.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return 0;
}

}  // namespace rt
