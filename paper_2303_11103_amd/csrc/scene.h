// Host scene preparation (see scene.cpp).
#pragma once
#include <string>
#include <vector>

#include "layout.h"

namespace rt {

struct HostScene {
    std::vector<Node> nodes;          // BVH, root at 0
    std::vector<Tri> tris;            // leaf order
    std::vector<Shade> shades;        // leaf order
    std::vector<Face> faces;
    std::vector<int32_t> face_tris;   // per face, its triangles (leaf-order indices)
    std::vector<int32_t> face_of_input;
    std::vector<Wedge> wedges;        // diffraction wedges, sorted by (face0, facen, a, end vertex)
    int32_t num_faces = 0;
    int depth = 0;                    // depth of the binary build tree
    int stack_need = 0;               // worst-case traversal stack entries of the 4-wide tree
    int depth_bound = 0;              // depth bound the accepted binary tree was built with
    bool collapse_by_height = false;  // 4-wide nodes formed by opening the tallest child (else the largest)
    double max_abs = 0.0;             // largest |coordinate| (at least 64 m)
    double pad = 0.0;                 // bounding-box inflation [m]
    double build_ms = 0.0;
};

// Validates the mesh, prepares triangle/shade/face records and builds the
// BVH.  Returns 0 on success, -1 with a message in err.
int build_scene(const float* V, int64_t nv, const int32_t* F, int64_t nt, const int32_t* tri_mat, int32_t nm,
                HostScene& out, std::string& err);

}  // namespace rt
