// Launch interface between the C ABI (api.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"
#include "layout.h"

namespace rt {

// State of one live ray between two bounces (96 bytes, read/written coalesced
// by consecutive lanes).
struct alignas(16) RayState {
    double o[3];    // origin (fp64)
    double d[3];    // unit direction (fp64)
    float E[6];     // field, complex Cartesian (re, im) per axis
    int32_t excl;   // face of the last reflection (-1 at the transmitter)
    int32_t prefix; // candidate-table slot of the face sequence so far (-1 none);
                    // reception-sphere mode: path length so far (float bits)
    int32_t ray;    // lattice position j: ray index = begin + j * stride;
    int32_t pad[3]; // reception-sphere mode: ray, pad = the face sequence, 24 bits per face
};
static_assert(sizeof(RayState) == 96, "ray state size");

constexpr uint64_t kEmptyKey = ~0ull;
constexpr int kQueueRegions = 64;
// The region counters sit 64 bytes apart: every wave's append is a
// device-scope atomic performed past the L2, and counters that share a line
// contend with each other.
constexpr int kCounterStride = 16;  // 32-bit words between two region counters

struct DevScene {
    const Node* nodes;
    const Tri* tris;
    const Shade* shades;
    const Face* faces;
    const int32_t* face_tris;
    int32_t num_faces;
    int32_t nt;
    int32_t num_nodes;
    int32_t stack_need;  // worst-case traversal stack entries of the tree
    const int32_t* leaf_of_input;  // [nt] leaf-order index of each input triangle
    const Wedge* wedges;           // [num_wedges] diffraction wedges
    int32_t num_wedges;
};

struct SbrArgs {
    DevScene sc;
    int64_t num_rays;   // lattice size N
    int64_t begin, stride;
    int64_t count;      // traced rays (positions 0..count-1)
    int64_t pos0, chunk; // positions handled by this launch sequence: [pos0, pos0 + chunk)
    int64_t perm_f, perm_g;  // band permutation (Fibonacci numbers F_m, F_{m-1}); 0 = identity
    int64_t perm_full;       // positions below this are permuted (whole bands)
    double perm_inv;         // 1 / F_m
    double tmin;
    uint64_t scat_seed;  // SplitMix64 seed of the diffuse-scattering draws
    double tx[3];
    Antenna tx_ant, rx_ant;
    // coverage
    double gx0, gy0, gcell, gz;
    int32_t gnx, gny;
    float wscale;       // (lambda/4pi)^2 (4pi/N) / cell^2
    float* gain;
    uint32_t* hits;
    // queues
    int32_t depth, max_depth;
    // The queues are split into kQueueRegions regions of region_cap rays; a
    // wave appends its survivors to region (wave % kQueueRegions) through
    // that region's counter, which spreads the queue atomics over 64 addresses.
    const RayState* in;
    // [kQueueRegions * kCounterStride]: word 0 of a region counts its rays, word 1
    // the rays its waves dropped before a last bounce (they add to the depth's count)
    const uint32_t* in_count;
    RayState* out;
    uint32_t* out_count;        // [kQueueRegions * kCounterStride]
    int64_t region_cap;
    uint64_t* stats;    // [max_depth + 1] traced rays per depth (nullable)
    uint64_t* work;     // stats mode: [4][max_depth + 1] rays, inner-node visits, child-box tests, triangle tests
    // record mode
    int32_t* rec_tri;
    double* rec_t;
    // candidate mode
    uint64_t* table;
    uint64_t table_mask;
    uint32_t* overflow;
    // reception-sphere mode: receivers binned on an xy grid (each receiver in
    // every cell within r_ins of it, CSR lists), the heights they span widened
    // by r_ins, and the set of (receiver, prefix slot) pairs
    const double* rx;            // [nrx][3]
    const int32_t* cell_start;   // [rnx * rny + 1]
    const int32_t* cell_rx;
    double rgx0, rgy0, rgcell;
    int32_t rgnx, rgny;
    double rz_lo, rz_hi;
    double sphere_k;             // kappa sqrt(4 pi / N): sphere radius per metre of path
    uint64_t* pairs;
    uint64_t pairs_mask;
    uint32_t* pairs_overflow;
};

// kModeSphere: rays carry their face sequence and path length; segments after
// the first reflection record (receiver, sequence) pairs within the spheres.
enum : int { kModeCoverage = 1, kModeRecord = 2, kModeCandidates = 4, kModeStats = 8, kModeSphere = 16 };
constexpr int kSphereMaxDepth = 5;       // faces packed 24 bits each into 128 bits
constexpr int32_t kSphereMaxFaces = 1 << 24;

// Rays one queue region must hold for a bounce launch of `grid` blocks over
// at most `chunk` rays: the waves of a region (every kQueueRegions-th) times
// their grid-stride iterations times 64 lanes.
int64_t sbr_region_capacity(int64_t chunk, int grid);
hipError_t launch_sbr_bounce(const SbrArgs& a, const MatTable& mats, int mode, int grid, hipStream_t s);
hipError_t launch_fib_dirs(int64_t N, int64_t begin, int64_t stride, int64_t count, double* out, hipStream_t s);
hipError_t launch_finalize_db(const float* gain, float* db, int64_t n, hipStream_t s);
// p[0 .. n) = v (32-bit words), as a kernel (usable inside captured graphs).
hipError_t launch_fill_u32(void* p, uint32_t v, size_t n, hipStream_t s);

// ---------------------------------------------------------------- paths
struct Cand {
    int32_t depth;
    int32_t faces[8];
};

struct PathArgs {
    DevScene sc;
    double freq, lambda;
    double tx[3];
    Antenna tx_ant;
    const double* rx;        // [nrx][3]
    const Antenna* rx_ant;   // [nrx]
    int32_t nrx;
    const Cand* cands;
    const uint32_t* ncand;   // device count
    const int32_t* pair_rx;  // reception-sphere mode: receiver of candidate j (null: every receiver)
    int32_t max_depth;
    int32_t P;               // slots per rx
    uint32_t* counts;        // [nrx] paths found
    // unsorted path records
    float* a;      // [nrx][P][2]
    float* T;      // [nrx][P][8]
    float* tau;    // [nrx][P]
    float* aod;    // [nrx][P][2]
    float* aoa;    // [nrx][P][2]
    int32_t* depth;   // [nrx][P]
    int32_t* faces;   // [nrx][P][FD]
    int32_t fd;       // faces stride = max(max_depth, 1)
};

hipError_t launch_paths_power(const float* a, const int32_t* depth, int64_t n, int P, double* power, hipStream_t s);
hipError_t launch_extract_pairs(const uint64_t* pairs, uint64_t pairs_cap, const uint64_t* table, Cand* out,
                                int32_t* out_rx, uint32_t* count, uint32_t max_out, hipStream_t s);
hipError_t launch_extract_candidates(const uint64_t* table, uint64_t cap, int32_t max_depth, Cand* out,
                                     uint32_t* count, uint32_t max_out, hipStream_t s);
hipError_t launch_image_paths(const PathArgs& a, const MatTable& mats, int64_t max_items, hipStream_t s);
// First-order diffraction: one thread per (receiver, wedge) writes the valid
// paths into the unsorted records of a (depth = 1, faces[0] = wedge id, fd = 1).
hipError_t launch_diffraction_paths(const PathArgs& a, const MatTable& mats, hipStream_t s);
// Diffraction part of a coverage map: gain[c] += sum over wedges of |a|^2 of the
// diffracted path from tx to the centre of cell c (one thread per cell).
hipError_t launch_coverage_diffraction(const DevScene& sc, const MatTable& mats, double lambda, const double* tx,
                                      const Antenna& txa, const Antenna& rxa, double gx0, double gy0, double gcell,
                                      double gz, int32_t gnx, int32_t gny, float* gain, hipStream_t s);
hipError_t launch_sort_paths(const PathArgs& a, int32_t nrx, float* a_out, float* T_out, float* tau_out,
                             float* aod_out, float* aoa_out, int32_t* depth_out, int32_t* faces_out,
                             int32_t* num_paths_out, hipStream_t s);

// Diffusely scattered paths: scattering points of a chunk of lattice rays,
// [ray][depth] (128 bytes).
struct alignas(16) ScatPoint {
    double p[3];    // the hit point
    double n[3];    // unit normal facing the incident ray
    double g[8];    // 2x2 complex G: (perp, par) from departure (theta, phi), times S w r_{perp,par}
    double s;       // ray length from the transmitter
    int32_t face;   // face of the hit (-1: no hit at this depth)
    int32_t scat;   // 1 when the hit scatters (S > 0)
};
static_assert(sizeof(ScatPoint) == 128, "scattering point size");

struct ScatArgs {
    DevScene sc;
    int64_t num_rays, begin, stride;
    int64_t pos0, n;          // lattice positions [pos0, pos0 + n) of this chunk
    int32_t max_depth, nrx;
    double tmin, lambda;
    double tx[3];
    Antenna tx_ant;
    const double* rx;         // [nrx][3]
    const Antenna* rx_ant;    // [nrx]
    ScatPoint* points;        // [n][max_depth]
    int64_t nrec_pad;         // n * max_depth rounded up to a multiple of 64
    uint64_t* masks;          // [nrx][nrec_pad / 64] visibility bits
    uint32_t* prefix;         // [nrx][nrec_pad / 64] visible records before each word (this chunk)
    int64_t* chunk_total;     // [nrx]
    int64_t* base;            // [nrx] paths of the earlier chunks (after the last chunk: the counts)
    int64_t P;                // slots per receiver
    float* a;                 // [nrx][P][2]
    float* T;                 // [nrx][P][8]
    float* tau;               // [nrx][P]
    float* aod;               // [nrx][P][2]
    float* aoa;               // [nrx][P][2]
    int32_t* depth;           // [nrx][P]
    int64_t* ray;             // [nrx][P]
    int32_t* faces;           // [nrx][P][fd]
    int32_t fd;               // max_depth
};
// Points, visibility, scan and write passes of one chunk; base must hold the
// counts of the earlier chunks (zero before the first).
hipError_t launch_scatter_chunk(const ScatArgs& a, const MatTable& mats, hipStream_t s);
// Empty-slot values for the slots at or after every receiver's final count.
hipError_t launch_scatter_tail(const ScatArgs& a, hipStream_t s);

struct GradArgs {
    DevScene sc;
    double freq, lambda;
    double tx[3];
    double yaw, pitch, roll;
    int32_t tx_pattern, tx_pol;
    const double* rx;
    const Antenna* rx_ant;
    int32_t nrx, P, fd;
    const int32_t* depth;   // [nrx][P]
    const int32_t* faces;   // [nrx][P][fd]
    const double* dL_dP;    // [nrx] (used when coef_adj is null)
    const double* coef_adj; // [nrx][P][2] complex adjoint g of each path's coefficient (nullable)
    double* grad;           // [2 nm + 5]
    int32_t nm;
};
hipError_t launch_power_grad(const GradArgs& a, const MatTable& mats, hipStream_t s);

// Channel frequency responses of paths (synthetic arrays, Doppler, OFDM).
struct CfrArgs {
    int64_t npairs;           // ntx * nrx
    int32_t nrx, P;
    const float* a;           // [npairs][P][2]
    const float* tau;         // [npairs][P]
    const float* aod;         // [npairs][P][2] (theta, phi)
    const float* aoa;
    const int32_t* depth;     // [npairs][P], < 0 for an empty slot
    double freq, lambda, spacing, fs;
    int32_t K, T, nt_el, nr_el;
    const double* tx_el;      // [nt_el][3] element offsets [m] (dev)
    const double* rx_el;      // [nr_el][3]
    const double* v_tx;       // [ntx][3] velocities [m/s] (dev)
    const double* v_rx;       // [nrx][3]
    float* H;                 // [npairs][T][nr_el][nt_el][K][2]
    int64_t total;            // entries of H
};
hipError_t launch_cfr(const CfrArgs& c, hipStream_t s);
hipError_t launch_cfr_adjoint(const CfrArgs& c, const float* G, double* g, hipStream_t s);

// Coverage-map gradient: replay of recorded rays with field tangents.
constexpr int kCovMaxMat = 4;                 // materials with tangents
constexpr int kCovT = 2 * kCovMaxMat + 2;     // (eps_r, sigma) per material, yaw, pitch
struct CovGradArgs {
    DevScene sc;
    int64_t num_rays, begin, stride, count;
    int32_t max_depth;
    int32_t nm;
    double tx[3];
    double yaw, pitch, roll;
    int32_t tx_pattern, tx_pol;
    int32_t gnx, gny;
    Antenna rx_ant;
    double gx0, gy0, gcell, gz;
    double wscale;            // (lambda/4pi)^2 (4pi/N) / cell^2
    double omega;             // 2 pi f
    uint64_t scat_seed;       // draws of diffuse scattering (as in the forward kernel)
    const uint8_t* region;    // [gny][gnx] (nullable: every cell)
    const int32_t* hit_tri;   // [max_depth+1][count] input triangle ids (-1 miss, -2 terminated)
    const double* hit_t;      // [max_depth+1][count]
    double* out;              // [2 nm + 3]: region sum, d/d(eps_r, sigma) per material, d/d yaw, d/d pitch
};
hipError_t launch_coverage_grad(const CovGradArgs& a, const MatTable& mats, int grid, hipStream_t s);

}  // namespace rt
