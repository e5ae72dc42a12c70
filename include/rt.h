/*
 * rt.h -- C ABI of the MI355X (gfx950) radio-propagation ray tracer.
 *
 * Implements the data-parallel hot path of the differentiable ray tracer of
 * Hoydis et al., "Sionna RT: Differentiable Ray Tracing for Radio Propagation
 * Modeling" (arXiv 2303.11103): shooting Fibonacci-lattice rays through a
 * triangle mesh with specular reflections (Sec. II-B), transforming the
 * polarised field at every interaction with Fresnel coefficients of materials
 * given by (eps_r, sigma), mu_r = 1 (Sec. II), accumulating coverage maps of
 * path gain (Sec. II-A, Fig. 2), finding exact specular paths with the image
 * method from candidate primitive sequences, removing duplicates and adding
 * line of sight (Sec. II-B), and returning path coefficients and delays
 * (Sec. II-A, the `a, tau` of the channel impulse response) with angles of
 * departure and arrival, plus gradients of received power with respect to
 * materials and transmitter pose (Sec. I, II; Sec. III-A and III-B).
 *
 * Conventions for every entry point
 *   - Return value: rt_status, RT_OK (0) on success, a negative code on
 *     failure; rt_last_error() returns a thread-local message for the last
 *     failure of the calling thread.  On failure no output is guaranteed to be
 *     written.
 *   - Arguments marked (host) are host pointers, read during the call only.
 *     Arguments marked (dev) are device pointers on the context's device,
 *     owned by the caller (e.g. torch tensors); the library never frees them.
 *     The library owns only the opaque handles it returns (rt_ctx, rt_scene),
 *     released by the matching *_destroy call, and its internal scratch.
 *   - All device work is enqueued on the context's HIP stream (rt_set_stream);
 *     calls return without waiting for it unless documented otherwise.
 *   - Argument errors (NaN/inf coordinates, out-of-range indices, sizes) are
 *     detected on the host before any launch and return RT_ERR_ARG.
 *   - A context is not thread safe: use one context per host thread.
 *   - Units: metres, seconds, hertz, radians, siemens per metre.
 *   - Layouts are row-major.  Float outputs are IEEE binary32 unless stated.
 */
#ifndef RT_MI355X_H
#define RT_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rt_status;
#define RT_OK            0
#define RT_ERR_ARG      -1  /* invalid argument (host-side validation) */
#define RT_ERR_CAPACITY -2  /* an output or internal table is too small; see rt_last_error */
#define RT_ERR_DEVICE   -3  /* a HIP call failed */
#define RT_ERR_OOM      -4  /* device memory allocation failed */

typedef struct rt_ctx rt_ctx;
typedef struct rt_scene rt_scene;

/* Radio material at the carrier frequency (Sec. II: relative permittivity and
 * conductivity, non-magnetic).  sigma = +INFINITY denotes a perfect electric
 * conductor (Fresnel coefficients r_perp = -1, r_par = +1). */
typedef struct {
    float eps_r;  /* relative permittivity, > 0 */
    float sigma;  /* conductivity [S/m], >= 0 or +INFINITY */
} rt_material;

/* Antenna patterns and polarisations (Sec. II, Listing 2: preconfigured
 * patterns such as the 3GPP TR 38.901 element and the dipole; single- and
 * dual-polarised antennas, "VH" and "cross").  A single-port antenna radiates
 * C_theta = g cos(zeta), C_phi = g sin(zeta) in its own frame, g the pattern's
 * amplitude and zeta the polarisation angle; a dual-polarised antenna is two
 * devices with orthogonal zeta (V and H, or +45 and -45 degrees). */
#define RT_PATTERN_ISO      0  /* isotropic, g = 1 */
#define RT_PATTERN_TR38901  1  /* TR 38.901 Table 7.3-1 element, 8 dBi, 65 deg beamwidths */
#define RT_PATTERN_DIPOLE   2  /* short dipole along the local z axis, g = sqrt(1.5) sin(theta) (1.76 dBi) */
#define RT_POL_V            0  /* zeta = 0: along theta-hat */
#define RT_POL_H            1  /* zeta = 90 degrees: along phi-hat */
#define RT_POL_SLANT_P45    2  /* zeta = +45 degrees */
#define RT_POL_SLANT_M45    3  /* zeta = -45 degrees */

/* A transmitter or receiver (Sec. II-A: position and orientation given by
 * yaw, pitch, roll; orientation R = Rz(yaw) Ry(pitch) Rx(roll), positive
 * pitch tilts the +x boresight towards -z). */
typedef struct {
    float pos[3];
    float yaw, pitch, roll;
    int32_t pattern;  /* RT_PATTERN_* */
    int32_t pol;      /* RT_POL_* */
} rt_device;

/* Tracing parameters. */
typedef struct {
    double freq_hz;           /* carrier frequency, > 0 */
    int32_t max_depth;        /* maximum number of reflections, 0..8 (0 = LOS only) */
    int32_t max_paths_per_rx; /* rt_compute_paths: path slots per (tx, rx), 1..256 */
    int64_t num_rays;         /* Fibonacci lattice size N, 1..2^40 */
    double t_min;             /* minimum accepted hit distance [m], >= 0 (1e-4 typical) */
    int64_t ray_begin;        /* trace rays ray_begin, ray_begin + ray_stride, ... < N */
    int64_t ray_stride;       /* >= 1 (1 = all rays from ray_begin) */
    int32_t cand_mode;        /* rt_compute_paths candidates: RT_CAND_ALL or RT_CAND_SPHERE */
    float sphere_kappa;       /* RT_CAND_SPHERE: reception-sphere factor kappa > 0 (2 typical) */
} rt_trace_params;

/* Candidate modes of rt_compute_paths.  RT_CAND_ALL (0): every distinct face
 * sequence found by the rays is tried for every receiver (Sec. II-B).
 * RT_CAND_SPHERE (1): a sequence is tried for a receiver only when a ray
 * segment with that sequence of reflections before it passes the receiver
 * within kappa (s + t) sqrt(4 pi / N), s being the path length before the
 * segment and t the distance along it to the closest approach (clamped to
 * [0, hit]): the ray tube of the lattice widened by kappa.  Needs max_depth
 * <= 5 and fewer than 2^24 faces. */
#define RT_CAND_ALL     0
#define RT_CAND_SPHERE  1

/* Horizontal coverage grid: cell (ix, iy) covers [x0 + ix*cell, x0 + (ix+1)*cell)
 * x [y0 + iy*cell, y0 + (iy+1)*cell) at height z; maps are stored [ny][nx]. */
typedef struct {
    double x0, y0, cell, z;
    int32_t nx, ny;
} rt_grid;

/* Scene information returned by rt_scene_info. */
typedef struct {
    int64_t num_triangles;
    int32_t num_faces;      /* coplanar same-material triangle groups */
    int32_t num_materials;
    int64_t bvh_nodes;
    int32_t bvh_depth;
    int32_t num_wedges;     /* edges that diffract (see rt_scene_wedges) */
    double build_ms;        /* host time of scene preparation + BVH build */
} rt_scene_info_t;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device` using the null stream. */
rt_status rt_create(rt_ctx** out, int32_t device);
rt_status rt_destroy(rt_ctx* ctx);
/* Enqueue all later work of this context on `hip_stream` (a hipStream_t, or
 * NULL for the null stream).  The stream must outlive its use. */
rt_status rt_set_stream(rt_ctx* ctx, void* hip_stream);
/* Block until all work enqueued by this context has finished. */
rt_status rt_synchronize(rt_ctx* ctx);
const char* rt_last_error(void);

/* ------------------------------------------------------------------ scene */

/* Build a scene from a triangle mesh (Sec. II: surfaces are triangle meshes,
 * each object has a radio material).
 *   V [nv][3] (host) float vertex positions; F [nt][3] (host) vertex indices
 *   in [0, nv); tri_mat [nt] (host) material index in [0, nm); mats [nm]
 *   (host).  Triangles with zero area are rejected (RT_ERR_ARG).
 * Prepares per-triangle records, groups coplanar same-material triangles into
 * faces (the primitives of candidate paths), builds a bounding volume
 * hierarchy on the host and uploads everything to the device (synchronous). */
rt_status rt_scene_create(rt_ctx* ctx, const float* V, int64_t nv, const int32_t* F, int64_t nt,
                          const int32_t* tri_mat, const rt_material* mats, int32_t nm, rt_scene** out);
/* Diffuse scattering (Sec. II-B lists diffuse reflections among the
 * interactions; the model here is Lambertian).  S [nm] (host) scattering
 * coefficient per material in [0, 1]: in coverage maps and rt_trace_record a
 * reflection is diffuse with probability S^2 (the scattered power fraction)
 * and the ray then leaves in a cosine-weighted direction around the normal,
 * carrying the reflected field components in that direction's transverse
 * basis; otherwise it is specular.  The draws come from the SplitMix64 stream
 * with the given seed: draw (i (max_depth + 1) + k) 3 + j for lattice ray i,
 * interaction depth k and j = 0 (diffuse or not), 1, 2 (direction);
 * rt_coverage_grad replays the same draws.  The paths of rt_compute_paths (and
 * their gradients) keep the specular share: a and T carry sqrt(1 - S^2) per
 * reflection; rt_compute_scattering returns the diffusely scattered paths.
 * RT_ERR_ARG for a count that differs from the scene's or S outside [0, 1]. */
rt_status rt_scene_set_scattering(rt_scene* scene, const float* S, int32_t nm, uint64_t seed);

/* Replace the material table (same count); no rebuild.  Synchronous. */
rt_status rt_scene_set_materials(rt_scene* scene, const rt_material* mats, int32_t nm);
rt_status rt_scene_info(const rt_scene* scene, rt_scene_info_t* out);
/* Face id per triangle, in input order: face_ids [nt] (host). */
rt_status rt_scene_face_ids(const rt_scene* scene, int32_t* face_ids);
rt_status rt_scene_destroy(rt_scene* scene);

/* ------------------------------------------------------------------ rays */

/* Fibonacci-lattice directions (Sec. II-B) of rays ray_begin + k*ray_stride,
 * k < count: dirs [count][3] (dev) float64.  Ray i of N points to
 * z = 1 - (2i+1)/N, azimuth 2 pi frac(i g) with frac(i g) computed as the
 * 64-bit product i * 0x9E3779B97F4A7C15 over 2^64. */
rt_status rt_fibonacci_directions(rt_ctx* ctx, int64_t num_rays, int64_t ray_begin, int64_t ray_stride,
                                  int64_t count, double* dirs);

/* Trace the lattice rays of one transmitter and record, per segment
 * k = 0..max_depth and traced ray j (ray index ray_begin + j*ray_stride), the
 * closest-hit triangle (input index; -1 miss, -2 ray already terminated) and
 * its distance (float64, +inf on a miss):
 *   hit_tri [max_depth+1][count] (dev) int32, hit_t [max_depth+1][count] (dev)
 *   float64, count = number of traced rays.
 * Uses the same kernels as rt_coverage_map. */
rt_status rt_trace_record(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                          int32_t* hit_tri, double* hit_t);

/* Coverage map (Sec. II-A, Fig. 2: path gain per cell of a plane).  Shoots
 * the lattice rays of one transmitter with up to max_depth specular
 * reflections and adds, for every crossing of the plane z = grid.z by a ray
 * segment, the ray-tube estimate
 *   (lambda/4pi)^2 (4pi/N) |F_rx(-d) . E|^2 / (cell^2 |d_z|)
 * to the crossed cell, where E is the ray's field (transmit pattern times the
 * reflection operators so far) and F_rx the receive pattern of rx_ant.
 *   gain [ny][nx] (dev) linear path gain, hits [ny][nx] (dev) crossings;
 *   gain_db [ny][nx] (dev, nullable) 10 log10(gain) (-inf where no hit);
 *   ray_bounces (dev, nullable) uint64 [max_depth+1]: rays that reached each
 *   depth.  The segments of depths below max_depth are closest-hit queries;
 *   a last-depth ray whose segment cannot cross the plane inside the grid is
 *   counted but dropped before that launch, and the others are searched only
 *   up to the crossing, which gives the same deposits.
 * The map is cleared first.  Sub-lattices (ray_begin, ray_stride) add only
 * their own rays with the weight of the full lattice N. */
rt_status rt_coverage_map(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                          const rt_device* rx_ant, const rt_grid* grid, float* gain, uint32_t* hits,
                          float* gain_db, uint64_t* ray_bounces);

/* Coverage maps of ntx transmitters in one call (Sec. II-A: several
 * transmitters per scene), each built as by rt_coverage_map with the same
 * parameters, receive pattern and grid:
 *   gain, hits [ntx][ny][nx] (dev); gain_db [ntx][ny][nx] (dev, nullable).
 * Stops at the first transmitter that fails validation, with that error. */
rt_status rt_coverage_maps(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx, int32_t ntx,
                           const rt_device* rx_ant, const rt_grid* grid, float* gain, uint32_t* hits, float* gain_db);

/* rt_coverage_map for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, outputs and errors as rt_coverage_map; the caller still
 * passes (and owns) every output.  The ray queues and queue counters live in
 * a fixed device array of the library (112 MiB + 64 KiB, one copy per GPU,
 * held until the process ends), so the lattice is traced in chunks of at most
 * 2^19 rays instead of 2^27; clears use fill kernels, not memsets.  Nothing is
 * allocated and no HIP events are created (rt_profile_enable does not apply).
 * Returns RT_ERR_CAPACITY if the queues for this device's launch width do not
 * fit the array.  Every call on one GPU shares that array: calls that overlap
 * on one GPU (other streams, other contexts or threads) race and must be
 * serialised by the caller. */
rt_status rt_coverage_map_noalloc(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                                  const rt_device* rx_ant, const rt_grid* grid, float* gain, uint32_t* hits,
                                  float* gain_db, uint64_t* ray_bounces);

/* rt_coverage_map that also counts, per depth k, the traced rays (at the last
 * depth without the rays dropped before it, see ray_bounces above), the BVH
 * inner nodes visited, the child boxes tested at those nodes (the node's
 * non-empty slots) and the triangles tested:
 *   work [4][max_depth+1] (dev) uint64 (rays, node visits, box tests,
 *   triangle tests).
 * The counters add atomics per ray; meant for measuring the work per
 * ray-bounce, not for production runs. */
rt_status rt_coverage_work(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                           const rt_device* rx_ant, const rt_grid* grid, float* gain, uint32_t* hits, uint64_t* work);

/* Launch timing for measurement tools: while enabled, every shoot-and-bounce
 * launch of this context is bracketed by HIP events on its stream.
 * rt_profile_read waits for the recorded launches and returns, for depths
 * k < n, the number of launches and their summed duration in milliseconds
 * (launches [n], ms [n], host), then clears the record. */
rt_status rt_profile_enable(rt_ctx* ctx, int32_t enable);
rt_status rt_profile_read(rt_ctx* ctx, int32_t n, int64_t* launches, double* ms);

/* Paths between ntx transmitters and nrx receivers (Sec. II-A
 * compute_paths; Sec. II-B): for every transmitter the lattice rays are shot
 * (max_depth reflections), the face sequence of every hit prefix becomes a
 * candidate, duplicates are removed, the image method is applied to every
 * candidate for every receiver and the line-of-sight path is added.  A path
 * is kept when its reflection points lie on their faces, on the front sides,
 * and every segment is unoccluded.  With scattering coefficients
 * (rt_scene_set_scattering) every reflection keeps its specular share
 * sqrt(1 - S^2).  Outputs, shape [ntx][nrx][P] with
 * P = max_paths_per_rx, paths of one (tx, rx) sorted by (depth, faces):
 *   a [..][2] (dev) complex coefficient (re, im) excluding exp(-j 2 pi f tau)
 *   T [..][2][2][2] (dev) 2x2 complex transfer matrix from (theta, phi) at
 *     departure to (theta, phi) at arrival (re, im)
 *   tau [..] (dev) delay [s];  aod [..][2], aoa [..][2] (dev) (theta, phi)
 *   depth [..] (dev) int32 number of reflections
 *   faces [..][max(max_depth,1)] (dev) int32 face ids (-1 padded)
 *   num_paths [ntx][nrx] (dev) int32 paths found (not truncated)
 * Unused slots get a = 0, tau = -1, depth = -1.  When some (tx, rx) has more
 * than P paths the call fails with RT_ERR_CAPACITY (message gives the
 * required P); num_paths is still written.  Synchronous (reads counters). */
rt_status rt_compute_paths(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                           int32_t ntx, const rt_device* rx, int32_t nrx, float* a, float* T, float* tau,
                           float* aod, float* aoa, int32_t* depth, int32_t* faces, int32_t* num_paths);

/* Received power per (tx, rx), incoherent over the paths (Sec. III-B
 * optimises an average received power): power [n] (dev) float64 =
 * sum over slots with depth >= 0 of |a|^2, for a [n][P][2] and depth [n][P]
 * (dev) as written by rt_compute_paths (n = ntx * nrx). */
rt_status rt_paths_power(rt_ctx* ctx, const float* a, const int32_t* depth, int64_t n, int32_t P, double* power);

/* Number of distinct candidate face sequences found by the last
 * rt_compute_paths call for its last transmitter. */
rt_status rt_last_candidate_count(rt_ctx* ctx, int64_t* count);

/* Diffusely scattered paths (Sec. II-B: diffuse reflections among the
 * interactions; Sec. II-A: scattering can be enabled for paths) with the
 * Lambertian model of rt_scene_set_scattering: for every transmitter the
 * lattice rays (num_rays, ray_begin, ray_stride, t_min of p; its
 * max_paths_per_rx and cand_mode are not used) are traced with
 * up to max_depth specular reflections, and hit k (1..max_depth) of lattice
 * ray i, at point h of a face with coefficient S > 0 (normal n facing the
 * ray, ray length s), scatters to every receiver R in front of the face
 * ((R - h) . n > 0) whose open segment h -> R is unoccluded:
 *   a = lambda/(4 pi) S w sqrt((4 pi / N) cos_s / pi) / r_s F_rx(-k) . E_s,
 * k = (R - h)/r_s, r_s = |R - h|, cos_s = k . n, E_s the reflected components
 * (r_perp a_perp, r_par a_par) of the ray's field on the transverse basis of
 * k (perp = k x n / |k x n|, par = perp x k), w the product of sqrt(1 - S^2)
 * over the earlier reflections.  Each ray stands for the solid angle 4 pi / N
 * of the full lattice, also in sub-lattices.  tau = (s + r_s)/c0; carrier
 * phase excluded, as for rt_compute_paths.  Outputs, shape [ntx][nrx][P] (dev):
 *   a [..][2], T [..][2][2][2] (a = lambda/(4 pi c0 tau) F_rx^T T F_tx in the
 *   (theta, phi) bases of departure and arrival, as for rt_compute_paths),
 *   tau [..], aod [..][2] (angles of the ray's departure), aoa [..][2]
 *   (angles of -k), depth [..] int32 k, ray [..] int64 lattice index i,
 *   faces [..][max(max_depth, 1)] int32 faces of the k hits (scattering face
 *   last, -1 padded), num_paths [ntx][nrx] int64 (not truncated).
 * Paths of a receiver are ordered by (ray, depth); unused slots get a = T = 0,
 * tau = -1, depth = -1, ray = -1.  P may exceed 256 (up to 2^40).
 * RT_ERR_CAPACITY when some receiver has more than P paths (the message gives
 * the required P; the first P are written).  No paths when no material
 * scatters.  Synchronous. */
rt_status rt_compute_scattering(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                                int32_t ntx, const rt_device* rx, int32_t nrx, int64_t P, float* a, float* T,
                                float* tau, float* aod, float* aoa, int32_t* depth, int64_t* ray, int32_t* faces,
                                int64_t* num_paths);

/* Wedges of the scene for first-order diffraction (Sec. II-B): edges shared
 * by exactly two triangles of two different faces, not on the ground (the
 * lowest z of the mesh), whose interior angle alpha between the faces'
 * half-planes (the smaller of the two: convex solids) is below pi.  Sorted by
 * (0-face, n-face, first vertex, second vertex); the 0-face is the face with
 * the smaller id.  count (host) receives the number of wedges; the first
 * min(capacity, count) records are written to out (host) [..][16] doubles:
 * first vertex a[3], unit edge direction e[3], t0[3] (unit vector in the
 * 0-face orthogonal to e, into the face), n0[3] (the 0-face normal on the
 * exterior side), length, n = 2 - alpha/pi (exterior angle n pi), 0-face id,
 * n-face id.  out may be NULL when capacity is 0. */
rt_status rt_scene_wedges(const rt_scene* scene, int32_t capacity, double* out, int32_t* count);

/* Diffraction part of a coverage map (Sec. II-A coverage maps with the
 * first-order diffraction of Sec. II-B): for every cell, the path gain
 * |a|^2 of the diffracted paths of rt_compute_diffraction from tx to the cell
 * centre (x0 + (ix + 1/2) cell, y0 + (iy + 1/2) cell, z), received with
 * rx_ant and summed over the wedges, is ADDED to gain [ny][nx] (dev, linear).
 * After rt_coverage_map it completes the map with diffraction.  These are
 * values at the cell centres; the reflected part of rt_coverage_map averages
 * over each cell.  Asynchronous on the context's stream. */
rt_status rt_coverage_diffraction(rt_ctx* ctx, rt_scene* scene, double freq_hz, const rt_device* tx,
                                  const rt_device* rx_ant, const rt_grid* grid, float* gain);

/* First-order diffraction paths (Sec. II-B: first-order diffraction; the
 * uniform theory of diffraction for a wedge, Kouyoumjian and Pathak, with the
 * Fresnel coefficients of the two faces in place of the perfect-conductor
 * signs, Luebbers): for every (tx, rx) and every wedge, the diffraction point
 * Q on the edge with equal angles of the incident and diffracted rays to the
 * edge (Keller's law), kept when Q lies inside the edge, tx and rx lie in the
 * wedge's exterior and both legs are unoccluded.  Its coefficient is
 *   a = lambda/(4 pi) F_rx(-s) . Dbar . F_tx(s') / sqrt(s' s (s' + s))
 * (carrier phase excluded, as for rt_compute_paths), with the dyadic
 * Dbar = -b' b D_s - p' p D_h of the UTD coefficients in edge-fixed unit
 * vectors, s' = |Q - tx|, s = |rx - Q|; tau = (s' + s)/c0.  Outputs, shape
 * [ntx][nrx][P] (dev), with the layouts of rt_compute_paths:
 *   a [..][2], T [..][2][2][2] (so that a = lambda/(4 pi (s + s')) F_rx^T T F_tx),
 *   tau [..], aod [..][2] (angles of s'), aoa [..][2] (angles of -s),
 *   wedge [..] int32 wedge index (rt_scene_wedges order, -1 unused),
 *   num_paths [ntx][nrx] int32 (not truncated).
 * Paths of one (tx, rx) are sorted by wedge index; unused slots get a = 0,
 * tau = -1.  RT_ERR_CAPACITY when some (tx, rx) has more than P paths (the
 * message gives the required P).  Synchronous. */
rt_status rt_compute_diffraction(rt_ctx* ctx, rt_scene* scene, double freq_hz, const rt_device* tx, int32_t ntx,
                                 const rt_device* rx, int32_t nrx, int32_t P, float* a, float* T, float* tau,
                                 float* aod, float* aoa, int32_t* wedge, int32_t* num_paths);

/* Gradient of a loss of received powers (Sec. I and III: gradients with
 * respect to material properties and transmitter orientation and position).
 * For one transmitter and the given paths (face sequences as returned by
 * rt_compute_paths, shape [nrx][P][max(max_depth,1)], with depth [nrx][P]),
 * the received power of rx r is P_r = sum_p |a_p|^2.  Given the upstream
 * adjoint dL_dP [nrx] (dev) float64, writes
 *   grad [2*nm + 5] (dev) float64 = sum_r dL_dP[r] dP_r/d(theta) for theta =
 *   (eps_r, sigma) of every material, tx x, y, z, tx yaw, tx pitch.
 * Faces and depths are the checkpoint of the forward pass: geometry and
 * fields are recomputed from them.  Enqueued, not synchronous. */
rt_status rt_paths_power_grad(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                              const rt_device* rx, int32_t nrx, int32_t P, const int32_t* depth,
                              const int32_t* faces, const double* dL_dP, double* grad);

/* Gradient of any real function L of the path coefficients: given for every
 * path slot the complex adjoint g = dL/da in the sense dL = Re(g da)
 * (coef_adj [nrx][P][2] (dev) float64), writes
 *   grad [2*nm + 5] (dev) float64 = sum over slots of Re(g da/dtheta)
 * for theta as in rt_paths_power_grad.  Only the coefficients a are
 * differentiated: the delays are held fixed, which is exact for the materials
 * (paths keep their geometry) but not for the transmitter position.  Other
 * arguments and behaviour as rt_paths_power_grad. */
rt_status rt_paths_coef_grad(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                             const rt_device* rx, int32_t nrx, int32_t P, const int32_t* depth,
                             const int32_t* faces, const double* coef_adj, double* grad);

/* ---------------------------------------------------------------- channels */

/* Channel frequency responses of paths (Sec. II-A: paths become channel
 * impulse responses, optionally with synthetic arrays, i.e. one traced
 * antenna per array with plane-wave phase shifts per element, and with
 * Doppler from device velocities; Sec. III-A: frequency responses of an OFDM
 * system).  Inputs as written by rt_compute_paths for ntx transmitters and
 * nrx receivers: a [ntx][nrx][P][2], tau, aod, aoa, depth (dev).  For time
 * step n < T (t = n / fs), receive element j, transmit element i and
 * subcarrier k < K (frequency f_k = (k - floor(K/2)) spacing_hz from the
 * carrier freq_hz):
 *   H = sum over paths of a exp(j 2 pi (-(f_c + f_k) tau + (k_t . r_i + k_r . r_j) / lambda + f_D t)),
 *   f_D = (v_tx . k_t + v_rx . k_r) / lambda,
 * with k_t the unit vector of the angles of departure, k_r that of the angles
 * of arrival (towards the arriving wave), r_i, r_j the element offsets from
 * the array centres (global frame, m).  tx_el [nt_el][3], rx_el [nr_el][3],
 * v_tx [ntx][3], v_rx [nrx][3] (m/s) are host arrays (nullable: a single
 * element at the centre, devices at rest).
 *   H [ntx][nrx][T][nr_el][nt_el][K][2] (dev) float32.
 * RT_ERR_ARG for empty dimensions, fs <= 0 with T > 1, or non-finite
 * offsets or velocities.  Enqueued after a synchronous upload of the small
 * host arrays. */
rt_status rt_paths_cfr(rt_ctx* ctx, int32_t ntx, int32_t nrx, int32_t P, const float* a, const float* tau,
                       const float* aod, const float* aoa, const int32_t* depth, double freq_hz, int32_t K,
                       double spacing_hz, int32_t nt_el, const double* tx_el, int32_t nr_el, const double* rx_el,
                       const double* v_tx, const double* v_rx, int32_t T, double fs, float* H);

/* Adjoint of rt_paths_cfr in the path coefficients: for an upstream
 * gradient G of a real loss with respect to H (G [..] (dev) float32 in H's
 * layout, dL = Re(conj(G) dH)), writes the coefficient adjoint
 *   g [ntx][nrx][P][2] (dev) float64 = sum over the (tx, rx) entries of
 *   conj(G) exp(j 2 pi phase), zero for empty slots,
 * so that dL = Re(g da) (the input of rt_paths_coef_grad).  Arguments as
 * rt_paths_cfr. */
rt_status rt_paths_cfr_adjoint(rt_ctx* ctx, int32_t ntx, int32_t nrx, int32_t P, const float* a, const float* tau,
                               const float* aod, const float* aoa, const int32_t* depth, double freq_hz, int32_t K,
                               double spacing_hz, int32_t nt_el, const double* tx_el, int32_t nr_el,
                               const double* rx_el, const double* v_tx, const double* v_rx, int32_t T, double fs,
                               const float* G, double* g);

/* Coverage-map gradient (Sec. III-B: gradient steps on a transmitter's
 * orientation; Sec. III-A: on radio materials).  For the coverage map of
 * rt_coverage_map with the same p, tx, rx_ant and grid, the path gain summed
 * over the region cells,
 *   G = sum over cells c with region[c] != 0 of gain[c]   (linear),
 * and its derivatives with respect to (eps_r, sigma) of every material and the
 * transmitter yaw and pitch.  The rays are fixed by their recorded hits
 * (hit_tri, hit_t from rt_trace_record with the same p and tx): ray geometry
 * does not depend on these parameters, and every ray is replayed in fp64 with
 * forward-mode field tangents.
 *   region [ny][nx] (dev, nullable: every cell) uint8;
 *   out [2*nm + 3] (dev) float64 = (G, dG/d eps_r_0, dG/d sigma_0, ...,
 *   dG/d yaw, dG/d pitch), cleared first.
 * RT_ERR_ARG for more than 4 materials.  Enqueued, not synchronous. */
rt_status rt_coverage_grad(rt_ctx* ctx, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                           const rt_device* rx_ant, const rt_grid* grid, const uint8_t* region,
                           const int32_t* hit_tri, const double* hit_t, double* out);

/* ------------------------------------------------------------------ surrogate */

/* Learned coverage-map surrogate (the paper motivates neural propagation
 * models, Sec. I, and closes Sec. III-A with learning as a calibration
 * tool; it specifies no network).  Function: inputs v = (tx x, y, z, cell
 * x, y), normalised as (v - in_center) / in_half; Fourier features
 * [sin 2 pi B v, cos 2 pi B v] with B (64 x 5) drawn N(0, s^2), s =
 * ff_scale on the transmitter columns and ff_scale_cell on the cell columns
 * (or structured, see ff_rows_tx);
 * 4 hidden layers of 256 with the tanh-form GELU; linear head.  The output
 * (path gain in dB) is the head plus, when prior_freq_hz > 0, the free-space
 * gain of the link, 20 log10(c0 / (4 pi f d)) with d the distance from the
 * transmitter to (cell x, cell y, prior_rx_z) (the Friis gain of an
 * isotropic pair, Sec. II-A); the network then learns the residual.
 * Parameters (fp32, rt_mlp_param_count() of them):
 * W1[256][128] b1[256] W2[256][256] b2 W3 b3 W4 b4 w5[256] b5[1].
 * Matrix products run on bf16 MFMA with fp32 accumulation; training uses
 * Adam (beta 0.9/0.999, eps 1e-8) on fp32 master weights and the masked
 * mean squared error sum m (y - t)^2 / sum m. */
typedef struct rt_mlp rt_mlp;
typedef struct {
    int32_t batch;        /* rows per call: multiple of 1024 (scratch is sized for it) */
    float ff_scale;       /* std of the Fourier entries on the transmitter inputs (x, y, z) */
    uint64_t seed;        /* initialisation seed */
    float in_center[5];
    float in_half[5];
    float ff_scale_cell;  /* std of the Fourier entries on the cell inputs (x, y); 0 = ff_scale */
    float prior_rx_z;     /* receiver height of the free-space prior [m] */
    double prior_freq_hz; /* carrier of the free-space prior [Hz]; 0 = no prior */
    /* Structured B (used when ff_rows_tx + ff_rows_rel > 0): the first ff_rows_tx
     * rows see the transmitter only (std ff_scale), the last ff_rows_rel rows the
     * cell relative to the transmitter in x, y (std ff_scale_rel, entries b and -b
     * on the cell and transmitter columns) and the transmitter height (std
     * ff_scale), the rows between the cell only (std ff_scale_cell). */
    int32_t ff_rows_tx;
    int32_t ff_rows_rel;
    float ff_scale_rel;
    int32_t reserved;     /* 0 */
} rt_mlp_config;

rt_status rt_mlp_param_count(int64_t* n);
/* Allocate and initialise (weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)),
 * biases 0). */
rt_status rt_mlp_create(rt_ctx* ctx, const rt_mlp_config* cfg, rt_mlp** out);
rt_status rt_mlp_destroy(rt_mlp* mlp);
/* Copy parameters [P] and Fourier matrix [64][5] (dev) out of / into the
 * handle; set also clears the Adam moments. */
rt_status rt_mlp_get_params(rt_mlp* mlp, float* params, float* ff);
rt_status rt_mlp_set_params(rt_mlp* mlp, const float* params, const float* ff);
/* Predictions y [n] (dev) for inputs v [n][5] (dev); n a multiple of 128,
 * at most batch. */
rt_status rt_mlp_forward(rt_mlp* mlp, const float* v, int64_t n, float* y);
/* Gradient of the masked MSE (targets t [n], mask m [n] in {0, 1}, dev):
 * grad [P] (dev); loss (dev, nullable) [1]. */
rt_status rt_mlp_grad(rt_mlp* mlp, const float* v, const float* t, const float* m, int64_t n, float* grad,
                      float* loss);
/* One Adam step with learning rate lr on the batch; loss (dev, nullable). */
rt_status rt_mlp_train_step(rt_mlp* mlp, const float* v, const float* t, const float* m, int64_t n, float lr,
                            float* loss);
/* Positions i < n (ascending) with mask[i] != 0 of a byte mask (dev, n <
 * 2^32) into index (dev, uint32, capacity entries); *count (host) receives
 * the number of such positions.  RT_ERR_CAPACITY (and nothing written) when
 * it exceeds capacity.  Synchronises the context's stream. */
rt_status rt_mlp_valid_index(rt_mlp* mlp, const uint8_t* mask, int64_t n, uint32_t* index, int64_t capacity,
                             int64_t* count);
/* Draw n training rows from a stack of T coverage maps (dev): maps [T][ny][nx]
 * in dB, tx [T][3], and the usable cells as flat positions into maps (index
 * [count], from rt_mlp_valid_index over the cell mask); row i takes index
 * entry (h mod count), h a counter-based hash of (seed, step, i).  Writes v
 * [n][5], t [n] and m [n] = 1 (dev). */
rt_status rt_mlp_sample_batch(rt_mlp* mlp, const float* maps, const uint32_t* index, int64_t count, const float* tx,
                              int32_t T, const rt_grid* grid, uint64_t seed, uint64_t step, float* v, float* t,
                              float* m, int64_t n);
/* Predicted maps [T][ny][nx] (dev, dB) for transmitters tx [T][3] (dev) on the
 * grid's cell centres.  RT_ERR_ARG for an empty stack or one of 2^40 cells or
 * more. */
rt_status rt_mlp_predict_maps(rt_mlp* mlp, const float* tx, int32_t T, const rt_grid* grid, float* maps);
/* Surrogate maps with the ray tracer as fallback: the predicted maps [T][ny][nx]
 * (dev, dB) of rt_mlp_predict_maps for the positions of tx [T] (host), then,
 * when any cell is marked, every transmitter's coverage map by the ray tracer
 * (rt_coverage_map with p, tx[k], rx_ant and the grid), whose dB values replace
 * the prediction in the cells with fallback [ny][nx] (dev, uint8) != 0 (-inf
 * where no ray crossed the cell).  fallback_cells (host, nullable) receives the
 * number of marked cells.  The scene must belong to the surrogate's context.
 * Grows per-handle scratch (positions and one map) as needed; synchronous. */
rt_status rt_mlp_predict_maps_fallback(rt_mlp* mlp, rt_scene* scene, const rt_trace_params* p, const rt_device* tx,
                                       int32_t T, const rt_device* rx_ant, const rt_grid* grid,
                                       const uint8_t* fallback, float* maps, int64_t* fallback_cells);

#ifdef __cplusplus
}
#endif

#endif /* RT_MI355X_H */
