"""FP64 CPU oracle for the radio ray tracer of arXiv 2303.11103 (Sionna RT).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The GPU library never calls it and shares no code with it; both read
only the seeded inputs produced by ``scenegen``.

Everything here is plain and slow on purpose: brute-force intersection of every
ray with every triangle (``hitref.c``), and NumPy float64 for the physics.  Each
function cites the passage of the paper (or the textbook result the paper
relies on) it follows.  The paper gives no equations; it names the components
(Sec. II: triangle meshes, materials (eps_r, sigma) with mu_r = 1, per-
interaction transformations of the polarised field, path coefficients and
delays; Sec. II-B: Fibonacci-lattice shooting, candidate primitive sequences,
image method, duplicate removal, LOS).  The formulas implemented for those
components are the textbook ones and every convention the paper leaves open is
fixed in one place, ``oracle.consts`` and the module docstrings.

Modules
  consts    physical constants and fixed conventions
  native    loader for the brute-force C kernels in hitref.c
  fib       Fibonacci-lattice ray directions
  geom      face grouping (coplanar same-material triangles)
  em        materials, Fresnel coefficients, antenna patterns, field transfer
  sbr       shoot-and-bounce tracing and the coverage-map estimator
  image     image-method paths (exhaustive and candidate-driven)
  grad      received-power loss and central finite differences
  covgrad   coverage-map region gain and its central finite differences
  channel   channel frequency responses of paths (synthetic arrays, Doppler, OFDM)
  scatter   Lambertian diffuse scattering for coverage maps (SplitMix64 draws)
  scatpaths diffusely scattered paths (Lambertian ray-tube model)
  diffraction  first-order wedge diffraction (UTD) paths
  mlp       float64 Fourier-feature MLP with manual backward (surrogate)
"""
