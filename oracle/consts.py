"""Physical constants and conventions shared by every oracle module.

Test infrastructure: see the package docstring.
"""
C0 = 299_792_458.0            # speed of light in vacuum [m/s]
EPS0 = 8.8541878128e-12       # vacuum permittivity [F/m]
GOLDEN_U64 = 0x9E3779B97F4A7C15  # round(2^64 * (sqrt(5) - 1) / 2)
TMIN_DEFAULT = 1e-4           # minimum accepted hit distance [m]
PLANE_QUANT = 2.0 ** 30       # face grouping: normals and offsets compared after rint(x * 2^30)
OCC_EPS = 1e-9                # occlusion test: open segment parameter range (eps, 1 - eps)
INFACE_TOL = 1e-9             # image method: in-face test tolerance [m]
