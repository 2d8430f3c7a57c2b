"""MI355X-native GMRES-GMG solver for the dG(k) x Q_r^d/Q_{r-1} space-time slab
systems of dynamic poro-/thermoelasticity (arXiv:2303.06742, Sec. 4).

The compute path is the HIP library libstgmg.so (C ABI in include/stgmg.h);
``capi`` is its ctypes binding and ``workloads`` the seeded configurations.
"""
