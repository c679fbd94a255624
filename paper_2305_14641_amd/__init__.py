"""Graph Quantum Clustering on MI355X (gfx950).

The HIP library (``libqc_hip.so``, C ABI in ``include/qc.h``) computes hop
distances, psi/V and Graph Gradient Descent labels; ``qc`` is its Python
binding and ``graphgen`` draws the seeded synthetic workloads.
"""
__all__ = ["qc", "graphgen", "build"]
