"""MI355X-native parallel intersection-free QEM mesh simplification.

The method is the simplification stage of PaMO (Sec. 5 of the paper): each
round computes per-vertex quadrics and per-edge costs (Eq. 1), selects the
edges that are local cost minima over their 1-ring, checks them (link
condition, flips, self-intersections against an LBVH) and commits the
survivors.  The compute path is the HIP library ``libpamo.so`` behind the C
ABI of ``include/pamo.h``; ``native`` is its ctypes binding.
"""
__all__ = ["native", "meshgen"]
