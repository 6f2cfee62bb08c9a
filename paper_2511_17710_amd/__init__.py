"""MI355X-native particle step (interpolate, rotate, Boris push, zig-zag
deposit, per-cell sort, adjoint) of the special-relativistic curvilinear PIC
method of Entity paper I (arXiv 2511.17710).

The HIP library is loaded lazily by ``paper_2511_17710_amd.picstep``; the
input generators in ``workloads`` need only numpy.
"""
