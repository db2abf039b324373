"""MI355X-native coupled lattice-Boltzmann / immersed-boundary time step (LBIBCell method).

The compute path is the HIP library ``liblbib.so`` (C ABI in ``include/lbib.h``);
``paper_1503_06726_amd.lbib`` is its thin ctypes binding and
``paper_1503_06726_amd.workloads`` builds seeded synthetic inputs.  Importing this
package loads nothing.
"""
