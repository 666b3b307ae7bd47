"""MI355X-native limited CG-WENO stage (arXiv:2509.04673).

The HIP library is loaded lazily by ``paper_2509_04673_amd.cem`` on first
use; importing the package itself touches no GPU code.
"""
