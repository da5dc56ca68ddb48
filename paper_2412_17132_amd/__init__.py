"""MI355X-native GW+C core-level path: contour-deformation Sigma^c of core
states with the RI polarisability built on FP64 MFMA, and the cumulant
spectral function.  The compute lives in libgwc.so (HIP, gfx950); this
package is its Python binding."""
from ._native import GwcError
from .api import (gwc_evgw0, gwc_sigma_analytic, gwc_sigma_core, gwc_spectral_cumulant,
                  gwc_spectral_cumulant_noalloc, probe_peak, timing_enable, timing_get, to_device,
                  version, wac_paper_settings)

__all__ = ["GwcError", "gwc_evgw0", "gwc_sigma_analytic", "gwc_sigma_core", "gwc_spectral_cumulant",
           "gwc_spectral_cumulant_noalloc", "probe_peak", "timing_enable", "timing_get", "to_device",
           "version", "wac_paper_settings"]
