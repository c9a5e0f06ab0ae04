"""MI355X-native local-ROI regularised tomography (arXiv 1604.02292).

The compute path is the HIP library libtomo.so (C ABI in include/tomo.h);
`tomo.Context` is its thin Python binding.
"""

from .tomo import Context, TomoError, make_params  # noqa: F401
from ._lib import (roi_params, tomo_rect, ROI_TV_NONNEG_CP, ROI_NONNEG_SIRT,  # noqa: F401
                   ROI_LOCAL_SIRT, ROI_LOCAL_FISTA_TV, ROI_LOCAL_FISTA_HAAR, ROI_FLAG_HALF_DATA, ROI_FLAG_ANISO_TV,
                   ROI_FLAG_BOX, ROI_FLAG_NO_MOMENTUM, ROI_FLAG_PIXEL_UNITS)
