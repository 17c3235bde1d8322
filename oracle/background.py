"""Background-tile test before reconstruction (Sec. 3.2, slide reconstruction
time): a patch whose low-resolution images show an intensity variance under a
threshold is treated as empty glass and not reconstructed.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading taken (the paper names the criterion but not the statistic's exact
form or the threshold): the statistic of a tile is the mean, over its
NA-matched images, of each image's population variance over its N x N pixels
divided by the square of that image's mean.  Dividing by the squared mean makes
it independent of LED brightness and exposure; the NA-matched images are the
ones whose contrast shows the sample.  A tile is background when the statistic
is below a caller-chosen threshold.
"""

import numpy as np


def relative_variance(img):
    """var(I) / mean(I)^2 of one image, population variance (divide by the
    pixel count), in float64."""
    x = np.asarray(img, dtype=np.float64)
    m = x.mean()
    return float(np.mean((x - m) ** 2) / (m * m))


def background_stat(images, n_bf):
    """Statistic of one tile: ``images`` is its (n_bf + n_df, N, N) stack,
    NA-matched first; returns the mean of relative_variance over the first
    n_bf images."""
    return float(np.mean([relative_variance(images[i]) for i in range(n_bf)]))


def is_background(images, n_bf, threshold):
    """True when the tile's statistic is below ``threshold``."""
    return background_stat(images, n_bf) < threshold
