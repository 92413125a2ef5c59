"""Error bars of time series by binning (batch means)."""
import numpy as np


def binned_mean(x, nbins=20):
    """Mean over axis 0 and its standard error from ``nbins`` consecutive
    batches (robust to autocorrelation shorter than a batch)."""
    x = np.asarray(x, dtype=float)
    n = (x.shape[0] // nbins) * nbins
    b = x[:n].reshape((nbins, n // nbins) + x.shape[1:]).mean(axis=1)
    return b.mean(axis=0), b.std(axis=0, ddof=1) / np.sqrt(nbins)


def jackknife_binder(m2, m4, nbins=20):
    """U = 1 - <m4>/(3 <m2>^2) with a jackknife error over batches."""
    m2 = np.asarray(m2, float)
    m4 = np.asarray(m4, float)
    n = (m2.size // nbins) * nbins
    b2 = m2[:n].reshape(nbins, -1).mean(axis=1)
    b4 = m4[:n].reshape(nbins, -1).mean(axis=1)
    U = 1 - b4.mean() / (3 * b2.mean() ** 2)
    jk = np.array([1 - np.delete(b4, i).mean() / (3 * np.delete(b2, i).mean() ** 2)
                   for i in range(nbins)])
    err = np.sqrt((nbins - 1) / nbins * np.sum((jk - jk.mean()) ** 2))
    return U, err
