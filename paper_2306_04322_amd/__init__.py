"""libpfspec: MI355X-native semi-implicit Fourier-spectral phase-field step.

Importing the package is cheap: the HIP library is loaded by
`paper_2306_04322_amd.pfspec` on first import of that module, and that
import fails loudly if the library has not been built.
"""

__version__ = "0.1.0"
