"""MI355X-native ExactSim: single-source SimRank with hand-written HIP kernels.

The compute path lives in ``libexactsim.so`` (C ABI: ``include/exactsim.h``);
``paper_2004_03493_amd.binding`` is its thin Python binding.  Importing this
package loads nothing; importing the binding loads the library and fails
loudly if it has not been built.
"""
__all__ = ["binding", "build"]
