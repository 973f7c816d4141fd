"""MI355X-native three-dimensional ray-bundle lensing (Killedar et al. 2011).

``rt`` binds the HIP library (``librt.so``); ``workloads`` builds seeded
synthetic inputs.  Importing the package itself loads nothing.
"""
__version__ = "0.1.0"
