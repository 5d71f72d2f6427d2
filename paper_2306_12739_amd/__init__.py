"""MI355X-native ensemble DNS of plane Couette and Poiseuille flow.

The compute path is a HIP shared library (``csrc/``) exposed through a C ABI
(``include/dns.h``); ``dns`` is its thin ctypes binding.  Importing this package
loads nothing: the library is opened on first use of ``dns``.
"""
