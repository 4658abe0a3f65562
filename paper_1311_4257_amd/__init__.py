"""MI355X-native directional fast multipole matvec (libdfmm + thin binding).

Import ``paper_1311_4257_amd.dfmm`` for the library binding and
``paper_1311_4257_amd.workloads`` for the seeded synthetic inputs.  This
package file imports nothing heavy on purpose.
"""
