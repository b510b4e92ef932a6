"""MI355X-native SNMPBB (symmetric NMF by nonmonotone projected Barzilai-Borwein).

Importing the package loads nothing native; ``paper_2606_02887_amd.snmf`` holds the
binding to the HIP library and ``paper_2606_02887_amd.gen`` the seeded workloads.
"""
