"""AccAltProj robust PCA on AMD Instinct MI355X (gfx950).

The compute path is the HIP library `librpca.so` (see `include/rpca.h`);
`paper_1711_05519_amd.rpca` is its thin Python binding and
`paper_1711_05519_amd.inputs` draws seeded synthetic instances. Importing the
package loads nothing; the library is opened on first use of the binding.
"""
