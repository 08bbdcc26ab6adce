/*
 * dr_h5.h - C ABI of the HDF5 file layer of the wire-scan reconstruction
 * (libdr_h5.so, built only where an HDF5 library is installed).
 *
 * The paper's input is a set of 2D detector images stored in HDF5, one image
 * per wire position (Sec. III-A, the HDF5 image of its figure; Sec. IV reads
 * the images from files), and its CPU side reads the files and writes the
 * results back out (Sec. III-C).  This layer reads such image sets into host
 * memory in the layout the reconstruction takes (uint16 [n_steps][ny][nx],
 * or row slabs of it), reads per-file scalars such as wire positions, and
 * writes depth-resolved images.  It has no GPU code and no dependency on
 * libdr.so: images it reads go to dr_reconstruct (host images are streamed to
 * the GPU in row slabs there).
 *
 * Reading: a file whose dataset is stored contiguously without filters is
 * read with positioned reads at the byte offset HDF5 reports, from several
 * threads at once; any other layout (chunked, compressed) goes through the
 * HDF5 library, one call at a time (the library serialises its calls).
 *
 * Errors: every entry point returns a dr_status (DR_OK or a negative code as
 * in dr.h); dr_h5_last_error() gives the calling thread's message.
 */
#ifndef DR_H5_H
#define DR_H5_H

#include <stddef.h>
#include <stdint.h>

#include "dr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dr_h5_stack_s* dr_h5_stack; /* an opened set of per-step image files */

/* Open n_files files (paths[k] holds wire step k), each with `dataset` a uint16
 * image [ny][nx] (rank 2, or rank 3 with a leading extent of 1), all of one
 * shape.  Reads only metadata; keeps copies of the paths.
 * Errors: DR_E_INVAL (NULL, n_files < 1, a file or dataset that cannot be
 * opened, a type other than unsigned 16-bit, a shape mismatch). */
dr_status dr_h5_open_stack(const char* const* paths, int32_t n_files, const char* dataset,
                           dr_h5_stack* out);

/* Shape of the stack; direct_files = how many files take the positioned-read
 * path. */
dr_status dr_h5_stack_shape(dr_h5_stack stack, int32_t* n_files, int32_t* ny, int32_t* nx,
                            int32_t* direct_files);

/* Read rows [row0, row0 + nrows) of every image into out, uint16
 * [n_files][nrows][nx] (host memory, e.g. pinned for streaming), with up to
 * nthreads threads (<= 0: 16).  Errors: DR_E_INVAL (NULL, rows outside the
 * image), DR_E_DEVICE (a read that fails or comes back short). */
dr_status dr_h5_read_rows(dr_h5_stack stack, int32_t row0, int32_t nrows, uint16_t* out,
                          int32_t nthreads);

dr_status dr_h5_close_stack(dr_h5_stack stack);

/* One numeric scalar `dataset` from each file (wire position coordinates,
 * beam-monitor counts, ...), converted to double: out[n_files]. */
dr_status dr_h5_read_scalars(const char* const* paths, int32_t n_files, const char* dataset,
                             double* out);

/* Write a stack as one file per step: paths[k] gets `dataset` = images[k]
 * (uint16 [ny][nx], little-endian), stored contiguously, or in chunks of
 * min(64, ny) rows with deflate when deflate_level is 1..9.  Files are
 * created or truncated. */
dr_status dr_h5_write_stack(const char* const* paths, int32_t n_files, const char* dataset,
                            const uint16_t* images, int32_t ny, int32_t nx, int32_t deflate_level);

/* Add a scalar dataset to each of n_files existing files: values[k] into
 * paths[k] (double). */
dr_status dr_h5_write_scalars(const char* const* paths, int32_t n_files, const char* dataset,
                              const double* values);

/* Write depth-resolved images (the reconstruction's output, float32
 * [n_bins][ny][nx]) into `path` as `dataset`, with the bin centres
 * first_center + b*width in `dataset`_depth (double [n_bins]).  The file is
 * created or truncated. */
dr_status dr_h5_write_depth_images(const char* path, const char* dataset, const float* images,
                                   int32_t n_bins, int32_t ny, int32_t nx, double first_center,
                                   double width);

/* Message of the last error on the calling thread ("" if none). */
const char* dr_h5_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DR_H5_H */
