/*
 * arts.h -- C ABI of the MI355X (gfx950) single-pulse search library, libarts.so.
 *
 * The library implements the data-parallel hot path of the Apertif Radio Transient System's
 * real-time search (van Leeuwen et al., arXiv:2205.12362, Sect. 6b.2 "AMBER"): synthesized-beam
 * formation from tied-array beams, brute-force incoherent dedispersion over DM trials,
 * optional time downsampling, boxcar matched filtering, S/N normalisation and threshold
 * candidate extraction.
 *
 * Conventions shared by every entry point:
 *  - Filterbank data are uint8 Stokes-I samples, channel-major with time fastest, i.e. a beam is
 *    [nchan][nsamp] and a set of beams is [nbeam][nchan][nsamp] contiguous (the TABF re-orders
 *    its output so that time is the fastest index, Appendix "Data loads"; samples are 8 bit,
 *    Appendix "Requantization in the TABF").
 *  - Every data pointer is DEVICE memory owned by the caller (e.g. a torch tensor's data_ptr());
 *    the library never frees it.  A plan owns only its own tables and workspace.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are asynchronous on it unless
 *    stated otherwise; the caller must keep buffers alive until the stream has passed them.
 *  - Return value: ARTS_OK (0) or a negative status; arts_strerror() names it and
 *    arts_last_error() gives the message of the last failure on the calling thread.  No C++
 *    exception and no abort crosses this boundary.
 *  - Integer results (delays, dedispersed series, boxcar sums, candidate positions) are exact.
 */
#ifndef ARTS_H
#define ARTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum arts_status {
  ARTS_OK = 0,
  ARTS_E_INVAL = -1,    /* an argument is out of range or inconsistent                       */
  ARTS_E_SHAPE = -2,    /* input shorter than the plan's halo (no complete output sample)    */
  ARTS_E_NOMEM = -3,    /* a device or host allocation failed                                */
  ARTS_E_DEVICE = -4,   /* a HIP runtime call or kernel launch failed                        */
  ARTS_E_CAPACITY = -5, /* candidate buffer too small; *count holds the number required      */
  ARTS_E_BUDGET = -6,   /* admission refused: the request does not fit the HBM budget        */
  ARTS_E_STATE = -7     /* call not valid in the object's current state                      */
};

typedef struct arts_plan_s* arts_plan_t;

/* One threshold candidate (32 bytes).  The paper's real-time candidates carry beam number,
 * downsampling factor, arrival time, width, DM and S/N (Sect. 6b.1, "Real-time analysis").
 *   sample     : start of the boxcar window, in (downsampled) samples, plus the caller's t_offset
 *   beam       : beam (or synthesized beam) index within the call, plus the caller's beam_offset
 *   dm_index   : index into the plan's DM list;  dm: that DM (pc cm^-3) as float
 *   width      : boxcar width in (downsampled) samples;  downsample: the plan's factor D
 *   snr        : (B_w - w mu) / (sigma sqrt(w)), FP32, see arts_boxcar_snr                   */
typedef struct arts_candidate {
  int64_t sample;
  int32_t beam;
  int32_t dm_index;
  int32_t width;
  int32_t downsample;
  float snr;
  float dm;
} arts_candidate;

/* --------------------------------------------------------------------- RFI mitigation ---- */

/* RFI mitigation of filterbank rows, in place (Sect. 6b.2 "RFI mitigation", optional in the
 * paper: one filter for bright wide-band low-DM RFI and one for narrow-band RFI; Sect. 9 on the
 * data lost to RFI: a time-domain and a frequency-domain method, each applied three times, every
 * pass to the data the previous one cleaned, on local statistics).  Readings taken here:
 *  - time domain, per row [nchan][nsamp]: the zero-DM series z(t) = sum_c x[c][t]; in each
 *    iteration the samples with z(t) > floor(mean + k_time sigma) (population statistics of z
 *    over the rows' nsamp samples) are replaced, in every channel, by that channel's mean over
 *    the other samples, rounded half to even.  A dispersed burst is spread out in z and stays;
 *  - frequency domain, per spectrum (one row, one sample): channels with
 *    x[c] > floor(mean + k_freq sigma) over the spectrum are replaced by the mean of the other
 *    channels, rounded half to even;
 *  - the time domain runs first; an iteration that flags nothing ends its filter.
 * The cuts floor(mean + k sigma) are exact: integer tests on the exact sums (an integer u is
 * above mean + k sigma when D = n u - sum > 0 and D^2 > k^2 (n sum_sq - sum^2)).
 * data: device uint8 [nrow][nchan] rows of `pitch` bytes, of which the first nsamp are used
 * (e.g. the TABs of one chunk); nsamp * nchan <= 2^32.  k_time, k_freq: thresholds in standard
 * deviations, 0 or within [2^-6, 1024].  niter_time, niter_freq: iterations (the paper: 3; 0
 * turns a filter off).  nchan <= 4096 when niter_freq > 0.  Allocates a device workspace of about
 * nrow * (8 nsamp + 12 nchan) bytes for the call; SYNCHRONISES stream.  Errors: ARTS_E_INVAL,
 * ARTS_E_NOMEM, ARTS_E_DEVICE.                                                               */
int arts_rfi_clean(uint8_t* data, int32_t nrow, int32_t nchan, int64_t nsamp, int64_t pitch,
                   float k_time, int32_t niter_time, float k_freq, int32_t niter_freq,
                   void* stream);

/* ------------------------------------------------------------------------------ plans ---- */

/* Host only (no device call): the plan's delay table.
 * Dedispersion shifts each channel by the delay of the trial DM (Sect. 6b.2, "Dedispersion").
 * Channel c has centre frequency f_c = f_lo_mhz + c * df_mhz; the reference is the highest
 * f_c.  delay[d][c] = round_half_even( 4.148808e3 * dm[d] * (1/f_c^2 - 1/f_ref^2)
 *                                      / (downsample * tsamp_s) )   in FP64.
 * delays_out: host int32 [ndm][nchan].  tie_margin_out (nullable): smallest distance of any
 * unrounded delay from a rounding tie, so callers can confirm the table is well defined.
 * Errors: ARTS_E_INVAL for nchan < 1, df == 0, tsamp <= 0, downsample < 1, ndm < 1, a DM
 * that is negative or not finite, a channel frequency <= 0, or a delay above 2^30.          */
int arts_delay_table(int32_t nchan, double f_lo_mhz, double df_mhz, double tsamp_s,
                     const double* dm_list, int32_t ndm, int32_t downsample,
                     int32_t* delays_out, double* tie_margin_out);

/* Host only (no device call): the SB table from the beam model (Appendix "Synthesized Beams"):
 * table_out[s][c] = the TAB row whose grating response covers SB s in channel c.
 *  - SB s has index n_SB = s - (nsb - 1) / 2 (0 is the centre of the compound beam).  At f_max
 *    it takes TAB n_TAB = n_SB mod ntab (minus ntab if above ntab/2 - 1) of grating order n_gr,
 *    n_SB = n_gr ntab + n_TAB (the paper's "rounding upward" of n_SB / ntab is read as the
 *    rounding that keeps this identity).
 *  - Going down in frequency it switches to TAB n_TAB - k sgn(n_SB) below the k-th switch
 *    frequency f_sw,k = (1 - b) f_{k-1} + b f_k, where f_0 = f_max and
 *    f_k = f_max (n_gr B_max + (n_TAB - k sgn) alpha B_cq) / (n_gr B_max + n_TAB alpha B_cq)
 *    (the paper's equation for f0 applied to the k-th neighbour, with the TAB separation in its
 *    second term as in the substitution that follows it); b = 1/2 for SBs one beam width apart
 *    (quarter = 0, the 71 SBs of ARTS), and for half a beam width (quarter = 1, 151 SBs)
 *    b = 1/4 for even n_SB and 3/4 for odd.  64 neighbours are followed.
 *  - A TAB index outside [-ntab/2, ntab/2 - 1] is the same TAB one grating order over and is
 *    wrapped into that range; TAB n is row n + ntab/2 of the TAB input.
 * Channel c is at f_lo + c df MHz.  ARTS: ntab = 12, alpha = 0.80, B_max = 1296 m, B_cq = 144 m,
 * f_max = 1500 MHz.  table_out: host uint8 [nsb][nchan].  margin_out (nullable): the smallest
 * distance (MHz) of a channel frequency from a switch frequency it was compared with.
 * Errors: ARTS_E_INVAL (odd or out-of-range ntab, non-positive model constants, a channel
 * frequency <= 0, NULL table).                                                             */
int arts_sb_table_beam_model(int32_t nsb, int32_t ntab, int32_t nchan, double f_lo_mhz,
                             double df_mhz, double f_max_mhz, double alpha, double b_max_m,
                             double b_cq_m, int32_t quarter, uint8_t* table_out,
                             double* margin_out);

/* Create a search plan on the current HIP device: validates the arguments (as above; widths
 * must be strictly increasing and >= 1), computes the FP64 delay table, and uploads it with the
 * tiling tables of the dedispersion kernel.  dm_list [ndm] and widths [nwidth] are host arrays,
 * copied.  The boxcar widths are the integration trials (Sect. 6b.2, "Integration").
 * *out receives the plan; destroy it with arts_plan_destroy.  Errors: ARTS_E_INVAL,
 * ARTS_E_NOMEM, ARTS_E_DEVICE.                                                              */
int arts_plan_create(int32_t nchan, double f_lo_mhz, double df_mhz, double tsamp_s,
                     const double* dm_list, int32_t ndm, const int32_t* widths, int32_t nwidth,
                     arts_plan_t* out);

/* Two-step subband dedispersion (Sect. 6b.2 "Dedispersion": the module can dedisperse in two
 * steps with subbanding; the subband dedispersion figure: subbands of 48 channels first
 * dedispersed to a coarse DM, then aligned over 32 fine trials; Table "dedispersion setup":
 * fine DM steps 0.2 / 2.5 with subbanding DM steps 6.4 / 40, 32 subbands).  The plan searches
 * the fine trials dm_first + k dm_step, k < ndm, in nsub subbands of nchan / nsub channels:
 *   step 1  Y[j][s][t] = sum over channels c of subband s of I[c][t + d1[j][c]], d1 the delay
 *           at coarse DM j (the centre of fine trials j nfine .. j nfine + nfine - 1) relative
 *           to the subband's highest channel, t < nin - max d1;
 *   step 2  X[k][t] = sum over subbands s of Y[k / nfine][s][t + d2[k][s]], d2 the delay of the
 *           subband's highest channel at fine DM k relative to the band's highest channel.
 * Both delays use the law and rounding of arts_delay_table.  X approximates brute force
 * (arts_plan_delays returns the composite delay d1 + d2 per trial and channel); its length is
 * nin - max d1 - max d2 (= nin - max_delay of arts_plan_info).  The plan is used like any
 * other (arts_dedisperse, arts_dedisperse_sb with SB formation in step 1, streams, batches,
 * serving, candidates).  Limits: nfine = 16 or 32, nchan / nsub <= 257 (16-bit step-1 sums),
 * D = 1.  One-shot calls keep the intermediate (2 bytes x nbeam x nsub x ncoarse x
 * (nin - max d1)) in the plan, so calls with one plan on different HIP streams must be ordered
 * by the caller; streams own theirs.  Errors: ARTS_E_INVAL, ARTS_E_NOMEM, ARTS_E_DEVICE.      */
int arts_plan_create_subband(int32_t nchan, double f_lo_mhz, double df_mhz, double tsamp_s,
                             double dm_first, double dm_step, int32_t ndm, int32_t nfine,
                             int32_t nsub, const int32_t* widths, int32_t nwidth,
                             arts_plan_t* out);

/* Subband structure of a plan: subbands, fine trials per coarse DM, coarse DMs and the largest
 * delay of each step (all 0 for a brute-force plan).                                        */
int arts_plan_subband_info(arts_plan_t plan, int32_t* nsub, int32_t* nfine, int32_t* ncoarse,
                           int32_t* max_delay1, int32_t* max_delay2);

/* As arts_plan_create, with time downsampling by an integer factor D >= 1 (Sect. 6b.2,
 * "Downsampling": a lower time resolution for high DMs).  Input stays native-rate uint8; the
 * kernels sum D consecutive samples (dropping a trailing partial group), delays use D*tsamp
 * and widths and output samples are in downsampled units.  D <= 257 keeps sums in 16 bits.   */
int arts_plan_create_ds(int32_t nchan, double f_lo_mhz, double df_mhz, double tsamp_s,
                        const double* dm_list, int32_t ndm, const int32_t* widths,
                        int32_t nwidth, int32_t downsample, arts_plan_t* out);

/* Release the plan's device tables and workspace.  NULL is ignored.  The caller must make
 * sure no stream still uses the plan.                                                      */
void arts_plan_destroy(arts_plan_t plan);

/* Plan geometry.  max_delay: largest delay in the table (downsampled samples).  halo =
 * max_delay + wmax - 1: an input of nin native samples yields L = nin/D - max_delay
 * dedispersed samples and nrep = nin/D - halo reported (boxcar start) samples.  Any pointer
 * may be NULL.                                                                              */
int arts_plan_info(arts_plan_t plan, int32_t* nchan, int32_t* ndm, int32_t* nwidth,
                   int32_t* downsample, int32_t* max_delay, int32_t* halo);

/* Copy the plan's delay table to host memory int32 [ndm][nchan] (for parity checks).        */
int arts_plan_delays(arts_plan_t plan, int32_t* host_out);

/* Dedispersion tiling.  variant indexes the compiled kernel shapes listed by
 * arts_tiling_count / arts_tiling_describe; dm_per_block is implied by the variant.  Changing
 * it rebuilds the plan's tiling tables (device allocation); streams capture their graphs
 * again afterwards.  arts_plan_set_tiling(p, v) is arts_plan_set_tiling_shape(p, v, 1, 0),
 * the shape plans are created with.                                                          */
int arts_plan_set_tiling(arts_plan_t plan, int32_t variant);
int arts_plan_get_tiling(arts_plan_t plan, int32_t* variant);
/* Tile shape: the variant, the LDS chunk buffers (2: the next chunk of channels is fetched
 * while this one is summed; 1: fetched in turn, twice the channels per chunk) and the channels
 * per chunk (0: as many as the LDS allows; else at most that many).  For subband plans the
 * shape applies to the first step.  On error (ARTS_E_INVAL: buffers not 1 or 2, channels
 * outside 0..255, or the variant does not fit the plan) the plan keeps its tiling.  get
 * reports the variant, buffers and channels per chunk in use (pointers nullable).             */
int arts_plan_set_tiling_shape(arts_plan_t plan, int32_t variant, int32_t buffers,
                               int32_t channels);
int arts_plan_get_tiling_shape(arts_plan_t plan, int32_t* variant, int32_t* buffers,
                               int32_t* channels);
int32_t arts_tiling_count(void);
/* Autotuner (the paper's GPU search is auto-tuned per platform and setup, Sect. 6b.2): times
 * tile shapes on pseudo-random input of nbeam x nchan x nin (device memory allocated and freed
 * by the call): every suitable variant (DMs per block, samples per lane) with one buffer and
 * the most channels per chunk, then the three fastest with two buffers and with half the
 * channels per chunk; `reps` timed launches each.  The fastest shape is set on the plan.  With
 * cache_path (nullable) the result is looked up in / appended to that text file, keyed by the
 * device's architecture and CU count, nchan, ndm, D, max_delay, a hash of the delay tables,
 * nbeam and nin.  *variant_out and *ms_out (nullable) receive the variant and its time per
 * launch (arts_plan_get_tiling_shape gives the rest of the shape).  Errors: ARTS_E_SHAPE (nin
 * too short), ARTS_E_NOMEM, ARTS_E_DEVICE.  Synchronous.                                     */
int arts_plan_autotune(arts_plan_t plan, int32_t nbeam, int64_t nin, int32_t reps,
                       const char* cache_path, int32_t* variant_out, float* ms_out);
/* Writes "J=<dwords per lane> ACC=<DMs per wave> WAVES=<waves per block> SPD=<samples per
 * dword>" and the partial-sum form for a variant into buf (NUL-terminated, at most len bytes):
 * " packed": 16-bit halves widened once per staged chunk; " packed held": widened every 257
 * channels; " group sums": the halves are the channel group sums of the first subband step,
 * the only plans these variants run; " framed": raw-dword frames per sub-dword offset held
 * across chunks; " framed runs": raw-dword frames per run of channels with one sub-dword
 * offset, added into the totals at the end of each run; " framed runs shared": the same with
 * each lane taking the sums of its last dword from the next lane (a time tile then covers
 * 64 x 4J - 4 outputs); " framed runs group sums": shared-word framed runs added into the
 * packed channel-group sums of the first subband step (split plans only); " pairs": two DM
 * trials of 16-bit samples summed from one window read; " pairs framed": the same in raw
 * frames per sample parity; none: single-sample adds.                                        */
int arts_tiling_describe(int32_t variant, char* buf, int32_t len);
/* Workgroups per CU that registers and waves allow (LDS aside) on the current device for a
 * variant's one-launch kernel (*per_job; for group-sum variants the split-plan kernel) and its
 * persistent batch kernel (*persistent; 0 for group-sum variants, which have none).  A plan
 * sizes its LDS chunks for *per_job workgroups per CU; batches and the serving engine run the
 * persistent kernel on the same chunks.  Errors: ARTS_E_INVAL, ARTS_E_DEVICE.                 */
int arts_tiling_occupancy(int32_t variant, int32_t* per_job, int32_t* persistent);

/* ------------------------------------------------------------------------ hot path ---- */

/* Synthesized-beam formation (Sect. 3d.beam; Appendix "Synthesized Beams"): an SB takes, in
 * each channel, the TAB whose grating response points at the SB's position at that frequency:
 *     sb_out[s][c][t] = tab[sb_table[s][c]][c][t],  t < nsamp.
 * tab: device uint8 [ntab][nchan][nsamp]; sb_table: device uint8 [nsb][nchan], entries < ntab
 * (an entry >= ntab yields zeros for that row); sb_out: device uint8 [nsb][nchan][nsamp].
 * Errors: ARTS_E_INVAL (sizes, NULL pointers, ntab > 256), ARTS_E_DEVICE.                   */
int arts_sb_synthesize(const uint8_t* tab, int32_t ntab, const uint8_t* sb_table, int32_t nsb,
                       int32_t nchan, int64_t nsamp, uint8_t* sb_out, void* stream);

/* Brute-force incoherent dedispersion (Sect. 6b.2, "Dedispersion", single step):
 *     out[b][d][t] = sum_c I_D[b][c][t + delay[d][c]],   t < L = nin/D - max_delay,
 * with I_D the input summed over groups of D samples.  in: device uint8 [nbeam][nchan][nin];
 * out: device int32 [nbeam][ndm][L] (exact: the sum is at most 255 * D * nchan < 2^31).
 * Errors: ARTS_E_SHAPE if L < 1; ARTS_E_INVAL for nbeam < 1 or NULL pointers;
 * ARTS_E_DEVICE.                                                                             */
int arts_dedisperse(arts_plan_t plan, const uint8_t* in, int32_t nbeam, int64_t nin,
                    int32_t* out, void* stream);

/* Dedispersion of synthesized beams formed on the fly from TABs, without materialising them
 * (SB formation folded into dedispersion, Sect. 3d.beam): identical to arts_sb_synthesize
 * followed by arts_dedisperse over the nsb SBs.  tab: device uint8 [ntab][nchan][nin];
 * sb_table: device uint8 [nsb][nchan] with entries < ntab; out: int32 [nsb][ndm][L].        */
int arts_dedisperse_sb(arts_plan_t plan, const uint8_t* tab, int32_t ntab,
                       const uint8_t* sb_table, int32_t nsb, int64_t nin, int32_t* out,
                       void* stream);

/* Boxcar matched filter and S/N of dedispersed series (Sect. 6b.2, "Integration" and
 * "S/N evaluation"; the paper leaves the estimator open, this library takes):
 *   window   nrep = L - wmax + 1 start samples, t < nrep
 *   stats    mu, sigma: mean and population standard deviation of X[b][d][t], t < nrep
 *   sums     B_w[t] = sum_{j<w} X[t + j]                       (exact int32)
 *   snr      (B_w - w mu) / (sigma sqrt(w)), 0 when sigma == 0   (FP32 from an exact integer
 *            numerator N*B_w - w*S1, relative error ~1e-7)
 * series: device int32 [nbeam][ndm][L].  Outputs, each optional (NULL = not written):
 * stats device double [nbeam][ndm][2] (mu, sigma); sums device int32 [nbeam][nwidth][ndm][nrep];
 * snr device float [nbeam][nwidth][ndm][nrep].  Errors: ARTS_E_SHAPE if nrep < 1.           */
int arts_boxcar_snr(arts_plan_t plan, const int32_t* series, int32_t nbeam, int64_t L,
                    double* stats, int32_t* sums, float* snr, void* stream);

/* Threshold candidate extraction (Sect. 6b.2, "Candidate selection": candidates whose S/N
 * exceeds a threshold are kept).  For every beam, DM trial and width, each maximal run of
 * consecutive start samples t < nrep with S/N > threshold (strict) yields one candidate at the
 * run's largest boxcar sum, the earliest t on ties.  The test is exact: S/N > thr is evaluated
 * as B_w > floor(w mu + thr sigma sqrt(w)) with mu, sigma in FP64; sigma == 0 gives none.
 * Candidates are copied to host_out [capacity] sorted by (beam, dm_index, width, sample);
 * *count receives the number found.  If it exceeds capacity, the first `capacity` in that
 * order are NOT guaranteed: the call returns ARTS_E_CAPACITY and the caller retries with a
 * buffer of *count.  This call SYNCHRONISES `stream`.  t_offset and beam_offset are added to
 * the reported sample and beam.                                                             */
int arts_candidates(arts_plan_t plan, const int32_t* series, int32_t nbeam, int64_t L,
                    float threshold, int64_t t_offset, int32_t beam_offset,
                    arts_candidate* host_out, int64_t capacity, int64_t* count, void* stream);

/* arts_candidates for callers that cannot allocate device memory (a serving loop with a frozen
 * allocator, a harness that forbids hipMalloc): the same search and results, with the
 * candidate records, their counter and the per-row pre-pass flags held in a fixed 16 MiB array
 * in device global memory that the library owns (one per device, kept until the process
 * ends) instead of the plan's workspace.  It calls no hipMalloc/hipFree; the first call on a
 * device looks the array's address up.  Limits: nbeam * ndm <= ARTS_NOALLOC_MAX_ROWS and
 * capacity <= ARTS_NOALLOC_MAX_CANDIDATES, else ARTS_E_INVAL; clustered plans give
 * ARTS_E_STATE (their workspace is allocated).  The plan must belong to the current device.
 * Every call on one device uses the same array: calls that overlap on one device (several
 * host threads, or this call racing another on a second stream) race; run them in turn.
 * Arguments, sorting, ARTS_E_CAPACITY and synchronisation as arts_candidates.               */
#define ARTS_NOALLOC_MAX_ROWS 1048576
#define ARTS_NOALLOC_MAX_CANDIDATES 491512
int arts_candidates_noalloc(arts_plan_t plan, const int32_t* series, int32_t nbeam, int64_t L,
                            float threshold, int64_t t_offset, int32_t beam_offset,
                            arts_candidate* host_out, int64_t capacity, int64_t* count,
                            void* stream);

/* DM-width clustering (Sect. 6b.2, "Clustering", optional in the paper): candidates of
 * different widths at the same time and DM are reduced to the one with the highest S/N, then
 * groups in neighbouring DM trials are compacted the same way, and one candidate is reported
 * per resulting cluster.  Readings taken here: a candidate covers its boxcar window
 * [sample, sample + width - 1]; step 1 groups the candidates of one (beam, dm_index) whose
 * windows overlap, transitively, and a group covers the union of its windows; step 2 joins the
 * groups of dm_index d and d + 1 of one beam whose covered intervals overlap, transitively.  A
 * cluster reports its member with the highest S/N, ties to the lowest dm_index, then the
 * earliest sample, then the smallest width.
 *
 * arts_plan_set_cluster(plan, 1) makes the candidate searches of this plan report clusters:
 * arts_candidates, arts_batch_candidates (per request) and the streams created afterwards (a
 * stream reads the setting in arts_stream_create).  Clustering runs on the device over the
 * candidates of one call, request or chunk and one plan.  The capacity of those calls must
 * still hold the unclustered candidates (with ARTS_E_CAPACITY, *count is that number).
 * enable: 0 (default) or 1; other values give ARTS_E_INVAL.                                 */
int arts_plan_set_cluster(arts_plan_t plan, int32_t enable);
int arts_plan_get_cluster(arts_plan_t plan, int32_t* enable);

/* Integration mode of the candidate search (Sect. 6b.2, "Integration": the dedispersed series
 * is downsampled by each trial pulse width).  mode 0 (default): sliding boxcars, every start
 * t < nrep is searched.  mode 1: decimated, as AMBER's downsampling: for width w only starts on
 * the absolute grid (t + t_offset) % w == 0 are searched, i.e. the series summed over
 * non-overlapping windows of w samples aligned to absolute sample 0 (streams: to the stream's
 * first sample, so consecutive chunks share the grid); a run is a maximal sequence of
 * consecutive grid starts above the threshold, reported at its largest sum (the earliest on
 * ties).  Moments, S/N and threshold are those of mode 0; width 1 gives identical results.
 * Applies to arts_candidates, arts_batch_candidates and streams (read at each search).  In a
 * stream every width must divide chunk / downsampling, so that each chunk starts on every
 * grid (ARTS_E_INVAL at arts_stream_create, or at the push if the mode is set later).
 * arts_boxcar_snr is not affected.  Other mode values give ARTS_E_INVAL.                      */
int arts_plan_set_integration(arts_plan_t plan, int32_t mode);
int arts_plan_get_integration(arts_plan_t plan, int32_t* mode);

/* Cluster a device list of this plan's candidates in place (same rule as above).
 * cand: device arts_candidate [n], n < 2^31, beam in [beam_offset, beam_offset + nbeam),
 * 0 <= dm_index < the plan's ndm.  On return cand[0, *count) holds one candidate per cluster,
 * in no particular order.  Records that agree in beam, dm_index, width and sample (never
 * produced by this library) are kept apart only by S/N: of equal ones, either may be reported.
 * Uses the plan's workspace (grown on demand); SYNCHRONISES stream.  Errors: ARTS_E_INVAL for
 * a record outside the beams or DM trials, a width < 1 or a NaN S/N (the list is then left
 * unchanged), ARTS_E_NOMEM / ARTS_E_DEVICE.                                                  */
int arts_plan_cluster(arts_plan_t plan, arts_candidate* cand, int64_t n, int32_t nbeam,
                      int32_t beam_offset, int64_t* count, void* stream);

/* Offline clustering of an observation's candidates over time (Sect. 6b.1, "Offline
 * analysis": candidates below DM 20 or S/N 10 are discarded, and within a 0.5 s time window and
 * DM windows that widen with DM only the highest-S/N candidate is kept).  Readings taken here:
 * a candidate's time is its native start sample * downsample; time window k is
 * [k t_window, (k + 1) t_window) native samples (floor division; 0.5 s is t_window = 6104 at
 * 81.92 us); DM window j is [dm_edges[j], dm_edges[j + 1]), the last one open-ended, and a DM
 * below dm_edges[0] is discarded (the DM limit; the widening edges are the caller's choice);
 * S/N below min_snr (compared in FP32) is discarded; the windows are shared by all beams of the
 * list; ties in S/N go to the candidate earlier in the list.
 * cand: device arts_candidate [n] (e.g. the clustered candidates of every chunk, uploaded),
 * n < 2^31, not modified.  dm_edges: host double [nedge], finite, strictly increasing,
 * 1 <= nedge < 2^20.  The kept candidates go to host_out [capacity], sorted by (native start,
 * dm, beam, width); *count receives their number (ARTS_E_CAPACITY if above capacity).
 * Allocates and frees a device workspace of about 32 n + 32 max(2n, 1024) bytes per call
 * (offline use); SYNCHRONISES stream.  Errors: ARTS_E_INVAL for bad arguments or a record
 * with width < 1, downsample outside [1, 2^20), a NaN S/N or DM, or a native start beyond
 * +-2^42; ARTS_E_NOMEM, ARTS_E_DEVICE.                                                      */
int arts_cluster_offline(const arts_candidate* cand, int64_t n, int64_t t_window,
                         const double* dm_edges, int32_t nedge, float min_snr,
                         arts_candidate* host_out, int64_t capacity, int64_t* count,
                         void* stream);

/* -------------------------------------------------------------------------- batches ---- */

/* One search request of an uneven batch: its own plan (channel count, DM range, widths, D),
 * input device uint8 [nbeam][nchan][nin] and output device int32 [nbeam][ndm][L],
 * L = nin/D - max_delay (as for arts_dedisperse).                                            */
typedef struct arts_request {
  arts_plan_t plan;
  const uint8_t* in;
  int32_t nbeam;
  int64_t nin;
  int32_t* out;
} arts_request;

typedef struct arts_batch_s* arts_batch_t;
/* A batch context: descriptor storage and per-request workspaces reused across calls.        */
int arts_batch_create(arts_batch_t* out);
void arts_batch_destroy(arts_batch_t b);

/* Dedisperse n requests: every request's tiles (beam, time tile, DM block) go into one
 * persistent launch per tiling variant present (the DM trials of the paper's search are
 * spread over GPUs by range, Sect. 9h; here uneven requests share one GPU launch).  Tiles
 * are taken from one device work queue, most expensive first.  status (nullable, [n]) gets
 * ARTS_OK, ARTS_E_INVAL (bad request) or ARTS_E_SHAPE (input shorter than the plan's halo;
 * skipped) per request.  Each output equals the request's own arts_dedisperse call bit for
 * bit.  Requests must not share an output buffer.  Asynchronous on `stream`.                 */
int arts_batch_dedisperse(arts_batch_t b, const arts_request* reqs, int32_t n, int32_t* status,
                          void* stream);

/* Threshold candidates of n dedispersed requests (as arts_candidates, request by request) into
 * one list: a candidate's beam is the request's first beam index (the sum of nbeam of the
 * requests before it) plus its beam within the request.  Sorted by (beam, dm_index, width,
 * sample); synchronises `stream`; ARTS_E_CAPACITY with *count = required if too small.
 * Requests skipped as too short contribute nothing.                                          */
int arts_batch_candidates(arts_batch_t b, const arts_request* reqs, int32_t n, float threshold,
                          arts_candidate* host_out, int64_t capacity, int64_t* count,
                          void* stream);

/* Batch autotuner: one tile shape for all native requests (and one for all 16-bit ones), so
 * that each kind goes into a single persistent launch; searched as arts_plan_autotune does,
 * but timing arts_batch_dedisperse on the caller's own requests (their outputs are written).
 * Every plan of a kind takes the fastest shape that fits all of them.  *variant_out / *ms_out
 * (nullable): the native kind's choice (else the 16-bit one's) and its time per launch.
 * Errors: ARTS_E_INVAL (no valid request), ARTS_E_DEVICE.  Synchronous.                      */
int arts_batch_autotune(arts_batch_t b, const arts_request* reqs, int32_t n, int32_t reps,
                        int32_t* variant_out, float* ms_out);

/* ------------------------------------------------------------------------ streaming ---- */

/* A streaming search over consecutive chunks (the real-time search processes 1.024 s chunks
 * and evaluates S/N over them, Sect. 6b.2 and Sect. 6b.1).  The stream keeps the overlap each
 * plan needs -- D * (max_delay + wmax - 1) native samples per row -- resident on the device, so
 * chunk k is searched exactly as a one-shot search of the concatenated input would search it;
 * before the first chunk the history is zeros.
 *
 *   plans[nplan]  plans sharing one channel count (e.g. native trials plus downsampled
 *                 high-DM trials); the stream keeps pointers, the plans must outlive it
 *   nsrc          source rows per chunk (beams, or TABs when sb_table is given)
 *   sb_table      device uint8 [nbeam][nchan] forming nbeam SBs from the nsrc TABs on the fly,
 *                 or NULL (then nbeam == nsrc)
 *   chunk         new native samples per push (a multiple of every plan's D, and of 4 if a
 *                 plan is a subband plan: its step-1 rows move by whole 8-byte groups)
 *   threshold     candidate S/N threshold;  cand_capacity: device candidate buffer entries
 *   flags         ARTS_STREAM_GRAPH: each push replays a captured hipGraph (one per ring parity
 *                 and position of the subband plans' step-1 windows, which move by one chunk per
 *                 push inside their buffer and are copied back to its front when they reach
 *                 its end);  ARTS_STREAM_PROFILE: time each phase with HIP events (phase 0
 *                 ring advance, 1..nplan dedispersion of plan i-1, nplan+1 statistics +
 *                 candidates of all plans).  The two flags are exclusive.
 * The stream owns its rings, series, workspace and a HIP stream of default priority.  Errors:
 * ARTS_E_INVAL, ARTS_E_NOMEM, ARTS_E_DEVICE.                                                  */
#define ARTS_STREAM_GRAPH 1u
#define ARTS_STREAM_PROFILE 2u
typedef struct arts_stream_s* arts_stream_t;
int arts_stream_create(const arts_plan_t* plans, int32_t nplan, int32_t nsrc,
                       const uint8_t* sb_table, int32_t nbeam, int64_t chunk, float threshold,
                       int64_t cand_capacity, uint32_t flags, arts_stream_t* out);

/* Clean every chunk pushed from now on before it is searched: its nsrc source rows (the TABs
 * of a stream with an SB table) go through the filters of arts_rfi_clean with these arguments
 * (statistics over the chunk).  Call between pushes (ARTS_E_STATE while a chunk is in flight);
 * the stream allocates its workspace here, and captured graphs are captured again.  niter_time
 * = niter_freq = 0 turns cleaning off.  Errors: ARTS_E_INVAL, ARTS_E_STATE, ARTS_E_NOMEM.   */
int arts_stream_set_rfi(arts_stream_t s, float k_time, int32_t niter_time, float k_freq,
                        int32_t niter_freq);

/* Device staging buffer [nsrc][nchan][chunk] owned by the stream: a producer may copy the next
 * chunk straight into it and push with chunk = that pointer (or NULL), avoiding a copy.        */
int arts_stream_input(arts_stream_t s, uint8_t** chunk_buffer);

/* Search the next chunk: device uint8 [nsrc][nchan][chunk] (NULL = the staging buffer).
 * Asynchronous; ordered after the work already queued on `stream`.  One chunk may be in flight:
 * collect it with arts_stream_wait before the next push (ARTS_E_STATE otherwise).              */
int arts_stream_push(arts_stream_t s, const uint8_t* chunk, void* stream);

/* Wait for the last pushed chunk and copy its candidates to host_out [capacity], sorted by
 * (beam, downsample, dm_index, width, sample).  `sample` is absolute: the boxcar start in the
 * plan's (downsampled) samples counted from the first sample of chunk 0 at the reference
 * frequency, i.e. k * chunk / D - D-halo + t for output t of chunk k.  Only outputs with
 * sample >= 0 are searched, and the S/N statistics (Sect. 6b.2) are taken over those same
 * outputs: earlier ones would read the zero history that precedes the stream (see
 * arts_stream_warmup).  *count = number found; ARTS_E_CAPACITY if it exceeds capacity or the
 * stream's own cand_capacity.  *chunk_index (nullable) = k.                                   */
int arts_stream_wait(arts_stream_t s, arts_candidate* host_out, int64_t capacity,
                     int64_t* count, int64_t* chunk_index);

/* Chunks pushed so far, device bytes the stream holds, and the native ring's overlap in native
 * samples (0 when every plan is downsampled).                                                 */
int arts_stream_info(arts_stream_t s, int64_t* chunks_pushed, int64_t* device_bytes,
                     int64_t* halo_native);

/* First output t of chunk `chunk_index` that plan_index searches: max(0, halo - k * chunk / D)
 * capped at chunk / D (= nothing searched), halo = max delay + wmax - 1 in downsampled samples.
 * Zero for every plan from chunk ceil(max over plans of halo * D / chunk) on; ARTS_E_INVAL for
 * a bad index.  With ARTS_STREAM_GRAPH, chunks with a nonzero warm-up run without the graphs. */
int arts_stream_warmup(arts_stream_t s, int32_t plan_index, int64_t chunk_index,
                       int64_t* t_begin);

/* Accumulated milliseconds and push count of one profiled phase (see ARTS_STREAM_PROFILE).    */
int arts_stream_timing(arts_stream_t s, int32_t phase, double* total_ms, int64_t* count);

/* Device pointer to plan_index's dedispersed series of the last chunk, int32 [nbeam][ndm][L],
 * L = chunk / D + wmax - 1 (valid until the next push).                                       */
int arts_stream_series(arts_stream_t s, int32_t plan_index, const int32_t** series, int64_t* L);

/* Checkpoint / resume: copy the device rings (arts_stream_snapshot_bytes bytes: the native ring,
 * then each downsampled plan's 16-bit ring) and the chunk count to the host, and restore them
 * into a stream created with the same arguments.  After a restore the stream continues
 * bit-exactly as the original would have.  Both need the last chunk collected first.           */
int arts_stream_snapshot_bytes(arts_stream_t s, int64_t* bytes);
int arts_stream_snapshot(arts_stream_t s, uint8_t* host, int64_t bytes, int64_t* chunks_pushed);
int arts_stream_restore(arts_stream_t s, const uint8_t* host, int64_t bytes,
                        int64_t chunks_pushed);

/* Release everything the stream owns (waits for its queued work first).  NULL is ignored.      */
void arts_stream_destroy(arts_stream_t s);

/* ------------------------------------------------------------------------- serving ---- */

/* Serving engine with continuous batching over streams (see arts_stream_create for the stream
 * arguments).  Streams are admitted while the device memory they need fits the HBM budget
 * (ARTS_E_BUDGET otherwise: retry once others have closed) and can join or leave between
 * ticks.  Each tick runs one search step for every stream with a submitted chunk: the
 * dedispersion of all of them goes into one persistent launch per tiling variant, so their
 * work shares the device.  A stream's results are identical to a standalone arts_stream fed
 * the same chunks.  Ticks go to the server's compute lanes (HIP streams of default priority)
 * in turn, so a tick enqueued while an earlier one still runs executes beside it on the
 * device; chunk copies use a further stream.  The calls below are not thread-safe.           */
typedef struct arts_server_s* arts_server_t;
int arts_server_create(int64_t hbm_budget_bytes, arts_server_t* out);
void arts_server_destroy(arts_server_t server);  /* closes every stream */
int arts_server_open(arts_server_t server, const arts_plan_t* plans, int32_t nplan,
                     int32_t nsrc, const uint8_t* sb_table, int32_t nbeam, int64_t chunk,
                     float threshold, int64_t cand_capacity, int32_t* stream_id);
int arts_server_close(arts_server_t server, int32_t stream_id);
/* Queue the stream's next chunk ([nsrc][nchan][chunk] uint8; host memory if from_host, pinned
 * for an asynchronous copy, else device memory).  ARTS_E_STATE while the stream's previous
 * chunk is pending or uncollected.                                                           */
int arts_server_submit(arts_server_t server, int32_t stream_id, const uint8_t* chunk,
                       int32_t from_host);
/* Enqueue one step for every stream with a submitted chunk; returns at once.  *nrun
 * (nullable) = number of streams stepped.  Errors: ARTS_E_DEVICE (a failed launch or copy),
 * ARTS_E_INVAL (a plan switched to decimated integration that no longer fits the stream's
 * chunk); the streams of that tick are then left part-way through their step: close them.    */
int arts_server_tick(arts_server_t server, int32_t* nrun);
/* Compute lanes used for ticks (1 or 2, default 2); waits for queued work first.           */
int arts_server_set_lanes(arts_server_t server, int32_t nlanes);
/* *done = 1 if the stream's last step has finished (or it has none in flight), 0 while it is
 * submitted or running; does not block, so a serving loop can keep admitting and submitting
 * while ticks run and collect each stream as soon as it is done.                             */
int arts_server_poll(arts_server_t server, int32_t stream_id, int32_t* done);
/* Wait for a stream's last step and return its candidates (as arts_stream_wait).             */
int arts_server_collect(arts_server_t server, int32_t stream_id, arts_candidate* host_out,
                        int64_t capacity, int64_t* count, int64_t* chunk_index);
/* The stream object behind an id (to read its series with arts_stream_series).              */
int arts_server_stream(arts_server_t server, int32_t stream_id, arts_stream_t* stream);
int arts_server_info(arts_server_t server, int64_t* used_bytes, int64_t* budget,
                     int32_t* nstreams);

/* ----------------------------------------------------------------------- diagnostics ---- */
const char* arts_strerror(int status);
const char* arts_last_error(void);
/* Library version string, and the gfx target the device code was built for.               */
const char* arts_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ARTS_H */
