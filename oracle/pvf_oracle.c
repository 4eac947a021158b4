/*
 * FP64 CPU oracle of the hybrid PVFinder inference path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * statement of what the path computes, used to check the HIP implementation.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product library never links or calls it, and it
 * shares no code, header or constant table with the product library.
 *
 * Every step follows the paper (arXiv:2602.19959):
 *   Section 2: nine features per track; a 400 mm region cut into 40 intervals
 *              of 100 bins; an FC network per track whose outputs are combined
 *              into the histogram; a UNet CNN; heuristic local-maximum peak
 *              finding with thresholds.
 *   Section 3: a track feeds the interval that holds it and, as a variant,
 *              a boundary track also feeds the neighbouring interval; the
 *              CNN input can also be batched by interval ([intervals, C,
 *              bins]) instead of one sequence per event.
 * Where the paper is silent the reading used is stated at the function.
 * Arithmetic is double precision throughout, starting from the float32
 * input values and float32 parameters.  Loops are direct: no blocking, no
 * fusion, no reordering of any sum beyond the order written here.
 *
 * Parameter vector: every tensor in the network's draw order (a weight then
 * its bias; MLP layers, then encoder levels 0..n-1 with conv1, conv2, then
 * decoder levels n-2..0 with the transposed conv, conv1, conv2, then the
 * head), each stored as float32 in the layouts linear [out][in],
 * conv [Cout][Cin][k], transposed conv [Cin][Cout][k].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- binning */

/* Interval index of a track, Section 2 (fixed spatial slicing).
 * Reading: interval i is the half-open [z_min + w*i, z_min + w*(i+1)); the
 * edges are integers in mm, so comparing on the float32 value is exact.  A
 * track outside the window, or with z not finite, belongs to no interval
 * (returns -1). */
int orc_bin(float z, double z_min, double interval_mm, int n_intervals)
{
    double zd = (double)z;
    if (!isfinite(zd)) return -1;
    for (int i = 0; i < n_intervals; ++i) {
        double lo = z_min + interval_mm * i;
        double hi = z_min + interval_mm * (i + 1);
        if (zd >= lo && zd < hi) return i;
    }
    return -1;
}

/* Non-zero when all nine features are finite (a track with a non-finite
 * feature is dropped, like a track outside the window). */
int orc_track_finite(const float *f, int n_feat, int64_t stride)
{
    for (int k = 0; k < n_feat; ++k)
        if (!isfinite((double)f[k * stride])) return 0;
    return 1;
}

/* Network input features of one track (reading of the silent preprocessing):
 * g0 = offset of z inside its interval mapped to [-1, 1),
 * gk = (fk - shift_k) * scale_k for the other features. */
void orc_features(const float *f, int64_t stride, int n_feat, int i,
                  double z_min, double interval_mm,
                  const float *shift, const float *scale, double *g)
{
    double lo = z_min + interval_mm * i;
    g[0] = ((double)f[0] - lo) / (interval_mm / 2.0) - 1.0;
    for (int k = 1; k < n_feat; ++k)
        g[k] = ((double)f[k * stride] - (double)shift[k]) * (double)scale[k];
}

/* ---------------------------------------------------------------- FC stage */

static double leaky(double x, double slope) { return x >= 0.0 ? x : slope * x; }

static double softplus(double x)
{
    /* log(1 + e^x), written to stay exact for large |x| */
    return (x > 0.0 ? x : 0.0) + log1p(exp(-fabs(x)));
}

/* y = W x + b for W [n_out][n_in] (float32), in double. */
static void linear(const double *x, int n_in, const float *W, const float *b,
                   int n_out, double *y)
{
    for (int o = 0; o < n_out; ++o) {
        double s = (double)b[o];
        for (int i = 0; i < n_in; ++i) s += (double)W[(int64_t)o * n_in + i] * x[i];
        y[o] = s;
    }
}

/* Number of floats the MLP occupies at the start of the parameter vector. */
int64_t orc_mlp_param_count(int n_feat, int hidden, int n_hidden, int n_out)
{
    int64_t n = (int64_t)hidden * n_feat + hidden;
    n += (int64_t)(n_hidden - 1) * (hidden * hidden + hidden);
    n += (int64_t)n_out * hidden + n_out;
    return n;
}

/* The per-track FC network of Section 2 ("six FC layers"): n_hidden layers of
 * width `hidden`, each LeakyReLU, then a linear layer of width n_out (one
 * value per bin of the interval) through softplus, so every contribution to
 * the histogram is positive. */
void orc_mlp(const double *g, const float *params, int n_feat, int hidden,
             int n_hidden, int n_out, double slope, double *out)
{
    double a[256], h[256];
    const float *p = params;
    int n_in = n_feat;
    memcpy(a, g, sizeof(double) * n_feat);
    for (int l = 0; l < n_hidden; ++l) {
        const float *W = p; p += (int64_t)hidden * n_in;
        const float *b = p; p += hidden;
        linear(a, n_in, W, b, hidden, h);
        for (int j = 0; j < hidden; ++j) a[j] = leaky(h[j], slope);
        n_in = hidden;
    }
    const float *W = p; p += (int64_t)n_out * n_in;
    const float *b = p;
    linear(a, n_in, W, b, n_out, out);
    for (int j = 0; j < n_out; ++j) out[j] = softplus(out[j]);
}

/* Histogram of one event, Section 2 (the FC outputs of all tracks are
 * combined into one histogram): H[n_out*i + j] is the sum over the tracks in
 * interval i of their output j, in track order; bins of intervals with no
 * track are exactly 0.  `f` points at the event's first track in plane 0 and
 * `stride` is the plane stride.  Returns the number of dropped tracks. */
/* Boundary tracks (Section 3 lets a track feed one or two intervals; the
 * paper gives no rule, this is the reading taken): a track closer than
 * boundary_mm to an edge of its interval that is shared with another
 * interval also feeds that neighbour.  Returns the neighbour's index, or -1
 * (boundary_mm <= 0, far from both edges, or the edge ends the histogram).
 * The distances are taken in double, like the binning. */
int orc_neighbour(float z, int i, double z_min, double interval_mm, int n_intervals, double boundary_mm)
{
    if (!(boundary_mm > 0.0) || i < 0) return -1;
    double zd = (double)z;
    double lo = z_min + interval_mm * i;
    double hi = z_min + interval_mm * (i + 1);
    if (zd - lo < boundary_mm && i > 0) return i - 1;
    if (hi - zd < boundary_mm && i < n_intervals - 1) return i + 1;
    return -1;
}

/* Histogram of one event: H [n_intervals][n_out] (zeroed here).  Each kept
 * track adds its network outputs to the bins of its interval; with
 * boundary_mm > 0 a boundary track also adds the network's outputs for the
 * neighbouring interval, its features taken in that interval's frame (the z
 * feature then lies just outside [-1, 1)).  Returns the number of dropped
 * tracks. */
int orc_histogram(const float *f, int64_t stride, int n_tracks, const float *params,
                  int n_feat, int hidden, int n_hidden, int n_out,
                  double z_min, double interval_mm, int n_intervals,
                  const float *shift, const float *scale, double slope, double boundary_mm, double *H)
{
    double g[64], o[1024];
    int dropped = 0;
    memset(H, 0, sizeof(double) * (size_t)n_out * n_intervals);
    for (int t = 0; t < n_tracks; ++t) {
        const float *ft = f + t;
        int i = orc_track_finite(ft, n_feat, stride)
                    ? orc_bin(ft[0], z_min, interval_mm, n_intervals) : -1;
        if (i < 0) { ++dropped; continue; }
        orc_features(ft, stride, n_feat, i, z_min, interval_mm, shift, scale, g);
        orc_mlp(g, params, n_feat, hidden, n_hidden, n_out, slope, o);
        for (int j = 0; j < n_out; ++j) H[(int64_t)n_out * i + j] += o[j];
        int nb = orc_neighbour(ft[0], i, z_min, interval_mm, n_intervals, boundary_mm);
        if (nb < 0) continue;
        orc_features(ft, stride, n_feat, nb, z_min, interval_mm, shift, scale, g);
        orc_mlp(g, params, n_feat, hidden, n_hidden, n_out, slope, o);
        for (int j = 0; j < n_out; ++j) H[(int64_t)n_out * nb + j] += o[j];
    }
    return dropped;
}

/* ---------------------------------------------------------------- UNet ops */

/* 1D cross-correlation with zero "same" padding (odd k):
 * y[o][t] = b[o] + sum_c sum_j W[o][c][j] * x[c][t + j - (k-1)/2],
 * x[c][s] = 0 outside [0, L).  x is [Cin][L], y is [Cout][L]. */
void orc_conv1d(const double *x, int Cin, int L, const float *W, const float *b,
                int Cout, int k, double *y)
{
    int r = (k - 1) / 2;
    for (int o = 0; o < Cout; ++o)
        for (int t = 0; t < L; ++t) {
            double s = (double)b[o];
            for (int c = 0; c < Cin; ++c)
                for (int j = 0; j < k; ++j) {
                    int u = t + j - r;
                    if (u < 0 || u >= L) continue;
                    s += (double)W[((int64_t)o * Cin + c) * k + j] * x[(int64_t)c * L + u];
                }
            y[(int64_t)o * L + t] = s;
        }
}

void orc_leaky_inplace(double *x, int64_t n, double slope)
{
    for (int64_t i = 0; i < n; ++i) x[i] = leaky(x[i], slope);
}

/* Max-pool of width 2 and stride 2: y[c][t] = max(x[c][2t], x[c][2t+1]). */
void orc_maxpool2(const double *x, int C, int L, double *y)
{
    int Lo = L / 2;
    for (int c = 0; c < C; ++c)
        for (int t = 0; t < Lo; ++t) {
            double a = x[(int64_t)c * L + 2 * t], b = x[(int64_t)c * L + 2 * t + 1];
            y[(int64_t)c * Lo + t] = a > b ? a : b;
        }
}

/* Transposed convolution with 2 taps and stride 2 (the decoder's upsampling):
 * y[o][2t + j] = b[o] + sum_c W[c][o][j] * x[c][t], j in {0, 1}.
 * x is [Cin][L], y is [Cout][2L], W is [Cin][Cout][2]. */
void orc_convT2(const double *x, int Cin, int L, const float *W, const float *b,
                int Cout, double *y)
{
    for (int o = 0; o < Cout; ++o)
        for (int t = 0; t < L; ++t)
            for (int j = 0; j < 2; ++j) {
                double s = (double)b[o];
                for (int c = 0; c < Cin; ++c)
                    s += (double)W[((int64_t)c * Cout + o) * 2 + j] * x[(int64_t)c * L + t];
                y[(int64_t)o * 2 * L + 2 * t + j] = s;
            }
}

/* Floats held by one activation stored by orc_unet in its tap buffer. */
static int64_t act(int C, int L) { return (int64_t)C * L; }

/* Size in doubles of the tap buffer orc_unet fills (every intermediate
 * activation, channels-first, in this order): per encoder level l:
 * conv1, conv2 (the skip), then the pooled map for l < n-1; per decoder level
 * l = n-2..0: the transposed conv output, conv1, conv2; finally the logit. */
int64_t orc_unet_tap_count(int L, int n_levels, int c0)
{
    int64_t n = 0;
    for (int l = 0; l < n_levels; ++l) {
        int C = c0 << l, Ll = L >> l;
        n += 2 * act(C, Ll);
        if (l < n_levels - 1) n += act(C, Ll / 2);
    }
    for (int l = n_levels - 2; l >= 0; --l) {
        int C = c0 << l, Ll = L >> l;
        n += 3 * act(C, Ll);
    }
    return n + L;
}

/* The UNet of Section 2: the encoder halves the length and doubles the
 * channels at each level, the decoder upsamples back, joining each level's
 * skip, and a 1x1 head gives one logit per bin.
 * Readings: every 5-tap conv is followed by LeakyReLU; no pool after the
 * deepest level; the transposed conv has no activation; the concatenation
 * puts the skip channels first; the head has no activation (the caller
 * applies the sigmoid).
 * x0 is the [L] network input (already scaled), params points at the first
 * UNet tensor, logit is [L].  taps, if not NULL, receives every activation
 * (orc_unet_tap_count doubles).  Returns 0, or -1 when out of memory. */
int orc_unet(const double *x0, int L, const float *params, int n_levels, int c0,
             int k, double slope, double *logit, double *taps)
{
    const float *p = params;
    double *skip[16] = {0};
    double *x = (double *)malloc(sizeof(double) * L);
    if (!x) return -1;
    memcpy(x, x0, sizeof(double) * L);
    int cin = 1, Ll = L;
    double *tp = taps;

    for (int l = 0; l < n_levels; ++l) {
        int C = c0 << l;
        double *a = (double *)malloc(sizeof(double) * act(C, Ll));
        double *s = (double *)malloc(sizeof(double) * act(C, Ll));
        if (!a || !s) return -1;
        const float *W1 = p; p += (int64_t)C * cin * k; const float *b1 = p; p += C;
        const float *W2 = p; p += (int64_t)C * C * k;   const float *b2 = p; p += C;
        orc_conv1d(x, cin, Ll, W1, b1, C, k, a);
        orc_leaky_inplace(a, act(C, Ll), slope);
        orc_conv1d(a, C, Ll, W2, b2, C, k, s);
        orc_leaky_inplace(s, act(C, Ll), slope);
        if (tp) { memcpy(tp, a, sizeof(double) * act(C, Ll)); tp += act(C, Ll);
                  memcpy(tp, s, sizeof(double) * act(C, Ll)); tp += act(C, Ll); }
        free(a);
        free(x);
        skip[l] = s;
        if (l < n_levels - 1) {
            x = (double *)malloc(sizeof(double) * act(C, Ll / 2));
            if (!x) return -1;
            orc_maxpool2(s, C, Ll, x);
            if (tp) { memcpy(tp, x, sizeof(double) * act(C, Ll / 2)); tp += act(C, Ll / 2); }
            Ll /= 2;
        } else {
            x = s;
        }
        cin = C;
    }
    /* x is the deepest skip; keep the pointer owned by skip[n-1]. */
    for (int l = n_levels - 2; l >= 0; --l) {
        int C = c0 << l, Cup = c0 << (l + 1);
        int Lo = Ll * 2;
        const float *WT = p; p += (int64_t)Cup * C * 2; const float *bT = p; p += C;
        const float *W1 = p; p += (int64_t)C * 2 * C * k; const float *b1 = p; p += C;
        const float *W2 = p; p += (int64_t)C * C * k;     const float *b2 = p; p += C;
        double *cat = (double *)malloc(sizeof(double) * act(2 * C, Lo));
        double *a = (double *)malloc(sizeof(double) * act(C, Lo));
        double *y = (double *)malloc(sizeof(double) * act(C, Lo));
        if (!cat || !a || !y) return -1;
        memcpy(cat, skip[l], sizeof(double) * act(C, Lo));
        orc_convT2(x, Cup, Ll, WT, bT, C, cat + act(C, Lo));
        if (tp) { memcpy(tp, cat + act(C, Lo), sizeof(double) * act(C, Lo)); tp += act(C, Lo); }
        orc_conv1d(cat, 2 * C, Lo, W1, b1, C, k, a);
        orc_leaky_inplace(a, act(C, Lo), slope);
        orc_conv1d(a, C, Lo, W2, b2, C, k, y);
        orc_leaky_inplace(y, act(C, Lo), slope);
        if (tp) { memcpy(tp, a, sizeof(double) * act(C, Lo)); tp += act(C, Lo);
                  memcpy(tp, y, sizeof(double) * act(C, Lo)); tp += act(C, Lo); }
        free(cat);
        free(a);
        if (x != skip[l + 1]) free(x);
        free(skip[l + 1]);
        skip[l + 1] = NULL;
        x = y;
        Ll = Lo;
    }
    free(skip[0]);
    /* 1x1 head: logit[t] = b + sum_c w[c] x[c][t] */
    const float *Wh = p; p += c0; const float *bh = p;
    for (int t = 0; t < L; ++t) {
        double s = (double)bh[0];
        for (int c = 0; c < c0; ++c) s += (double)Wh[c] * x[(int64_t)c * L + t];
        logit[t] = s;
    }
    if (tp) memcpy(tp, logit, sizeof(double) * L);
    free(x);
    return 0;
}

double orc_sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* ---------------------------------------------------------------- peaks */

/* Heuristic peak finding of Section 2 (local maxima with thresholds) on the
 * per-bin probability p[0..L).  Readings: a candidate is a strict local
 * maximum p[t-1] < p[t] > p[t+1] with 1 <= t <= L-2 and p[t] > p_min; its
 * window is [t-hw, t+hw] clipped to the histogram; S = plain sum of p over
 * the window; the candidate is a vertex when S > s_min; its position is the
 * p-weighted mean of the window's bin centres z_min + bw*(j + 0.5).
 * Windows may overlap (no suppression).  Vertices come out in ascending t.
 * Writes at most max_out vertices; returns how many there are in total. */
int orc_peaks(const double *p, int L, double z_min, double bw, double p_min,
              double s_min, int hw, int max_out, int *t_out, double *z_out,
              double *prob_out, double *integral_out)
{
    int n = 0;
    for (int t = 1; t + 1 < L; ++t) {
        if (!(p[t - 1] < p[t] && p[t] > p[t + 1])) continue;
        if (!(p[t] > p_min)) continue;
        int lo = t - hw < 0 ? 0 : t - hw;
        int hi = t + hw > L - 1 ? L - 1 : t + hw;
        double S = 0.0, M = 0.0;
        for (int j = lo; j <= hi; ++j) {
            S += p[j];
            M += p[j] * (z_min + bw * (j + 0.5));
        }
        if (!(S > s_min)) continue;
        if (n < max_out) {
            if (t_out) t_out[n] = t;
            if (z_out) z_out[n] = M / S;
            if (prob_out) prob_out[n] = p[t];
            if (integral_out) integral_out[n] = S;
        }
        ++n;
    }
    return n;
}

/* ---------------------------------------------------------------- event */

/* The whole path for one event: histogram -> input scale -> UNet -> sigmoid
 * -> peaks.  Geometry: n_intervals intervals of n_out bins of width bw
 * starting at z_min (L = n_intervals * n_out bins).  layout 0 runs the UNet
 * once over all L bins; layout 1 (the interval-batched [intervals, C, bins]
 * form of Section 3) runs it on every interval's n_out bins on their own,
 * with zero padding at the interval edges, and concatenates the logits.
 * Outputs H [L], logit [L], p [L] and up to max_out vertices; returns the
 * vertex count, or -1 on an allocation failure.  *dropped receives the
 * number of dropped tracks. */
int orc_event(const float *f, int64_t stride, int n_tracks, const float *params,
              int n_feat, int hidden, int n_hidden, int n_out,
              int n_levels, int c0, int k, double slope, double s_in,
              const float *shift, const float *scale,
              double z_min, double bw, int n_intervals, double boundary_mm, int layout,
              double p_min, double s_min, int hw, int max_out,
              double *H, double *logit, double *p, int *dropped,
              int *t_out, double *z_out, double *prob_out, double *integral_out)
{
    int L = n_intervals * n_out;
    double interval_mm = bw * n_out;
    int d = orc_histogram(f, stride, n_tracks, params, n_feat, hidden, n_hidden, n_out,
                          z_min, interval_mm, n_intervals, shift, scale, slope, boundary_mm, H);
    if (dropped) *dropped = d;
    double *x0 = (double *)malloc(sizeof(double) * L);
    if (!x0) return -1;
    for (int t = 0; t < L; ++t) x0[t] = s_in * H[t];
    const float *unet = params + orc_mlp_param_count(n_feat, hidden, n_hidden, n_out);
    int rc = 0;
    if (layout == 1) {
        for (int i = 0; i < n_intervals && rc == 0; ++i)
            rc = orc_unet(x0 + (int64_t)i * n_out, n_out, unet, n_levels, c0, k, slope,
                          logit + (int64_t)i * n_out, NULL);
    } else {
        rc = orc_unet(x0, L, unet, n_levels, c0, k, slope, logit, NULL);
    }
    free(x0);
    if (rc != 0) return -1;
    for (int t = 0; t < L; ++t) p[t] = orc_sigmoid(logit[t]);
    return orc_peaks(p, L, z_min, bw, p_min, s_min, hw, max_out,
                     t_out, z_out, prob_out, integral_out);
}
